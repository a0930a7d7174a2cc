"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad descriptors before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1703_10119_amd import dfhm, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dfhm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dfhm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = dfhm.load()
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dfhm.EXPORTS)


def test_struct_sizes_match_header_layout():
    # 12 doubles per layer, 4 per sinusoid; int32 pairs where declared
    assert C.sizeof(dfhm.Layer) == 12 * 8
    assert C.sizeof(dfhm.Sine) == 4 * 8
    assert C.sizeof(dfhm.Wall) == 8 + 3 * 96 + 8 * 8 + 4 * 32 + 3 * 8 + 2 * 8 + 2 * 32
    assert C.sizeof(dfhm.Room) == 4 * 8 + 2 * 32 + 8 + 8 + 2 * 8 + 8
    assert dfhm._LAYER_ORDER == wl.LAYER_FIELDS


def _cfg(dt=1.0):
    c = dfhm.Config()
    c.dt_s = dt
    return c


def _create(walls, cfg):
    L = dfhm.load()
    arr = dfhm.walls_struct(walls)
    h = C.c_void_p()
    st = L.dfhm_create(C.byref(cfg), arr, len(walls["nx"]), None, 0, C.byref(h))
    return st, h


@pytest.mark.parametrize("mutate", [
    lambda w: w["nx"].__setitem__(0, 2),
    lambda w: w["nx"].__setitem__(0, 4096),
    lambda w: w["n_layers"].__setitem__(0, 4),
    lambda w: w["layer"].__setitem__((0, 0, 0), -0.1),
    lambda w: w["layer"].__setitem__((0, 0, 6), 0.0),
    lambda w: w["hT"].__setitem__((0, 0), -1.0),
    lambda w: w["Tamb"].__setitem__((0, 0, 2), 0.0),
    lambda w: w["RH0"].__setitem__(0, 0.0),
    lambda w: w["T0"].__setitem__(0, float("nan")),
])
def test_bad_descriptor_is_rejected_before_device_use(mutate):
    w = wl.single_wall()
    mutate(w)
    st, h = _create(w, _cfg())
    assert st == 1 and not h.value


def test_bad_config_is_rejected():
    w = wl.single_wall()
    for bad in (dict(dt_s=0.0), dict(dt_s=-1.0), dict(precision=5), dict(startup=3),
                dict(schedule=9), dict(chunk_steps=-2)):
        c = _cfg()
        for k, v in bad.items():
            setattr(c, k, v)
        st, h = _create(w, c)
        assert st == 1 and not h.value, bad


def test_null_arguments():
    L = dfhm.load()
    h = C.c_void_p()
    assert L.dfhm_create(None, None, 0, None, 0, C.byref(h)) == 1
    assert L.dfhm_step_n(None, 1) == 1
    assert L.dfhm_step_index(None) == -1
    assert L.dfhm_status_string(6) == b"unstable explicit zone step"
    L.dfhm_destroy(None)


def test_arena_size_accounts_for_levels():
    L = dfhm.load()
    w = wl.uniform_batch(4, nx=1001)
    arr = dfhm.walls_struct(w)
    c64, c32 = _cfg(), _cfg()
    c32.precision = dfhm.FP32
    b64 = L.dfhm_arena_bytes(C.byref(c64), arr, 4)
    b32 = L.dfhm_arena_bytes(C.byref(c32), arr, 4)
    assert b64 >= 4 * 4 * 1001 * 8 and b32 >= 4 * 4 * 1001 * 4 and b64 > b32
