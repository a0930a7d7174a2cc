"""Checkpoint / restart through the C ABI (dfhm_save / dfhm_load), on the GPU.

A context restored from a checkpoint must continue exactly -- bit for bit --
as the context that wrote it: the DF recurrence needs only levels n and n-1,
and everything else that evolves (flux sums and their compensations, the
zone air) is in the checkpoint.  Runs cross chunk boundaries and both level
parities.  A checkpoint of other walls or another precision is refused.
"""
import numpy as np
import pytest

from paper_1703_10119_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1703_10119_amd import dfhm  # noqa: E402

CASES = [(p, s) for p in (dfhm.FP64, dfhm.FP32) for s in (dfhm.SCHED_RESIDENT, dfhm.SCHED_STREAM)]


def state(s):
    T0, P0 = s.all_fields(0)
    T1, P1 = s.all_fields(1)
    now, integ = s.fluxes()
    out = [T0, P0, T1, P1, now, integ]
    if s.R:
        out += list(s.rooms())
    return out


@pytest.mark.parametrize("prec,sched", CASES)
@pytest.mark.parametrize("before", [137, 0, 1])
def test_restart_continues_bit_identically(prec, sched, before):
    walls = wl.layered_batch(24, seed=31, dt=2.0)
    cfg = wl.default_config(dt=2.0)
    a = dfhm.Solver(walls, cfg, precision=prec, schedule=sched, chunk=50)
    a.step(before)
    ck = a.save()
    a.step(150)
    want = state(a)
    b = dfhm.Solver(walls, cfg, precision=prec, schedule=sched, chunk=50)
    b.step(3)                        # some other state first, other parity
    b.load(ck)
    assert b.n == before
    b.step(150)
    got = state(b)
    for x, y in zip(got, want):
        assert np.array_equal(x, y)
    # rewinding the context that wrote it
    a.load(ck)
    a.step(150)
    for x, y in zip(state(a), want):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_restart_with_zones():
    walls, rooms = wl.building_batch(3, seed=44, dt=10.0)
    cfg = wl.default_config(dt=10.0)
    a = dfhm.Solver(walls, cfg, rooms=rooms, schedule=dfhm.SCHED_RESIDENT)
    a.step(1201)
    ck = a.save()
    a.step(999)
    want = state(a)
    b = dfhm.Solver(walls, cfg, rooms=rooms, schedule=dfhm.SCHED_RESIDENT)
    b.load(ck)
    b.step(999)
    for x, y in zip(state(b), want):
        assert np.array_equal(x, y)


def test_checkpoint_of_other_walls_or_precision_is_refused():
    walls = wl.uniform_batch(4, seed=5, nx=51)
    cfg = wl.default_config(dt=1.0)
    a = dfhm.Solver(walls, cfg, precision=dfhm.FP64)
    a.step(10)
    ck = a.save()
    other = wl.uniform_batch(4, seed=6, nx=51)
    b = dfhm.Solver(other, cfg, precision=dfhm.FP64)
    with pytest.raises(dfhm.DfhmError):
        b.load(ck)
    c = dfhm.Solver(walls, cfg, precision=dfhm.FP32)
    with pytest.raises(dfhm.DfhmError):
        c.load(ck)
    with pytest.raises(dfhm.DfhmError):
        a.load(ck[:-8])
    bad = bytearray(ck)
    bad[0] ^= 1
    with pytest.raises(dfhm.DfhmError):
        a.load(bytes(bad))
    assert b.n == 0 and c.n == 0


def test_checkpoint_of_another_dt_or_zone_is_refused():
    """The digest covers the run constants and the zone descriptors: a
    checkpoint written at another dt (levels n and n-1 one old dt apart), or
    for a zone of another volume, another schedule or without its links, is
    refused and leaves the context unchanged."""
    walls, rooms = wl.building_batch(2, seed=46, dt=10.0)
    cfg = wl.default_config(dt=10.0)
    a = dfhm.Solver(walls, cfg, rooms=rooms, schedule=dfhm.SCHED_STREAM)
    a.step(25)
    ck = a.save()
    b = dfhm.Solver(walls, wl.default_config(dt=5.0), rooms=rooms, schedule=dfhm.SCHED_STREAM)
    with pytest.raises(dfhm.DfhmError):
        b.load(ck)
    assert b.n == 0
    r2 = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in rooms.items()}
    r2["volume"][1] *= 1.01
    c = dfhm.Solver(walls, cfg, rooms=r2, schedule=dfhm.SCHED_STREAM)
    with pytest.raises(dfhm.DfhmError):
        c.load(ck)
    r3 = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in rooms.items()}
    r3["g_o"][0, 5] += 1e-6
    d = dfhm.Solver(walls, cfg, rooms=r3, schedule=dfhm.SCHED_STREAM)
    with pytest.raises(dfhm.DfhmError):
        d.load(ck)
    w2 = {k: v.copy() for k, v in walls.items()}
    w2["Tamb"][3, 0, 1] += 0.5          # another outdoor amplitude
    e = dfhm.Solver(w2, cfg, rooms=rooms, schedule=dfhm.SCHED_STREAM)
    with pytest.raises(dfhm.DfhmError):
        e.load(ck)
    # the same setup accepts it
    f = dfhm.Solver(walls, cfg, rooms=rooms, schedule=dfhm.SCHED_STREAM)
    f.load(ck)
    assert f.n == 25
    for s in (a, b, c, d, e, f):
        s.close()
