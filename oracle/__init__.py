"""Plain FP64 CPU oracle for the Dufort-Frankel hygrothermal wall / room method.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product library never imports,
links or runs anything from here; the two share no code, only the seeded input
arrays of the workload generator.

The arithmetic lives in ``dfhm_ref.c`` (built to ``libdfhm_ref.so`` with plain
``gcc -O2``, no fast-math, no FMA contraction); this module only marshals the
generator's arrays into that library's own structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfhm_ref.c")
_LIB = os.path.join(_HERE, "libdfhm_ref.so")

LAYER_FIELDS = ("thick", "k0", "aT", "kM0", "aM", "bTM", "c0", "cT", "cM0",
                "aC", "eTM", "fTM")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over walls)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Layer(C.Structure):
    _fields_ = [(n, C.c_double) for n in LAYER_FIELDS]


class _Sine(C.Structure):
    _fields_ = [("mean", C.c_double), ("amp", C.c_double),
                ("period", C.c_double), ("phase", C.c_double)]


class _Wall(C.Structure):
    _fields_ = [("nx", C.c_int32), ("n_layers", C.c_int32),
                ("layer", _Layer * 3),
                ("hT", C.c_double * 2), ("hM", C.c_double * 2),
                ("qinf", C.c_double * 2), ("ginf", C.c_double * 2),
                ("Tamb", _Sine * 2), ("RHamb", _Sine * 2),
                ("T0", C.c_double), ("RH0", C.c_double), ("area", C.c_double),
                ("emis", C.c_double * 2), ("qsun", _Sine * 2),
                ("law", C.c_int32), ("pad_law", C.c_int32), ("Lv", C.c_double), ("cw", C.c_double)]


class _Room(C.Structure):
    _fields_ = [("volume", C.c_double), ("ach", C.c_double), ("T0", C.c_double),
                ("RH0", C.c_double), ("Tout", _Sine), ("RHout", _Sine),
                ("n_sched", C.c_int32), ("sched_dt", C.c_double),
                ("g_o", C.POINTER(C.c_double)), ("Q_h", C.POINTER(C.c_double)),
                ("view", C.c_double)]


class _Cfg(C.Structure):
    _fields_ = [("dt", C.c_double), ("Lv", C.c_double), ("cw", C.c_double),
                ("rho_a", C.c_double), ("c_pa", C.c_double), ("c_pv", C.c_double),
                ("Pv_ref", C.c_double), ("startup", C.c_int32), ("law", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # DFHM_REF_LIB names another build of dfhm_ref.c: the mutation tests
        # load copies of the oracle with a planted mistake this way
        path = os.environ.get("DFHM_REF_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(path):
                build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.ref_create.restype = P
        L.ref_create.argtypes = [C.POINTER(_Cfg), C.POINTER(_Wall), C.c_int64,
                                 C.POINTER(_Room), C.c_int64, P, P]
        L.ref_destroy.argtypes = [P]
        L.ref_step.argtypes = [P, C.c_int64, C.c_int]
        L.ref_step_index.restype = C.c_int64
        L.ref_step_index.argtypes = [P]
        L.ref_set_step_index.argtypes = [P, C.c_int64]
        L.ref_total_nodes.restype = C.c_int64
        L.ref_total_nodes.argtypes = [P]
        L.ref_get_fields.argtypes = [P, C.c_int64, C.c_int, P, P]
        L.ref_set_fields.argtypes = [P, C.c_int64, C.c_int, P, P]
        L.ref_get_fluxes.argtypes = [P, P, P]
        L.ref_get_rooms.argtypes = [P, P, P]
        L.ref_get_layers.argtypes = [P, C.c_int64, P]
        L.ref_get_coeffs.argtypes = [P, C.c_int64, P, P]
        L.ref_startup_substeps.restype = C.c_int64
        L.ref_startup_substeps.argtypes = [P, C.c_int64]
        L.ref_psat.restype = C.c_double
        L.ref_psat.argtypes = [C.c_double]
        L.ref_set_links.argtypes = [P, P, P, P, C.c_int64]
        L.ref_implicit_run.restype = C.c_double
        L.ref_implicit_run.argtypes = [C.POINTER(_Wall), C.c_double, C.c_double,
                                       C.c_int64, C.c_double, C.c_double, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _fill_sine(s, row):
    s.mean, s.amp, s.period, s.phase = (float(x) for x in row)


def _walls_struct(walls: dict):
    W = len(walls["nx"])
    arr = (_Wall * max(W, 1))()
    lay = np.asarray(walls["layer"], np.float64)
    # radiation inputs are optional in a wall set (absent = none)
    emis = walls.get("emis", np.zeros((W, 2)))
    qsun = walls.get("qsun")
    if qsun is None:
        qsun = np.zeros((W, 2, 4))
        qsun[..., 2] = 86400.0
    for w in range(W):
        x = arr[w]
        x.nx = int(walls["nx"][w])
        x.n_layers = int(walls["n_layers"][w])
        for l in range(3):
            for i, n in enumerate(LAYER_FIELDS):
                setattr(x.layer[l], n, float(lay[w, l, i]))
        for s in range(2):
            x.hT[s] = float(walls["hT"][w, s])
            x.hM[s] = float(walls["hM"][w, s])
            x.qinf[s] = float(walls["qinf"][w, s])
            x.ginf[s] = float(walls["ginf"][w, s])
            _fill_sine(x.Tamb[s], walls["Tamb"][w, s])
            _fill_sine(x.RHamb[s], walls["RHamb"][w, s])
            x.emis[s] = float(emis[w, s])
            _fill_sine(x.qsun[s], qsun[w, s])
        x.T0 = float(walls["T0"][w])
        x.RH0 = float(walls["RH0"][w])
        x.area = float(walls["area"][w])
    return arr


def _cfg_struct(cfg: dict):
    c = _Cfg()
    for n in ("dt", "Lv", "cw", "rho_a", "c_pa", "c_pv", "Pv_ref"):
        setattr(c, n, float(cfg[n]))
    c.startup = int(cfg.get("startup", 0))
    c.law = int(cfg.get("law", 0))
    return c


def psat(T: float) -> float:
    """Magnus saturation pressure of the oracle (Pa)."""
    return lib().ref_psat(float(T))


class RefSim:
    """A batch of walls (and optionally rooms) advanced by the oracle."""

    def __init__(self, walls: dict, cfg: dict, rooms: dict | None = None):
        L = lib()
        self.W = len(walls["nx"])
        self.nx = np.asarray(walls["nx"], np.int64)
        self._walls = _walls_struct(walls)
        self._cfg = _cfg_struct(cfg)
        self.R = 0
        room_arr = None
        self._keep = []
        if rooms is not None:
            self.R = len(rooms["volume"])
            room_arr = (_Room * max(self.R, 1))()
            for r in range(self.R):
                x = room_arr[r]
                x.volume = float(rooms["volume"][r])
                x.ach = float(rooms["ach"][r])
                x.T0 = float(rooms["T0"][r])
                x.RH0 = float(rooms["RH0"][r])
                _fill_sine(x.Tout, rooms["Tout"][r])
                _fill_sine(x.RHout, rooms["RHout"][r])
                go = np.ascontiguousarray(rooms["g_o"][r], np.float64)
                qh = np.ascontiguousarray(rooms["Q_h"][r], np.float64)
                self._keep += [go, qh]
                x.n_sched = len(go)
                x.sched_dt = float(rooms["sched_dt"][r])
                x.g_o = go.ctypes.data_as(C.POINTER(C.c_double))
                x.Q_h = qh.ctypes.data_as(C.POINTER(C.c_double))
                x.view = float(rooms["view"][r]) if "view" in rooms else 0.0
        self._wr = np.ascontiguousarray(walls.get("wall_room", np.full(self.W, -1)), np.int64)
        self._rs = np.ascontiguousarray(walls.get("room_side", np.ones(self.W)), np.int8)
        if rooms is None:
            self._wr[:] = -1
        self._h = L.ref_create(C.byref(self._cfg), self._walls, self.W,
                               room_arr, self.R, _ptr(self._wr), _ptr(self._rs))
        if not self._h:
            raise MemoryError("oracle create failed")
        if rooms is not None and len(rooms.get("link_a", ())) > 0:
            la = np.ascontiguousarray(rooms["link_a"], np.int32)
            lb = np.ascontiguousarray(rooms["link_b"], np.int32)
            lg = np.ascontiguousarray(rooms["link_g"], np.float64)
            L.ref_set_links(self._h, _ptr(la), _ptr(lb), _ptr(lg), len(la))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ref_destroy(h)
            self._h = None

    @property
    def n(self) -> int:
        return lib().ref_step_index(self._h)

    @n.setter
    def n(self, value: int):
        lib().ref_set_step_index(self._h, int(value))

    def step(self, nsteps: int, threads: int = 0):
        lib().ref_step(self._h, int(nsteps), int(threads))

    def fields(self, w: int, level: int = 0):
        nx = int(self.nx[w])
        T = np.empty(nx)
        P = np.empty(nx)
        lib().ref_get_fields(self._h, int(w), int(level), _ptr(T), _ptr(P))
        return T, P

    def set_fields(self, w: int, level: int, T, P):
        T = np.ascontiguousarray(T, np.float64)
        P = np.ascontiguousarray(P, np.float64)
        lib().ref_set_fields(self._h, int(w), int(level), _ptr(T), _ptr(P))

    def all_fields(self, level: int = 0):
        """Concatenated (T, P) of all walls, wall after wall."""
        Ts, Ps = zip(*(self.fields(w, level) for w in range(self.W)))
        return np.concatenate(Ts), np.concatenate(Ps)

    def fluxes(self):
        now = np.empty((self.W, 2, 2))
        integ = np.empty((self.W, 2, 2))
        lib().ref_get_fluxes(self._h, _ptr(now), _ptr(integ))
        return now, integ

    def rooms(self):
        Ta = np.empty(max(self.R, 1))
        Pa = np.empty(max(self.R, 1))
        lib().ref_get_rooms(self._h, _ptr(Ta), _ptr(Pa))
        return Ta[: self.R], Pa[: self.R]

    def layers(self, w: int):
        lay = np.empty(int(self.nx[w]), np.int32)
        lib().ref_get_layers(self._h, int(w), _ptr(lay))
        return lay

    def coeffs(self, w: int):
        nx = int(self.nx[w])
        node = np.empty((nx, 3))
        face = np.empty((nx - 1, 3))
        lib().ref_get_coeffs(self._h, int(w), _ptr(node), _ptr(face))
        return node, face

    def startup_substeps(self, w: int) -> int:
        return lib().ref_startup_substeps(self._h, int(w))


def implicit_run(walls: dict, w: int, dt: float, Lv: float, nsteps: int,
                 theta: float = 0.5, eta: float = 1e-12, law: int = 0, cw: float = 4180.0):
    """Theta-scheme comparator with fixed-point sub-iterations on wall ``w``
    (law 0: the shape law; 1: the Table 1 material).

    Returns (T, P, mean fixed-point iterations per step)."""
    one = {k: (v[w:w + 1] if hasattr(v, "__len__") else v) for k, v in walls.items()}
    arr = _walls_struct(one)
    arr[0].law, arr[0].Lv, arr[0].cw = int(law), float(Lv), float(cw)
    nx = int(walls["nx"][w])
    T = np.empty(nx)
    P = np.empty(nx)
    it = lib().ref_implicit_run(arr, float(dt), float(Lv), int(nsteps), float(theta),
                                float(eta), _ptr(T), _ptr(P))
    return T, P, it
