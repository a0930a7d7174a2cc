"""Thin ctypes binding of ``include/dfhm.h`` (argument marshalling only).

Every step of the method runs in the HIP kernels of ``libdfhm.so``; this
module converts the workload arrays into the ABI's structs, hands device
memory (a torch tensor) and the current torch stream to the library, and
converts results back to numpy.  It raises if the library is missing: there
is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfhm.so")

FP64, FP32 = 0, 1
START_FTCS, START_REPEAT = 0, 1
SCHED_AUTO, SCHED_STREAM, SCHED_RESIDENT = 0, 1, 2

_LAYER_ORDER = ("thick", "k0", "aT", "kM0", "aM", "bTM", "c0", "cT", "cM0", "aC", "eTM", "fTM")


class DfhmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dfhm status {status}: {msg}")
        self.status = status


class Sine(C.Structure):
    _fields_ = [("mean", C.c_double), ("amp", C.c_double), ("period_s", C.c_double),
                ("phase", C.c_double)]


class Layer(C.Structure):
    _fields_ = [("thickness_m", C.c_double), ("k0", C.c_double), ("a_T", C.c_double),
                ("kM0", C.c_double), ("a_M", C.c_double), ("b_TM", C.c_double),
                ("c0", C.c_double), ("c_T", C.c_double), ("cM0", C.c_double),
                ("c_M", C.c_double), ("e_TM", C.c_double), ("f_TM", C.c_double)]


class Wall(C.Structure):
    _fields_ = [("nx", C.c_int32), ("n_layers", C.c_int32), ("layer", Layer * 3),
                ("h_T", C.c_double * 2), ("h_M", C.c_double * 2),
                ("q_inf", C.c_double * 2), ("g_inf", C.c_double * 2),
                ("T_amb", Sine * 2), ("RH_amb", Sine * 2),
                ("T0", C.c_double), ("RH0", C.c_double), ("area_m2", C.c_double),
                ("emissivity", C.c_double * 2), ("q_sun", Sine * 2)]


class Room(C.Structure):
    _fields_ = [("volume_m3", C.c_double), ("ach_per_h", C.c_double), ("T0", C.c_double),
                ("RH0", C.c_double), ("T_out", Sine), ("RH_out", Sine),
                ("n_sched", C.c_int32), ("sched_dt_s", C.c_double),
                ("g_o_kg_s", C.POINTER(C.c_double)), ("Q_h_W", C.POINTER(C.c_double)),
                ("view_factor", C.c_double)]


class Config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("startup", C.c_int32), ("schedule", C.c_int32),
                ("chunk_steps", C.c_int32), ("dt_s", C.c_double), ("Lv", C.c_double),
                ("cw", C.c_double), ("rho_a", C.c_double), ("c_pa", C.c_double),
                ("c_pv", C.c_double), ("Pv_ref", C.c_double), ("stream", C.c_void_p),
                ("block_threads", C.c_int32), ("nodes_per_thread", C.c_int32),
                ("use_graph", C.c_int32), ("law", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("precision", C.c_int32),
                ("block_threads", C.c_int32), ("nodes_per_thread", C.c_int32),
                ("chunk_steps", C.c_int32), ("n_blocks", C.c_int32),
                ("max_walls_per_block", C.c_int32), ("use_graph", C.c_int32),
                ("n_walls", C.c_int64), ("n_rooms", C.c_int64), ("total_nodes", C.c_int64),
                ("step_index", C.c_int64), ("pack_efficiency", C.c_double),
                ("max_rooms_per_block", C.c_int32), ("reserved", C.c_int32),
                ("n_links", C.c_int64)]


class ImplicitConfig(C.Structure):
    """dfhm_implicit_config"""
    _fields_ = [("dt_s", C.c_double), ("theta", C.c_double), ("eta", C.c_double),
                ("max_iters", C.c_int32), ("law", C.c_int32), ("Lv", C.c_double),
                ("stream", C.c_void_p), ("cw", C.c_double)]


class MlpConfig(C.Structure):
    """dfhm_mlp_config"""
    _fields_ = [("n_in", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("n_out", C.c_int32), ("max_batch", C.c_int32),
                ("seed", C.c_uint64), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("weight_decay", C.c_float), ("stream", C.c_void_p)]


class FeatureDesc(C.Structure):
    """dfhm_feature_desc"""
    _fields_ = [("n_hist", C.c_int32), ("stride", C.c_int32), ("dt_hist", C.c_float),
                ("T_mean", C.c_float), ("T_scale", C.c_float), ("RH_mean", C.c_float),
                ("RH_scale", C.c_float), ("p_mean", C.c_float * 8), ("p_scale", C.c_float * 8)]


class ZoneLink(C.Structure):
    _fields_ = [("zone_a", C.c_int32), ("zone_b", C.c_int32), ("g_kg_s", C.c_double)]


EXPORTS = ("dfhm_arena_bytes", "dfhm_create", "dfhm_room_couple", "dfhm_zone_links",
           "dfhm_step_n", "dfhm_sync",
           "dfhm_fluxes", "dfhm_get_fields", "dfhm_get_all_fields", "dfhm_set_fields",
           "dfhm_set_step_index", "dfhm_get_rooms", "dfhm_get_info", "dfhm_autotune",
           "dfhm_step_index", "dfhm_last_error", "dfhm_status_string", "dfhm_destroy",
           "dfhm_save", "dfhm_load",
           "dfhm_implicit_create", "dfhm_implicit_step_n", "dfhm_implicit_get_fields",
           "dfhm_implicit_iterations", "dfhm_implicit_step_index", "dfhm_implicit_destroy",
           "dfhm_mlp_create", "dfhm_mlp_param_count", "dfhm_mlp_get_params",
           "dfhm_mlp_set_params", "dfhm_mlp_forward", "dfhm_mlp_gradients",
           "dfhm_mlp_train_step", "dfhm_mlp_last_error", "dfhm_mlp_destroy",
           "dfhm_mlp_features", "dfhm_mlp_decode", "dfhm_mlp_decode_ensemble",
           "dfhm_mlp_get_intermediate", "dfhm_mlp_infer", "dfhm_mlp_infer_noalloc",
           "dfhm_mlp_infer_ensemble",
           "dfhm_mlp_noalloc_max_batch")

_lib = None


def load(path: str = LIB_PATH):
    """Load libdfhm.so and declare the ABI; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(path)
    P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
    L.dfhm_arena_bytes.restype = C.c_size_t
    L.dfhm_arena_bytes.argtypes = [C.POINTER(Config), C.POINTER(Wall), I64]
    L.dfhm_create.argtypes = [C.POINTER(Config), C.POINTER(Wall), I64, P, C.c_size_t,
                              C.POINTER(P)]
    L.dfhm_room_couple.argtypes = [P, C.POINTER(Room), I64, P, P]
    L.dfhm_zone_links.argtypes = [P, C.POINTER(ZoneLink), I64]
    L.dfhm_step_n.argtypes = [P, I64]
    L.dfhm_sync.argtypes = [P]
    L.dfhm_fluxes.argtypes = [P, P, P]
    L.dfhm_get_fields.argtypes = [P, I64, C.c_int, P, P]
    L.dfhm_get_all_fields.argtypes = [P, C.c_int, P, P]
    L.dfhm_set_fields.argtypes = [P, I64, C.c_int, P, P]
    L.dfhm_set_step_index.argtypes = [P, I64]
    L.dfhm_get_rooms.argtypes = [P, P, P]
    L.dfhm_get_info.argtypes = [P, C.POINTER(Info)]
    L.dfhm_autotune.argtypes = [P, I32]
    L.dfhm_step_index.restype = I64
    L.dfhm_step_index.argtypes = [P]
    L.dfhm_last_error.restype = C.c_char_p
    L.dfhm_last_error.argtypes = [P]
    L.dfhm_status_string.restype = C.c_char_p
    L.dfhm_status_string.argtypes = [C.c_int]
    L.dfhm_destroy.restype = None
    L.dfhm_destroy.argtypes = [P]
    for f in (L.dfhm_create, L.dfhm_room_couple, L.dfhm_zone_links, L.dfhm_step_n,
              L.dfhm_sync, L.dfhm_fluxes,
              L.dfhm_get_fields, L.dfhm_get_all_fields, L.dfhm_set_fields,
              L.dfhm_set_step_index, L.dfhm_get_rooms, L.dfhm_get_info, L.dfhm_autotune):
        f.restype = C.c_int
    L.dfhm_save.argtypes = [P, P, C.POINTER(C.c_size_t)]
    L.dfhm_load.argtypes = [P, P, C.c_size_t]
    L.dfhm_save.restype = C.c_int
    L.dfhm_load.restype = C.c_int
    L.dfhm_implicit_create.argtypes = [C.POINTER(ImplicitConfig), C.POINTER(Wall), I64, C.POINTER(P)]
    L.dfhm_implicit_step_n.argtypes = [P, I64]
    L.dfhm_implicit_get_fields.argtypes = [P, I64, P, P]
    L.dfhm_implicit_iterations.argtypes = [P, C.POINTER(C.c_double)]
    L.dfhm_implicit_step_index.restype = I64
    L.dfhm_implicit_step_index.argtypes = [P]
    L.dfhm_implicit_destroy.restype = None
    L.dfhm_implicit_destroy.argtypes = [P]
    for f in (L.dfhm_implicit_create, L.dfhm_implicit_step_n, L.dfhm_implicit_get_fields,
              L.dfhm_implicit_iterations):
        f.restype = C.c_int
    # surface-flux surrogate
    L.dfhm_mlp_create.argtypes = [C.POINTER(MlpConfig), C.POINTER(P)]
    L.dfhm_mlp_param_count.restype = I64
    L.dfhm_mlp_param_count.argtypes = [P]
    L.dfhm_mlp_get_params.argtypes = [P, P]
    L.dfhm_mlp_set_params.argtypes = [P, P]
    L.dfhm_mlp_forward.argtypes = [P, P, I64, P]
    L.dfhm_mlp_gradients.argtypes = [P, P, P, I64, P, P]
    L.dfhm_mlp_train_step.argtypes = [P, P, P, I64, C.c_float, P]
    L.dfhm_mlp_last_error.restype = C.c_char_p
    L.dfhm_mlp_last_error.argtypes = [P]
    L.dfhm_mlp_destroy.restype = None
    L.dfhm_mlp_destroy.argtypes = [P]
    L.dfhm_mlp_features.argtypes = [P, P, P, P, I64, C.POINTER(FeatureDesc), P, P]
    L.dfhm_mlp_decode.argtypes = [P, I64, P, C.c_float, P, P, P]
    L.dfhm_mlp_decode_ensemble.argtypes = [P, I32, I64, P, C.c_float, P, P, P]
    L.dfhm_mlp_infer.argtypes = [P, P, I64, P, P, P]
    L.dfhm_mlp_get_intermediate.argtypes = [P, I32, I32, I64, P]
    for f in (L.dfhm_mlp_create, L.dfhm_mlp_get_params, L.dfhm_mlp_set_params,
              L.dfhm_mlp_forward, L.dfhm_mlp_gradients, L.dfhm_mlp_train_step,
              L.dfhm_mlp_features, L.dfhm_mlp_decode, L.dfhm_mlp_decode_ensemble,
              L.dfhm_mlp_infer, L.dfhm_mlp_get_intermediate):
        f.restype = C.c_int
    L.dfhm_mlp_infer_ensemble.argtypes = [P, I32, P, I64, P, P, P]
    L.dfhm_mlp_infer_ensemble.restype = C.c_int
    L.dfhm_mlp_infer_noalloc.argtypes = [P, P, I64, P, P, P]
    L.dfhm_mlp_infer_noalloc.restype = C.c_int
    L.dfhm_mlp_noalloc_max_batch.argtypes = [P]
    L.dfhm_mlp_noalloc_max_batch.restype = I64
    _lib = L
    return L


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _sine(s, row):
    s.mean, s.amp, s.period_s, s.phase = (float(x) for x in row)


def _radiation(walls: dict, W: int):
    """Emissivities and incident sinusoids of a wall set (absent = none)."""
    emis = walls.get("emis")
    if emis is None:
        emis = np.zeros((W, 2))
    qsun = walls.get("qsun")
    if qsun is None:
        qsun = np.zeros((W, 2, 4))
        qsun[..., 2] = 86400.0
    return np.asarray(emis, np.float64), np.asarray(qsun, np.float64)


def walls_struct(walls: dict):
    """dfhm_wall array from a workload wall set."""
    W = len(walls["nx"])
    arr = (Wall * W)()
    emis, qsun = _radiation(walls, W)
    lay = np.asarray(walls["layer"], np.float64)
    fields = [f for f, _ in Layer._fields_]
    for w in range(W):
        x = arr[w]
        x.nx = int(walls["nx"][w])
        x.n_layers = int(walls["n_layers"][w])
        for l in range(3):
            for i, name in enumerate(fields):
                setattr(x.layer[l], name, float(lay[w, l, i]))
        for s in range(2):
            x.h_T[s] = float(walls["hT"][w, s])
            x.h_M[s] = float(walls["hM"][w, s])
            x.q_inf[s] = float(walls["qinf"][w, s])
            x.g_inf[s] = float(walls["ginf"][w, s])
            _sine(x.T_amb[s], walls["Tamb"][w, s])
            _sine(x.RH_amb[s], walls["RHamb"][w, s])
            x.emissivity[s] = float(emis[w, s])
            _sine(x.q_sun[s], qsun[w, s])
        x.T0 = float(walls["T0"][w])
        x.RH0 = float(walls["RH0"][w])
        x.area_m2 = float(walls["area"][w])
    return arr


def walls_struct_fast(walls: dict):
    """Same as walls_struct, filled through a structured numpy view (large W)."""
    W = len(walls["nx"])
    arr = (Wall * W)()
    buf = np.frombuffer(arr, dtype=np.uint8).reshape(W, C.sizeof(Wall))
    o_nx = Wall.nx.offset
    buf[:, o_nx:o_nx + 4] = np.asarray(walls["nx"], np.int32).view(np.uint8).reshape(W, 4)
    o_nl = Wall.n_layers.offset
    buf[:, o_nl:o_nl + 4] = np.asarray(walls["n_layers"], np.int32).view(np.uint8).reshape(W, 4)

    def put(off, vals):
        v = np.ascontiguousarray(vals, np.float64).reshape(W, -1)
        buf[:, off:off + 8 * v.shape[1]] = v.view(np.uint8).reshape(W, -1)

    put(Wall.layer.offset, np.asarray(walls["layer"], np.float64).reshape(W, -1))
    put(Wall.h_T.offset, walls["hT"])
    put(Wall.h_M.offset, walls["hM"])
    put(Wall.q_inf.offset, walls["qinf"])
    put(Wall.g_inf.offset, walls["ginf"])
    put(Wall.T_amb.offset, np.asarray(walls["Tamb"]).reshape(W, -1))
    put(Wall.RH_amb.offset, np.asarray(walls["RHamb"]).reshape(W, -1))
    put(Wall.T0.offset, walls["T0"])
    put(Wall.RH0.offset, walls["RH0"])
    put(Wall.area_m2.offset, walls["area"])
    emis, qsun = _radiation(walls, W)
    put(Wall.emissivity.offset, emis)
    put(Wall.q_sun.offset, qsun.reshape(W, -1))
    return arr


class Solver:
    """One dfhm context on the current HIP device.

    walls, rooms: workload dicts; cfg: dict with dt and the constants
    (``workloads.default_config``).  precision, schedule, startup, chunk,
    threads, npt, use_graph map to dfhm_config.  ``arena`` = "torch"
    allocates the wall state in a torch uint8 tensor (PyTorch owns the
    memory), None lets the library allocate."""

    def __init__(self, walls: dict, cfg: dict, rooms: dict | None = None, precision=FP64,
                 schedule=SCHED_AUTO, startup=None, chunk=0, threads=0, npt=0,
                 use_graph=0, arena="torch", stream=None):
        import torch
        L = load()
        self._torch = torch
        self.W = len(walls["nx"])
        self.nx = np.asarray(walls["nx"], np.int64)
        self.off = np.concatenate([[0], np.cumsum(self.nx)])
        self.N = int(self.off[-1])
        self.precision = precision
        c = Config()
        c.precision = precision
        c.startup = int(cfg.get("startup", 0) if startup is None else startup)
        c.schedule = schedule
        c.chunk_steps = int(chunk)
        c.dt_s = float(cfg["dt"])
        c.Lv = float(cfg.get("Lv", 0.0))
        c.cw = float(cfg.get("cw", 0.0))
        c.rho_a = float(cfg.get("rho_a", 0.0))
        c.c_pa = float(cfg.get("c_pa", 0.0))
        c.c_pv = float(cfg.get("c_pv", 0.0))
        c.Pv_ref = float(cfg.get("Pv_ref", 0.0))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        c.stream = stream
        c.block_threads = int(threads)
        c.nodes_per_thread = int(npt)
        c.use_graph = int(use_graph)
        c.law = int(cfg.get("law", 0))
        self._cfg = c
        self._walls = walls_struct_fast(walls) if self.W > 256 else walls_struct(walls)
        self._arena = None
        aptr, abytes = None, 0
        if arena == "torch":
            abytes = L.dfhm_arena_bytes(C.byref(c), self._walls, self.W)
            self._arena = torch.empty(abytes, dtype=torch.uint8, device="cuda")
            aptr = self._arena.data_ptr()
        h = C.c_void_p()
        st = L.dfhm_create(C.byref(c), self._walls, self.W, aptr, abytes, C.byref(h))
        if st != 0:
            raise DfhmError(st, "dfhm_create: " + L.dfhm_status_string(st).decode())
        self._h = h
        self.R = 0
        if rooms is not None:
            self._couple(walls, rooms)

    def _check(self, st, what):
        if st != 0:
            L = load()
            raise DfhmError(st, f"{what}: {L.dfhm_last_error(self._h).decode()}")

    def _couple(self, walls, rooms):
        L = load()
        R = len(rooms["volume"])
        arr = (Room * R)()
        self._keep = []
        for r in range(R):
            x = arr[r]
            x.volume_m3 = float(rooms["volume"][r])
            x.ach_per_h = float(rooms["ach"][r])
            x.T0 = float(rooms["T0"][r])
            x.RH0 = float(rooms["RH0"][r])
            _sine(x.T_out, rooms["Tout"][r])
            _sine(x.RH_out, rooms["RHout"][r])
            go = np.ascontiguousarray(rooms["g_o"][r], np.float64)
            qh = np.ascontiguousarray(rooms["Q_h"][r], np.float64)
            self._keep += [go, qh]
            x.n_sched = len(go)
            x.sched_dt_s = float(rooms["sched_dt"][r])
            x.g_o_kg_s = go.ctypes.data_as(C.POINTER(C.c_double))
            x.Q_h_W = qh.ctypes.data_as(C.POINTER(C.c_double))
            x.view_factor = float(rooms["view"][r]) if "view" in rooms else 0.0
        wr = np.ascontiguousarray(walls["wall_room"], np.int64)
        rs = np.ascontiguousarray(walls["room_side"], np.int8)
        self._check(L.dfhm_room_couple(self._h, arr, R, _ptr(wr), _ptr(rs)), "dfhm_room_couple")
        if len(rooms.get("link_a", ())) > 0:
            self.link_zones(rooms["link_a"], rooms["link_b"], rooms["link_g"])
        self.R = R

    def link_zones(self, a, b, g):
        """dfhm_zone_links: g[l] kg/s of dry air each way between zones a[l], b[l]."""
        n = len(a)
        arr = (ZoneLink * n)()
        for l in range(n):
            arr[l].zone_a, arr[l].zone_b, arr[l].g_kg_s = int(a[l]), int(b[l]), float(g[l])
        self._check(load().dfhm_zone_links(self._h, arr, n), "dfhm_zone_links")

    def close(self):
        if getattr(self, "_h", None):
            load().dfhm_destroy(self._h)
            self._h = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self) -> int:
        return int(load().dfhm_step_index(self._h))

    def step(self, nsteps: int):
        self._check(load().dfhm_step_n(self._h, int(nsteps)), "dfhm_step_n")

    def sync(self):
        self._check(load().dfhm_sync(self._h), "dfhm_sync")

    def fluxes(self):
        now = np.empty((self.W, 2, 2))
        integ = np.empty((self.W, 2, 2))
        self._check(load().dfhm_fluxes(self._h, _ptr(now), _ptr(integ)), "dfhm_fluxes")
        return now, integ

    def fields(self, w: int, level: int = 0):
        nx = int(self.nx[w])
        T = np.empty(nx)
        P = np.empty(nx)
        self._check(load().dfhm_get_fields(self._h, int(w), int(level), _ptr(T), _ptr(P)),
                    "dfhm_get_fields")
        return T, P

    def all_fields(self, level: int = 0):
        T = np.empty(self.N)
        P = np.empty(self.N)
        self._check(load().dfhm_get_all_fields(self._h, int(level), _ptr(T), _ptr(P)),
                    "dfhm_get_all_fields")
        return T, P

    def set_fields(self, w: int, level: int, T, P):
        T = np.ascontiguousarray(T, np.float64)
        P = np.ascontiguousarray(P, np.float64)
        self._check(load().dfhm_set_fields(self._h, int(w), int(level), _ptr(T), _ptr(P)),
                    "dfhm_set_fields")

    def set_step_index(self, n: int):
        self._check(load().dfhm_set_step_index(self._h, int(n)), "dfhm_set_step_index")

    def rooms(self):
        Ta = np.empty(self.R)
        Pa = np.empty(self.R)
        self._check(load().dfhm_get_rooms(self._h, _ptr(Ta), _ptr(Pa)), "dfhm_get_rooms")
        return Ta, Pa

    def info(self) -> dict:
        inf = Info()
        self._check(load().dfhm_get_info(self._h, C.byref(inf)), "dfhm_get_info")
        return {f: getattr(inf, f) for f, _ in Info._fields_}

    def save(self) -> bytes:
        """Checkpoint of the evolving state (dfhm_save)."""
        L = load()
        n = C.c_size_t(0)
        self._check(L.dfhm_save(self._h, None, C.byref(n)), "dfhm_save")
        buf = C.create_string_buffer(n.value)
        self._check(L.dfhm_save(self._h, buf, C.byref(n)), "dfhm_save")
        return buf.raw[:n.value]

    def load(self, ckpt: bytes):
        """Restore a checkpoint written by a context of the same walls (dfhm_load)."""
        buf = C.create_string_buffer(ckpt, len(ckpt))
        self._check(load().dfhm_load(self._h, buf, len(ckpt)), "dfhm_load")

    def autotune(self, probe_steps: int = 50):
        self._check(load().dfhm_autotune(self._h, int(probe_steps)), "dfhm_autotune")


class Implicit:
    """Batched implicit comparator (theta-scheme with fixed-point
    sub-iterations) on the current HIP device: dfhm_implicit_*."""

    def __init__(self, walls: dict, dt: float, theta: float = 1.0, eta: float = 1e-10,
                 max_iters: int = 200, Lv: float = 0.0, stream=None, law: int = 0,
                 cw: float = 0.0):
        import torch
        L = load()
        c = ImplicitConfig()
        c.dt_s, c.theta, c.eta, c.max_iters, c.Lv = float(dt), float(theta), float(eta), int(max_iters), float(Lv)
        c.law, c.cw = int(law), float(cw)
        c.stream = torch.cuda.current_stream().cuda_stream if stream is None else stream
        self.W = len(walls["nx"])
        self.nx = np.asarray(walls["nx"], np.int64)
        arr = walls_struct_fast(walls) if self.W > 256 else walls_struct(walls)
        h = C.c_void_p()
        st = L.dfhm_implicit_create(C.byref(c), arr, self.W, C.byref(h))
        if st != 0:
            raise DfhmError(st, "dfhm_implicit_create")
        self._h = h

    def step(self, nsteps: int):
        st = load().dfhm_implicit_step_n(self._h, int(nsteps))
        if st != 0:
            raise DfhmError(st, "dfhm_implicit_step_n")

    def fields(self, w: int):
        nx = int(self.nx[w])
        T = np.empty(nx)
        P = np.empty(nx)
        st = load().dfhm_implicit_get_fields(self._h, int(w), T.ctypes.data_as(C.c_void_p),
                                             P.ctypes.data_as(C.c_void_p))
        if st != 0:
            raise DfhmError(st, "dfhm_implicit_get_fields")
        return T, P

    def iterations(self) -> float:
        m = C.c_double(0.0)
        st = load().dfhm_implicit_iterations(self._h, C.byref(m))
        if st != 0:
            raise DfhmError(st, "dfhm_implicit_iterations")
        return m.value

    @property
    def n(self) -> int:
        return int(load().dfhm_implicit_step_index(self._h))

    def close(self):
        if getattr(self, "_h", None):
            load().dfhm_implicit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
