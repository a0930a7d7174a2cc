"""Seeded synthetic workloads for the wall / room batches.

This module only draws input parameters (geometry, material scales, surface
coefficients, outdoor sinusoids, room schedules) with ``numpy``'s PCG64
generator.  It holds none of the method's arithmetic, imports nothing from the
GPU library or the oracle, and is the one module both of them are fed from.

The paper (Sec. 4 and Sec. 6) drives its walls with measured weather and
material data that are only shown in figures; the batches below stand in for
them with sinusoidal outdoor air and material scales drawn around a nominal
wall whose coefficients equal the east/west wall of Table 2 at 50 % relative
humidity.

A wall set is a dict of arrays (W walls, 3 layer slots):

    nx [W] int32, n_layers [W] int32, layer [W, 3, len(LAYER_FIELDS)] f64,
    hT, hM, qinf, ginf [W, 2] f64  (side 0 = x = 0, side 1 = x = L),
    Tamb, RHamb [W, 2, 4] f64      (mean, amplitude, period s, phase rad),
    T0, RH0, area [W] f64,
    emis [W, 2] f64                (surface emissivity, used on a room side),
    qsun [W, 2, 4] f64             (incident radiation sinusoid, clipped at 0),
    wall_room [W] int64 (-1 = no room), room_side [W] int8.

A room set is a dict:  volume, ach, T0, RH0 [R]; Tout, RHout [R, 4];
sched_dt [R]; g_o, Q_h [R, S] (kg/s and W, periodic piecewise constant);
view [R] (view factor between two surfaces of the room; 0 = no long-wave
exchange); optionally link_a, link_b [L] int32 and link_g [L] f64 (kg/s of
dry air exchanged each way between two rooms).
"""
from __future__ import annotations

import math

import numpy as np

LAYER_FIELDS = ("thick", "k0", "aT", "kM0", "aM", "bTM", "c0", "cT", "cM0",
                "aC", "eTM", "fTM")
SINE_FIELDS = ("mean", "amp", "period", "phase")

# physical constants used as inputs (J/kg latent heat, J/(kg K) water)
LV = 2.5e6
CW = 4180.0

# nominal wall (east/west wall of Table 2 at phi = 0.5 under the law shapes)
NOMINAL = dict(k0=0.3096, kM0=3.126e-9, c0=7.827e5, cM0=3.045e-2)
# law shape coefficients of the nonlinear walls
SHAPE = dict(aT=0.5, aM=3.0, bTM=0.1 * LV, cT=0.2, aC=2.0, eTM=0.0, fTM=CW)

DAY = 86400.0

# Largest dt/dx (s/m) the batches use.  With the conductivities taken at
# level n, their state dependence enters a perturbation as an explicitly and
# centrally treated transport term, and the DF update then has a
# Courant-type limit on dt/dx whatever lambda is (shown by the oracle alone);
# at 5000 s/m the most diffusive walls of a 65,536-wall batch (nu ~ 9x
# nominal) still diverge, at 3333 s/m none do.  The paper's own grid (3.6 s,
# 1 mm) sits at 3600 s/m.  Generators keep dx >= dt / this.
DT_OVER_DX_MAX = 1.0 / 3.0e-4


def default_config(dt: float = 1.0, startup: int = 0, law: int = 0) -> dict:
    """Global constants of a run (room air defaults rho_a, c_pa, c_pv, Pv_ref);
    law 0 = the per-layer shape law, 1 = the Table 1 material."""
    return dict(dt=float(dt), Lv=LV, cw=CW, rho_a=1.2, c_pa=1006.0, c_pv=1860.0,
                Pv_ref=1.61e5, startup=int(startup), law=int(law))


def _zero_sine(shape) -> np.ndarray:
    s = np.zeros(tuple(shape) + (4,))
    s[..., 2] = DAY
    return s


def _empty_walls(W: int) -> dict:
    return dict(
        nx=np.zeros(W, np.int32),
        n_layers=np.ones(W, np.int32),
        layer=np.zeros((W, 3, len(LAYER_FIELDS)), np.float64),
        hT=np.zeros((W, 2)), hM=np.zeros((W, 2)),
        qinf=np.zeros((W, 2)), ginf=np.zeros((W, 2)),
        Tamb=np.zeros((W, 2, 4)), RHamb=np.zeros((W, 2, 4)),
        T0=np.zeros(W), RH0=np.zeros(W), area=np.ones(W),
        emis=np.zeros((W, 2)), qsun=_zero_sine((W, 2)),
        wall_room=np.full(W, -1, np.int64), room_side=np.ones(W, np.int8),
    )


def _set_layer(walls: dict, w, l, **vals):
    for name, v in vals.items():
        walls["layer"][w, l, LAYER_FIELDS.index(name)] = v


def _shape_all(walls: dict, W: int, nl: int = 3):
    for name, v in SHAPE.items():
        walls["layer"][:W, :nl, LAYER_FIELDS.index(name)] = v


def _sine(arr, mean, amp, period, phase):
    arr[..., 0] = mean
    arr[..., 1] = amp
    arr[..., 2] = period
    arr[..., 3] = phase


def _interior_side(walls: dict):
    """Side 1: interior-type exchange, constant air at the initial state."""
    walls["hT"][:, 1] = 8.0
    walls["hM"][:, 1] = 3e-8
    _sine(walls["Tamb"][:, 1], 293.0, 0.0, DAY, 0.0)
    _sine(walls["RHamb"][:, 1], 0.5, 0.0, DAY / 2, 0.0)


def single_wall(seed: int = 101, nx: int = 101) -> dict:
    """One 10 cm homogeneous wall, k0 and kM0 within +-10 % of nominal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _empty_walls(1)
    w["nx"][:] = nx
    w["n_layers"][:] = 1
    _shape_all(w, 1)
    _set_layer(w, 0, 0, thick=0.1,
               k0=NOMINAL["k0"] * rng.uniform(0.9, 1.1),
               kM0=NOMINAL["kM0"] * rng.uniform(0.9, 1.1),
               c0=NOMINAL["c0"], cM0=NOMINAL["cM0"])
    w["hT"][:, 0] = 25.0
    w["hM"][:, 0] = 2e-7
    _sine(w["Tamb"][:, 0], 293.0, 10.0, DAY, 0.0)
    _sine(w["RHamb"][:, 0], 0.5, 0.2, DAY / 2, 0.0)
    _interior_side(w)
    w["T0"][:] = 293.0
    w["RH0"][:] = 0.5
    return w


def _outdoor(rng, W):
    """Random outdoor sinusoids: T amplitude 2-15 K, RH 0.6 +- up to 0.3."""
    AT = rng.uniform(2.0, 15.0, W)
    pT = rng.uniform(0.0, 2 * math.pi, W)
    AR = rng.uniform(0.0, 0.3, W)
    pR = rng.uniform(0.0, 2 * math.pi, W)
    return AT, pT, AR, pR


def uniform_batch(n_walls: int, seed: int = 202, nx: int = 1001, L: float = 0.3) -> dict:
    """Identical-grid batch: walls of thickness L (30 cm: with 1001 nodes and
    dt = 1 s that is dt/dx = 3333 s/m), scales log-uniform over a decade."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = int(n_walls)
    w = _empty_walls(W)
    w["nx"][:] = nx
    w["n_layers"][:] = 1
    _shape_all(w, W)
    s10 = math.sqrt(10.0)

    def logu(nom):
        return np.exp(rng.uniform(math.log(nom / s10), math.log(nom * s10), W))

    k0, kM0, c0, cM0 = (logu(NOMINAL[k]) for k in ("k0", "kM0", "c0", "cM0"))
    for name, v in (("k0", k0), ("kM0", kM0), ("c0", c0), ("cM0", cM0)):
        w["layer"][:, 0, LAYER_FIELDS.index(name)] = v
    w["layer"][:, 0, LAYER_FIELDS.index("thick")] = L
    AT, pT, AR, pR = _outdoor(rng, W)
    w["hT"][:, 0] = 25.0
    w["hM"][:, 0] = 2e-7
    _sine(w["Tamb"][:, 0], 293.0, AT, DAY, pT)
    _sine(w["RHamb"][:, 0], 0.6, AR, DAY / 2, pR)
    _interior_side(w)
    w["T0"][:] = 293.0
    w["RH0"][:] = 0.5
    return w


def table1_batch(n_walls: int, seed: int = 707, nx: int = 1001, L: float = 0.3,
                 spread: float = 1.5) -> dict:
    """Identical-grid batch under the Table 1 law (run with cfg["law"] = 1):
    the load-bearing material of Sec. 6 with its four scale multipliers
    (lambda, k_M and k_TM, rho_0 c_0, c_M and c_TM) log-uniform within a
    factor ``spread`` of 1, the outdoor air of ``uniform_batch`` on side 0,
    20 degC / 50 % inside and initially.  30 cm and 1001 nodes give
    dt/dx = 3333 s/m at dt = 1 s.  Under this law (its k_TM = L_v delta_v is
    about 20x the shape law's) the nonlinear DF step is more fragile: with
    spread 2 at dt = 1 s, 4 of 65,536 walls (heat diffusivity about 3x the
    material's) diverge within 50 steps, in the oracle and on the GPU alike;
    with spread 1.5 all 65,536 stay bounded for 6000 steps, as they do with
    spread 2 at dt = 0.5 s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = int(n_walls)
    w = _empty_walls(W)
    w["nx"][:] = nx
    w["n_layers"][:] = 1
    w["layer"][:, 0, LAYER_FIELDS.index("thick")] = L
    for name in ("k0", "kM0", "c0", "cM0"):
        w["layer"][:, 0, LAYER_FIELDS.index(name)] = np.exp(
            rng.uniform(-math.log(spread), math.log(spread), W))
    AT, pT, AR, pR = _outdoor(rng, W)
    w["hT"][:, 0] = 25.0
    w["hM"][:, 0] = 2e-7
    _sine(w["Tamb"][:, 0], 293.15, AT, DAY, pT)
    _sine(w["RHamb"][:, 0], 0.6, AR, DAY / 2, pR)
    w["hT"][:, 1] = 8.0
    w["hM"][:, 1] = 3e-8
    _sine(w["Tamb"][:, 1], 293.15, 0.0, DAY, 0.0)
    _sine(w["RHamb"][:, 1], 0.5, 0.0, DAY / 2, 0.0)
    w["T0"][:] = 293.15
    w["RH0"][:] = 0.5
    return w


def paper_wall_batch(n_walls: int, seed: int = 808, nx: int = 101) -> dict:
    """The wall of Sec. 4 and Table 3 (run with cfg["law"] = 1): 10 cm of the
    Table 1 material (scales 1), nx nodes, h_T = 25 / 8 W/(m2 K) and h_M =
    2e-7 / 3e-8 s/m outside / inside, 20 degC and 50 % inside and initially.
    The paper's outdoor series exist only as figures; each wall sees
    T = 293.15 + 10 sin(2 pi t / 24 h + a) K and RH = 0.5 + 0.2 sin(2 pi t /
    12 h + b), with phases a, b drawn uniformly (one wall per phase pair, so
    that a batch is not one wall repeated)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = int(n_walls)
    w = _empty_walls(W)
    w["nx"][:] = nx
    w["n_layers"][:] = 1
    for name in ("k0", "kM0", "c0", "cM0"):
        w["layer"][:, 0, LAYER_FIELDS.index(name)] = 1.0
    w["layer"][:, 0, LAYER_FIELDS.index("thick")] = 0.1
    w["hT"][:] = (25.0, 8.0)
    w["hM"][:] = (2e-7, 3e-8)
    _sine(w["Tamb"][:, 0], 293.15, 10.0, DAY, rng.uniform(0.0, 2 * math.pi, W))
    _sine(w["RHamb"][:, 0], 0.5, 0.2, DAY / 2, rng.uniform(0.0, 2 * math.pi, W))
    _sine(w["Tamb"][:, 1], 293.15, 0.0, DAY, 0.0)
    _sine(w["RHamb"][:, 1], 0.5, 0.0, DAY / 2, 0.0)
    w["T0"][:] = 293.15
    w["RH0"][:] = 0.5
    return w


def _cap_nodes(w: dict, dx_min: float):
    """Limit Nx so that dx >= dx_min (at least 3 nodes)."""
    L = np.array([w["layer"][i, :w["n_layers"][i], 0].sum() for i in range(len(w["nx"]))])
    cap = np.maximum(3, np.floor(L / dx_min).astype(np.int64) + 1)
    w["nx"][:] = np.minimum(w["nx"], cap).astype(np.int32)


def layered_batch(n_walls: int, seed: int = 303, nx_lo: int = 51,
                  nx_hi: int = 2001, nx_median: float = 300.0,
                  nx_sigma: float = 0.6, dt: float = 1.0) -> dict:
    """Uneven batch: lognormal Nx, 1-3 layers of 1-20 cm, +-10 % k scales;
    Nx capped so that dt/dx <= DT_OVER_DX_MAX."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = int(n_walls)
    w = _empty_walls(W)
    nx = np.rint(np.exp(rng.normal(math.log(nx_median), nx_sigma, W)))
    w["nx"][:] = np.clip(nx, nx_lo, nx_hi).astype(np.int32)
    w["n_layers"][:] = rng.integers(1, 4, W).astype(np.int32)
    _shape_all(w, W)
    for l in range(3):
        live = l < w["n_layers"]
        thick = np.where(live, rng.uniform(0.01, 0.2, W), 0.0)
        w["layer"][:, l, LAYER_FIELDS.index("thick")] = thick
        w["layer"][:, l, LAYER_FIELDS.index("k0")] = NOMINAL["k0"] * rng.uniform(0.9, 1.1, W)
        w["layer"][:, l, LAYER_FIELDS.index("kM0")] = NOMINAL["kM0"] * rng.uniform(0.9, 1.1, W)
        w["layer"][:, l, LAYER_FIELDS.index("c0")] = NOMINAL["c0"]
        w["layer"][:, l, LAYER_FIELDS.index("cM0")] = NOMINAL["cM0"]
    _cap_nodes(w, dt / DT_OVER_DX_MAX)
    AT, pT, AR, pR = _outdoor(rng, W)
    w["hT"][:, 0] = 25.0
    w["hM"][:, 0] = 2e-7
    _sine(w["Tamb"][:, 0], 293.0, AT, DAY, pT)
    _sine(w["RHamb"][:, 0], 0.6, AR, DAY / 2, pR)
    _interior_side(w)
    w["T0"][:] = 293.0
    w["RH0"][:] = 0.5
    return w


def building_batch(n_rooms: int, seed: int = 404, nx_lo: int = 101,
                   nx_hi: int = 801, n_sched: int = 24, dt: float = 1.0,
                   radiation: bool = False, link_group: int = 1):
    """Box rooms (2.5 m high, square floor) with 6 layered walls each.

    Side 0 of every wall faces the outdoor air of its room, side 1 the room.
    Hourly moisture (0-500 g/h) and heat (0-1000 W) schedules, seeded.  Nx is
    capped so that dt/dx <= DT_OVER_DX_MAX.  Returns (walls, rooms).

    radiation=True adds the radiative sources of the paper's two-zone case
    (Sec. 6.2): room-side emissivity 0.5 with one wall per room at 0.9, view
    factor 0.2, and on the outdoor side a daily half-wave incident flux
    (amplitude 100-600 W/m2 per wall, standing in for the orientation; the
    paper's own series is only shown in a figure); initial wall
    temperatures are then spread over 291-295 K so that the long-wave
    exchange is active from the first step.

    link_group = k > 1 joins consecutive rooms into chains of k zones
    (0-1-...-(k-1), k-...) with an airflow of 0.3 air changes per hour of the
    smaller zone each way (the inter-zone flow of the paper's two-zone case,
    Sec. 6.2, is 0.3 h^-1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    R = int(n_rooms)
    W = 6 * R
    w = _empty_walls(W)
    w["nx"][:] = rng.integers(nx_lo, nx_hi + 1, W).astype(np.int32)
    w["n_layers"][:] = rng.integers(1, 4, W).astype(np.int32)
    _shape_all(w, W)
    for l in range(3):
        live = l < w["n_layers"]
        thick = np.where(live, rng.uniform(0.01, 0.2, W), 0.0)
        w["layer"][:, l, LAYER_FIELDS.index("thick")] = thick
        w["layer"][:, l, LAYER_FIELDS.index("k0")] = NOMINAL["k0"] * rng.uniform(0.9, 1.1, W)
        w["layer"][:, l, LAYER_FIELDS.index("kM0")] = NOMINAL["kM0"] * rng.uniform(0.9, 1.1, W)
        w["layer"][:, l, LAYER_FIELDS.index("c0")] = NOMINAL["c0"]
        w["layer"][:, l, LAYER_FIELDS.index("cM0")] = NOMINAL["cM0"]
    _cap_nodes(w, dt / DT_OVER_DX_MAX)
    volume = rng.uniform(30.0, 300.0, R)
    ach = rng.uniform(0.2, 2.0, R)
    AT, pT, AR, pR = _outdoor(rng, R)
    side = np.sqrt(volume / 2.5)
    areas = np.stack([side * 2.5] * 4 + [side * side] * 2, axis=1)  # [R, 6]
    w["area"][:] = areas.reshape(-1)
    w["wall_room"][:] = np.repeat(np.arange(R, dtype=np.int64), 6)
    w["room_side"][:] = 1
    w["hT"][:, 0] = 25.0
    w["hM"][:, 0] = 2e-7
    w["hT"][:, 1] = 8.0
    w["hM"][:, 1] = 3e-8
    _sine(w["Tamb"][:, 0], 293.0, np.repeat(AT, 6), DAY, np.repeat(pT, 6))
    _sine(w["RHamb"][:, 0], 0.6, np.repeat(AR, 6), DAY / 2, np.repeat(pR, 6))
    _sine(w["Tamb"][:, 1], 293.0, 0.0, DAY, 0.0)   # unused: room side
    _sine(w["RHamb"][:, 1], 0.5, 0.0, DAY / 2, 0.0)
    w["T0"][:] = 293.0
    w["RH0"][:] = 0.5
    rooms = dict(
        volume=volume, ach=ach, T0=np.full(R, 293.0), RH0=np.full(R, 0.5),
        Tout=np.zeros((R, 4)), RHout=np.zeros((R, 4)),
        sched_dt=np.full(R, 3600.0),
        g_o=rng.uniform(0.0, 0.5, (R, n_sched)) / 3600.0,   # kg/s
        Q_h=rng.uniform(0.0, 1000.0, (R, n_sched)),
        view=np.zeros(R),
    )
    _sine(rooms["Tout"], 293.0, AT, DAY, pT)
    _sine(rooms["RHout"], 0.6, AR, DAY / 2, pR)
    if radiation:
        w["emis"][:, 1] = 0.5
        w["emis"][::6, 1] = 0.9
        rooms["view"][:] = 0.2
        _sine(w["qsun"][:, 0], 0.0, rng.uniform(100.0, 600.0, W), DAY,
              np.repeat(pT, 6) - math.pi / 2)
        w["T0"][:] = rng.uniform(291.0, 295.0, W)
    if link_group > 1:
        a = [r for r in range(R - 1) if (r + 1) % link_group != 0]
        rooms["link_a"] = np.array(a, np.int32)
        rooms["link_b"] = np.array([r + 1 for r in a], np.int32)
        rooms["link_g"] = 0.3 * 1.2 * np.minimum(volume[a], volume[[r + 1 for r in a]]) / 3600.0
    return w, rooms


def subset(walls: dict, idx) -> dict:
    """Walls ``idx`` of a wall set (room links dropped)."""
    idx = np.asarray(idx)
    out = {k: np.ascontiguousarray(v[idx]) for k, v in walls.items()}
    out["wall_room"][:] = -1
    return out


def concat(*sets: dict) -> dict:
    return {k: np.concatenate([s[k] for s in sets]) for k in sets[0]}


def total_nodes(walls: dict) -> int:
    return int(np.asarray(walls["nx"], np.int64).sum())
