"""Oracle pins on the lumped room-air balance (CPU only).

Forward Euler on the zone balance (eq. LAV_equation, explicit coupling of
Sec. 5.3) has exact geometric discrete solutions when the room is decoupled
from its walls, and its fixed point through linear walls is the
series-resistance steady state.  Both are closed forms independent of the
oracle's code."""
import math

import numpy as np
import pytest

import oracle
from helpers import linear_wall
from paper_1703_10119_amd import workloads as wl


def _room(volume=54.0, ach=0.5, T0=293.15, RH0=0.5, Tout=283.0, RHout=0.8,
          g_o=(0.0,), Q_h=(0.0,), sched_dt=3600.0):
    r = dict(volume=np.array([volume]), ach=np.array([ach]), T0=np.array([T0]),
             RH0=np.array([RH0]), Tout=np.zeros((1, 4)), RHout=np.zeros((1, 4)),
             sched_dt=np.array([sched_dt]), g_o=np.array([g_o], np.float64),
             Q_h=np.array([Q_h], np.float64))
    wl._sine(r["Tout"], Tout, 0.0, wl.DAY, 0.0)
    wl._sine(r["RHout"], RHout, 0.0, wl.DAY, 0.0)
    return r


def _adiabatic_wall():
    w = linear_wall(11, hT=(0.0, 0.0), hM=(0.0, 0.0))
    w["wall_room"][:] = 0
    w["room_side"][:] = 1
    return w


def test_room_moisture_geometric():
    cfg = wl.default_config(dt=60.0)
    r = _room(g_o=(0.4 / 3600,))
    sim = oracle.RefSim(_adiabatic_wall(), cfg, r)
    mass = cfg["rho_a"] * 54.0
    gv = 0.5 * mass / 3600.0
    Pout = 0.8 * oracle.psat(283.0)
    Peq = Pout + (0.4 / 3600) * cfg["Pv_ref"] / gv
    P0 = 0.5 * oracle.psat(293.15)
    q = 1.0 - cfg["dt"] * 0.5 / 3600.0
    for n in (1, 10, 100, 1000):
        sim.step(n - sim.n)
        _, Pa = sim.rooms()
        assert Pa[0] == pytest.approx(Peq + (P0 - Peq) * q ** n, rel=1e-12)


def _equilibrium_source(cfg, P0, Pout, ach=0.5, volume=54.0):
    mass = cfg["rho_a"] * volume
    gv = ach * mass / 3600.0
    return gv, gv * (P0 - Pout) / cfg["Pv_ref"]


def test_room_temperature_geometric_and_schedule():
    """Vapour pressure held at its fixed point; a two-slot heat schedule gives
    a piecewise geometric approach to T_out + Q_h / (g_v c_ma) per slot."""
    cfg = wl.default_config(dt=30.0)
    P0 = 0.5 * oracle.psat(293.15)
    Pout = 0.8 * oracle.psat(283.0)
    gv, go = _equilibrium_source(cfg, P0, Pout)
    Qh = (400.0, 1500.0)
    r = _room(g_o=(go, go), Q_h=Qh, sched_dt=600.0)        # 20 steps per slot
    sim = oracle.RefSim(_adiabatic_wall(), cfg, r)
    cma = cfg["c_pa"] + cfg["c_pv"] * P0 / cfg["Pv_ref"]
    q = 1.0 - cfg["dt"] * 0.5 / 3600.0
    T = 293.15
    for slot in range(6):
        Teq = 283.0 + Qh[slot % 2] / (gv * cma)
        T = Teq + (T - Teq) * q ** 20
        sim.step(20)
        Ta, Pa = sim.rooms()
        assert Pa[0] == pytest.approx(P0, rel=1e-13)
        assert Ta[0] == pytest.approx(T, rel=1e-13)


def _room_with_linear_walls(hM_walls):
    specs = [(18.0, 0.294, 5.0), (18.0, 0.841, 25.0), (9.0, 0.387, 12.0), (9.0, 0.387, 12.0)]
    ws = []
    for A, k, hout in specs:
        w = linear_wall(21, cM=6.09e-3, kM=5.47e-9, cTT=2e5, kTT=k, cTM=0.0, kTM=0.0,
                        hT=(hout, 8.0), hM=(hM_walls[0], hM_walls[1]),
                        Tinf=(283.0, 283.0), RHinf=(0.8, 0.8), T0=283.0, RH0=0.5)
        w["area"][:] = A
        w["wall_room"][:] = 0
        w["room_side"][:] = 1
        ws.append(w)
    return wl.concat(*ws), specs


def test_room_heat_steady_state_through_walls():
    """Heat only (no vapour exchange): the fixed point balances Q_h against
    ventilation and the wall conductances 1 / (1/h_out + L/k + 1/h_in)."""
    cfg = wl.default_config(dt=60.0)
    walls, specs = _room_with_linear_walls((0.0, 0.0))
    Pout = 0.8 * oracle.psat(283.0)
    RH0 = Pout / oracle.psat(283.0)
    r = _room(T0=283.0, RH0=RH0, Tout=283.0, RHout=0.8, Q_h=(800.0,))
    sim = oracle.RefSim(walls, cfg, r)
    sim.step(20000)
    Ta, Pa = sim.rooms()
    gv = 0.5 * cfg["rho_a"] * 54.0 / 3600.0
    cma = cfg["c_pa"] + cfg["c_pv"] * Pout / cfg["Pv_ref"]
    UA = sum(A / (1 / hout + 0.1 / k + 1 / 8.0) for A, k, hout in specs)
    assert Pa[0] == pytest.approx(Pout, rel=1e-12)
    assert Ta[0] == pytest.approx(283.0 + 800.0 / (gv * cma + UA), rel=1e-10)


def test_room_moisture_steady_state_through_walls():
    """Vapour only matters for P_a: g_o balances ventilation and the wall
    vapour conductances 1 / (1/hM_out + L/k_M + 1/hM_in)."""
    cfg = wl.default_config(dt=60.0)
    hMo, hMi = 2e-7, 3e-8
    walls, specs = _room_with_linear_walls((hMo, hMi))
    go = 0.2 / 3600.0
    r = _room(T0=283.0, RH0=0.6, Tout=283.0, RHout=0.8, g_o=(go,))
    sim = oracle.RefSim(walls, cfg, r)
    sim.step(20000)
    _, Pa = sim.rooms()
    Pout = 0.8 * oracle.psat(283.0)
    gv = 0.5 * cfg["rho_a"] * 54.0 / 3600.0
    UM = sum(A / (1 / hMo + 0.1 / 5.47e-9 + 1 / hMi) for A, _, _ in specs)
    assert Pa[0] == pytest.approx(Pout + go / (gv / cfg["Pv_ref"] + UM), rel=1e-9)
