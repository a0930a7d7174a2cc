"""Oracle pins on the radiative surface sources (CPU only).

The surface heat source of eq. (2.3) (Sec. 2, boundary conditions) carries
incident radiation on any side and, on a zone side, the long-wave exchange
s eps sigma sum_w (T_w^4 - T^4) among the zone's surfaces.  The pins below
come from physics and arithmetic the oracle does not share:

  * two walls that see each other only by radiation reach a steady state
    that is a pair of scalar nonlinear equations (series resistances of the
    linear walls, outdoor convection, the radiative balance) solved here by
    root finding; the DF scheme reproduces linear steady profiles exactly, so
    the oracle must converge to that root;
  * with equal emissivities the long-wave powers of a zone sum to zero at
    every step, with unequal ones the sum of q / eps does;
  * walls at one temperature exchange nothing, bit for bit;
  * the incident flux integrated over a period equals the closed form of
    the half-wave rectified sinusoid, A P / pi, to the Riemann-sum error of
    the step.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from helpers import linear_wall
from paper_1703_10119_amd import workloads as wl

SIGMA = 5.670374419e-8


def _room(view, T0=293.0):
    r = dict(volume=np.array([50.0]), ach=np.array([0.5]), T0=np.array([T0]),
             RH0=np.array([0.5]), Tout=np.zeros((1, 4)), RHout=np.zeros((1, 4)),
             sched_dt=np.array([3600.0]), g_o=np.zeros((1, 1)), Q_h=np.zeros((1, 1)),
             view=np.array([view]))
    wl._sine(r["Tout"], T0, 0.0, wl.DAY, 0.0)
    wl._sine(r["RHout"], 0.5, 0.0, wl.DAY, 0.0)
    return r


def _radiating_walls(Tout, emis, L=0.02, k=0.5, c=2.0e5, h_out=50.0, nx=21):
    """Linear heat-only walls (no moisture exchange), outdoor convection on
    side 0, radiation only on side 1 (the zone side)."""
    ws = []
    for T, e in zip(Tout, emis):
        w = linear_wall(nx, L=L, cTT=c, kTT=k, cTM=0.0, kTM=0.0,
                        hT=(h_out, 0.0), hM=(0.0, 0.0), Tinf=(T, 293.0), T0=293.0)
        w["emis"][0] = (0.0, e)
        w["wall_room"][:] = 0
        w["room_side"][:] = 1
        ws.append(w)
    return wl.concat(*ws)


def test_two_wall_radiative_steady_state():
    Ta, Tb = 313.0, 273.0
    ea, eb = 0.5, 0.9
    s = 0.2
    L, k, h = 0.02, 0.2, 50.0
    R = 1.0 / h + L / k                      # series resistance, m2 K / W
    walls = _radiating_walls((Ta, Tb), (ea, eb), L=L, k=k, h_out=h)
    sim = oracle.RefSim(walls, wl.default_config(dt=2.0, startup=1), _room(s))
    sim.step(12000)
    TA = sim.fields(0)[0][-1]
    TB = sim.fields(1)[0][-1]
    sim.step(100)
    assert abs(sim.fields(0)[0][-1] - TA) < 1e-10      # converged

    # independent steady state: conduction in = radiation out on each wall,
    # (T_out - T_s) / R + s eps sigma (T_other^4 - T_s^4) = 0
    def TB_of(TA_):
        return brentq(lambda x: (Tb - x) / R + s * eb * SIGMA * (TA_ ** 4 - x ** 4), 200.0, 400.0)

    TA_ss = brentq(lambda x: (Ta - x) / R + s * ea * SIGMA * (TB_of(x) ** 4 - x ** 4), 200.0, 400.0)
    TB_ss = TB_of(TA_ss)
    assert sim.fields(0)[0][-1] == pytest.approx(TA_ss, abs=1e-8)
    assert sim.fields(1)[0][-1] == pytest.approx(TB_ss, abs=1e-8)
    # the radiation is a visible effect here (several K off the outdoor air)
    assert Ta - TA_ss > 2.0 and TB_ss - Tb > 2.0
    # the zone-side flux reported is the radiative one (no convection there)
    now, _ = sim.fluxes()
    assert now[0, 1, 0] == pytest.approx(-(Ta - TA_ss) / R, rel=1e-7)
    assert now[1, 1, 0] == pytest.approx((TB_ss - Tb) / R, rel=1e-7)


@pytest.mark.parametrize("emis", [(0.7, 0.7, 0.7), (0.5, 0.9, 0.3)])
def test_longwave_balance_per_step(emis):
    walls = _radiating_walls((313.0, 273.0, 300.0), emis)
    sim = oracle.RefSim(walls, wl.default_config(dt=2.0, startup=0), _room(0.2))
    e = np.asarray(emis)
    seen = 0.0
    for _ in range(30):
        sim.step(7)
        now, _ = sim.fluxes()
        q = now[:, 1, 0]                   # zone side heat flux = long-wave only
        seen = max(seen, np.abs(q).max())
        assert abs(np.sum(q / e)) <= 1e-12 * np.abs(q / e).sum() + 1e-14
    assert seen > 1.0


def test_equal_surfaces_exchange_nothing():
    w1 = _radiating_walls((300.0, 300.0), (0.5, 0.9))
    w0 = _radiating_walls((300.0, 300.0), (0.0, 0.0))
    cfg = wl.default_config(dt=2.0, startup=0)
    a = oracle.RefSim(w1, cfg, _room(0.2))
    b = oracle.RefSim(w0, cfg, _room(0.0))
    a.step(50)
    b.step(50)
    for w in range(2):
        np.testing.assert_array_equal(a.fields(w)[0], b.fields(w)[0])
        np.testing.assert_array_equal(a.fields(w)[1], b.fields(w)[1])
    np.testing.assert_array_equal(a.fluxes()[1], b.fluxes()[1])


def test_incident_radiation_period_integral():
    """Half-wave rectified incident flux on an adiabatic wall: the applied
    flux integral over one period is A P / pi."""
    A, P, dt = 400.0, 86400.0, 60.0
    w = linear_wall(11, hT=(0.0, 0.0), hM=(0.0, 0.0))
    wl._sine(w["qsun"][0, 0], 0.0, A, P, 0.3)
    sim = oracle.RefSim(w, wl.default_config(dt=dt, startup=1))
    sim.step(int(P / dt))
    _, integ = sim.fluxes()
    assert integ[0, 0, 0] == pytest.approx(A * P / math.pi, rel=1e-6)
    assert integ[0, 1, 0] == 0.0


def test_constant_incident_equals_constant_source():
    """amp = 0: the incident flux is its mean (clipped at zero), so a wall
    with q_sun = q0 steps bit for bit like one with q_inf = q0, and a
    negative mean gives no flux at all."""
    cfg = wl.default_config(dt=30.0, startup=0)
    base = linear_wall(21, hT=(10.0, 8.0), hM=(1e-8, 2e-8), Tinf=(280.0, 293.0))
    a, b, c = (dict((k, v.copy()) for k, v in base.items()) for _ in range(3))
    wl._sine(a["qsun"][0, 0], 150.0, 0.0, wl.DAY, 0.0)
    b["qinf"][0, 0] = 150.0
    wl._sine(c["qsun"][0, 1], -80.0, 0.0, wl.DAY, 0.0)
    sa, sb, sc, s0 = (oracle.RefSim(x, cfg) for x in (a, b, c, base))
    for s in (sa, sb, sc, s0):
        s.step(40)
    np.testing.assert_array_equal(sa.fields(0)[0], sb.fields(0)[0])
    np.testing.assert_array_equal(sa.fluxes()[1], sb.fluxes()[1])
    np.testing.assert_array_equal(sc.fields(0)[0], s0.fields(0)[0])
    assert not np.array_equal(sa.fields(0)[0], s0.fields(0)[0])
