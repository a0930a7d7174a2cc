"""Oracle pins on the airflow between zones (Sec. 5.1, the inter-zone
sources of eq. LAV_equation), CPU only.

A link moves g kg/s of dry air each way between two zones.  Pins that do not
come from the oracle's code:

  * the moist-air enthalpy of the textbook, h = c_pa theta + w (L_v + c_pv
    theta) (theta in degC, w ~ Pv / Pv_ref): zone i gains g (h_j - h_i) of
    heat per unit time, whatever the two air states are;
  * two zones exchanging only air: the vapour-pressure difference decays by
    the exact factor 1 - dt g (1/m_1 + 1/m_2) per forward-Euler step and the
    mass-weighted sum is conserved (likewise the temperatures at equal Pv);
  * a chain source zone -> middle zone -> ventilated zone reaches the steady
    state that a series of flow resistances gives in closed form.
"""
import numpy as np
import pytest

import oracle
from helpers import linear_wall
from paper_1703_10119_amd import workloads as wl


def _zones(T0, RH0, volume, ach=None, g_o=None):
    R = len(T0)
    r = dict(volume=np.asarray(volume, float), ach=np.zeros(R) if ach is None else np.asarray(ach, float),
             T0=np.asarray(T0, float), RH0=np.asarray(RH0, float),
             Tout=np.zeros((R, 4)), RHout=np.zeros((R, 4)), sched_dt=np.full(R, 3600.0),
             g_o=np.zeros((R, 1)) if g_o is None else np.asarray(g_o, float).reshape(R, 1),
             Q_h=np.zeros((R, 1)), view=np.zeros(R))
    wl._sine(r["Tout"], 283.0, 0.0, wl.DAY, 0.0)
    wl._sine(r["RHout"], 0.8, 0.0, wl.DAY, 0.0)
    return r


def _link(r, pairs):
    r["link_a"] = np.array([a for a, _, _ in pairs], np.int32)
    r["link_b"] = np.array([b for _, b, _ in pairs], np.int32)
    r["link_g"] = np.array([g for _, _, g in pairs], np.float64)
    return r


def _free_wall():
    """A wall coupled to no zone (the zones exchange only air)."""
    return linear_wall(5, hT=(0.0, 0.0), hM=(0.0, 0.0))


def test_enthalpy_of_exchanged_air():
    cfg = wl.default_config(dt=5.0)
    T0, RH0, V = (296.0, 287.5), (0.35, 0.8), (40.0, 90.0)
    g = 0.02
    r = _link(_zones(T0, RH0, V), [(0, 1, g)])
    sim = oracle.RefSim(_free_wall(), cfg, r)
    Ta0, Pa0 = sim.rooms()
    sim.step(1)
    Ta1, Pa1 = sim.rooms()
    Pref = cfg["Pv_ref"]

    def h(T, P):                      # J per kg of dry air, theta in degC
        th, w = T - 273.15, P / Pref
        return cfg["c_pa"] * th + w * (cfg["Lv"] + cfg["c_pv"] * th)

    for i, j in ((0, 1), (1, 0)):
        m = cfg["rho_a"] * V[i]
        c = cfg["c_pa"] + cfg["c_pv"] * Pa0[i] / Pref
        Q = (Ta1[i] - Ta0[i]) * m * c / cfg["dt"]
        assert Q == pytest.approx(g * (h(Ta0[j], Pa0[j]) - h(Ta0[i], Pa0[i])), rel=1e-10)
        G = (Pa1[i] - Pa0[i]) * m / Pref / cfg["dt"]
        assert G == pytest.approx(g * (Pa0[j] - Pa0[i]) / Pref, rel=1e-10)


@pytest.mark.parametrize("field", ["P", "T"])
def test_two_zone_exchange_is_geometric_and_conservative(field):
    cfg = wl.default_config(dt=20.0)
    V = (30.0, 120.0)
    m1, m2 = (cfg["rho_a"] * v for v in V)
    g = 0.01
    if field == "P":
        T0, RH0 = (293.0, 293.0), (0.3, 0.8)
    else:
        # equal vapour pressure in both zones: RH chosen so that Pv matches
        P = 0.5 * oracle.psat(300.0)
        T0, RH0 = (300.0, 288.0), (0.5, P / oracle.psat(288.0))
    sim = oracle.RefSim(_free_wall(), cfg, _link(_zones(T0, RH0, V), [(0, 1, g)]))
    Ta, Pa = sim.rooms()
    x0 = Pa if field == "P" else Ta
    q = 1.0 - cfg["dt"] * g * (1.0 / m1 + 1.0 / m2)
    D0, S0 = x0[1] - x0[0], m1 * x0[0] + m2 * x0[1]
    for n in (1, 10, 100, 400):
        sim.step(n - sim.n)
        Ta, Pa = sim.rooms()
        x = Pa if field == "P" else Ta
        assert x[1] - x[0] == pytest.approx(D0 * q ** n, rel=1e-9, abs=1e-9 * abs(D0))
        assert m1 * x[0] + m2 * x[1] == pytest.approx(S0, rel=1e-13)
        if field == "T":
            assert Pa[0] == pytest.approx(Pa[1], rel=1e-13)


def test_chain_steady_state():
    """Zone 0 holds a vapour source, zone 2 is ventilated; 0-1 and 1-2 are
    linked.  In the steady state the source flows through the chain:
    w_2 = w_out + g_o / g_v, w_1 = w_2 + g_o / g_12, w_0 = w_1 + g_o / g_01."""
    cfg = wl.default_config(dt=30.0)
    V = (50.0, 30.0, 80.0)
    go, g01, g12 = 0.2 / 3600, 0.004, 0.006
    ach2 = 1.0
    r = _zones((293.0, 293.0, 293.0), (0.5, 0.5, 0.5), V, ach=(0.0, 0.0, ach2),
               g_o=(go, 0.0, 0.0))
    r = _link(r, [(1, 0, g01), (1, 2, g12)])
    sim = oracle.RefSim(_free_wall(), cfg, r)
    sim.step(40000)
    _, Pa = sim.rooms()
    Pref = cfg["Pv_ref"]
    gv = ach2 * cfg["rho_a"] * V[2] / 3600.0
    Pout = 0.8 * oracle.psat(283.0)
    P2 = Pout + go * Pref / gv
    P1 = P2 + go * Pref / g12
    P0 = P1 + go * Pref / g01
    np.testing.assert_allclose(Pa, [P0, P1, P2], rtol=1e-9)


def test_no_links_and_zero_flow_are_identical():
    cfg = wl.default_config(dt=10.0)
    walls, rooms = wl.building_batch(2, seed=9, nx_lo=11, nx_hi=31, dt=10.0)
    a = oracle.RefSim(walls, cfg, rooms)
    b = oracle.RefSim(walls, cfg, _link(dict(rooms), [(0, 1, 0.0)]))
    a.step(200)
    b.step(200)
    np.testing.assert_array_equal(a.rooms()[0], b.rooms()[0])
    np.testing.assert_array_equal(a.all_fields(0)[0], b.all_fields(0)[0])
