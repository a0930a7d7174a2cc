"""Pins of the oracle's coefficient law (CPU only).

The balance identity and the per-node residual of the scheme hold for any
coefficient law, so they cannot tell a wrong law from the right one.  These
tests pin the law itself, from outside the oracle:

  * Table 2 (Sec. 6.1): at 20 degC and 50 % relative humidity the nominal
    wall must give the east/west wall's k_TT, k_M, c_TT, c_M and c_TM;
  * the config's law shapes at literal states (uniform T, given phi), where
    each coefficient is a fixed multiple of its scale;
  * Sec. 3.1: a face coefficient is the law evaluated at the face-averaged
    state ((T_j + T_{j+1}) / 2, (P_j + P_{j+1}) / 2), not the mean of the two
    node values; states are chosen so that the face state has phi = 0.5
    exactly while the nodes do not;
  * across a layer interface, the harmonic mean of the two layers' laws at the
    face state.

``test_oracle_mutations.py`` plants mistakes in a copy of the oracle and
checks that this file fails on each.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1703_10119_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
F = wl.LAYER_FIELDS


def _wall(nx=3, thick=(0.1,), scales=None, T0=293.15, RH0=0.5):
    """A wall of unit (or given) law scales under the shape law."""
    w = wl._empty_walls(1)
    w["nx"][:] = nx
    w["n_layers"][:] = len(thick)
    wl._shape_all(w, 1)
    for l, th in enumerate(thick):
        sc = dict(k0=1.0, kM0=1.0, c0=1.0, cM0=1.0) if scales is None else scales[l]
        w["layer"][0, l, F.index("thick")] = th
        for k, v in sc.items():
            w["layer"][0, l, F.index(k)] = v
    for s in range(2):
        wl._sine(w["Tamb"][0, s], T0, 0.0, wl.DAY, 0.0)
        wl._sine(w["RHamb"][0, s], RH0, 0.0, wl.DAY, 0.0)
    w["T0"][:] = T0
    w["RH0"][:] = RH0
    return w


def _coeffs_at(w, T, P):
    """Oracle node (c_TT, c_M, c_TM) and face (k_TT, k_M, k_TM) coefficients
    with level n set to (T, P)."""
    sim = oracle.RefSim(w, wl.default_config(dt=1.0))
    sim.set_fields(0, 0, np.asarray(T, float), np.asarray(P, float))
    return sim.coeffs(0)


def test_law_reproduces_table2_east_west_wall():
    """Nominal scales at 293.15 K, phi = 0.5 give Table 2's east/west wall
    within 0.3 % (k_TT 0.387, k_M 5.47e-9, c_TT 8.61e5, c_M 6.09e-2, c_TM
    5.09e3); k_TM = 0.1 L_v k_M (the config's k_TM)."""
    d = json.load(open(os.path.join(GOLD, "table2_appendix_b.json")))["walls"]["east_west"]
    w = _wall(nx=5, scales=[dict(wl.NOMINAL)])
    node, face = oracle.RefSim(w, wl.default_config()).coeffs(0)
    for j in range(5):
        assert node[j, 0] == pytest.approx(d["cTT"], rel=3e-3)
        assert node[j, 1] == pytest.approx(d["cM"], rel=3e-3)
        assert node[j, 2] == pytest.approx(d["cTM"], rel=3e-3)
    for j in range(4):
        assert face[j, 0] == pytest.approx(d["kTT"], rel=3e-3)
        assert face[j, 1] == pytest.approx(d["kM"], rel=3e-3)
        assert face[j, 2] == pytest.approx(0.1 * 2.5e6 * face[j, 1], rel=1e-14)


# (phi, k_TT/k0, k_M/kM0, c_TT/c0, c_M/cM0): 1 + 0.5 phi, 1 + 3 phi^2,
# 1 + 0.2 phi, 1 + 2 phi written out as numbers
LITERAL = [(0.2, 1.1, 1.12, 1.04, 1.4),
           (0.5, 1.25, 1.75, 1.1, 2.0),
           (0.8, 1.4, 2.92, 1.16, 2.6),
           (0.95, 1.475, 3.7075, 1.19, 2.9)]


@pytest.mark.parametrize("phi,kT,kM,cT,cM", LITERAL)
@pytest.mark.parametrize("theta", [5.0, 20.0, 30.0])
def test_law_shape_at_literal_states(phi, kT, kM, cT, cM, theta):
    """Uniform state at theta degC and the given phi: every coefficient is a
    literal multiple of its scale, and c_TM / c_M = c_w theta (theta in degC)."""
    T = 273.15 + theta
    w = _wall(nx=4, T0=T, RH0=phi)
    P = phi * oracle.psat(T)
    node, face = _coeffs_at(w, [T] * 4, [P] * 4)
    assert np.allclose(face[:, 0], kT, rtol=1e-13, atol=0)
    assert np.allclose(face[:, 1], kM, rtol=1e-13, atol=0)
    assert np.allclose(face[:, 2], 0.1 * 2.5e6 * kM, rtol=1e-13, atol=0)
    assert np.allclose(node[:, 0], cT, rtol=1e-13, atol=0)
    assert np.allclose(node[:, 1], cM, rtol=1e-13, atol=0)
    assert np.allclose(node[:, 2], 4180.0 * theta * cM, rtol=1e-12, atol=0)


def test_face_coefficients_at_face_averaged_state():
    """Sec. 3.1: faces take the law at the face-averaged state.

    Face 0 joins 283.15 K and 303.15 K at equal vapour pressure p = 0.5
    Ps(293.15): its state is (293.15 K, p), phi = 0.5 exactly, so k_TT = 1.25,
    k_M = 1.75, while the two nodes sit at phi 0.95 and 0.28 (mean of the node
    values: k_TT 1.31, k_M 2.47).  Face 1 joins phi 0.2 and 0.8 at 303.15 K:
    face phi 0.5 again, where the mean of the node values would give
    k_M = 2.02."""
    p = 0.5 * oracle.psat(293.15)
    ps30 = oracle.psat(303.15)
    T = [283.15, 303.15, 303.15]
    P = [p, p, 0.8 * ps30]
    node, face = _coeffs_at(_wall(nx=3), T, P)
    assert face[0, 0] == pytest.approx(1.25, rel=1e-13)
    assert face[0, 1] == pytest.approx(1.75, rel=1e-13)
    assert face[0, 2] == pytest.approx(0.1 * 2.5e6 * 1.75, rel=1e-13)
    T = [303.15, 303.15, 303.15]
    P = [0.2 * ps30, 0.8 * ps30, 0.8 * ps30]
    node, face = _coeffs_at(_wall(nx=3), T, P)
    assert face[0, 0] == pytest.approx(1.25, rel=1e-13)
    assert face[0, 1] == pytest.approx(1.75, rel=1e-13)
    assert face[1, 1] == pytest.approx(1 + 3 * 0.64, rel=1e-13)
    # node coefficients stay at the node states
    assert node[0, 1] == pytest.approx(1.4, rel=1e-13)
    assert node[1, 1] == pytest.approx(2.6, rel=1e-13)


def test_interface_face_is_harmonic_mean_at_face_state():
    """Two 5 cm layers, 3 nodes: node 1 (x = 5 cm) belongs to layer 0, so face
    1 is the interface.  Layer scales k0 = 1 and 3 (kM0 = 2 and 0.5) at the
    face state phi = 0.5: k_TT = 2 (1.25)(3.75) / 5 = 1.875, k_M = 2 (3.5)
    (0.875) / 4.375 = 1.4."""
    sc = [dict(k0=1.0, kM0=2.0, c0=1.0, cM0=1.0), dict(k0=3.0, kM0=0.5, c0=1.0, cM0=1.0)]
    w = _wall(nx=3, thick=(0.05, 0.05), scales=sc)
    ps = oracle.psat(293.15)
    T = [293.15, 283.15, 303.15]
    # face 1 state: T = 293.15, P = 0.5 ps
    P = [0.5 * ps, 0.3 * ps, 0.7 * ps]
    sim = oracle.RefSim(w, wl.default_config())
    assert sim.layers(0).tolist() == [0, 0, 1]
    sim.set_fields(0, 0, np.asarray(T, float), np.asarray(P, float))
    node, face = sim.coeffs(0)
    assert face[1, 0] == pytest.approx(1.875, rel=1e-13)
    assert face[1, 1] == pytest.approx(1.4, rel=1e-13)
    assert face[1, 2] == pytest.approx(0.1 * 2.5e6 * 1.4, rel=1e-13)
