"""Where the nonlinear Dufort-Frankel step stops being stable (CPU only).

Sec. 3.1 proves unconditional stability for constant coefficients (pinned in
``test_oracle_linear.py``), and Sec. 4 reports solutions for every dt* of its
sweep on the Table 1 wall.  With the coefficients taken at level n, the
state dependence of a *conductivity* enters the equation of a perturbation
as a transport term, k'(u) u_x d(du)/dx, which the three-level update treats
explicitly and centrally; at large dt/dx the scheme itself carries
information at about dx/dt (its modified equation, eq. expansion_dufort, is
a telegraph equation), so the step stays stable only while that transport
is slower: a Courant-type limit on dt/dx, not on lambda.  The pins:

  * state-dependent capacities with constant conductivities stay bounded at
    dt* = 0.1 (360 s on a 1 mm grid), where state-dependent conductivities
    with constant capacities diverge (shape law, same wall and forcing);
  * the Table 1 wall (10 cm, 101 nodes, the paper's material) stays bounded
    at the paper's grid, dt* = 1e-3 (3.6 s, 3600 s/m), with forcing strong
    enough to drive the surface past saturation, and diverges at dt* = 1e-2;
  * on the Table 1 wall the divergence sets in at the same dt/dx on grids of
    2, 1 and 0.5 mm: bounded at 1.8e4 s/m and diverged at 3.6e5 s/m on all
    three, while the 0.5 mm grid stays bounded at 72 s, a lambda three times
    that of the diverging 2 mm run at 360 s;
  * with forcing that keeps the state away from saturation (RH 0.5 +- 0.1 at
    constant temperature) the Table 1 wall stays bounded to dt* = 5e-2, the
    top of the range Sec. 4 recommends.
"""
import numpy as np
import pytest

import oracle
from paper_1703_10119_amd import workloads as wl

F = wl.LAYER_FIELDS


def _wall(nx=101, law=1, amp_rh=0.2, amp_t=10.0, mean_rh=0.5, k_shape=None, c_shape=None):
    """10 cm wall, outdoor sinusoids on side 0 (h_T 25, h_M 2e-7), 20 degC /
    50 % inside (h_T 8, h_M 3e-8), uniform initial 20 degC / 50 %.  law 1:
    the Table 1 material; law 0: the nominal shape law with the given
    (a_T, a_M) and (c_T, c_M) shape coefficients."""
    w = wl._empty_walls(1)
    w["nx"][:] = nx
    w["n_layers"][:] = 1
    if law == 0:
        wl._shape_all(w, 1)
        for k, v in wl.NOMINAL.items():
            w["layer"][0, 0, F.index(k)] = v
        w["layer"][0, 0, F.index("aT")], w["layer"][0, 0, F.index("aM")] = k_shape
        w["layer"][0, 0, F.index("cT")], w["layer"][0, 0, F.index("aC")] = c_shape
    else:
        for k in ("k0", "kM0", "c0", "cM0"):
            w["layer"][0, 0, F.index(k)] = 1.0
    w["layer"][0, 0, F.index("thick")] = 0.1
    w["hT"][0] = (25.0, 8.0)
    w["hM"][0] = (2e-7, 3e-8)
    wl._sine(w["Tamb"][0, 0], 293.15, amp_t, wl.DAY, 0.0)
    wl._sine(w["RHamb"][0, 0], mean_rh, amp_rh, wl.DAY / 2, 0.0)
    wl._sine(w["Tamb"][0, 1], 293.15, 0.0, wl.DAY, 0.0)
    wl._sine(w["RHamb"][0, 1], 0.5, 0.0, wl.DAY / 2, 0.0)
    w["T0"][:] = 293.15
    w["RH0"][:] = 0.5
    return w


def _bounded(w, dt, hours=120.0, law=1):
    """True if the wall stays finite within 200-400 K for `hours`."""
    s = oracle.RefSim(w, wl.default_config(dt=dt, law=law))
    n = int(round(hours * 3600.0 / dt))
    chunk = max(1, int(round(3600.0 / dt)))
    done = 0
    while done < n:
        k = min(chunk, n - done)
        s.step(k)
        done += k
        T, P = s.fields(0, 0)
        if not (np.all(np.isfinite(T)) and np.all(np.isfinite(P))) or T.min() < 200 or T.max() > 400:
            return False
    return True


def test_conductivities_not_capacities_set_the_limit():
    """Shape law, RH 0.6 +- 0.3 and T 293 +- 15 K outside, dt = 360 s on the
    1 mm grid (dt* = 0.1, lambda_T ~ 300): constant conductivities with
    capacities 2x and 11x from dry to wet stay bounded; conductivities 3x and
    31x from dry to wet with constant capacities diverge; at dt = 3.6 s both
    stay bounded."""
    kw = dict(law=0, amp_rh=0.3, amp_t=15.0, mean_rh=0.6)
    caps = _wall(k_shape=(0.0, 0.0), c_shape=(1.0, 10.0), **kw)
    cond = _wall(k_shape=(2.0, 30.0), c_shape=(0.0, 0.0), **kw)
    assert _bounded(caps, 360.0, law=0)
    assert not _bounded(cond, 360.0, law=0)
    assert _bounded(cond, 3.6, hours=48.0, law=0)


def test_table1_wall_at_the_papers_grid_and_beyond():
    """Table 1 wall, RH 0.5 +- 0.2 and T 293 +- 10 K outside (the surface
    cools below the dew point of the initial vapour pressure: phi > 1 there,
    where this material's c_M vanishes): bounded at dt* = 1e-3, diverged at
    dt* = 1e-2."""
    assert _bounded(_wall(), 3.6, hours=72.0)
    assert not _bounded(_wall(), 36.0)


@pytest.mark.parametrize("nx", [51, 101, 201])
def test_table1_onset_follows_dt_over_dx(nx):
    """RH 0.5 +- 0.2 at constant temperature: bounded at dt/dx = 1.8e4 s/m and
    diverged at 3.6e5 s/m on every grid."""
    dx = 0.1 / (nx - 1)
    w = lambda: _wall(nx=nx, amp_t=0.0)   # noqa: E731
    assert _bounded(w(), 1.8e4 * dx)
    assert not _bounded(w(), 3.6e5 * dx)


def test_table1_onset_is_not_a_lambda_limit():
    """The 0.5 mm grid stays bounded at dt = 72 s (lambda_T = 2 nu dt / dx^2
    ~ 260 with nu_T = 4.5e-7 m2/s) while the 2 mm grid diverges at 360 s
    (lambda_T ~ 80): what sets the limit is dt/dx (1.4e5 against 1.8e5 s/m)."""
    assert _bounded(_wall(nx=201, amp_t=0.0), 72.0)
    assert not _bounded(_wall(nx=51, amp_t=0.0), 360.0)


def test_table1_wall_with_moderate_forcing_over_the_papers_range():
    """RH 0.5 +- 0.1 at constant temperature: bounded for 120 h at dt* = 5e-2
    (180 s, 1.8e5 s/m) on the 1 mm grid."""
    assert _bounded(_wall(amp_rh=0.1, amp_t=0.0), 180.0)
