"""Pins of the constants and readings the method depends on (CPU only)."""
import json
import math
import os

import pytest

import oracle
from paper_1703_10119_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_magnus_against_steam_tables():
    """Ps(T) of the oracle within 0.4 % of the IAPWS-95 saturation pressure."""
    d = json.load(open(os.path.join(GOLD, "psat_water_table.json")))
    for tc, ps in zip(d["T_celsius"], d["Ps_Pa"]):
        assert oracle.psat(273.15 + tc) == pytest.approx(ps, rel=4e-3)


def test_appendix_b_recomputed_from_table2():
    """Table 2 + L = 0.1 m, t0 = 3600 s, Ti = 20 degC, phi_i = 0.5, with
    L_v = 2.5e6 J/kg and Magnus Ps reproduce every Fourier, Biot and gamma
    number App. B prints for the three walls, at both surfaces, within 1 %."""
    d = json.load(open(os.path.join(GOLD, "table2_appendix_b.json")))
    sc = d["reference_scales"]
    L, t0, Ti = sc["L_m"], sc["t0_s"], sc["Ti_K"]
    Pvi = sc["phi_i"] * oracle.psat(Ti)
    Lv = wl.LV
    hin = d["interior_exchange"]
    for name, v in d["walls"].items():
        b = d["appendix_b"][name]
        got = dict(
            FoM=t0 * v["kM"] / (L * L * v["cM"]),
            FoTT=t0 * v["kTT"] / (L * L * v["cTT"]),
            FoTM=t0 * v["kTM"] / (L * L * v["cTM"]),
            gamma=v["cTM"] * Pvi / (v["cTT"] * Ti),
            BiM0=v["hM"] * L / v["kM"], BiTT0=v["hT"] * L / v["kTT"],
            BiTM0=Lv * v["hM"] * L * Pvi / (v["kTT"] * Ti),
            BiM1=hin["hM"] * L / v["kM"], BiTT1=hin["hT"] * L / v["kTT"],
            BiTM1=Lv * hin["hM"] * L * Pvi / (v["kTT"] * Ti),
        )
        for k, val in got.items():
            assert val == pytest.approx(b[k], rel=1e-2), (name, k, val, b[k])


def test_coupling_storage_uses_celsius():
    """Table 2: c_TM / (c_w c_M) = 20 for every wall, i.e. the temperature in
    c_TM = c_w T f'/Ps is read in degC at Ti = 20 degC (fTM = c_w, theta =
    T - 273.15 in the law)."""
    d = json.load(open(os.path.join(GOLD, "table2_appendix_b.json")))
    for v in d["walls"].values():
        assert v["cTM"] / (wl.CW * v["cM"]) == pytest.approx(20.0, rel=1e-2)
    assert wl.SHAPE["fTM"] == wl.CW and wl.SHAPE["eTM"] == 0.0


def test_nominal_wall_equals_table2_east_west_at_half_humidity():
    """The nominal law scales reproduce Table 2's east/west wall at phi = 0.5."""
    d = json.load(open(os.path.join(GOLD, "table2_appendix_b.json")))["walls"]["east_west"]
    N, S = wl.NOMINAL, wl.SHAPE
    phi = 0.5
    assert N["k0"] * (1 + S["aT"] * phi) == pytest.approx(d["kTT"], rel=2e-3)
    assert N["kM0"] * (1 + S["aM"] * phi * phi) == pytest.approx(d["kM"], rel=2e-3)
    assert N["c0"] * (1 + S["cT"] * phi) == pytest.approx(d["cTT"], rel=2e-3)
    assert N["cM0"] * (1 + S["aC"] * phi) == pytest.approx(d["cM"], rel=2e-3)
