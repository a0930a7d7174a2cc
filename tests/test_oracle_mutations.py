"""Planted mistakes in the oracle must fail its pins (CPU only).

Each case copies ``oracle/dfhm_ref.c`` to a temporary directory, plants one
plausible mistake by a textual substitution, builds the copy with the
oracle's own compiler flags and runs the law pins of
``test_oracle_law_pins.py`` against it in a fresh process (the oracle loads
the copy named by ``DFHM_REF_LIB``).  The pins must fail for every mistake
and pass for the unmodified copy.  The network oracle's activation is pinned
the same way in ``test_mlp_oracle.py``.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dfhm_ref.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_law_pins.py")

_FACE = ("    double Tf = 0.5 * (T[j] + T[j + 1]);\n"
         "    double Pf = 0.5 * (P[j] + P[j + 1]);\n"
         "    ref_kcoef a = law_k(w, &w->layer[lay[j]], Tf, Pf);\n")
_FACE_NODE_MEAN = (
    "    double Tf = 0.5 * (T[j] + T[j + 1]);\n"
    "    double Pf = 0.5 * (P[j] + P[j + 1]);\n"
    "    ref_kcoef a0 = law_k(w, &w->layer[lay[j]], T[j], P[j]);\n"
    "    ref_kcoef a1 = law_k(w, &w->layer[lay[j]], T[j + 1], P[j + 1]);\n"
    "    ref_kcoef a = {0.5 * (a0.kTT + a1.kTT), 0.5 * (a0.kM + a1.kM), 0.5 * (a0.kTM + a1.kTM)};\n")

MUTANTS = {
    "k_M linear in phi": ("k.kM = m->kM0 * (1.0 + m->aM * phi * phi);",
                          "k.kM = m->kM0 * (1.0 + m->aM * phi);"),
    "10x k_TT slope": ("k.kTT = m->k0 * (1.0 + m->aT * phi);",
                       "k.kTT = m->k0 * (1.0 + 10.0 * m->aT * phi);"),
    "10x c_TT slope": ("c.cTT = m->c0 * (1.0 + m->cT * phi);",
                       "c.cTT = m->c0 * (1.0 + 10.0 * m->cT * phi);"),
    "10x c_M slope": ("c.cM = m->cM0 * (1.0 + m->aC * phi);",
                      "c.cM = m->cM0 * (1.0 + 10.0 * m->aC * phi);"),
    "theta in K in c_TM": ("c.cTM = (m->eTM + m->fTM * th) * c.cM;",
                           "c.cTM = (m->eTM + m->fTM * T) * c.cM;"),
    "k_TM from the scale only": ("k.kTM = m->bTM * k.kM;", "k.kTM = m->bTM * m->kM0;"),
    "node-averaged faces": (_FACE, _FACE_NODE_MEAN),
    "arithmetic interface mean": ("return s > 0.0 ? 2.0 * a * b / s : 0.0;",
                                  "return 0.5 * s;"),
    "relative humidity against the wrong Magnus slope": (
        "return 610.94 * exp(17.625 * th / (th + 243.04));",
        "return 610.94 * exp(17.625 * th / (th + 273.15));"),
}


def _build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    if old is not None:
        assert src.count(old) == 1, f"{name}: pattern not found exactly once"
        src = src.replace(old, new)
    d = tmp_path / name.replace(" ", "_")
    d.mkdir()
    c = d / "dfhm_ref.c"
    c.write_text(src)
    so = d / "libdfhm_ref.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off",
                           "-fPIC", "-shared", str(c), "-o", str(so), "-lm"])
    return str(so)


def _run_pins(so):
    env = dict(os.environ, DFHM_REF_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        PINS, os.path.join(ROOT, "tests", "test_constants.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout[-2000:]


def test_unmodified_copy_passes(tmp_path):
    rc, out = _run_pins(_build_variant(tmp_path, "unmodified", None, None))
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    old, new = MUTANTS[name]
    rc, out = _run_pins(_build_variant(tmp_path, name, old, new))
    assert rc != 0, f"planted mistake '{name}' passed every law pin:\n{out}"
