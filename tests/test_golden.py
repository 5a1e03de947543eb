"""The oracle against stored values: the constants the paper prints
(tests/golden/paper_constants.json, each with its passage) and the oracle's
own results on the seeded config-1 box (tests/golden/config1_oracle.json,
written by tests/golden/make_golden.py from the oracle alone)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import opes as Op
from paper_2608_12691_amd import systems as S

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _poly(coeffs, x):
    return sum(c * x ** int(p) for p, c in coeffs.items())


PAPER = _load("paper_constants.json")
ORACLE = _load("config1_oracle.json")


# ---------------------------------------------------------------- printed constants

def test_ucap_matches_printed_polynomial():
    inner = PAPER["ucap_polynomial"]["coefficients_by_power"]
    outer = PAPER["ucap_outer_branch"]["coefficients_by_power"]
    for x in np.linspace(0.0, 0.999, 23):
        assert O.ucap(x)[0] == pytest.approx(_poly(inner, x), rel=1e-13, abs=1e-12)
    for x in (1.0, 1.05, 1.3, 2.0, 3.5):
        assert O.ucap(x)[0] == pytest.approx(_poly(outer, x), rel=1e-13, abs=1e-13)
    assert O.ucap(0.0)[0] == PAPER["ucap_value_at_zero"]["value"]


def test_lbf_switches_match_printed_smoothsteps():
    a = PAPER["hA_argument"]
    s22 = PAPER["S22_polynomial"]["coefficients_by_power"]
    s32 = PAPER["S32_polynomial"]["coefficients_by_power"]
    for lam in np.linspace(0.0, 1.0, 41):
        x = (lam - a["onset"]) / a["width"]
        hA_ref = _poly(s32, x) if x > 0 else 0.0
        hB_ref = _poly(s22, lam) - hA_ref
        hA, hB, _, _ = O.lbf_switches(lam)
        assert hA == pytest.approx(hA_ref, abs=1e-14)
        assert hB == pytest.approx(hB_ref, abs=1e-14)
    e = PAPER["end_states"]
    for lam in np.linspace(0.0, e["hA_zero_up_to"], 8):
        assert O.lbf_switches(lam)[0] == 0.0
    hA, hB, _, _ = O.lbf_switches(1.0)
    assert hA == pytest.approx(e["hA_at_1"], abs=1e-15) and hB == pytest.approx(e["hB_at_1"], abs=1e-15)


def test_theta_map_printed_cases():
    for theta, lam in PAPER["theta_map"]["theta_lambda_pairs"]:
        assert Op.theta_to_lambda(theta)[1] == pytest.approx(lam, abs=1e-15)


def test_opes_settings_are_the_printed_ones():
    o = PAPER["opes_settings"]
    assert Op.GRID == o["grid_points"]
    op = Op.DualOpes(kT=0.6)
    assert op.sigma == o["gaussian_width"]
    kT = 0.6
    g_std, nu_std, _ = op.c_std
    g_expl, nu_expl, _ = op.c_expl
    assert g_std == pytest.approx(o["barrier_standard_rigid"] / kT) and g_expl == pytest.approx(o["barrier_explore"] / kT)
    assert nu_std == pytest.approx(1.0 - 1.0 / g_std) and nu_expl == pytest.approx(g_expl - 1.0)


# ---------------------------------------------------------------- oracle regression

def test_golden_inputs_are_reproduced():
    """The seeded generator still builds the box the stored values belong to."""
    w = S.make_config(1)
    s = w.systems[0]
    fp = ORACLE["inputs"]
    p = np.asarray(s.positions, dtype=np.float64)
    assert p.shape[0] == fp["n_atoms"] and int(np.sum(s.is_solute)) == fp["n_solute"]
    assert np.asarray(s.exclusions).shape[0] == fp["n_exclusions"]
    assert list(map(float, s.box)) == fp["box"]
    assert float(p.sum()) == pytest.approx(fp["sum"], rel=1e-14)
    assert float((p * p).sum()) == pytest.approx(fp["sum_sq"], rel=1e-14)
    assert np.array_equal(p[0], fp["first"]) and np.array_equal(p[-1], fp["last"])


def test_oracle_reproduces_golden():
    w = S.make_config(1)
    s = w.systems[0]
    atoms = ORACLE["force_atoms"]
    sched = {"beutler": O.BEUTLER, "lbf": O.LBF}
    for c in ORACLE["cases"]:
        r = O.evaluate_system(s, w.ff, O.Params.of(w, sched[c["schedule"]]), c["lam"])
        scale = np.asarray(c["abs_terms"])
        err = np.abs(r["terms"] - np.asarray(c["terms"]))
        assert np.all(err <= 1e-12 * np.maximum(scale, 1.0)), (c["schedule"], c["lam"], err)
        assert r["n_pairs"] == c["n_pairs"]
        F = r["forces"][atoms]
        Fg = np.asarray(c["forces"])
        assert np.sqrt(np.sum((F - Fg) ** 2) / np.sum(Fg * Fg)) < 1e-12
