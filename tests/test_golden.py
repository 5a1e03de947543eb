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


# ---------------------------------------------------------------- closed forms (mpmath, no oracle)

CLOSED = _load("closed_forms.json")


def test_closed_form_fixture_is_reproduced():
    """The stored table is what its committed script computes (no oracle involved)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("mcf", os.path.join(GOLDEN, "make_closed_forms.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    fresh = m.table()
    assert len(fresh["pairs"]) == len(CLOSED["pairs"])
    for a, b in zip(fresh["pairs"], CLOSED["pairs"]):
        assert (a["form"], a["r"], a["lam"]) == (b["form"], b["r"], b["lam"])
        assert np.allclose(a["values"], b["values"], rtol=1e-14, atol=0)


@pytest.mark.parametrize("form", ["beutler", "lbf", "plain"])
def test_oracle_single_pair_against_closed_forms(form):
    """Energy, -du/dr, the left du/dlambda and the parameter derivatives of
    one pair at interior lambda (Beutler 1/2 < lambda < 1 included: the
    electrostatic stage) and inside the u_cap core, against 40-digit values."""
    sched = O.LBF if form == "lbf" else O.BEUTLER
    prm = CLOSED["params"]
    P = O.Params(prm["cutoff"], prm["switch_width"], prm["dsf_alpha"], prm["sc_alpha"], sched)
    rows = [r for r in CLOSED["pairs"] if r["form"] == form]
    assert rows
    for row in rows:
        got = O.pair_probe(row["r"], prm["sigma"], prm["epsilon"], prm["qq"], form != "plain", P, row["lam"])
        want = np.asarray(row["values"])
        scale = np.maximum(np.abs(want), 1e-9 * np.abs(want).max())
        assert np.all(np.abs(got - want) <= 1e-10 * scale), (row, got)


def test_lbf_switches_against_closed_forms():
    for row in CLOSED["lbf_switches"]["rows"]:
        got = O.lbf_switches(row["lam"])
        assert np.allclose(got, row["values"], rtol=1e-12, atol=1e-15), (row["lam"], got)


def test_survey_two_particle_values_are_in_the_fixture():
    """The Beutler values at r = 3.5 A for lambda = 0.25, 0.5, 0.75, 1 and
    the LBF values at r = 2.0 A (lambda = 1/2, inside the cap) and 3.5 A
    (lambda = 3/4), as (u, -du/dr, du/dlambda)."""
    want = {("beutler", 3.5, 0.25): (-0.0599775149151449, 0.00354216174004655, -0.238703144380784),
            ("beutler", 3.5, 0.5): (-0.116604573669458, 0.0808486142144937, -0.205661724322461),
            ("beutler", 3.5, 0.75): (-4.33560631530104, -3.14116426025866, -16.8760069665263),
            ("beutler", 3.5, 1.0): (-8.55460805693263, -6.36317713473181, -16.8760069665263),
            ("lbf", 2.0, 0.5): (6.01621994111549, 25.7411909367237, 74.9360523040282),
            ("lbf", 3.5, 0.75): (-4.96647097336035, -3.64053694937599, -26.9746205340027)}
    rows = {(r["form"], r["r"], r["lam"]): r["values"] for r in CLOSED["pairs"]}
    for key, v in want.items():
        assert np.allclose(rows[key][:3], v, rtol=1e-13), key
    # lambda = 1 is the plain potential (Beutler: lv = 1 gives x = (s/r)^6)
    plain = O.pair_probe(3.5, 3.2, 0.12, -0.3, False, O.Params(9.0, 1.0, 0.2, 0.5, O.BEUTLER), 0.5)[0]
    assert plain == pytest.approx(want[("beutler", 3.5, 1.0)][0], rel=1e-13)
