"""Pins of the Ewald/PME oracle (oracle/pme.py) against facts that do not
come from the oracle itself: textbook values of cardinal B-splines, the
Madelung constant of rock salt, the Wigner lattice constant of a single
charge in a cubic box, the independence of an Ewald sum from its
splitting parameter, and convergence of PME to the Ewald sum."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import pme as P

from conftest import workload

# Madelung constant of the rock-salt structure (per ion pair, nearest-neighbour distance)
MADELUNG_NACL = 1.7475645946331822
# Wigner lattice constant of the simple cubic lattice: a unit charge in a cubic
# box of edge L with a neutralising background has Ewald energy -xi/(2L)
WIGNER_SC = 2.8372974794806202


def test_bspline_textbook_values():
    # M_2 is the hat function, M_3 and M_4 the quadratic and cubic B-splines
    assert P.bspline(1.0, 2) == 1.0 and P.bspline(0.5, 2) == 0.5
    assert P.bspline(1.0, 3) == pytest.approx(0.5) and P.bspline(1.5, 3) == pytest.approx(0.75)
    assert [float(P.bspline(k, 4)) for k in (1, 2, 3)] == pytest.approx([1 / 6, 2 / 3, 1 / 6], abs=1e-15)
    u = np.linspace(0.0, 1.0, 7)
    assert P.bspline(u, 4) == pytest.approx(u ** 3 / 6, abs=1e-15)          # first piece of the cubic
    assert P.bspline(u + 3.0, 4) == pytest.approx((1 - u) ** 3 / 6, abs=1e-15)
    assert float(P.bspline(-0.1, 5)) == 0.0 and float(P.bspline(5.1, 5)) == 0.0


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_bspline_partition_of_unity_symmetry_and_derivative(n):
    rng = np.random.Generator(np.random.PCG64(11))
    w = rng.uniform(0.0, 1.0, 50)
    j = np.arange(n)
    assert P.bspline(w[:, None] + j, n).sum(axis=1) == pytest.approx(np.ones(50), abs=1e-14)
    assert P.bspline_d(w[:, None] + j, n).sum(axis=1) == pytest.approx(np.zeros(50), abs=1e-13)
    u = rng.uniform(0.0, n, 50)
    assert P.bspline(u, n) == pytest.approx(P.bspline(n - u, n), abs=1e-14)
    h = 1e-6
    fd = (P.bspline(u + h, n) - P.bspline(u - h, n)) / (2 * h)
    assert P.bspline_d(u, n) == pytest.approx(fd, abs=1e-8)


def test_bspline_moduli_at_zero_and_at_nyquist():
    for n in (4, 5, 6):
        b = P.bspline_moduli(32, n)
        assert b[0] == pytest.approx(1.0)                     # sum_k M_n(k+1) = 1
        assert np.all(np.isfinite(b)) and np.all(b >= 1.0 - 1e-12)
        assert b[1:] == pytest.approx(b[1:][::-1])            # |b(m)| = |b(K - m)|
    # odd order on an even grid: the Nyquist denominator vanishes; the reading
    # takes the mean of the neighbouring |D|^2
    b5 = P.bspline_moduli(32, 5)
    assert 1.0 / b5[16] == pytest.approx(0.5 * (1.0 / b5[15] + 1.0 / b5[17]))


def _rock_salt(cells=4, a0=5.64):
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    shifts = np.array([[i, j, k] for i in range(cells) for j in range(cells) for k in range(cells)])
    na = (fcc[None] + shifts[:, None]).reshape(-1, 3) * a0
    cl = na + np.array([0.5 * a0, 0.0, 0.0])
    pos = np.concatenate([na, cl])
    types = np.array([0] * len(na) + [1] * len(cl), np.int32)
    return pos, types, a0 * cells, a0 / 2


def test_madelung_constant_of_rock_salt():
    """Real space (the C oracle's Ewald mode) + exact reciprocal sum + self
    term of 512 ions in 4x4x4 conventional cells: -M k_e/d per ion pair."""
    pos, types, L, d = _rock_salt()
    n = len(pos)
    sol = np.zeros(n, np.uint8)
    alpha = 0.42
    prm = O.Params(11.2, 0.0, alpha, 0.5, O.BEUTLER, ewald=True)
    r = O.evaluate(pos, types, sol, np.zeros((0, 2), np.int32), [L] * 3, np.array([1.0, 1.0]),
                   np.array([0.0, 0.0]), np.array([1.0, -1.0]), prm, 0.5)
    q = np.array([1.0, -1.0])[types]
    rec = P.ewald_reciprocal(pos, q, sol, [L] * 3, alpha, [19] * 3)
    cor = P.ewald_corrections(pos, q, sol, np.zeros((0, 2)), [L] * 3, alpha)
    E = r["terms"][0] + rec["e_ww"] + cor["e_ww"]
    assert E == pytest.approx(-(n / 2) * MADELUNG_NACL * P.KE / d, rel=1e-9)
    # every ion sits at a centre of symmetry: no force
    assert np.abs(r["forces"] + rec["forces"]).max() < 1e-9


@pytest.mark.parametrize("L", [10.0, 13.0])
def test_wigner_constant_of_a_charge_in_a_cubic_box(L):
    """One unit charge, no pairs: reciprocal + self + background = -k_e xi/(2L)."""
    x = np.array([[1.0, 2.0, 3.0]])
    rec = P.ewald_reciprocal(x, [1.0], [0], [L] * 3, 1.0, [22] * 3)
    cor = P.ewald_corrections(x, [1.0], [0], np.zeros((0, 2)), [L] * 3, 1.0)
    assert rec["e_ww"] + cor["e_ww"] == pytest.approx(-P.KE * WIGNER_SC / (2 * L), rel=1e-12)


def _ewald_total(w, lam, alpha, schedule, mmax):
    s = w.systems[0]
    prm = O.Params(w.cutoff, w.switch_width, alpha, w.sc_alpha, schedule, ewald=True)
    return P.evaluate_system(s, w.ff, prm, lam, None, None, reciprocal=("exact", mmax))


@pytest.mark.parametrize("schedule", [O.BEUTLER, O.LBF], ids=["beutler", "lbf"])
def test_ewald_sum_is_independent_of_the_splitting_parameter(schedule):
    """The 660-atom box (9 A cutoff, water exclusions, a fully excluded
    solute) at lambda = 0.8: the total energy, dU/dlambda and the forces
    with the exact reciprocal sum agree at a = 0.55 and 0.65 A^-1, which
    fixes the self, exclusion and background parts against the real and
    reciprocal ones (both truncations below 1e-11)."""
    w = workload(1)
    a = _ewald_total(w, 0.8, 0.55, schedule, [20] * 3)
    b = _ewald_total(w, 0.8, 0.65, schedule, [24] * 3)
    scale = np.abs(a["terms"]).max()
    assert np.abs(a["terms"] - b["terms"]).max() < 1e-9 * scale
    # the S-W electrostatics (real + reciprocal + corrections) is a slot of its own
    assert a["terms"][3] == pytest.approx(b["terms"][3], rel=1e-8)
    fr = np.sqrt(np.sum((a["forces"] - b["forces"]) ** 2) / np.sum(a["forces"] ** 2))
    assert fr < 1e-8


def test_pme_converges_to_the_ewald_reciprocal_sum():
    w = workload(1)
    s = w.systems[0]
    q = w.ff.charge[s.types]
    alpha = 0.35
    ref = P.ewald_reciprocal(s.positions, q, s.is_solute, s.box, alpha, [16] * 3, c=0.3)
    errs = []
    for K, n in (((20, 20, 20), 4), ((32, 30, 32), 5), ((48, 48, 45), 6)):
        p = P.pme_reciprocal(s.positions, q, s.is_solute, s.box, alpha, K, n, c=0.3)
        e = max(abs(p[k] - ref[k]) / abs(ref[k]) for k in ("e_ss", "e_ww", "e_sw"))
        f = math.sqrt(np.sum((p["forces"] - ref["forces"]) ** 2) / np.sum(ref["forces"] ** 2))
        errs.append((e, f))
    assert errs[0][0] > errs[1][0] > errs[2][0] and errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[2][0] < 1e-6 and errs[2][1] < 1e-5


def test_cross_term_split_sums_to_the_one_group_energy():
    w = workload(1)
    s = w.systems[0]
    q = w.ff.charge[s.types]
    none = np.zeros(len(q), bool)
    for fn, arg in ((P.pme_reciprocal, dict(K=(24, 24, 24), n=5)), (P.ewald_reciprocal, dict(mmax=[8] * 3))):
        split = fn(s.positions, q, s.is_solute, s.box, 0.35, **arg)
        one = fn(s.positions, q, none, s.box, 0.35, **arg)
        assert split["e_ss"] + split["e_ww"] + split["e_sw"] == pytest.approx(one["e_ww"], rel=1e-12)
        assert one["e_ss"] == 0.0 and one["e_sw"] == 0.0
        assert split["forces"] == pytest.approx(one["forces"], rel=1e-10, abs=1e-10)   # c = 1


def test_pme_forces_and_potential_are_derivatives_of_its_energy():
    w = workload(1)
    s = w.systems[0]
    q = w.ff.charge[s.types].astype(float)
    c, K, n = 0.37, (24, 25, 24), 5

    def U(pos, qq):
        p = P.pme_reciprocal(pos, qq, s.is_solute, s.box, 0.35, K, n, c)
        return p["e_ss"] + p["e_ww"] + c * p["e_sw"]

    base = P.pme_reciprocal(s.positions, q, s.is_solute, s.box, 0.35, K, n, c)
    sol = int(np.nonzero(s.is_solute)[0][2])
    h = 1e-5
    for atom, ax in ((sol, 0), (sol, 2), (40, 1), (300, 0)):
        xp, xm = s.positions.copy(), s.positions.copy()
        xp[atom, ax] += h
        xm[atom, ax] -= h
        fd = -(U(xp, q) - U(xm, q)) / (2 * h)
        assert base["forces"][atom, ax] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    for atom in (sol, 40):
        qp, qm = q.copy(), q.copy()
        qp[atom] += 1e-5
        qm[atom] -= 1e-5
        fd = (U(s.positions, qp) - U(s.positions, qm)) / 2e-5
        assert base["potential"][atom] == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("schedule,lam", [(O.BEUTLER, 0.8), (O.LBF, 0.6)], ids=["beutler", "lbf"])
def test_pme_dudl_is_the_lambda_derivative_of_the_energy(schedule, lam):
    w = workload(1)
    s = w.systems[0]
    prm = O.Params(w.cutoff, w.switch_width, 0.35, w.sc_alpha, schedule, ewald=True)
    ev = lambda l: P.evaluate_system(s, w.ff, prm, l, (24, 24, 24), 5)
    r = ev(lam)
    h = 1e-5
    fd = (ev(lam + h)["terms"][8] - ev(lam - h)["terms"][8]) / (2 * h)
    assert r["terms"][9] == pytest.approx(fd, rel=1e-7)
    # the cross term enters dU/dlambda with c'(lambda), the energy with c(lambda)
    c, dc = P.elec_factor(schedule, lam)
    r0 = O.evaluate_system(s, w.ff, prm, lam)
    assert r["terms"][7] - r0["terms"][7] == pytest.approx(dc * r["cross"], rel=1e-12)
    assert r["terms"][3] - r0["terms"][3] == pytest.approx(c * r["cross"], rel=1e-12)
