"""Pins of the CPU oracle to facts outside itself.

Each test checks the oracle against something it does not contain: a
textbook closed form, a statement the paper prints, a library routine
(scipy, mpmath), a brute-force construction, or an invariant of the
potential.  Between them a dropped term, a wrong sign, a wrong index or a
transposed operand anywhere in the oracle fails at least one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle as O
from paper_2608_12691_amd import systems as S

mp.mp.dps = 30
P_BEU = O.Params(cutoff=9.0, switch_width=1.0, dsf_alpha=0.2, sc_alpha=0.5, schedule=O.BEUTLER)
P_LBF = O.Params(cutoff=9.0, switch_width=1.0, dsf_alpha=0.2, sc_alpha=0.5, schedule=O.LBF)


def num_diff(f, x, h=1e-6):
    return (f(x + h) - f(x - h)) / (2 * h)


# ---------------------------------------------------------------- LJ pieces

def test_lj_minimum_textbook():
    """Plain LJ has its minimum -eps at r = 2^(1/6) sigma with zero force."""
    for sig, eps in [(3.2, 0.12), (3.15, 0.152), (2.5, 0.03)]:
        r = 2 ** (1 / 6) * sig
        out = O.pair_probe(r, sig, eps, 0.0, False, P_BEU, 0.5)
        assert out[0] == pytest.approx(-eps, rel=1e-13)
        assert abs(out[1]) < 1e-12


def test_lj_zero_crossing_textbook():
    """At r = sigma the LJ energy is 0 and the force is 24 eps / sigma."""
    sig, eps = 3.4, 0.2
    out = O.pair_probe(sig, sig, eps, 0.0, False, P_BEU, 0.5)
    assert abs(out[0]) < 1e-14
    assert out[1] == pytest.approx(24 * eps / sig, rel=1e-13)


def test_combining_rule_lorentz_berthelot():
    """A two-atom box equals the pair with sigma=(si+sj)/2, eps=sqrt(ei ej)."""
    sig = np.array([3.0, 3.6])
    eps = np.array([0.1, 0.25])
    q = np.array([0.0, 0.0])
    box = np.full(3, 30.0)
    pos = np.array([[1.0, 2.0, 3.0], [4.2, 2.0, 3.0]])
    out = O.evaluate(pos, [0, 1], [0, 0], np.zeros((0, 2)), box, sig, eps, q, P_BEU, 0.5)
    r = 3.2
    s, e = 3.3, math.sqrt(0.025)
    lj = 4 * e * ((s / r) ** 12 - (s / r) ** 6)
    assert out["terms"][0] == pytest.approx(lj, rel=1e-13)


# ---------------------------------------------------------------- switch

def test_smoothstep_s22_paper_properties():
    """S22 has two vanishing derivatives at 0 and at 1 and runs from 0 to 1 (eq. 9)."""
    rc, w = 9.0, 1.0
    rs = rc - w
    assert O.switch(rs, rc, w)[0] == 1.0
    assert abs(O.switch(rc - 1e-15, rc, w)[0]) < 1e-12
    assert O.switch(rs + w / 2, rc, w)[0] == pytest.approx(0.5, abs=1e-15)  # odd symmetry about 1/2
    for r in (rs, rc):
        assert abs(O.switch(r, rc, w)[1]) < 1e-12
    # second derivative vanishes at both ends (numerically)
    d2 = lambda r: num_diff(lambda x: O.switch(x, rc, w)[1], r, 1e-5)
    assert abs(d2(rs + 1e-4)) < 1e-2 and abs(d2(rc - 1e-4)) < 1e-2
    for r in np.linspace(rs + 0.01, rc - 0.01, 9):
        assert O.switch(r, rc, w)[1] == pytest.approx(num_diff(lambda x: O.switch(x, rc, w)[0], r, 1e-5), rel=1e-6)


def test_switch_hard_truncation():
    assert tuple(O.switch(8.99, 9.0, 0.0)) == (1.0, 0.0)


# ---------------------------------------------------------------- DSF

def test_dsf_vanishes_with_slope_at_cutoff():
    for a in (0.2, 0.3):
        v, dv = O.dsf(9.0, 9.0, a)
        assert abs(v) < 1e-15 and abs(dv) < 1e-15


def test_dsf_is_shifted_force_of_damped_coulomb():
    """D(r) = V(r) - V(rc) - V'(rc)(r - rc) with V = erfc(a r)/r (mpmath, numeric V')."""
    a, rc = 0.2, 9.0
    V = lambda r: mp.erfc(a * r) / r
    dVc = mp.diff(V, rc)
    for r in (1.0, 2.7, 4.4, 8.3):
        ref = V(r) - V(rc) - dVc * (r - rc)
        v, dv = O.dsf(r, rc, a)
        assert v == pytest.approx(float(ref), rel=1e-13, abs=1e-15)
        assert dv == pytest.approx(float(mp.diff(V, r) - dVc), rel=1e-12)


def test_dsf_alpha_zero_is_shifted_force_coulomb():
    """a -> 0 gives the textbook shifted-force Coulomb 1/r - 1/rc + (r - rc)/rc^2."""
    rc = 10.0
    for r in (1.5, 3.0, 7.0):
        v, dv = O.dsf(r, rc, 0.0)
        assert v == pytest.approx(1 / r - 1 / rc + (r - rc) / rc ** 2, rel=1e-14)
        assert dv == pytest.approx(-1 / r ** 2 + 1 / rc ** 2, rel=1e-14)


def test_erfc_libm_matches_scipy():
    from scipy.special import erfc
    for x in (0.2, 1.0, 1.8, 2.4):
        r = x / 0.2
        v = O.dsf(r, 12.0, 0.2)[0]
        # recover erfc(a r)/r from D: D(r) - slope (r - rc) + erfc(a rc)/rc
        ec = erfc(0.2 * 12.0)
        slope = ec / 144.0 + 0.2 * 2 / math.sqrt(math.pi) * math.exp(-0.04 * 144.0) / 12.0
        assert (v - slope * (r - 12.0) + ec / 12.0) * r == pytest.approx(erfc(x), rel=1e-13)


# ---------------------------------------------------------------- u_cap (eq. 6)

def test_ucap_printed_values_and_join():
    """u_cap(0) = 119.2 (printed) and a C^3 join with 4x^-12 - 4x^-6 at x = 1."""
    assert O.ucap(0.0)[0] == pytest.approx(119.2, abs=1e-12)
    assert abs(O.ucap(1.0)[0]) < 1e-12 and abs(O.ucap(1.0 - 1e-13)[0]) < 1e-9
    poly = lambda x: -868 * x ** 6 + mp.mpf("2188.8") * x ** 5 - 1440 * x ** 4 + mp.mpf("119.2")
    lj = lambda x: 4 * x ** -12 - 4 * x ** -6
    for k in (1, 2, 3):
        assert float(mp.diff(poly, 1, k)) == pytest.approx(float(mp.diff(lj, 1, k)), rel=1e-12)
    # the oracle's derivative agrees with both branches' numerical derivative
    for x in (0.3, 0.8, 0.999, 1.001, 1.3):
        assert O.ucap(x)[1] == pytest.approx(num_diff(lambda y: O.ucap(y)[0], x, 1e-7), rel=1e-6)
    # monotone decreasing on (0, 1): the cap has no spurious minimum
    xs = np.linspace(0.01, 0.99, 50)
    assert all(O.ucap(x)[1] < 0 for x in xs)


# ---------------------------------------------------------------- h_A, h_B (eqs. 7-10)

def test_lbf_switches_paper_statements():
    for l in (0.0, 0.1, 0.35):
        hA, hB, dA, dB = O.lbf_switches(l)
        assert hA == 0.0 and dA == 0.0           # hA = 0 for lambda <= 0.35
    hA, hB, dA, dB = O.lbf_switches(1.0)
    assert hA == pytest.approx(1.0, abs=1e-15) and abs(hB) < 1e-15   # fully interacting end state
    hA, hB, dA, dB = O.lbf_switches(0.0)
    assert hB == 0.0                              # non-interacting end state
    for l in (0.2, 0.5, 0.75, 0.9):
        h = O.lbf_switches(l)
        assert h[2] == pytest.approx(num_diff(lambda x: O.lbf_switches(x)[0], l), rel=1e-7, abs=1e-9)
        assert h[3] == pytest.approx(num_diff(lambda x: O.lbf_switches(x)[1], l), rel=1e-7, abs=1e-9)


def test_s32_vanishing_derivatives():
    """S32 (eq. 10) has three vanishing derivatives at 0 and two at 1: near the ends
    h_A grows like x^4 and 1 - h_A like 20 (1-x)^3, x = (lambda - 0.35)/0.65."""
    hA = lambda l: O.lbf_switches(l)[0]
    for x in (1e-2, 2e-2):
        assert hA(0.35 + 0.65 * x) == pytest.approx(15 * x ** 4, rel=0.2)
    for x in (1e-2, 2e-2):
        assert 1 - hA(1 - 0.65 * x) == pytest.approx(20 * x ** 3, rel=0.2)
    assert abs(O.lbf_switches(1.0)[2]) < 1e-12


# ---------------------------------------------------------------- Beutler soft core

@pytest.mark.parametrize("lv", [0.25, 0.5, 0.9, 1.0])
def test_beutler_minimum_closed_form(lv):
    """4 eps lv (x^2 - x) is minimal (-lv eps) at x = 1/2, i.e. (r/s)^6 = 2 - a(1 - lv)."""
    sig, eps, a = 3.2, 0.12, 0.5
    lam = lv / 2.0  # lambda <= 1/2 gives lv = 2 lambda, le = 0
    r = sig * (2 - a * (1 - lv)) ** (1 / 6)
    out = O.pair_probe(r, sig, eps, 0.7, True, P_BEU, lam)
    assert out[0] == pytest.approx(-lv * eps, rel=1e-12)
    assert abs(out[1]) < 1e-12


def test_beutler_core_value_at_contact():
    """r -> 0 with lv = 1/2, a = 1/2: x = 4 and u = 4 eps lv (16 - 4) = 24 eps."""
    out = O.pair_probe(1e-7, 3.2, 0.12, 0.0, True, P_BEU, 0.25)
    assert out[0] == pytest.approx(24 * 0.12, rel=1e-12)


def test_end_states_single_pair():
    """lambda = 1 reproduces the plain pair; lambda = 0 decouples it (both schedules)."""
    for P in (P_BEU, P_LBF):
        for r in (2.1, 3.5, 8.5):
            plain = O.pair_probe(r, 3.2, 0.12, -0.3, False, P, 0.5)
            one = O.pair_probe(r, 3.2, 0.12, -0.3, True, P, 1.0)
            zero = O.pair_probe(r, 3.2, 0.12, -0.3, True, P, 0.0)
            assert one[0] == pytest.approx(plain[0], rel=1e-13)
            assert one[1] == pytest.approx(plain[1], rel=1e-12)
            assert zero[0] == 0.0 and zero[1] == 0.0


@pytest.mark.parametrize("P", [P_BEU, P_LBF], ids=["beutler", "lbf"])
@pytest.mark.parametrize("lam", [0.2, 0.4, 0.7, 0.95])
@pytest.mark.parametrize("r", [1.6, 2.9, 3.6, 8.6])
def test_pair_derivatives_consistent_with_energy_differences(P, lam, r):
    """-du/dr, du/dlambda, du/dsig, du/deps, du/dqq agree with central
    differences of the oracle's own pair energy (a consistency check between
    its energy and its derivatives; the values themselves are pinned in
    test_golden.py against 40-digit closed forms)."""
    sig, eps, qq = 3.2, 0.12, -0.3

    def u(r_=r, lam_=lam, sig_=sig, eps_=eps, qq_=qq):
        return O.pair_probe(float(r_), float(sig_), float(eps_), float(qq_), True, P, float(lam_))[0]

    out = O.pair_probe(r, sig, eps, qq, True, P, lam)
    h = 1e-5
    assert out[1] == pytest.approx(-(u(r_=r + h) - u(r_=r - h)) / (2 * h), rel=1e-6, abs=1e-9)
    assert out[2] == pytest.approx((u(lam_=lam + h) - u(lam_=lam - h)) / (2 * h), rel=1e-6, abs=1e-9)
    assert out[3] == pytest.approx((u(sig_=sig + h) - u(sig_=sig - h)) / (2 * h), rel=1e-6, abs=1e-9)
    assert out[4] == pytest.approx((u(eps_=eps + h) - u(eps_=eps - h)) / (2 * h), rel=1e-6, abs=1e-9)
    assert out[5] == pytest.approx((u(qq_=qq + h) - u(qq_=qq - h)) / (2 * h), rel=1e-6, abs=1e-9)


def test_beutler_left_derivative_at_kink():
    """At lambda = 1/2 the vdw stage is finishing (left derivative) and elec has not started."""
    out = O.pair_probe(3.5, 3.2, 0.12, -0.3, True, P_BEU, 0.5)
    left = O.pair_probe(3.5, 3.2, 0.12, -0.3, True, P_BEU, 0.5 - 1e-7)
    u = lambda l: O.pair_probe(3.5, 3.2, 0.12, -0.3, True, P_BEU, l)[0]
    assert out[2] == pytest.approx((u(0.5) - u(0.5 - 1e-6)) / 1e-6, rel=1e-5)
    assert out[2] == pytest.approx(left[2], rel=1e-5)


def test_lbf_below_035_is_pure_softened_basis():
    """For lambda <= 0.35 only h_B eps u_cap S acts; for r >= sigma that is h_B times the switched LJ."""
    for r in (3.3, 4.0, 8.5):
        l = 0.3
        hB = O.lbf_switches(l)[1]
        u = O.pair_probe(r, 3.2, 0.12, -0.3, True, P_LBF, l)[0]
        plain_lj = O.pair_probe(r, 3.2, 0.12, 0.0, False, P_LBF, l)[0]
        assert u == pytest.approx(hB * plain_lj, rel=1e-12)


# ---------------------------------------------------------------- whole boxes

def _box(cfg1):
    return cfg1.systems[0], cfg1.ff, O.Params.of(cfg1)


def test_newton_third_law_and_translation(cfg1):
    s, ff, P = _box(cfg1)
    out = O.evaluate_system(s, ff, P, 0.5)
    F = out["forces"]
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).sum()
    shift = np.array([7.3, -2.9, 11.1])
    out2 = O.evaluate(s.positions + shift, s.types, s.is_solute, s.exclusions, s.box, ff.sigma, ff.epsilon,
                      ff.charge, P, 0.5)
    assert np.allclose(out2["terms"], out["terms"], rtol=1e-12, atol=1e-10)
    assert np.allclose(out2["forces"], F, rtol=1e-10, atol=1e-9)


def test_permutation_invariance(cfg1):
    """Relabelling the atoms permutes the forces and leaves the energies."""
    s, ff, P = _box(cfg1)
    rng = np.random.default_rng(3)
    perm = rng.permutation(s.n_atoms)
    inv = np.argsort(perm)
    ex = inv[s.exclusions]
    ex = np.sort(ex, axis=1)
    ex = ex[np.lexsort((ex[:, 1], ex[:, 0]))]
    for sched in (O.BEUTLER, O.LBF):
        P.schedule = sched
        a = O.evaluate_system(s, ff, P, 0.7)
        b = O.evaluate(s.positions[perm], s.types[perm], s.is_solute[perm], ex, s.box, ff.sigma, ff.epsilon,
                       ff.charge, P, 0.7)
        assert np.allclose(a["terms"], b["terms"], rtol=1e-12, atol=1e-10)
        assert np.allclose(a["forces"][perm], b["forces"], rtol=1e-10, atol=1e-9)
    P.schedule = O.BEUTLER


def test_lambda_one_is_fully_plain(cfg1):
    """lambda = 1 equals the box with no alchemical group (both schedules)."""
    s, ff, P = _box(cfg1)
    plain = O.evaluate(s.positions, s.types, np.zeros_like(s.is_solute), s.exclusions, s.box, ff.sigma,
                       ff.epsilon, ff.charge, P, 1.0)
    for sched in (O.BEUTLER, O.LBF):
        P.schedule = sched
        one = O.evaluate_system(s, ff, P, 1.0)
        assert one["terms"][8] == pytest.approx(plain["terms"][8], rel=1e-12)
        assert np.allclose(one["forces"], plain["forces"], rtol=1e-10, atol=1e-9)
    P.schedule = O.BEUTLER


def test_lambda_zero_decouples(cfg1):
    s, ff, P = _box(cfg1)
    for sched in (O.BEUTLER, O.LBF):
        P.schedule = sched
        z = O.evaluate_system(s, ff, P, 0.0)
        assert z["terms"][2] == 0.0 and z["terms"][3] == 0.0
        solu = np.nonzero(s.is_solute)[0]
        # a rigid solute with all intra pairs excluded feels no force at lambda = 0
        assert np.abs(z["forces"][solu]).max() == 0.0
    P.schedule = O.BEUTLER


def test_energy_fd_in_positions(cfg1):
    s, ff, P = _box(cfg1)
    rng = np.random.default_rng(7)
    for sched, lam in ((O.BEUTLER, 0.3), (O.BEUTLER, 0.8), (O.LBF, 0.6)):
        P.schedule = sched
        F = O.evaluate_system(s, ff, P, lam)["forces"]
        atoms = list(np.nonzero(s.is_solute)[0][:4]) + list(rng.choice(s.n_atoms, 8, replace=False))
        h = 1e-5
        for a in atoms:
            for k in range(3):
                xp = s.positions.copy(); xp[a, k] += h
                xm = s.positions.copy(); xm[a, k] -= h
                fd = -(O.atom_energy(a, s, ff, P, lam, xp) - O.atom_energy(a, s, ff, P, lam, xm)) / (2 * h)
                assert F[a, k] == pytest.approx(fd, rel=2e-6, abs=2e-7)
    P.schedule = O.BEUTLER


def test_energy_fd_in_lambda_and_params(cfg1):
    s, ff, P = _box(cfg1)
    h = 1e-5
    for sched, lam in ((O.BEUTLER, 0.3), (O.BEUTLER, 0.8), (O.LBF, 0.45), (O.LBF, 0.8)):
        P.schedule = sched
        out = O.evaluate_system(s, ff, P, lam, param_grads=True)
        E = lambda l: O.evaluate_system(s, ff, P, l, forces=False)["terms"][8]
        assert out["terms"][9] == pytest.approx((E(lam + h) - E(lam - h)) / (2 * h), rel=1e-6)
        for t in [0, 1, 2, 5, 9]:
            for name, arr in (("d_sigma", "sigma"), ("d_charge", "charge"), ("d_eps", "epsilon")):
                if name == "d_eps" and ff.epsilon[t] == 0:
                    continue
                def Et(v):
                    ff2 = S.ForceField(ff.sigma.copy(), ff.epsilon.copy(), ff.charge.copy(), ff.names)
                    getattr(ff2, arr)[t] = v
                    return O.evaluate_system(s, ff2, P, lam, forces=False)["terms"][8]
                v0 = getattr(ff, arr)[t]
                fd = (Et(v0 + h) - Et(v0 - h)) / (2 * h)
                assert out[name][t] == pytest.approx(fd, rel=1e-5, abs=1e-6), (sched, name, t)
    P.schedule = O.BEUTLER


def test_pair_set_vs_kdtree_bruteforce(cfg1):
    """The list pair set equals scipy's periodic KD-tree query minus exclusions."""
    s = cfg1.systems[0]
    L = s.box[0]
    for r_list in (6.0, 9.0):
        ours = O.pair_set(s.positions, s.exclusions, s.box, r_list)
        w = np.mod(s.positions, L)
        tree = cKDTree(w, boxsize=L)
        ref = tree.query_pairs(r_list, output_type="ndarray")
        ref = np.sort(ref, axis=1)
        excl = set(map(tuple, s.exclusions.tolist()))
        ref = np.array([p for p in ref.tolist() if tuple(p) not in excl])
        ref = ref[np.lexsort((ref[:, 1], ref[:, 0]))]
        assert ours.shape == ref.shape
        assert np.array_equal(ours, ref)


def test_pair_count_vs_kdtree(cfg1):
    s, ff, P = _box(cfg1)
    out = O.evaluate_system(s, ff, P, 0.5, forces=False)
    tree = cKDTree(np.mod(s.positions, s.box[0]), boxsize=s.box[0])
    n = len(tree.query_pairs(P.cutoff)) - len(s.exclusions)  # every excluded pair is within the cutoff
    assert out["n_pairs"] == n


def test_exclusion_removes_exactly_the_pair():
    """Excluding a pair subtracts that pair's energy (two-atom box vs three-atom box)."""
    box = np.full(3, 25.0)
    pos = np.array([[1.0, 1.0, 1.0], [4.5, 1.2, 0.8], [1.5, 4.1, 2.0]])
    sig, eps, q = np.array([3.2, 3.0, 3.6]), np.array([0.1, 0.2, 0.15]), np.array([0.4, -0.3, -0.1])
    types = [0, 1, 2]
    full = O.evaluate(pos, types, [0, 0, 0], np.zeros((0, 2)), box, sig, eps, q, P_BEU, 0.5)["terms"][8]
    ex = O.evaluate(pos, types, [0, 0, 0], np.array([[0, 2]]), box, sig, eps, q, P_BEU, 0.5)["terms"][8]
    pair02 = O.evaluate(pos[[0, 2]], [0, 2], [0, 0], np.zeros((0, 2)), box, sig, eps, q, P_BEU, 0.5)["terms"][8]
    assert full - ex == pytest.approx(pair02, rel=1e-12)


def test_minimum_image_across_boundary():
    """Two atoms 3.5 A apart through the periodic face equal the bare pair."""
    box = np.full(3, 20.0)
    pos = np.array([[0.5, 10.0, 10.0], [17.0, 10.0, 10.0]])
    out = O.evaluate(pos, [0, 0], [0, 1], np.zeros((0, 2)), box, [3.2], [0.12], [0.0], P_BEU, 0.75)
    ref = O.pair_probe(3.5, 3.2, 0.12, 0.0, True, P_BEU, 0.75)
    assert out["terms"][8] == pytest.approx(ref[0], rel=1e-13)
    # atom 1 sits at x = -3 relative to atom 0: the force on it points along -x when repulsive
    assert out["forces"][1, 0] == pytest.approx(-ref[1], rel=1e-12)


def test_input_validation():
    with pytest.raises(ValueError):
        O.evaluate(np.zeros((2, 3)), [0, 0], [0, 0], np.zeros((0, 2)), np.full(3, 10.0), [3.0], [0.1], [0.0],
                   P_BEU, 0.5)  # box smaller than twice the cutoff
    with pytest.raises(ValueError):
        O.evaluate(np.zeros((2, 3)), [0, 0], [0, 0], np.array([[1, 0]]), np.full(3, 30.0), [3.0], [0.1], [0.0],
                   P_BEU, 0.5)  # exclusion with i > j


def test_atoms_terms_restrict_the_full_sum(cfg1):
    """Per-atom sums: forces equal the full evaluation's, the solute atoms'
    lambda derivatives add up to dU/dlambda (each solute-solvent pair has one
    solute atom), and the atom energies count every pair twice."""
    s, ff, P = _box(cfg1)
    for sched, lam in ((O.BEUTLER, 0.3), (O.BEUTLER, 0.8), (O.LBF, 0.6)):
        P.schedule = sched
        full = O.evaluate_system(s, ff, P, lam)
        every = np.arange(s.n_atoms)
        at = O.atoms_terms(every, s, ff, P, lam)
        np.testing.assert_allclose(at["forces"], full["forces"], rtol=1e-12, atol=1e-11)
        assert at["n_pairs"].sum() == 2 * full["n_pairs"]
        assert at["energy"].sum() == pytest.approx(2 * full["terms"][8], rel=1e-12)
        solu = np.nonzero(s.is_solute)[0]
        assert O.atoms_terms(solu, s, ff, P, lam)["dudl"].sum() == pytest.approx(full["terms"][9], rel=1e-12)
        # the per-atom energy is the atom-energy function of the FD tests
        for a in (0, int(solu[0]), s.n_atoms - 1):
            assert at["energy"][a] == pytest.approx(O.atom_energy(a, s, ff, P, lam), rel=1e-13)
    P.schedule = O.BEUTLER


def test_atoms_terms_force_is_minus_gradient(cfg1):
    s, ff, P = _box(cfg1)
    lam, h = 0.65, 1e-5
    atoms = np.array([1, 40, int(np.nonzero(s.is_solute)[0][2])])
    f = O.atoms_terms(atoms, s, ff, P, lam)["forces"]
    for i, a in enumerate(atoms):
        for k in range(3):
            xp = s.positions.copy(); xp[a, k] += h
            xm = s.positions.copy(); xm[a, k] -= h
            fd = -(O.atom_energy(a, s, ff, P, lam, xp) - O.atom_energy(a, s, ff, P, lam, xm)) / (2 * h)
            assert f[i, k] == pytest.approx(fd, rel=2e-6, abs=2e-7)
