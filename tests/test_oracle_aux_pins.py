"""Pins of the dihedral/d-AFED and lambda/OPES oracles to facts outside them."""
import math

import numpy as np
import pytest

from oracle import dihedral as D
from oracle import opes as Op

BOX = np.full(3, 50.0)


def _quad(phi_deg):
    """Atoms 1-4 with 2->3 along +x and dihedral phi (1 in the xy plane)."""
    r2 = np.array([10.0, 10.0, 10.0])
    r3 = r2 + [1.5, 0, 0]
    r1 = r2 + [-0.5, 1.4, 0]
    p = math.radians(phi_deg)
    r4 = r3 + [0.5, 1.4 * math.cos(p), 1.4 * math.sin(p)]
    return r1, r2, r3, r4


@pytest.mark.parametrize("phi", [0.0, 180.0, 90.0, -90.0, 60.0, -150.0])
def test_dihedral_textbook_angles(phi):
    """The angle between the two bond planes, measured about 2->3, is recovered."""
    xi, _ = D.dihedral(*_quad(phi), BOX)
    want = math.radians(phi)
    assert abs(D.wrap_angle(xi - want)) < 1e-12


def test_dihedral_gradient_fd_and_invariances():
    rng = np.random.default_rng(5)
    for _ in range(10):
        r = [np.array([10.0, 10.0, 10.0]) + rng.normal(0, 1.2, 3) for _ in range(4)]
        xi, g = D.dihedral(*r, BOX)
        h = 1e-6
        for a in range(4):
            for k in range(3):
                rp = [v.copy() for v in r]
                rm = [v.copy() for v in r]
                rp[a][k] += h
                rm[a][k] -= h
                fd = D.wrap_angle(D.dihedral(*rp, BOX)[0] - D.dihedral(*rm, BOX)[0]) / (2 * h)
                assert g[a, k] == pytest.approx(fd, rel=1e-6, abs=1e-7)
        # translation and rotation invariance of xi fix sum_i g_i = 0 and sum_i r_i x g_i = 0
        assert np.abs(g.sum(axis=0)).max() < 1e-10
        torque = sum(np.cross(r[a], g[a]) for a in range(4))
        assert np.abs(torque).max() < 1e-9


def test_dihedral_minimum_image():
    r1, r2, r3, r4 = _quad(75.0)
    shift = np.array([50.0, -50.0, 0.0])
    xi0, g0 = D.dihedral(r1, r2, r3, r4, BOX)
    xi1, g1 = D.dihedral(r1 + shift, r2, r3 - shift, r4, BOX)
    assert xi1 == pytest.approx(xi0, abs=1e-12)
    assert np.allclose(g1, g0, atol=1e-12)


def test_dafed_energy_force_and_mass_sum():
    rng = np.random.default_rng(9)
    pos = 10.0 + rng.normal(0, 1.5, (8, 3))
    idx = np.array([[0, 1, 2, 3], [2, 3, 4, 5], [4, 5, 6, 7]])
    s = np.array([2.5, -3.0, 0.4])       # 2.5 - xi can exceed pi: exercises the wrap
    kappa = np.array([400.0, 250.0, 100.0])
    minv = rng.uniform(0.05, 1.0, 8)
    out = D.cvs(pos, idx, BOX, minv, s, kappa)
    # the wrap keeps each displacement in (-pi, pi]
    d = D.wrap_angle(out["xi"] - s)
    assert np.all(np.abs(d) <= math.pi)
    assert out["u_dafed"] == pytest.approx(0.5 * np.sum(kappa * d * d), rel=1e-14)
    # force = -dU/dx by central differences of the energy
    h = 1e-6
    for a in range(8):
        for k in range(3):
            pp = pos.copy(); pp[a, k] += h
            pm = pos.copy(); pm[a, k] -= h
            fd = -(D.cvs(pp, idx, BOX, None, s, kappa)["u_dafed"] - D.cvs(pm, idx, BOX, None, s, kappa)["u_dafed"]) / (2 * h)
            assert out["forces"][a, k] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    # eq. 16 denominator with unit masses is the squared gradient norm
    one = D.cvs(pos, idx, BOX, np.ones(8))
    assert np.allclose(one["msum"], (out["dxi"] ** 2).sum(axis=(1, 2)), rtol=1e-14)


def test_wrap_angle():
    assert D.wrap_angle(np.array([3 * math.pi / 2]))[0] == pytest.approx(-math.pi / 2)
    assert D.wrap_angle(np.array([-math.pi]))[0] == pytest.approx(math.pi)
    assert D.wrap_angle(np.array([math.pi]))[0] == pytest.approx(math.pi)


# ---------------------------------------------------------------- OPES

KT = Op.KB_KCAL * 298.0


def test_theta_map_eq3():
    assert Op.theta_to_lambda(0.3) == pytest.approx((0.3, 0.3, 1.0))
    assert Op.theta_to_lambda(1.0) == pytest.approx((1.0, 1.0, 1.0))
    assert Op.theta_to_lambda(1.3) == pytest.approx((1.3, 0.7, -1.0))
    assert Op.theta_to_lambda(2.4) == pytest.approx((0.4, 0.4, 1.0))     # periodic
    assert Op.theta_to_lambda(-0.5) == pytest.approx((1.5, 0.5, -1.0))


def test_opes_constants_eqs_12_13():
    """gamma = beta dE, eps = exp(-beta dE/nu), and (nu/beta) ln eps = -dE exactly."""
    for dE, var in ((30.0, "standard"), (5.0, "explore"), (50.0, "standard")):
        g, nu, eps = Op.opes_constants(dE, KT, var)
        assert g == pytest.approx(dE / KT, rel=1e-15)
        assert nu == pytest.approx(1 - 1 / g if var == "standard" else g - 1, rel=1e-15)
        assert nu * KT * math.log(eps) == pytest.approx(-dE, rel=1e-13)
    # well-tempered target: both variants give the same exponent 1/gamma at equal barrier
    g, nu_s, _ = Op.opes_constants(30.0, KT, "standard")


def test_opes_far_from_kernels_is_minus_barriers():
    """Where rho_hat vanishes the bias is (nu/beta) ln eps = -dE per variant."""
    op = Op.DualOpes(KT, sigma=0.05, barrier_std=30.0, barrier_expl=5.0)
    op.deposit(0.2)
    u, du = op.bias(1.2)
    assert u == pytest.approx(-35.0, abs=1e-9)
    assert abs(du) < 1e-9


def test_opes_single_kernel_closed_form():
    op = Op.DualOpes(KT, sigma=0.1)
    op.deposit(0.7)
    u, du = op.bias(0.7)
    _, nus, es = op.c_std
    _, nue, ee = op.c_expl
    assert u == pytest.approx(nus * KT * math.log(1 + es) + nue * KT * math.log(1 + ee), rel=1e-12)
    assert abs(du) < 1e-12  # the kernel's maximum


def test_opes_derivative_fd_and_periodicity():
    op = Op.DualOpes(KT, sigma=0.1)
    for th in (0.1, 0.15, 0.3, 1.9, 1.95, 0.05):
        op.deposit(th)
    for th in (0.02, 0.4, 1.0, 1.97):
        u, du = op.bias(th)
        h = 1e-6
        fd = (op.bias(th + h)[0] - op.bias(th - h)[0]) / (2 * h)
        assert du == pytest.approx(fd, rel=1e-6, abs=1e-8)
    assert op.bias(0.3)[0] == pytest.approx(op.bias(2.3)[0], rel=1e-13)


def test_opes_explore_idempotent_duplicates():
    """Equal-weight kernels: duplicating every centre leaves rho_hat/rho_bar unchanged."""
    a = Op.DualOpes(KT, barrier_std=1e9)  # standard part negligible-weight test uses explore only
    b = Op.DualOpes(KT, barrier_std=1e9)
    for th in (0.2, 0.9, 1.5):
        a.centers.append(th); a.w_std.append(1.0)
        b.centers += [th, th]; b.w_std += [1.0, 1.0]
    for th in (0.1, 0.8, 1.6):
        assert a._bias_one(th, [1.0] * 3, a.c_expl)[0] == pytest.approx(b._bias_one(th, [1.0] * 6, b.c_expl)[0],
                                                                        rel=1e-13)


def test_opes_generalized_force_sign_flip():
    """On (1, 2] the generalized force on theta is the mirror of that on [0, 1]."""
    op = Op.DualOpes(KT)
    a = op.update(0.4, dudl=10.0)
    b = op.update(1.6, dudl=10.0)
    assert a["lam"] == pytest.approx(b["lam"])
    assert a["f_theta"] == pytest.approx(-10.0) and b["f_theta"] == pytest.approx(10.0)


def test_opes_rho_bar_is_the_mean_over_three_centres():
    """Explore kernels (equal weights) at 0.2, 0.3 and 1.0 with sigma = 0.05:
    the close pair overlaps by exp(-2), the far one is isolated (every other
    overlap, images included, is below exp(-100)).  Worked by hand:
    rho_hat(0.2) = rho_hat(0.3) = (1 + e^-2)/3, rho_hat(1.0) = 1/3, so the
    mean over the centres is (3 + 2 e^-2)/9 (a median or maximum would give
    (1 + e^-2)/3) and at theta = 1 the ratio is 3/(3 + 2 e^-2) (eq. 11)."""
    op = Op.DualOpes(KT, sigma=0.05)
    for th in (0.2, 0.3, 1.0):
        op.centers.append(th)
        op.w_std.append(1.0)
    g, nu, eps = op.c_expl
    e2 = math.exp(-2.0)
    want_ratio = 3.0 / (3.0 + 2.0 * e2)
    u, _ = op._bias_one(1.0, [1.0, 1.0, 1.0], op.c_expl)
    assert u == pytest.approx(nu * KT * math.log(want_ratio + eps), rel=1e-13)
    u2, _ = op._bias_one(0.2, [1.0, 1.0, 1.0], op.c_expl)
    assert u2 == pytest.approx(nu * KT * math.log(3.0 * (1.0 + e2) / (3.0 + 2.0 * e2) + eps), rel=1e-13)


def test_standard_weights_recover_the_unbiased_density():
    """OPES-Standard reweights its kernels so that rho_hat converges to the
    unbiased distribution (text after eq. 13).  Samples drawn from a known
    biased density p(theta) ~ p*(theta) exp(-V(theta)/kT), deposited with
    the bias V in place, must give rho_hat = (p* convolved with the kernel)
    within sampling error; with p* ~ 1 + cos(pi theta)/2 on [0, 2) that
    smoothed target is sigma sqrt(2 pi) (1 + e^(-pi^2 sigma^2/2) cos(pi theta)/2)/2.
    Weights exp(-V/kT) or equal weights miss it by factors of e^(+-3) and
    e^(+-1.5)."""
    rng = np.random.default_rng(2608)
    sigma = 0.1
    amp = 1.5 * KT
    V = lambda t: amp * math.sin(math.pi * t)
    # rejection sampling from p* exp(-V/kT) on [0, 2)
    n, xs = 20000, []
    bound = 1.5 * math.exp(amp / KT)
    while len(xs) < n:
        t = rng.uniform(0.0, 2.0, 4 * n)
        y = rng.uniform(0.0, bound, 4 * n)
        keep = y < (1.0 + 0.5 * np.cos(np.pi * t)) * np.exp(-amp * np.sin(np.pi * t) / KT)
        xs.extend(t[keep].tolist())
    xs = xs[:n]
    op = Op.DualOpes(KT, sigma=sigma)
    op.bias = lambda th: (V(th), 0.0)   # the bias in force when each sample was taken
    for th in xs:
        op.deposit(th)
    w = np.asarray(op.w_std)
    assert np.allclose(w, np.exp(np.array([V(t) for t in xs]) / KT), rtol=1e-12)
    c = np.asarray(op.centers)
    for th in (0.1, 0.5, 0.9, 1.3, 1.7):
        d = th - c
        g = sum(np.exp(-0.5 * (d + img) ** 2 / sigma ** 2) for img in (-2.0, 0.0, 2.0))
        rho = float((w * g).sum() / w.sum())
        want = sigma * math.sqrt(2 * math.pi) * (1 + math.exp(-(math.pi * sigma) ** 2 / 2) *
                                                 math.cos(math.pi * th) / 2) / 2
        assert rho == pytest.approx(want, rel=0.08), th
        assert Op.DualOpes._rho(op, th, op.w_std)[0] == pytest.approx(rho, rel=1e-10)
