"""Pins of the lambda-dynamics / d-AFED oracle (oracle/ldyn.py) to facts
outside it: exact kinematics of the splitting, the stationary distributions
a Langevin thermostat must produce, the moment identities of kernel
merging, the uncompressed OPES reference, and exact quadratures."""
import math

import numpy as np
import pytest

from oracle import ldyn as L
from oracle import opes as Op

KT = L.KB_KCAL * 298.0


def test_baoab_without_friction_is_exact_for_a_constant_force():
    """gamma = 0 reduces BAOAB to velocity Verlet, exact for a constant force:
    q_N = q0 + v0 t + F t^2/(2m), and the stored momentum is the half-step p0 + (N - 1/2) h F."""
    q, p, m, h, F = 0.3, 0.7, 2.5, 0.4, -1.3
    q0, p0 = q, p
    for n in range(1, 51):
        q, p = L.baoab(q, p, m, KT, 0.0, h, F, 123.0, n == 1)
        t = n * h
        assert q == pytest.approx(q0 + p0 / m * t + F * t * t / (2 * m), rel=1e-13, abs=1e-13)
        assert p == pytest.approx(p0 + (n - 0.5) * h * F, rel=1e-13)


def test_baoab_harmonic_configurations_are_boltzmann():
    """BAOAB samples the configurational distribution of a harmonic well
    without step-size bias: <q^2> = kT/k (Leimkuhler & Matthews)."""
    rng = np.random.default_rng(7)
    m, k, h, gamma = 1.0, 4.0, 0.3, 1.0
    q, p = 0.0, 0.0
    n = 200000
    z = rng.standard_normal(n)
    acc = 0.0
    for i in range(n):
        q, p = L.baoab(q, p, m, KT, gamma, h, -k * q, z[i], i == 0)
        if i >= 1000:
            acc += q * q
    q2 = acc / (n - 1000)
    assert q2 == pytest.approx(KT / k, rel=0.03)


def test_o_step_keeps_the_maxwell_distribution():
    """With no force the momentum is driven to N(0, m kT) by the O step."""
    rng = np.random.default_rng(11)
    m, h, gamma = 3.0, 0.5, 1.0
    q, p = 0.0, 0.0
    z = rng.standard_normal(100000)
    ps = []
    for i in range(len(z)):
        q, p = L.baoab(q, p, m, KT, gamma, h, 0.0, z[i], i == 0)
        ps.append(p)
    assert np.var(ps[100:]) == pytest.approx(m * KT, rel=0.02)


def _mixture_moments(comps):
    """Total weight, mean and variance of a sum of normalised-relative kernels by quadrature."""
    x = np.linspace(-3.0, 3.0, 600001)
    f = np.zeros_like(x)
    for w, c, s, s0 in comps:
        f += w * (s0 / s) * np.exp(-0.5 * (x - c) ** 2 / s ** 2)
    dx = x[1] - x[0]
    W = f.sum() * dx
    mu = (x * f).sum() * dx / W
    var = ((x - mu) ** 2 * f).sum() * dx / W
    return W, mu, var


@pytest.mark.parametrize("c1,theta", [(0.70, 0.74), (0.02, 1.97), (1.99, 0.03)])
def test_kernel_merge_conserves_weight_mean_and_variance(c1, theta):
    """Compression replaces two kernels by one with the same total weight,
    mean and variance (moment matching), across the periodic boundary too."""
    s0 = 0.1
    ks = L.KernelSet(s0, compress=1.0)
    ks.add(c1, 2.0)
    ks.c[0], ks.s[0] = c1, 0.13          # an earlier merge left a wider kernel
    k = ks.add(theta, 0.5)
    assert k == 0 and len(ks.c) == 1
    t2 = c1 + L.periodic_delta(theta, c1)    # the new kernel at its image next to c1
    W, mu, var = _mixture_moments([(2.0, c1, 0.13, s0), (0.5, t2, s0, s0)])
    Wm, mum, varm = _mixture_moments([(ks.w[0], c1 + L.periodic_delta(ks.c[0], c1), ks.s[0], s0)])
    assert Wm == pytest.approx(W, rel=1e-9)
    assert mum == pytest.approx(mu, abs=1e-9)
    assert varm == pytest.approx(var, rel=1e-7)
    assert 0.0 <= ks.c[0] < 2.0


def test_kernel_merge_threshold_and_nearest_choice():
    ks = L.KernelSet(0.1, compress=1.0)
    for c in (0.2, 0.5, 1.95):
        ks.add(c, 1.0)
    assert len(ks.c) == 3
    assert ks.add(0.32, 1.0) == 3            # 1.2 widths from the nearest: a new kernel
    assert ks.add(0.03, 1.0) == 2            # 0.08 from 1.95 across the boundary
    assert ks.add(0.42, 1.0) == 1 and len(ks.c) == 4   # 0.08 from 0.5, 0.10 from 0.32
    # an exact tie goes to the lower index
    tie = L.KernelSet(0.5, compress=1.0)
    tie.add(0.25, 1.0)
    tie.add(0.75, 1.0)
    assert tie.add(0.5, 1.0) == 0
    none = L.KernelSet(0.1, compress=0.0)
    for c in (0.2, 0.2, 0.2):
        none.add(c, 1.0)
    assert len(none.c) == 3


def test_uncompressed_bias_equals_the_pinned_reference():
    """compress = 0: bias and derivative equal the uncompressed dual OPES
    reference (itself pinned by closed forms) after every deposition."""
    rng = np.random.default_rng(3)
    a = L.DualOpesCompressed(KT, 0.1, 30.0, 5.0, compress=0.0)
    b = Op.DualOpes(KT, sigma=0.1, barrier_std=30.0, barrier_expl=5.0)
    for th in rng.uniform(0.0, 2.0, 25):
        a.deposit(th)
        b.deposit(th)
        for x in (0.05, 0.6, 1.0, 1.55, 1.99):
            ua, da = a.bias(x)
            ub, db = b.bias(x)
            assert ua == pytest.approx(ub, rel=1e-12, abs=1e-12)
            assert da == pytest.approx(db, rel=1e-10, abs=1e-10)


def test_compressed_bias_keeps_far_from_kernels_value():
    """Where rho_hat vanishes the bias is -(dE_std + dE_expl) with or without merging."""
    a = L.DualOpesCompressed(KT, 0.05, 30.0, 5.0, compress=1.0)
    for th in (0.2, 0.22, 0.24, 0.21):
        a.deposit(th)
    assert len(a.std.c) < 4
    u, du = a.bias(1.2)
    assert u == pytest.approx(-35.0, abs=1e-9) and abs(du) < 1e-9


def test_ti_midpoint_rule_exact_values():
    """Samples at the bin centres: a linear mean force integrates exactly;
    x^2 gives the midpoint rule's known 1/3 - 1/(12 n^2)."""
    n = 10
    for f, want in ((lambda x: 2.0 - 3.0 * x, 2.0 - 1.5), (lambda x: x * x, 1.0 / 3.0 - 1.0 / (12 * n * n))):
        ld = L.LambdaDynamics(KT, 1.0, 1.0, 1.0, 0.1, 30.0, 5.0, 1.0, 0, n, 0.0)
        for b in range(n):
            c = (b + 0.5) / n
            bb = min(int(c * n), n - 1)
            ld.ti_sum[bb] += f(c)
            ld.ti_cnt[bb] += 1
        assert ld.free_energy() == pytest.approx(want, rel=1e-13)
    empty = L.LambdaDynamics(KT, 1.0, 1.0, 1.0, 0.1, 30.0, 5.0, 1.0, 0, n, 0.0)
    assert math.isnan(empty.free_energy())


def test_lambda_distribution_under_a_linear_potential():
    """With dU/dlambda = a (a linear potential in lambda) and no OPES, lambda
    dynamics samples p(lambda) ~ exp(-a lambda / kT) on [0, 1] through the
    mirror map: <lambda> = kT/a - 1/(exp(a/kT) - 1).  A wrong sign of the
    force on theta or of the mirror derivative moves the mean to the other side."""
    rng = np.random.default_rng(5)
    a = 2.0 * KT
    ld = L.LambdaDynamics(KT, mass=50.0, friction=0.05, dt=1.0, sigma=0.1, barrier_std=30.0, barrier_expl=5.0,
                          compress=1.0, stride=0, ti_bins=10, theta0=0.5)
    n = 300000
    z = rng.standard_normal(n)
    acc = 0.0
    for i in range(n):
        lam = ld.step(a, z[i])
        if i >= 2000:
            acc += lam
    mean = acc / (n - 2000)
    want = KT / a - 1.0 / (math.exp(a / KT) - 1.0)
    assert mean == pytest.approx(want, abs=0.012)
    assert ld.free_energy() == pytest.approx(a, rel=1e-12)


def test_auxiliary_variables_follow_the_coupling_at_their_temperature():
    """A fixed xi: s_k fluctuates about xi with <wrap(xi - s)^2> = kT_s/kappa (eq. 15 at T_s)."""
    rng = np.random.default_rng(9)
    kT_s = L.KB_KCAL * 1000.0
    kappa = 239.0
    aux = L.AuxiliaryDynamics(kT_s, [2.0e4], [kappa], friction=0.025, dt=1.0, s0=[2.9])
    n = 200000
    z = rng.standard_normal((n, 1))
    acc = 0.0
    xi = np.array([3.1])
    for i in range(n):
        s = aux.step(xi, z[i])
        if i >= 5000:
            acc += L.wrap_angle(xi[0] - s[0]) ** 2
    assert acc / (n - 5000) == pytest.approx(kT_s / kappa, rel=0.05)


def test_dafed_mass_and_coupling_formulas():
    """eq. 16 and the period of two coupled masses: with m_s = 300 m_xi the
    40 fs period needs kappa = mu (2 pi / 40)^2, mu = 300/301 m_xi."""
    m_xi = 1.0 / 0.05
    m_s = L.auxiliary_mass(300.0, 0.05)
    assert m_s == pytest.approx(300.0 * m_xi)
    k = L.coupling_for_period(m_s, m_xi, 40.0)
    mu = m_s * m_xi / (m_s + m_xi)
    # two masses joined by a spring kappa oscillate with omega^2 = kappa / mu
    assert 2.0 * math.pi / math.sqrt(k / mu) == pytest.approx(40.0, rel=1e-14)
