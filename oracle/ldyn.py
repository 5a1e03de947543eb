"""Lambda dynamics and d-AFED extended dynamics (FP64 reference).

TEST INFRASTRUCTURE (see the package docstring).

What the paper's method does with the nonbonded kernel's dU/dlambda
(Methodology: the extended Hamiltonian; Linear Basis Function; OPES;
Adiabatic Free Energy Dynamics; Simulation Details):
- lambda and the d-AFED auxiliary variables s_k are extended dynamical
  variables with their own masses and kinetic energies (the extended
  Hamiltonian), each set coupled to its own thermostat; they advance with
  the same time step as the atoms, and after each step the new values give
  the coupling forces of the next.
- lambda is the mirror image of a periodic theta in [0, 2) (eq. 3); the
  force on theta is -dlambda/dtheta dU/dlambda - dU_OPES/dtheta.
- the dual OPES bias on theta (eqs. 11-14) is built from kernels deposited
  every `stride` steps; rho_bar is the average of rho_hat over the centres
  of the compressed kernels.
- d-AFED: U = sum_k kappa_k/2 wrap(xi_k - s_k)^2 (eq. 15), so the force on
  s_k is kappa_k wrap(xi_k - s_k); s_k is kept at T_s (hotter than T).
- Delta G = integral over lambda of the conditional mean of dU/dlambda
  (eq. 2), accumulated in bins along lambda and integrated numerically.

Readings where the paper names a method without giving it, or is silent:
- thermostat: the paper couples the extended variables to a regulated
  Nose-Hoover-Langevin thermostat whose equations it does not state; here
  Langevin dynamics with the BAOAB splitting (Leimkuhler & Matthews, 2013,
  a published method): B p += h/2 F; A q += h/2 p/m; O p = c p +
  sqrt((1 - c^2) m kT) xi with c = exp(-gamma h); A; force; B.  The normal
  deviates xi are inputs (one per variable per step).
- kernel compression (OPES, Invernizzi & Parrinello 2020; named, not
  described, in the paper): a new kernel whose centre lies within
  `compress` deposition widths (periodic distance) of the nearest existing
  kernel centre of the same variant is merged into that kernel (ties: the
  lowest index), conserving weight, mean and variance:
      w = w1 + w2,  c = (w1 c1 + w2 c2)/w,
      s^2 = (w1 (s1^2 + c1^2) + w2 (s2^2 + c2^2))/w - c^2,
  with c2 taken at its periodic image nearest c1 and c wrapped into [0, 2);
  one merge per deposition.  compress = 0 keeps every kernel.
- kernels are Gaussians normalised relative to the deposition width s0:
  w (s0/s) exp(-d^2 / (2 s^2)) with images at +-2 (equal to the
  uncompressed reference when nothing merges); rho_hat = sum over kernels
  / sum of weights; Standard weights exp(U_total(theta)/kT) with the total
  bias at deposition, Explore weights 1; no bias before the first kernel.
- a deposition happens at the step's current theta before the step's
  force is formed, on steps 0, stride, 2 stride, ... (stride <= 0: none).
- TI: midpoint rule over n equal bins of lambda in [0, 1] (lambda = 1 in
  the last bin); a bin without samples makes Delta G undefined (NaN).
Units: kcal/mol, fs, theta dimensionless, s_k in radians.
"""
import math

import numpy as np

KB_KCAL = 0.0019872042586408316          # kcal/(mol K)
DA_NM2_TO_KCAL_FS2 = 1.0e6 / 4.184        # 1 Da nm^2 = 1 kJ/mol ps^2 in kcal/mol fs^2
KJ_TO_KCAL = 1.0 / 4.184


def opes_constants(barrier, kT, variant):
    """(gamma, nu, eps) of eqs. 12-13 for one variant."""
    gamma = barrier / kT
    nu = 1.0 - 1.0 / gamma if variant == "standard" else gamma - 1.0
    return gamma, nu, math.exp(-gamma / nu)


def theta_to_lambda(theta):
    """Wrapped theta, lambda and dlambda/dtheta (eq. 3)."""
    th = theta - 2.0 * math.floor(theta / 2.0)
    if th <= 1.0:
        return th, th, 1.0
    return th, 2.0 - th, -1.0


def periodic_delta(a, b):
    """a - b on the period-2 line, in [-1, 1)."""
    d = a - b
    return d - 2.0 * math.floor((d + 1.0) / 2.0)


def wrap_angle(x):
    """Into (-pi, pi]."""
    y = x - 2.0 * math.pi * math.floor((x + math.pi) / (2.0 * math.pi))
    return math.pi if y == -math.pi else y


class KernelSet:
    """One OPES variant's kernels on the periodic theta line."""

    def __init__(self, sigma0, compress):
        self.s0, self.compress = sigma0, compress
        self.c, self.w, self.s = [], [], []

    def value(self, theta):
        """(sum_k w_k g_k(theta), its theta derivative)."""
        v = dv = 0.0
        for c, w, s in zip(self.c, self.w, self.s):
            for img in (-2.0, 0.0, 2.0):
                x = theta - c + img
                g = w * (self.s0 / s) * math.exp(-0.5 * x * x / (s * s))
                v += g
                dv += -x / (s * s) * g
        return v, dv

    def add(self, theta, weight):
        """Deposit a kernel at theta; merge into the nearest one when close."""
        if self.compress > 0 and self.c:
            dist = [abs(periodic_delta(theta, c)) for c in self.c]
            k = min(range(len(dist)), key=lambda i: (dist[i], i))
            if dist[k] < self.compress * self.s0:
                # the moment formulas above, taken about c1 (d = c2 - c1)
                c1, w1, s1 = self.c[k], self.w[k], self.s[k]
                d = periodic_delta(theta, c1)
                w = w1 + weight
                c = c1 + weight * d / w
                var = (w1 * s1 * s1 + weight * self.s0 * self.s0) / w + w1 * weight * d * d / (w * w)
                self.c[k] = c - 2.0 * math.floor(c / 2.0)
                self.w[k] = w
                self.s[k] = math.sqrt(var)
                return k
        self.c.append(theta)
        self.w.append(weight)
        self.s.append(self.s0)
        return len(self.c) - 1

    def rho(self, theta):
        W = sum(self.w)
        v, dv = self.value(theta)
        return v / W, dv / W

    def rho_bar(self):
        return sum(self.rho(c)[0] for c in self.c) / len(self.c)


class DualOpesCompressed:
    def __init__(self, kT, sigma, barrier_std, barrier_expl, compress):
        self.kT = kT
        self.std = KernelSet(sigma, compress)
        self.expl = KernelSet(sigma, compress)
        self.c_std = opes_constants(barrier_std, kT, "standard")
        self.c_expl = opes_constants(barrier_expl, kT, "explore")
        self.rbar_std = self.rbar_expl = None

    def _one(self, ks, rbar, consts, theta):
        _, nu, eps = consts
        rho, drho = ks.rho(theta)
        arg = rho / rbar + eps
        return nu * self.kT * math.log(arg), nu * self.kT * (drho / rbar) / arg

    def bias(self, theta):
        if not self.std.c:
            return 0.0, 0.0
        us, ds = self._one(self.std, self.rbar_std, self.c_std, theta)
        ue, de = self._one(self.expl, self.rbar_expl, self.c_expl, theta)
        return us + ue, ds + de

    def deposit(self, theta):
        th = theta - 2.0 * math.floor(theta / 2.0)
        u, _ = self.bias(th)
        self.std.add(th, math.exp(u / self.kT))
        self.expl.add(th, 1.0)
        self.rbar_std = self.std.rho_bar()
        self.rbar_expl = self.expl.rho_bar()


def baoab(q, p, m, kT, gamma, h, force, noise, first):
    """One BAOAB step from the force at the current q: the closing half kick
    of the previous step (skipped on the first step), then B, A, O, A of
    this one; returns the new (q, p), whose closing half kick waits for the
    force at the new q."""
    if not first:
        p += 0.5 * h * force
    p += 0.5 * h * force
    q += 0.5 * h * p / m
    c = math.exp(-gamma * h)
    p = c * p + math.sqrt((1.0 - c * c) * m * kT) * noise
    q += 0.5 * h * p / m
    return q, p


class LambdaDynamics:
    """One replica's theta with dual OPES (compressed) and TI accumulators."""

    def __init__(self, kT, mass, friction, dt, sigma, barrier_std, barrier_expl, compress, stride, ti_bins,
                 theta0, p0=0.0):
        self.kT, self.m, self.gamma, self.h = kT, mass, friction, dt
        self.stride, self.nb = stride, ti_bins  # stride <= 0: no OPES kernels
        self.opes = DualOpesCompressed(kT, sigma, barrier_std, barrier_expl, compress)
        self.theta, self.p = theta0 - 2.0 * math.floor(theta0 / 2.0), p0
        self.n = 0
        self.ti_sum = np.zeros(ti_bins)
        self.ti_cnt = np.zeros(ti_bins)

    def lam(self):
        return theta_to_lambda(self.theta)[1]

    def step(self, dudl, noise):
        """Consume the step's dU/dlambda (at the current lambda) and one normal deviate;
        returns the next lambda."""
        if self.stride > 0 and self.n % self.stride == 0:
            self.opes.deposit(self.theta)
        th, lam, dl = theta_to_lambda(self.theta)
        u, du = self.opes.bias(th)
        f = -dl * dudl - du
        b = min(int(lam * self.nb), self.nb - 1)
        self.ti_sum[b] += dudl
        self.ti_cnt[b] += 1.0
        q, p = baoab(th, self.p, self.m, self.kT, self.gamma, self.h, f, noise, self.n == 0)
        self.theta = q - 2.0 * math.floor(q / 2.0)
        self.p = p
        self.n += 1
        self.last = dict(theta=th, lam=lam, dlam=dl, u_opes=u, du_opes=du, f_theta=f)
        return self.lam()

    def free_energy(self):
        """Midpoint-rule integral of the bin means of dU/dlambda (eq. 2); NaN if a bin is empty."""
        if np.any(self.ti_cnt == 0):
            return float("nan")
        return float(np.sum(self.ti_sum / self.ti_cnt) / self.nb)


class AuxiliaryDynamics:
    """d-AFED auxiliary variables s_k (eq. 15) at temperature kT_s."""

    def __init__(self, kT_s, masses, kappas, friction, dt, s0):
        self.kT, self.gamma, self.h = kT_s, friction, dt
        self.m = np.asarray(masses, float)
        self.kappa = np.asarray(kappas, float)
        self.s = np.array([wrap_angle(v) for v in s0], float)
        self.p = np.zeros_like(self.s)
        self.n = 0

    def step(self, xi, noise):
        f = np.array([self.kappa[k] * wrap_angle(xi[k] - self.s[k]) for k in range(len(self.s))])
        for k in range(len(self.s)):
            q, p = baoab(self.s[k], self.p[k], self.m[k], self.kT, self.gamma, self.h, f[k], noise[k], self.n == 0)
            self.s[k] = wrap_angle(q)
            self.p[k] = p
        self.n += 1
        self.last_force = f
        return self.s.copy()


def auxiliary_mass(c, msum):
    """m_s = c / sum_i m_i^-1 |dxi/dr_i|^2 (eq. 16)."""
    return c / msum


def coupling_for_period(m_s, m_xi, period):
    """kappa giving the coupled xi-s pair the oscillation period `period`
    (reduced mass of the two; eq. 16's inverse sum is m_xi)."""
    mu = m_s * m_xi / (m_s + m_xi)
    return mu * (2.0 * math.pi / period) ** 2
