"""Mirror-periodic theta map and the dual OPES bias on theta (FP64 reference).

TEST INFRASTRUCTURE (see the package docstring).

The paper's steps, in its notation:
- theta in [0, 2) is periodic; lambda = theta on [0, 1] and 2 - theta on
  (1, 2] (eq. 3); the generalized force on theta changes sign on (1, 2].
- U_OPES(theta) = (nu/beta) ln(rho_hat(theta)/rho_bar + eps) (eq. 11) with
  gamma = beta dE (eq. 12) and eps = exp(-beta dE / nu) (eq. 13);
  OPES-Standard: nu = 1 - 1/gamma and reweighted kernels; OPES-Explore:
  nu = gamma - 1 and equal kernel weights (text after eq. 13); the dual bias
  is their sum (eq. 14).
Readings where the paper is silent (kernel compression is not described):
- Gaussian kernels of width sigma on the periodic theta line (images at
  +-2 summed), unnormalized, stored uncompressed.
- rho_hat(theta) = sum_k w_k G(theta - theta_k) / sum_k w_k.
- rho_bar = (1/n) sum_i rho_hat(theta_i), the average over the kernel
  centres.
- Standard weights w_k = exp(beta U_total(theta_k)) with the total bias at
  deposition (this unbiases the estimate); Explore weights are 1.
- No kernel deposited yet: U_OPES = 0.
- Output grid: 101 nodes theta_g = 2 g / 101 on the periodic domain.
"""
import math

import numpy as np

KB_KCAL = 0.0019872042586408316  # Boltzmann constant, kcal/(mol K)
GRID = 101


def opes_constants(barrier, kT, variant):
    """(gamma, nu, eps) for a barrier dE (eqs. 12-13)."""
    gamma = barrier / kT
    nu = 1.0 - 1.0 / gamma if variant == "standard" else gamma - 1.0
    eps = math.exp(-gamma / nu)
    return gamma, nu, eps


def theta_to_lambda(theta):
    """Wrapped theta, lambda and dlambda/dtheta (eq. 3)."""
    th = theta - 2.0 * math.floor(theta / 2.0)
    if th <= 1.0:
        return th, th, 1.0
    return th, 2.0 - th, -1.0


def gauss(d, sigma):
    """Periodic Gaussian on [0, 2): images at -2, 0, +2, and its derivative."""
    v = dv = 0.0
    for img in (-2.0, 0.0, 2.0):
        x = d + img
        g = math.exp(-0.5 * x * x / (sigma * sigma))
        v += g
        dv += -x / (sigma * sigma) * g
    return v, dv


class DualOpes:
    def __init__(self, kT, sigma=0.10, barrier_std=30.0, barrier_expl=5.0):
        self.kT, self.sigma = kT, sigma
        self.c_std = opes_constants(barrier_std, kT, "standard")
        self.c_expl = opes_constants(barrier_expl, kT, "explore")
        self.centers, self.w_std = [], []

    def _rho(self, theta, weights):
        W = sum(weights)
        v = dv = 0.0
        for c, w in zip(self.centers, weights):
            g, dg = gauss(theta - c, self.sigma)
            v += w * g
            dv += w * dg
        return v / W, dv / W

    def _bias_one(self, theta, weights, consts):
        gamma, nu, eps = consts
        rho, drho = self._rho(theta, weights)
        rbar = sum(self._rho(c, weights)[0] for c in self.centers) / len(self.centers)
        arg = rho / rbar + eps
        return nu * self.kT * math.log(arg), nu * self.kT * (drho / rbar) / arg

    def bias(self, theta):
        """(U_total, dU_total/dtheta) at theta."""
        if not self.centers:
            return 0.0, 0.0
        us, ds = self._bias_one(theta, self.w_std, self.c_std)
        ue, de = self._bias_one(theta, [1.0] * len(self.centers), self.c_expl)
        return us + ue, ds + de

    def deposit(self, theta):
        th = theta - 2.0 * math.floor(theta / 2.0)
        u, _ = self.bias(th)
        self.centers.append(th)
        self.w_std.append(math.exp(u / self.kT))

    def update(self, theta, dudl, deposit=False):
        """One thin update: optional deposition, then lambda, bias and F_theta."""
        if deposit:
            self.deposit(theta)
        th, lam, dl = theta_to_lambda(theta)
        u, du = self.bias(th)
        return dict(theta=th, lam=lam, dlam_dtheta=dl, u_opes=u, du_opes=du, f_theta=-dl * dudl - du)

    def grid(self):
        th = 2.0 * np.arange(GRID) / GRID
        vals = np.array([self.bias(t) for t in th])
        return th, vals[:, 0], vals[:, 1]
