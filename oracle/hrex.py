"""Hamiltonian replica exchange between lambda states (FP64 reference).

TEST INFRASTRUCTURE (see the package docstring).

The paper's reference calculations exchange configurations between 21
evenly spaced lambda states every 1 ps (Simulation Details).  With the LBF
potential of eq. 4, U(x, lambda) = U_solv + U_solu + h_A(lambda) U_A(x) +
h_B(lambda) U_B(x), so the energy of box a at any other state follows from
its two basis energies:
    U_a(l') - U_a(l) = (h_A(l') - h_A(l)) U_A,a + (h_B(l') - h_B(l)) U_B,a.
A swap of the states s and s+1 held by boxes a and b is accepted with the
Metropolis probability min(1, exp(-D)),
    D = [U_a(l_s+1) - U_a(l_s) + U_b(l_s) - U_b(l_s+1)] / kT
      = [(h_A(l_s+1) - h_A(l_s)) (U_A,a - U_A,b)
         + (h_B(l_s+1) - h_B(l_s)) (U_B,a - U_B,b)] / kT.
Readings: neighbour swaps only, all pairs (s, s+1) with s of the attempt's
parity (even on even attempts, odd on odd) in one attempt; the uniform
deviate of pair s on attempt n is uniforms[n][s] (an input); accepted when
D <= 0 or u < exp(-D).
"""
import math

import numpy as np

import oracle as O


def lbf_h(lam):
    """(h_A, h_B) of eqs. 7-8 from the oracle's switching functions."""
    v = O.lbf_switches(lam)
    return float(v[0]), float(v[1])


def exchange_delta(ua_a, ub_a, ua_b, ub_b, lam_lo, lam_hi, kT):
    """D of a swap of the states lam_lo (held by a) and lam_hi (held by b)."""
    ha0, hb0 = lbf_h(lam_lo)
    ha1, hb1 = lbf_h(lam_hi)
    return ((ha1 - ha0) * (ua_a - ua_b) + (hb1 - hb0) * (ub_a - ub_b)) / kT


class Hrex:
    def __init__(self, lambdas, kT):
        self.lam = np.asarray(lambdas, float)
        self.kT = kT
        M = len(self.lam)
        self.state_of = np.arange(M)          # box -> state
        self.n = 0
        self.attempts = np.zeros(M - 1, np.int64)
        self.accepts = np.zeros(M - 1, np.int64)
        self.log = []                          # (attempt, pair, D, u, accepted)

    def exchange(self, ua, ub, uniforms):
        """One attempt over the pairs of this attempt's parity; ua, ub per box."""
        M = len(self.lam)
        box_of = np.empty(M, int)
        box_of[self.state_of] = np.arange(M)
        for s in range(self.n % 2, M - 1, 2):
            a, b = box_of[s], box_of[s + 1]
            D = exchange_delta(ua[a], ub[a], ua[b], ub[b], self.lam[s], self.lam[s + 1], self.kT)
            u = float(uniforms[s])
            ok = D <= 0.0 or u < math.exp(-D)
            self.attempts[s] += 1
            if ok:
                self.accepts[s] += 1
                self.state_of[a], self.state_of[b] = s + 1, s
            self.log.append((self.n, s, D, u, ok))
        self.n += 1
        return self.lam[self.state_of].copy()
