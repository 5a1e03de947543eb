"""Pins of the replica-exchange oracle (oracle/hrex.py): the swap energy
from the LBF bases equals the one from full evaluations at both lambdas
(eq. 4 is linear in its bases), and the attempts leave the Boltzmann
distribution over state assignments stationary."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle import hrex as H
from paper_2608_12691_amd import systems as S

KT = 0.0019872042586408316 * 298.0


def test_swap_energy_from_bases_equals_full_evaluations():
    """D from U_A, U_B of two boxes equals [U_a(l1) - U_a(l0) + U_b(l0) - U_b(l1)]/kT
    from the oracle's full LBF evaluations at l0 and l1."""
    rng = np.random.Generator(np.random.PCG64(44))
    w1 = S.make_config(1)
    boxes = [S.random_tiny_system(rng, n, 20.0, n_solute=4, n_types=w1.ff.n_types, min_dist=2.2) for n in (120, 150)]
    P = O.Params(9.0, 1.0, 0.2, 0.5, O.LBF)
    ev = lambda s, lam: O.evaluate(s.positions, s.types, s.is_solute, s.exclusions, s.box, w1.ff.sigma,
                                   w1.ff.epsilon, w1.ff.charge, P, lam, forces=False)["terms"]
    ta, tb = ev(boxes[0], 0.5), ev(boxes[1], 0.5)
    for l0, l1 in ((0.3, 0.4), (0.45, 0.55), (0.9, 1.0), (0.0, 0.05)):
        D = H.exchange_delta(ta[4], ta[5], tb[4], tb[5], l0, l1, KT)
        full = (ev(boxes[0], l1)[8] - ev(boxes[0], l0)[8] + ev(boxes[1], l0)[8] - ev(boxes[1], l1)[8]) / KT
        assert D == pytest.approx(full, rel=1e-9, abs=1e-9)


def test_exchanges_keep_the_boltzmann_distribution_of_assignments():
    """Three boxes with fixed bases: the frequency of each state assignment
    approaches exp(-sum_r U_r(lambda_state(r))/kT), normalised over the six."""
    lam = np.array([0.4, 0.6, 0.8])
    ua = np.array([-2.0, -3.1, -2.6]) * KT
    ub = np.array([1.0, 0.2, 0.6]) * KT
    hx = H.Hrex(lam, KT)
    rng = np.random.Generator(np.random.PCG64(12))
    n = 120000
    U = rng.uniform(0.0, 1.0, (n, 2))
    counts = {}
    for i in range(n):
        hx.exchange(ua, ub, U[i])
        key = tuple(hx.state_of)
        counts[key] = counts.get(key, 0) + 1
    def energy(perm):
        return sum(H.lbf_h(lam[perm[r]])[0] * ua[r] + H.lbf_h(lam[perm[r]])[1] * ub[r] for r in range(3))
    perms = list(itertools.permutations(range(3)))
    wts = np.array([math.exp(-energy(p) / KT) for p in perms])
    wts /= wts.sum()
    for p, want in zip(perms, wts):
        assert counts.get(p, 0) / n == pytest.approx(want, abs=0.01), (p, want)


def test_acceptance_rule_limits():
    hx = H.Hrex([0.5, 0.6], KT)
    # box 0 gains at the higher state: D < 0 accepted whatever the deviate
    hx.exchange(np.array([-10.0, 0.0]), np.array([0.0, 0.0]), [0.999999])
    assert list(hx.state_of) == [1, 0]
    hx2 = H.Hrex([0.5, 0.6], KT)
    hx2.exchange(np.array([1e4, 0.0]), np.array([0.0, 0.0]), [1e-300])
    assert list(hx2.state_of) == [0, 1] and hx2.accepts[0] == 0
    # odd attempts pair states 1-2 only
    hx3 = H.Hrex([0.2, 0.4, 0.6], KT)
    hx3.exchange(np.zeros(3), np.zeros(3), [0.5, 0.5])
    hx3.exchange(np.zeros(3), np.zeros(3), [0.5, 0.5])
    assert list(hx3.attempts) == [1, 1]
