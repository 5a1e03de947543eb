"""Synthetic input generators: counts, densities, minimum distances, charges, seeds."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2608_12691_amd import systems as S


def _min_intermolecular(s):
    L = s.box
    tree = cKDTree(np.mod(s.positions, L), boxsize=L)
    pairs = tree.query_pairs(2.2, output_type="ndarray")
    pairs = pairs[s.molecule[pairs[:, 0]] != s.molecule[pairs[:, 1]]]
    if len(pairs) == 0:
        return np.inf
    d = s.positions[pairs[:, 1]] - s.positions[pairs[:, 0]]
    d -= L * np.round(d / L)
    return np.linalg.norm(d, axis=1).min()


@pytest.mark.parametrize("k", [1, 2])
def test_water_configs(k):
    w = S.make_config(k)
    s = w.systems[0]
    assert s.positions.shape == (s.n_atoms, 3)
    assert s.is_solute.sum() == (12 if k == 1 else 24)
    n_w = s.info["n_waters"]
    assert s.n_atoms == s.is_solute.sum() + 3 * n_w
    assert n_w >= 0.95 * s.info["n_waters_requested"]
    q = w.ff.charge[s.types]
    assert abs(q.sum()) < 1e-9
    assert _min_intermolecular(s) >= 1.5
    # exclusions: sorted unique i<j; every water contributes its three intramolecular pairs
    ex = s.exclusions
    assert np.all(ex[:, 0] < ex[:, 1])
    assert np.array_equal(ex, ex[np.lexsort((ex[:, 1], ex[:, 0]))])
    n_sol = int(s.is_solute.sum())
    assert len(ex) == n_sol * (n_sol - 1) // 2 + 3 * n_w
    # density: 100 atoms/nm^3 for config 2 (graded box), liquid water for config 1
    rho = s.n_atoms / np.prod(s.box) * 1000
    assert 85 < rho < 105


def test_seed_reproducible():
    a = S.make_config(1)
    b = S.make_config(1)
    assert np.array_equal(a.systems[0].positions, b.systems[0].positions)
    c = S.make_config(1, seed=5)
    assert not np.array_equal(a.systems[0].positions[:5], c.systems[0].positions[:5])


def test_solute_parameters_ranges():
    w = S.make_config(2)
    s = w.systems[0]
    t = np.unique(s.types[s.is_solute == 1])
    assert len(t) == 24
    assert np.all((w.ff.sigma[t] >= 3.0) & (w.ff.sigma[t] <= 4.0))
    assert np.all((w.ff.epsilon[t] >= 0.05) & (w.ff.epsilon[t] <= 0.2))
    assert abs(w.ff.charge[t].sum()) < 1e-12


def test_perturbation_walk_and_lambdas():
    w = S.make_config(1)
    xs = S.perturbation_walk(w.systems[0], 5, 0.01, 11)
    assert xs.shape == (5, w.systems[0].n_atoms, 3)
    assert np.array_equal(xs[0], w.systems[0].positions)
    step = xs[1] - xs[0]
    assert 0.008 < step.std() < 0.012
    lam = S.lambda_draws(100, 3)
    assert lam.min() >= 0 and lam.max() <= 1
