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


def _check_clash_free(s):
    """No intermolecular heavy-heavy pair below 2.2 A, no H-involving pair below 1.5 A."""
    L = s.box
    heavy = np.ones(s.n_atoms, bool)
    tree = cKDTree(np.mod(s.positions, L), boxsize=L)
    pairs = tree.query_pairs(2.2, output_type="ndarray")
    pairs = pairs[s.molecule[pairs[:, 0]] != s.molecule[pairs[:, 1]]]
    d = s.positions[pairs[:, 1]] - s.positions[pairs[:, 0]]
    d -= L * np.round(d / L)
    return np.linalg.norm(d, axis=1).min() if len(pairs) else np.inf


def test_config3_octanol_box():
    w = S.make_config(3)
    s = w.systems[0]
    n_oct = s.info["n_octanol"]
    assert s.is_solute.sum() == 20
    assert s.n_atoms == 20 + 27 * n_oct
    # the packer may drop a few chains but never more than 2 % of the request
    assert n_oct >= 0.98 * s.info["n_octanol_requested"]
    rho = s.n_atoms / np.prod(s.box) * 1000
    assert 100.0 <= rho <= 104.0
    assert _check_clash_free(s) >= 1.5
    # octanol exclusions: bond-graph distance <= 3 inside each chain
    names, bonds = S.octanol_topology()
    per_chain = len(S._exclusions_within(27, bonds, 3))
    ex = s.exclusions
    solu = s.is_solute.astype(bool)
    in_oct = ~solu[ex[:, 0]] & ~solu[ex[:, 1]]
    assert in_oct.sum() == per_chain * n_oct
    assert np.all(s.molecule[ex[:, 0]] == s.molecule[ex[:, 1]])
    assert (~in_oct).sum() <= 20 * 19 // 2
    # charges: the hydroxyl group and C1 carry -0.68 + 0.42 + 0.26 = 0 per chain
    q = w.ff.charge[s.types]
    assert abs(q[~s.is_solute.astype(bool)].sum()) < 1e-9


def test_octanol_aligned_conformers_geometry():
    rng = np.random.Generator(np.random.PCG64(5))
    conf = S.octanol_conformers_aligned(rng, 64)
    assert len(conf) >= 48
    names, bonds = S.octanol_topology()
    want = {("O", "HO"): S.OCT_OH, ("O", "C1"): S.OCT_CO, ("C1", "C"): S.OCT_CC, ("C", "C"): S.OCT_CC,
            ("C", "H"): S.OCT_CH, ("C1", "H"): S.OCT_CH}
    for x in conf[:8]:
        for i, j in bonds:
            key = (names[i], names[j]) if (names[i], names[j]) in want else (names[j], names[i])
            assert np.linalg.norm(x[i] - x[j]) == pytest.approx(want[key], abs=1e-9)
        # heavy-atom principal axis along z
        heavy = np.array([n not in ("H", "HO") for n in names])
        _, v = np.linalg.eigh(np.cov((x[heavy] - x[heavy].mean(0)).T))
        assert abs(abs(v[2, -1]) - 1.0) < 1e-9


def test_config5_slab():
    """Water in z < L/2, octanol-like chains above, the peptide-like solute in the water half."""
    w = S.make_config(5)
    s = w.systems[0]
    L = s.box[0]
    info = s.info
    assert s.is_solute.sum() == 22
    assert s.n_atoms == 22 + 3 * info["n_waters"] + 27 * info["n_octanol"]
    assert info["n_waters"] >= 0.99 * info["n_waters_requested"]
    assert info["n_octanol"] >= 0.98 * info["n_octanol_requested"]
    assert s.n_atoms >= 0.98 * 250_000
    z = np.mod(s.positions[:, 2], L)
    water = (w.ff.names[0] == "OW") & np.isin(s.types, [0, 1])
    oct_atoms = (s.is_solute == 0) & ~water
    # molecule centres on their side of the slab (chains may straddle z = L by periodicity)
    zc_w = np.mod(s.positions[water][::3, 2], L)
    assert np.all(zc_w < 0.5 * L + 0.5)
    assert np.mean(z[oct_atoms] >= 0.5 * L - 1.0) > 0.97
    sol_z = np.mod(s.positions[s.is_solute.astype(bool), 2], L)
    assert np.all(sol_z < 0.5 * L)
    assert _check_clash_free(s) >= 1.5
    assert tuple(w.info["cv_atoms"].shape) == (4, 4)
