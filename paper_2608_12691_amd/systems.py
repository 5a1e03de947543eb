"""Seeded synthetic systems for the alchemical nonbonded path.

This module only draws random numbers and builds geometry: atom positions,
types, the solute flag, exclusion lists, boxes and per-type parameters.  It
holds none of the pair-potential arithmetic, so it can feed both the CPU
oracle and the GPU library without coupling them.

The workloads stand in for the paper's systems (one solute in a few hundred
waters or 80 octanols, simulated with a 1.2 nm cutoff; Simulation Details
section).  None of the paper's molecules or force-field files are used: the
solutes are random trees, the water is a rigid three-site model with
TIP3P-like geometry, and the octanol-like solvent is a 27-atom C8H17OH chain
with random dihedrals.  Units are Angstrom, kcal/mol and elementary charges.

Every draw comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np
from scipy.spatial import cKDTree

# --------------------------------------------------------------------------
# data containers
# --------------------------------------------------------------------------


@dataclasses.dataclass
class ForceField:
    """Per-type Lennard-Jones and charge parameters (shared by all boxes)."""

    sigma: np.ndarray    # [n_types] Angstrom
    epsilon: np.ndarray  # [n_types] kcal/mol
    charge: np.ndarray   # [n_types] e
    names: List[str]

    @property
    def n_types(self) -> int:
        return int(self.sigma.shape[0])


@dataclasses.dataclass
class System:
    """One periodic box (one replica)."""

    positions: np.ndarray   # [n, 3] float64, not necessarily wrapped
    types: np.ndarray       # [n] int32
    is_solute: np.ndarray   # [n] uint8, 1 = alchemically coupled group
    exclusions: np.ndarray  # [m, 2] int32, i < j, lexicographically sorted
    box: np.ndarray         # [3] float64 edge lengths
    molecule: np.ndarray    # [n] int32 molecule id (informational)
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])


@dataclasses.dataclass
class Workload:
    """A named configuration: boxes, parameters and the call protocol."""

    name: str
    systems: List[System]
    ff: ForceField
    cutoff: float
    skin: float
    switch_width: float
    dsf_alpha: float
    sc_alpha: float
    lambdas: np.ndarray          # [K] lambda of each box for the first call
    seed: int
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return sum(s.n_atoms for s in self.systems)


# --------------------------------------------------------------------------
# constants of the synthetic models
# --------------------------------------------------------------------------

WATER_OH = 0.957
WATER_HOH_DEG = 104.5
WATER_O = dict(sigma=3.15, epsilon=0.152, charge=-0.834)
WATER_H = dict(sigma=1.0, epsilon=0.0, charge=0.417)   # no LJ on H

OCT_CC, OCT_CH, OCT_CO, OCT_OH = 1.53, 1.09, 1.43, 0.957
TETRA_DEG = 109.47
OCT_TYPES = {
    "C": dict(sigma=3.5, epsilon=0.066, charge=0.0),
    "C1": dict(sigma=3.5, epsilon=0.066, charge=0.26),
    "H": dict(sigma=2.5, epsilon=0.03, charge=0.0),
    "O": dict(sigma=3.15, epsilon=0.152, charge=-0.68),
    "HO": dict(sigma=1.0, epsilon=0.0, charge=0.42),
}

# minimum intermolecular distances enforced by the packers
MIN_HEAVY = 2.2
MIN_WITH_H = 1.5
SOLUTE_WATER_DELETE = 2.0

BASE_SEED = 12691 * 10


def config_seed(k: int) -> int:
    """Seed of configuration k (1-based)."""
    return BASE_SEED + k


# --------------------------------------------------------------------------
# small geometry helpers
# --------------------------------------------------------------------------


def _place(a, b, c, bond, angle_deg, torsion_deg):
    """Atom d with |cd| = bond, angle(b,c,d) = angle, dihedral(a,b,c,d) = torsion."""
    a, b, c = (np.asarray(v, dtype=np.float64) for v in (a, b, c))
    bc = c - b
    bc /= np.linalg.norm(bc)
    n = np.cross(b - a, bc)
    nn = np.linalg.norm(n)
    if nn < 1e-8:  # collinear reference: pick any perpendicular
        trial = np.array([1.0, 0.0, 0.0]) if abs(bc[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        n = np.cross(trial, bc)
        nn = np.linalg.norm(n)
    n /= nn
    m = np.cross(n, bc)
    th = np.deg2rad(angle_deg)
    ph = np.deg2rad(torsion_deg)
    d2 = np.array([-bond * np.cos(th), bond * np.sin(th) * np.cos(ph), bond * np.sin(th) * np.sin(ph)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * n


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _graph_distances(n: int, bonds: Sequence[tuple]) -> np.ndarray:
    adj = [[] for _ in range(n)]
    for i, j in bonds:
        adj[i].append(j)
        adj[j].append(i)
    dist = np.full((n, n), 10 ** 6, dtype=np.int64)
    for s in range(n):
        dist[s, s] = 0
        frontier = [s]
        while frontier:
            nxt = []
            for u in frontier:
                for v in adj[u]:
                    if dist[s, v] > dist[s, u] + 1:
                        dist[s, v] = dist[s, u] + 1
                        nxt.append(v)
            frontier = nxt
    return dist


def _exclusions_within(n: int, bonds, max_graph_dist: int) -> np.ndarray:
    d = _graph_distances(n, bonds)
    ii, jj = np.nonzero(np.triu(d <= max_graph_dist, k=1))
    return np.stack([ii, jj], axis=1).astype(np.int32)


def _all_pairs(n: int) -> np.ndarray:
    ii, jj = np.triu_indices(n, k=1)
    return np.stack([ii, jj], axis=1).astype(np.int32)


def _wrap(x, box):
    w = np.mod(x, box)
    w[w >= box] = 0.0  # guard the rounding case x mod L == L
    return w


# --------------------------------------------------------------------------
# molecules
# --------------------------------------------------------------------------


def random_tree_solute(rng, n_atoms: int, bond=1.5, angle=109.5, min_nonbonded=2.5):
    """Random tree of n_atoms with fixed bond length and bond angle.

    Returns (coords [n,3], bonds list).  Pairs three or more bonds apart are
    kept at least ``min_nonbonded`` apart (rejection).
    """
    for _attempt in range(1000):
        coords = [np.zeros(3), np.array([bond, 0.0, 0.0])]
        parent = {1: 0}
        nbrs = {0: [1], 1: [0]}
        bonds = [(0, 1)]
        ok = True
        for k in range(2, n_atoms):
            placed = False
            for _try in range(200):
                cand = [i for i in range(k) if len(nbrs[i]) < 4]
                p = int(rng.choice(cand))
                g = nbrs[p][0] if p != 0 else nbrs[0][0]
                if g == p:
                    continue
                # dihedral reference: another neighbour of g, else a fixed point
                refs = [a for a in nbrs[g] if a != p]
                a_ref = coords[refs[0]] if refs else coords[g] + np.array([0.0, 1.0, 0.3])
                tors = rng.uniform(0.0, 360.0)
                x = _place(a_ref, coords[g], coords[p], bond, angle, tors)
                # distance check against atoms not bonded to p (skip 1-2, 1-3)
                good = True
                for i in range(k):
                    if i == p:
                        continue
                    lim = 2.0 if i in nbrs[p] else min_nonbonded  # 1-3 pairs vs the rest
                    if np.linalg.norm(coords[i] - x) < lim:
                        good = False
                        break
                if good:
                    coords.append(x)
                    nbrs[k] = [p]
                    nbrs[p].append(k)
                    parent[k] = p
                    bonds.append((p, k))
                    placed = True
                    break
            if not placed:
                ok = False
                break
        if ok:
            c = np.array(coords)
            return c - c.mean(axis=0), bonds
    raise RuntimeError("random_tree_solute: could not grow a clash-free tree")


def water_molecule_frame() -> np.ndarray:
    half = np.deg2rad(WATER_HOH_DEG / 2.0)
    return np.array([
        [0.0, 0.0, 0.0],
        [WATER_OH * np.sin(half), WATER_OH * np.cos(half), 0.0],
        [-WATER_OH * np.sin(half), WATER_OH * np.cos(half), 0.0],
    ])


def octanol_topology():
    """27-atom C8H17OH: names, bonds.  Index plan: O, HO, C1..C8, H's."""
    names = ["O", "HO"] + ["C1"] + ["C"] * 7
    bonds = [(0, 1), (0, 2)] + [(1 + k, 2 + k) for k in range(1, 8)]
    h_idx = 10
    for k in range(1, 9):
        c = 1 + k
        nh = 3 if k == 8 else 2
        for _ in range(nh):
            names.append("H")
            bonds.append((c, h_idx))
            h_idx += 1
    assert len(names) == 27
    return names, bonds


def octanol_conformer(rng, max_tries=500):
    names, bonds = octanol_topology()
    gd = _graph_distances(27, bonds)
    heavy = np.array([n not in ("H", "HO") for n in names])
    for _ in range(max_tries):
        x = np.zeros((27, 3))
        x[0] = [0.0, 0.0, 0.0]              # O
        x[2] = [OCT_CO, 0.0, 0.0]           # C1
        x[3] = _place([0.0, 1.0, 0.0], x[0], x[2], OCT_CC, TETRA_DEG, 180.0)   # C2
        x[1] = _place(x[3], x[2], x[0], OCT_OH, TETRA_DEG, rng.uniform(0, 360))  # HO
        # backbone C3..C8 (indices 4..9); the dihedral reference of C3 is O
        for c in range(4, 10):
            a = 0 if c == 4 else c - 3
            x[c] = _place(x[a], x[c - 2], x[c - 1], OCT_CC, TETRA_DEG, rng.uniform(0, 360))
        h = 10
        for k in range(1, 9):
            c = 1 + k
            prev = 0 if k == 1 else c - 1
            if k < 8:
                nxt = c + 1
                for tors in (120.0, -120.0):
                    x[h] = _place(x[nxt], x[prev], x[c], OCT_CH, TETRA_DEG, tors)
                    h += 1
            else:
                t0 = rng.uniform(0, 360)
                for tors in (t0, t0 + 120.0, t0 + 240.0):
                    x[h] = _place(x[c - 2], x[prev], x[c], OCT_CH, TETRA_DEG, tors)
                    h += 1
        d = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=-1)
        far = gd >= 4
        hh = heavy[:, None] & heavy[None, :]
        if np.any(far & hh & (d < 2.5)) or np.any(far & ~hh & (d < 1.5)):
            continue
        return x - x.mean(axis=0), names, bonds
    raise RuntimeError("octanol_conformer: no clash-free conformer")


PEPTIDE_CV = {"phi": (4, 6, 8, 17), "psi": (6, 8, 17, 19), "chi": (6, 8, 10, 13), "omega": (0, 4, 6, 8)}


def peptide_solute(rng, max_tries=500):
    """22-atom N-acetyl amide with an ethyl side chain (Ac-X-NH2).

    Index plan: 0 CH3, 1-3 H, 4 C_Ac, 5 O_Ac, 6 N, 7 H_N, 8 CA, 9 HA, 10 CB,
    11-12 HB, 13 CG, 14-16 HG, 17 C, 18 O, 19 N2, 20-21 H_N2.
    """
    bonds = [(0, 1), (0, 2), (0, 3), (0, 4), (4, 5), (4, 6), (6, 7), (6, 8), (8, 9), (8, 10),
             (10, 11), (10, 12), (10, 13), (13, 14), (13, 15), (13, 16), (8, 17), (17, 18),
             (17, 19), (19, 20), (19, 21)]
    is_h = np.zeros(22, dtype=bool)
    is_h[[1, 2, 3, 7, 9, 11, 12, 14, 15, 16, 20, 21]] = True
    gd = _graph_distances(22, bonds)
    for _ in range(max_tries):
        phi, psi, chi = rng.uniform(-180, 180, size=3)
        omega = 180.0 + rng.uniform(-10, 10)
        x = np.zeros((22, 3))
        x[0] = [0.0, 0.0, 0.0]
        x[4] = [1.52, 0.0, 0.0]
        x[6] = _place([0.0, 1.0, 0.0], x[0], x[4], 1.33, 116.0, 180.0)
        x[5] = _place(x[6], x[0], x[4], 1.23, 121.0, 180.0)
        x[8] = _place(x[0], x[4], x[6], 1.46, 122.0, omega)
        x[7] = _place(x[8], x[4], x[6], 1.01, 119.0, 180.0)
        x[17] = _place(x[4], x[6], x[8], 1.52, 110.0, phi)
        x[19] = _place(x[6], x[8], x[17], 1.33, 116.0, psi)
        x[18] = _place(x[19], x[8], x[17], 1.23, 121.0, 180.0)
        x[10] = _place(x[17], x[6], x[8], 1.53, TETRA_DEG, 120.0)
        x[9] = _place(x[17], x[6], x[8], 1.09, TETRA_DEG, -120.0)
        x[13] = _place(x[6], x[8], x[10], 1.53, TETRA_DEG, chi)
        x[11] = _place(x[13], x[8], x[10], 1.09, TETRA_DEG, 120.0)
        x[12] = _place(x[13], x[8], x[10], 1.09, TETRA_DEG, -120.0)
        t0 = rng.uniform(0, 360)
        for h, t in zip((14, 15, 16), (t0, t0 + 120, t0 + 240)):
            x[h] = _place(x[8], x[10], x[13], 1.09, TETRA_DEG, t)
        t0 = rng.uniform(0, 360)
        for h, t in zip((1, 2, 3), (t0, t0 + 120, t0 + 240)):
            x[h] = _place(x[6], x[4], x[0], 1.09, TETRA_DEG, t)
        x[20] = _place(x[8], x[17], x[19], 1.01, 120.0, 0.0)
        x[21] = _place(x[8], x[17], x[19], 1.01, 120.0, 180.0)
        d = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=-1)
        far = gd >= 4
        hh = ~is_h[:, None] & ~is_h[None, :]
        if np.any(far & hh & (d < 2.5)) or np.any(far & ~hh & (d < 1.5)):
            continue
        return x - x.mean(axis=0), bonds, is_h
    raise RuntimeError("peptide_solute: no clash-free conformer")


# --------------------------------------------------------------------------
# packers
# --------------------------------------------------------------------------


def _clash_pairs(pos, box, mol, heavy):
    """Intermolecular atom pairs closer than the packing thresholds."""
    tree = cKDTree(_wrap(pos, box), boxsize=box)
    pairs = tree.query_pairs(r=MIN_HEAVY, output_type="ndarray")
    if pairs.size == 0:
        return pairs
    pairs = pairs[mol[pairs[:, 0]] != mol[pairs[:, 1]]]
    if pairs.size == 0:
        return pairs
    d = pos[pairs[:, 1]] - pos[pairs[:, 0]]
    d -= box * np.round(d / box)
    r = np.linalg.norm(d, axis=1)
    both_heavy = heavy[pairs[:, 0]] & heavy[pairs[:, 1]]
    bad = np.where(both_heavy, r < MIN_HEAVY, r < MIN_WITH_H)
    return pairs[bad]


def _lattice_sites(rng, n_sites, lo, hi):
    """n_sites points on the smallest cubic-ish lattice filling [lo, hi)."""
    ext = np.asarray(hi, float) - np.asarray(lo, float)
    vol_per = np.prod(ext) / n_sites
    a = vol_per ** (1.0 / 3.0)
    counts = np.maximum(1, np.round(ext / a).astype(int))
    while np.prod(counts) < n_sites:
        counts[np.argmax(ext / counts)] += 1
    grids = [lo[d] + (np.arange(counts[d]) + 0.5) * ext[d] / counts[d] for d in range(3)]
    g = np.stack(np.meshgrid(*grids, indexing="ij"), axis=-1).reshape(-1, 3)
    if g.shape[0] > n_sites:
        g = g[np.sort(rng.choice(g.shape[0], size=n_sites, replace=False))]
    return g, ext / counts


class _Packer:
    """Rigid-body placement of molecules with clash repair by redrawing."""

    def __init__(self, rng, box):
        self.rng = rng
        self.box = np.asarray(box, float)
        self.mol_templates = []   # per molecule: callable returning local coords
        self.centers = []
        self.coords = []          # per molecule [n,3] absolute
        self.heavy = []
        self.fixed = []

    def add(self, local, center, heavy, template=None, fixed=False, jitter=0.0):
        rot = np.eye(3) if fixed else _random_rotation(self.rng)
        c = np.asarray(center, float) + (0 if fixed else self.rng.uniform(-jitter, jitter, 3))
        self.coords.append(local @ rot.T + c)
        self.centers.append(np.asarray(center, float))
        self.mol_templates.append((template, jitter))
        self.heavy.append(heavy)
        self.fixed.append(fixed)

    def flat(self):
        pos = np.concatenate(self.coords)
        mol = np.concatenate([np.full(len(c), i) for i, c in enumerate(self.coords)])
        heavy = np.concatenate(self.heavy)
        return pos, mol, heavy

    def repair(self, max_iter=400):
        for it in range(max_iter):
            pos, mol, heavy = self.flat()
            bad = _clash_pairs(pos, self.box, mol, heavy)
            if bad.size == 0:
                return it
            mols = np.unique(np.concatenate([mol[bad[:, 0]], mol[bad[:, 1]]]))
            # redraw one partner of each clashing pair, never a fixed molecule
            redo = set()
            for a, b in zip(mol[bad[:, 0]], mol[bad[:, 1]]):
                cand = [m for m in (int(b), int(a)) if not self.fixed[m]]
                if cand and not (set(cand) & redo):
                    redo.add(cand[0])
            for m in redo:
                template, jitter = self.mol_templates[m]
                local = template() if template is not None else None
                if local is None:
                    c0 = self.coords[m].mean(axis=0)
                    local = self.coords[m] - c0
                else:
                    local = local - local.mean(axis=0)
                rot = _random_rotation(self.rng)
                c = self.centers[m] + self.rng.uniform(-jitter, jitter, 3)
                self.coords[m] = local @ rot.T + c
            del mols
        raise RuntimeError("packer: clashes remain after %d redraws" % max_iter)


def _water_forcefield_types():
    names = ["OW", "HW"]
    sig = [WATER_O["sigma"], WATER_H["sigma"]]
    eps = [WATER_O["epsilon"], WATER_H["epsilon"]]
    chg = [WATER_O["charge"], WATER_H["charge"]]
    return names, sig, eps, chg


def _solute_params(rng, n, q_half_range):
    sig = rng.uniform(3.0, 4.0, n)
    eps = rng.uniform(0.05, 0.2, n)
    q = rng.uniform(-q_half_range, q_half_range, n)
    q -= q.mean()
    return sig, eps, q


def _assemble(parts, box):
    pos = np.concatenate([p["pos"] for p in parts])
    types = np.concatenate([p["types"] for p in parts]).astype(np.int32)
    solute = np.concatenate([p["solute"] for p in parts]).astype(np.uint8)
    mol = np.concatenate([p["mol"] for p in parts]).astype(np.int32)
    excl = []
    off = 0
    for p in parts:
        if len(p["excl"]):
            excl.append(np.asarray(p["excl"], np.int32) + off)
        off += len(p["pos"])
    excl = np.concatenate(excl) if excl else np.zeros((0, 2), np.int32)
    excl = np.unique(excl, axis=0) if len(excl) else excl
    order = np.lexsort((excl[:, 1], excl[:, 0])) if len(excl) else np.arange(0)
    excl = excl[order].astype(np.int32)
    return System(positions=pos, types=types, is_solute=solute, exclusions=excl,
                  box=np.asarray(box, float), molecule=mol)


def solvated_rigid_solute(rng, n_waters, box, solute_local, solute_types, type_ow=0, type_hw=1,
                          water_region=None):
    """Rigid solute at the box centre in lattice water (deleting overlaps)."""
    box = np.asarray(box, float)
    centre = box / 2.0
    sol = solute_local + centre
    lo, hi = (np.zeros(3), box) if water_region is None else water_region
    sites, _ = _lattice_sites(rng, n_waters, lo, hi)
    wf = water_molecule_frame()
    pk = _Packer(rng, box)
    heavy_sol = np.ones(len(sol), bool)
    pk.add(sol - sol.mean(axis=0), sol.mean(axis=0), heavy_sol, fixed=True)
    for s in sites:
        pk.add(wf, s, np.array([True, False, False]), jitter=0.3)
    # delete waters overlapping the solute before repairing the rest
    keep = [0]
    tree = cKDTree(_wrap(sol, box), boxsize=box)
    for m in range(1, len(pk.coords)):
        d, _ = tree.query(_wrap(pk.coords[m], box), k=1)
        if np.min(d) >= SOLUTE_WATER_DELETE:
            keep.append(m)
    pk.coords = [pk.coords[m] for m in keep]
    pk.centers = [pk.centers[m] for m in keep]
    pk.mol_templates = [pk.mol_templates[m] for m in keep]
    pk.heavy = [pk.heavy[m] for m in keep]
    pk.fixed = [pk.fixed[m] for m in keep]
    n_iter = pk.repair()
    # re-check the solute distance after repairs (repairs may move waters)
    parts = [dict(pos=pk.coords[0], types=np.asarray(solute_types), solute=np.ones(len(sol)),
                  mol=np.zeros(len(sol)), excl=_all_pairs(len(sol)))]
    for m in range(1, len(pk.coords)):
        parts.append(dict(pos=pk.coords[m], types=np.array([type_ow, type_hw, type_hw]),
                          solute=np.zeros(3), mol=np.full(3, m), excl=[(0, 1), (0, 2), (1, 2)]))
    sysm = _assemble(parts, box)
    sysm.info.update(n_waters_requested=int(n_waters), n_waters=len(pk.coords) - 1,
                     repair_iterations=int(n_iter))
    return sysm


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------


def _rigid_solute_ff(rng, n_solute):
    names, sig, eps, chg = _water_forcefield_types()
    s_sig, s_eps, s_q = _solute_params(rng, n_solute, 0.5)
    ff = ForceField(sigma=np.array(sig + list(s_sig)), epsilon=np.array(eps + list(s_eps)),
                    charge=np.array(chg + list(s_q)),
                    names=names + ["S%d" % i for i in range(n_solute)])
    return ff


def make_config1(seed=None):
    """12-atom rigid solute in 216 waters, 18.6 A cube, cutoff 9 A, lambda 0.5."""
    seed = config_seed(1) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    sol, _ = random_tree_solute(rng, 12)
    ff = _rigid_solute_ff(rng, 12)
    box = np.full(3, 18.6)
    s = solvated_rigid_solute(rng, 216, box, sol, np.arange(2, 14))
    return Workload(name="water216_solute12", systems=[s], ff=ff, cutoff=9.0, skin=0.0,
                    switch_width=1.0, dsf_alpha=0.2, sc_alpha=0.5, lambdas=np.array([0.5]), seed=seed)


def make_config2(seed=None, literal_box=False):
    """24-atom rigid solute in 3000 waters, cutoff 10 A, skin 1 A.

    The graded box is 44.85 A (100 atoms/nm^3, liquid-water density); the
    literal 31.0 A box is three times that density and is only a stress
    variant (it fails the packers' minimum-distance checks).
    """
    seed = config_seed(2) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    sol, _ = random_tree_solute(rng, 24)
    ff = _rigid_solute_ff(rng, 24)
    L = 31.0 if literal_box else 44.85
    s = solvated_rigid_solute(rng, 3000, np.full(3, L), sol, np.arange(2, 26))
    lam = rng.uniform(0.0, 1.0, 1)
    return Workload(name="water3000_solute24", systems=[s], ff=ff, cutoff=10.0, skin=1.0,
                    switch_width=1.0, dsf_alpha=0.2, sc_alpha=0.5, lambdas=lam, seed=seed,
                    info=dict(n_calls=1000, perturb_sigma=0.01, box_reading="literal" if literal_box else "graded"))


def make_config4(seed=None, n_replicas=16):
    """16 boxes of 2,000-12,000 atoms at 100 atoms/nm^3, lambda_k = k/15."""
    seed = config_seed(4) if seed is None else seed
    rng0 = np.random.Generator(np.random.PCG64(seed))
    sol, _ = random_tree_solute(rng0, 24)
    ff = _rigid_solute_ff(rng0, 24)
    n_atoms = rng0.integers(2000, 12001, size=n_replicas)
    systems = []
    for r in range(n_replicas):
        rng = np.random.Generator(np.random.PCG64(seed + 1000 * (r + 1)))
        L = (n_atoms[r] / 0.1) ** (1.0 / 3.0)
        n_w = int(round((n_atoms[r] - 24) / 3))
        systems.append(solvated_rigid_solute(rng, n_w, np.full(3, L), sol, np.arange(2, 26)))
    lam = np.arange(n_replicas) / max(1, n_replicas - 1)
    return Workload(name="hrex16_water", systems=systems, ff=ff, cutoff=10.0, skin=1.0,
                    switch_width=1.0, dsf_alpha=0.2, sc_alpha=0.5, lambdas=lam, seed=seed,
                    info=dict(target_atoms=n_atoms.tolist()))


def single_box_like(workload: Workload, seed=None):
    """One water box holding as many atoms as all boxes of ``workload``."""
    seed = config_seed(4) + 77 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    n_total = workload.n_atoms
    sol_sys = workload.systems[0]
    sol_idx = np.nonzero(sol_sys.is_solute)[0]
    sol = sol_sys.positions[sol_idx] - sol_sys.positions[sol_idx].mean(axis=0)
    L = (n_total / 0.1) ** (1.0 / 3.0)
    n_w = int(round((n_total - len(sol_idx)) / 3))
    s = solvated_rigid_solute(rng, n_w, np.full(3, L), sol, sol_sys.types[sol_idx])
    return Workload(name="single_box_%d" % s.n_atoms, systems=[s], ff=workload.ff, cutoff=workload.cutoff,
                    skin=workload.skin, switch_width=workload.switch_width, dsf_alpha=workload.dsf_alpha,
                    sc_alpha=workload.sc_alpha, lambdas=workload.lambdas[:1].copy(), seed=seed)


def _octanol_ff_types():
    names = list(OCT_TYPES.keys())
    return (names, [OCT_TYPES[n]["sigma"] for n in names], [OCT_TYPES[n]["epsilon"] for n in names],
            [OCT_TYPES[n]["charge"] for n in names])


def _place_batch(a, b, c, bond, angle_deg, torsion_deg):
    """_place for M reference triples at once: a, b, c [M,3], torsion [M] (degrees)."""
    bc = c - b
    bc /= np.linalg.norm(bc, axis=1, keepdims=True)
    n = np.cross(b - a, bc)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    m = np.cross(n, bc)
    th = np.deg2rad(angle_deg)
    ph = np.deg2rad(np.asarray(torsion_deg, float))[:, None]
    return c - bond * np.cos(th) * bc + bond * np.sin(th) * (np.cos(ph) * m + np.sin(ph) * n)


def octanol_conformers_aligned(rng, n_draw):
    """Octanol-like chains for dense packing, drawn as a batch: backbone
    dihedrals trans-biased (180 deg with probability 0.8, else +-65 deg
    gauche, each +N(0, 8 deg)), hydroxyl and methyl torsions uniform;
    self-clashing draws are rejected as in octanol_conformer.  Each kept
    chain is centred with its heavy-atom principal axis along z.  Returns
    [M, 27, 3] with M <= n_draw."""
    names, bonds = octanol_topology()
    gd = _graph_distances(27, bonds)
    heavy = np.array([n not in ("H", "HO") for n in names])
    M = n_draw
    x = np.zeros((M, 27, 3))
    x[:, 2] = [OCT_CO, 0.0, 0.0]
    x[:, 3] = _place([0.0, 1.0, 0.0], x[0, 0], x[0, 2], OCT_CC, TETRA_DEG, 180.0)
    x[:, 1] = _place_batch(x[:, 3], x[:, 2], x[:, 0], OCT_OH, TETRA_DEG, rng.uniform(0, 360, M))
    for c in range(4, 10):
        a = 0 if c == 4 else c - 3
        u = rng.uniform(size=M)
        base = np.where(u < 0.8, 180.0, np.where(u < 0.9, 65.0, -65.0))
        x[:, c] = _place_batch(x[:, a], x[:, c - 2], x[:, c - 1], OCT_CC, TETRA_DEG, base + rng.normal(0.0, 8.0, M))
    h = 10
    for k in range(1, 9):
        c = 1 + k
        prev = 0 if k == 1 else c - 1
        if k < 8:
            for tors in (120.0, -120.0):
                x[:, h] = _place_batch(x[:, c + 1], x[:, prev], x[:, c], OCT_CH, TETRA_DEG, np.full(M, tors))
                h += 1
        else:
            t0 = rng.uniform(0, 360, M)
            for dt in (0.0, 120.0, 240.0):
                x[:, h] = _place_batch(x[:, c - 2], x[:, prev], x[:, c], OCT_CH, TETRA_DEG, t0 + dt)
                h += 1
    d = np.linalg.norm(x[:, :, None, :] - x[:, None, :, :], axis=-1)
    far = gd >= 4
    hh = heavy[:, None] & heavy[None, :]
    ok = ~(np.any(far & hh & (d < 2.5), axis=(1, 2)) | np.any(far & ~hh & (d < 1.5), axis=(1, 2)))
    x = x[ok] - x[ok].mean(axis=1, keepdims=True)
    out = np.empty_like(x)
    for i in range(len(x)):
        _, v = np.linalg.eigh(np.cov(x[i][heavy].T))
        axis = v[:, -1] if v[2, -1] >= 0 else -v[:, -1]
        out[i] = x[i] @ _rotation_onto_z(axis).T
    return out


def _rotation_onto_z(u):
    """Rotation matrix taking the unit vector u onto +z (Rodrigues)."""
    z = np.array([0.0, 0.0, 1.0])
    v = np.cross(u, z)
    s, c = np.linalg.norm(v), float(u @ z)
    if s < 1e-12:
        return np.eye(3) if c > 0 else np.diag([1.0, -1.0, -1.0])
    k = v / s
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    ang = np.arctan2(s, c)
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def _z_turn(rng):
    """Uniform rotation about z, then an end-over-end flip with probability 1/2."""
    t = rng.uniform(0.0, 2.0 * np.pi)
    c, s = np.cos(t), np.sin(t)
    r = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    return r @ np.diag([1.0, -1.0, -1.0]) if rng.uniform() < 0.5 else r


class _SlotPacker:
    """Molecules on lattice slots with clash removal by redrawing.

    Each movable molecule has a draw function returning its absolute
    coordinates.  Intermolecular pairs closer than MIN_HEAVY (heavy-heavy)
    or MIN_WITH_H (involving H) are clashes; per round one partner of every
    clash is redrawn.  A molecule redrawn max_redraws times is removed (the
    achieved count is recorded by the caller: the density is never changed
    silently).
    """

    def __init__(self, rng, box):
        self.rng = rng
        self.box = np.asarray(box, float)
        self.coords, self.heavy, self.draw, self.redraws = [], [], [], []

    def add(self, heavy, draw=None, coords=None):
        self.coords.append(draw() if coords is None else np.asarray(coords, float))
        self.heavy.append(np.asarray(heavy, bool))
        self.draw.append(draw)
        self.redraws.append(0)

    def _flat(self, alive):
        idx = np.nonzero(alive)[0]
        pos = np.concatenate([self.coords[m] for m in idx])
        mol = np.concatenate([np.full(len(self.coords[m]), m) for m in idx])
        heavy = np.concatenate([self.heavy[m] for m in idx])
        return pos, mol, heavy

    def _clashes(self, pos, mol, heavy, tree, query_mask=None):
        """Clashing molecule pairs; with query_mask, only atoms it selects are queried."""
        if query_mask is None:
            pairs = tree.query_pairs(r=MIN_HEAVY, output_type="ndarray")
        else:
            qi = np.nonzero(query_mask)[0]
            lists = tree.query_ball_point(_wrap(pos[qi], self.box), r=MIN_HEAVY)
            a = np.repeat(qi, [len(l) for l in lists])
            b = np.concatenate([np.asarray(l, int) for l in lists]) if len(lists) else np.zeros(0, int)
            pairs = np.stack([a, b], 1) if len(a) else np.zeros((0, 2), int)
        if pairs.size == 0:
            return np.zeros((0, 2), int)
        pairs = pairs[mol[pairs[:, 0]] != mol[pairs[:, 1]]]
        if pairs.size == 0:
            return np.zeros((0, 2), int)
        d = pos[pairs[:, 1]] - pos[pairs[:, 0]]
        d -= self.box * np.round(d / self.box)
        r = np.linalg.norm(d, axis=1)
        bad = np.where(heavy[pairs[:, 0]] & heavy[pairs[:, 1]], r < MIN_HEAVY, r < MIN_WITH_H)
        return np.stack([mol[pairs[bad, 0]], mol[pairs[bad, 1]]], 1)

    def run(self, max_rounds=3000, max_redraws=200):
        alive = np.ones(len(self.coords), bool)
        moved = None
        for rnd in range(max_rounds):
            pos, mol, heavy = self._flat(alive)
            tree = cKDTree(_wrap(pos, self.box), boxsize=self.box)
            qmask = None if moved is None else np.isin(mol, list(moved))
            bad = self._clashes(pos, mol, heavy, tree, qmask)
            if len(bad) == 0:
                if moved is None:
                    return alive, rnd
                moved = None  # confirm with a full check
                continue
            # redraw one partner per clash: the molecule just moved when the
            # check was local (bad[:, 0] holds it), else the second one
            redo = set()
            for a, b in bad:
                order = (a, b) if moved is not None else (b, a)
                cand = [int(m) for m in order if self.draw[m] is not None]
                if cand and not (set(cand) & redo):
                    redo.add(cand[0])
            if not redo:
                raise RuntimeError("packer: clash between fixed molecules")
            for m in redo:
                self.redraws[m] += 1
                if self.redraws[m] > max_redraws:
                    alive[m] = False
                else:
                    self.coords[m] = self.draw[m]()
            moved = {m for m in redo if alive[m]}
        raise RuntimeError("packer: clashes remain after %d rounds" % max_rounds)


def _octanol_slots(rng, pk, n_mol, lo, hi, counts, pool_size=4096):
    """n_mol aligned octanol chains on a random subset of a counts[0] x
    counts[1] x counts[2] lattice in [lo, hi): a conformer drawn from a pool
    of pool_size batch draws, a random turn about z, flip, jitter U(+-0.3) A
    in x, y and U(+-0.45) A in z."""
    pool = octanol_conformers_aligned(rng, pool_size)
    names, bonds = octanol_topology()
    heavy = np.array([n not in ("H", "HO") for n in names])
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    ext = hi - lo
    grids = [lo[d] + (np.arange(counts[d]) + 0.5) * ext[d] / counts[d] for d in range(3)]
    g = np.stack(np.meshgrid(*grids, indexing="ij"), axis=-1).reshape(-1, 3)
    if g.shape[0] < n_mol:
        raise ValueError("lattice too small for %d molecules" % n_mol)
    sites = g[np.sort(rng.choice(g.shape[0], size=n_mol, replace=False))]
    first = len(pk.coords)
    for site in sites:
        def draw(site=site):
            j = rng.uniform(-1.0, 1.0, 3) * np.array([0.3, 0.3, 0.45])
            return pool[rng.integers(len(pool))] @ _z_turn(rng).T + site + j
        pk.add(heavy, draw)
    return first


def _delete_near(pk, ref_index, dmin, first):
    """Remove movable molecules (index >= first) with an atom closer than dmin to molecule ref_index."""
    tree = cKDTree(_wrap(pk.coords[ref_index], pk.box), boxsize=pk.box)
    keep = list(range(first))
    for m in range(first, len(pk.coords)):
        d, _ = tree.query(_wrap(pk.coords[m], pk.box), k=1)
        if np.min(d) >= dmin:
            keep.append(m)
    for name in ("coords", "heavy", "draw", "redraws"):
        lst = getattr(pk, name)
        setattr(pk, name, [lst[m] for m in keep])


def make_config3(seed=None, n_octanol=1480, L=73.0):
    """20-atom flexible solute in 1,480 octanol-like chains, 73 A cube (104 atoms/nm^3)."""
    seed = config_seed(3) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    onames, osig, oeps, ochg = _octanol_ff_types()
    sol, sbonds = random_tree_solute(rng, 20)
    s_sig, s_eps, s_q = _solute_params(rng, 20, 0.5)
    ff = ForceField(sigma=np.array(osig + list(s_sig)), epsilon=np.array(oeps + list(s_eps)),
                    charge=np.array(ochg + list(s_q)), names=onames + ["S%d" % i for i in range(20)])
    type_of = {n: i for i, n in enumerate(onames)}
    names, bonds = octanol_topology()
    oexcl = _exclusions_within(27, bonds, 3)
    otypes = np.array([type_of[n] for n in names])
    box = np.full(3, L)
    pk = _SlotPacker(rng, box)
    pk.add(np.ones(20, bool), coords=sol - sol.mean(axis=0) + box / 2)
    counts = np.array([16, 16, 6])   # 4.56 x 4.56 x 12.2 A cells for ~12 A chains
    _octanol_slots(rng, pk, n_octanol, np.zeros(3), box, counts)
    _delete_near(pk, 0, SOLUTE_WATER_DELETE, 1)
    alive, rounds = pk.run()
    parts = [dict(pos=pk.coords[0], types=np.arange(5, 25), solute=np.ones(20), mol=np.zeros(20),
                  excl=_exclusions_within(20, sbonds, 3))]
    for m in np.nonzero(alive)[0][1:]:
        parts.append(dict(pos=pk.coords[m], types=otypes, solute=np.zeros(27), mol=np.full(27, m), excl=oexcl))
    s = _assemble(parts, box)
    s.info.update(n_octanol_requested=n_octanol, n_octanol=len(parts) - 1, packing_rounds=int(rounds))
    return Workload(name="octanol1480_solute20", systems=[s], ff=ff, cutoff=10.0, skin=1.0, switch_width=1.0,
                    dsf_alpha=0.2, sc_alpha=0.5, lambdas=np.array([0.3]), seed=seed,
                    info=dict(fd_lambdas=[0.3, 0.7, 1.0]))


def make_config5(seed=None, L=135.0, n_total=250_000):
    """250k-atom water/octanol slab with a 22-atom peptide-like solute in the water half."""
    seed = config_seed(5) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    wn, wsig, weps, wchg = _water_forcefield_types()
    onames, osig, oeps, ochg = _octanol_ff_types()
    sol, sbonds, _ = peptide_solute(rng)
    s_sig, s_eps, s_q = _solute_params(rng, 22, 0.6)
    ff = ForceField(sigma=np.array(wsig + osig + list(s_sig)), epsilon=np.array(weps + oeps + list(s_eps)),
                    charge=np.array(wchg + ochg + list(s_q)),
                    names=wn + onames + ["P%d" % i for i in range(22)])
    type_of = {n: 2 + i for i, n in enumerate(onames)}
    names, bonds = octanol_topology()
    oexcl = _exclusions_within(27, bonds, 3)
    otypes = np.array([type_of[n] for n in names])
    box = np.full(3, L)
    n_w = int(round(0.1 * L * L * L / 2)) // 3
    n_oct = (n_total - 22 - 3 * n_w) // 27
    pk = _SlotPacker(rng, box)
    pk.add(np.ones(22, bool), coords=sol - sol.mean(axis=0) + np.array([L / 2, L / 2, L / 4]))
    sites, _ = _lattice_sites(rng, n_w, np.zeros(3), np.array([L, L, L / 2]))
    wf = water_molecule_frame()
    wheavy = np.array([True, False, False])
    for site in sites:
        pk.add(wheavy, lambda site=site: wf @ _random_rotation(rng).T + site + rng.uniform(-0.3, 0.3, 3))
    first_oct = len(pk.coords)
    counts = np.array([31, 31, 5])   # 4.35 x 4.35 x 13.5 A cells
    _octanol_slots(rng, pk, n_oct, np.array([0.0, 0.0, L / 2]), np.array([L, L, L]), counts)
    _delete_near(pk, 0, SOLUTE_WATER_DELETE, 1)
    alive, rounds = pk.run()
    parts = [dict(pos=pk.coords[0], types=np.arange(7, 29), solute=np.ones(22), mol=np.zeros(22),
                  excl=_exclusions_within(22, sbonds, 3))]
    nw = no = 0
    for m in np.nonzero(alive)[0][1:]:
        if len(pk.coords[m]) == 3:
            parts.append(dict(pos=pk.coords[m], types=np.array([0, 1, 1]), solute=np.zeros(3), mol=np.full(3, m),
                              excl=[(0, 1), (0, 2), (1, 2)]))
            nw += 1
        else:
            parts.append(dict(pos=pk.coords[m], types=otypes, solute=np.zeros(27), mol=np.full(27, m), excl=oexcl))
            no += 1
    s = _assemble(parts, box)
    s.info.update(n_waters_requested=n_w, n_waters=nw, n_octanol_requested=n_oct, n_octanol=no,
                  packing_rounds=int(rounds), cv=PEPTIDE_CV)
    del first_oct
    return Workload(name="slab250k_peptide22", systems=[s], ff=ff, cutoff=12.0, skin=1.0, switch_width=1.0,
                    dsf_alpha=0.2, sc_alpha=0.5, lambdas=np.array([0.7]), seed=seed,
                    info=dict(cv_atoms=np.array(list(PEPTIDE_CV.values()), np.int32)))


def make_config(k: int, seed: Optional[int] = None, **kw) -> Workload:
    return {1: make_config1, 2: make_config2, 3: make_config3, 4: make_config4, 5: make_config5}[k](seed=seed, **kw)


# --------------------------------------------------------------------------
# call protocols
# --------------------------------------------------------------------------


def perturbation_walk(system: System, n_calls: int, sigma: float, seed: int):
    """Positions of n_calls successive calls: x_t = x_{t-1} + N(0, sigma) per coordinate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    steps = rng.normal(0.0, sigma, size=(n_calls, system.n_atoms, 3))
    steps[0] = 0.0
    return system.positions[None, :, :] + np.cumsum(steps, axis=0)


def lambda_draws(n_calls: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=n_calls)


def random_tiny_system(rng, n_atoms: int, box: float, n_solute: int, n_types: int, min_dist=1.6):
    """Small random box for edge-case tests: random positions with a minimum distance."""
    pos = []
    while len(pos) < n_atoms:
        x = rng.uniform(0, box, 3)
        ok = True
        for p in pos:
            d = x - p
            d -= box * np.round(d / box)
            if np.linalg.norm(d) < min_dist:
                ok = False
                break
        if ok:
            pos.append(x)
    pos = np.array(pos)
    types = rng.integers(0, n_types, n_atoms).astype(np.int32)
    sol = np.zeros(n_atoms, np.uint8)
    sol[:n_solute] = 1
    return System(positions=pos, types=types, is_solute=sol, exclusions=np.zeros((0, 2), np.int32),
                  box=np.full(3, float(box)), molecule=np.arange(n_atoms, dtype=np.int32))
