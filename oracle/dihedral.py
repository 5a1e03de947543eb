"""Dihedral collective variables and the d-AFED coupling (FP64 reference).

TEST INFRASTRUCTURE (see the package docstring).

- Dihedral xi of atoms (1, 2, 3, 4) with bond vectors F = r1 - r2,
  G = r2 - r3, H = r4 - r3 and normals A = F x G, B = H x G:
  xi = atan2((B x A) . G/|G|, A . B), in (-pi, pi]; 0 for the cis
  arrangement, pi for trans.
- Cartesian gradient: the closed form of Blondel & Karplus (J. Comput. Chem.
  17, 1132, 1996), a published method restated here:
      dxi/dr1 = -|G|/|A|^2 A
      dxi/dr4 = +|G|/|B|^2 B
      dxi/dr2 =  |G|/|A|^2 A + (F.G)/(|A|^2 |G|) A - (H.G)/(|B|^2 |G|) B
      dxi/dr3 = -|G|/|B|^2 B - (F.G)/(|A|^2 |G|) A + (H.G)/(|B|^2 |G|) B
- d-AFED coupling (the paper's eq. 15): U = sum_k kappa_k/2 d_k^2 with
  d_k = xi_k - s_k wrapped into (-pi, pi]; force on atom i is
  -sum_k kappa_k d_k dxi_k/dr_i.
- Effective-mass denominator (eq. 16): sum_i m_i^-1 |dxi_k/dr_i|^2 over the
  four atoms of CV k (the auxiliary mass is c times its inverse).
Bond vectors use the minimum image of an orthorhombic box.
"""
import numpy as np


def _mi(v, box):
    return v - box * np.round(v / box)


def dihedral(r1, r2, r3, r4, box):
    F = _mi(np.asarray(r1, float) - r2, box)
    G = _mi(np.asarray(r2, float) - r3, box)
    H = _mi(np.asarray(r4, float) - r3, box)
    A = np.cross(F, G)
    B = np.cross(H, G)
    gn = np.linalg.norm(G)
    xi = np.arctan2(np.dot(np.cross(B, A), G) / gn, np.dot(A, B))
    a2, b2 = np.dot(A, A), np.dot(B, B)
    fg, hg = np.dot(F, G), np.dot(H, G)
    d1 = -gn / a2 * A
    d4 = gn / b2 * B
    d2 = gn / a2 * A + fg / (a2 * gn) * A - hg / (b2 * gn) * B
    d3 = -gn / b2 * B - fg / (a2 * gn) * A + hg / (b2 * gn) * B
    return xi, np.stack([d1, d2, d3, d4])


def wrap_angle(d):
    """Wrap into (-pi, pi]."""
    w = np.mod(d + np.pi, 2 * np.pi) - np.pi
    return np.where(w == -np.pi, np.pi, w)


def cvs(positions, idx, box, mass_inv=None, s=None, kappa=None):
    """All CVs: xi [C], dxi [C,4,3], msum [C] (eq. 16 denominator), u_dafed, forces [N,3]."""
    pos = np.asarray(positions, float)
    idx = np.asarray(idx, int).reshape(-1, 4)
    C = idx.shape[0]
    xi = np.zeros(C)
    dxi = np.zeros((C, 4, 3))
    for k in range(C):
        xi[k], dxi[k] = dihedral(*(pos[i] for i in idx[k]), box)
    out = dict(xi=xi, dxi=dxi)
    if mass_inv is not None:
        mi = np.asarray(mass_inv, float)
        out["msum"] = np.array([sum(mi[idx[k, j]] * np.dot(dxi[k, j], dxi[k, j]) for j in range(4))
                                for k in range(C)])
    if s is not None:
        d = wrap_angle(xi - np.asarray(s, float))
        kap = np.asarray(kappa, float)
        out["u_dafed"] = float(np.sum(0.5 * kap * d * d))
        f = np.zeros_like(pos)
        for k in range(C):
            for j in range(4):
                f[idx[k, j]] -= kap[k] * d[k] * dxi[k, j]
        out["forces"] = f
    return out
