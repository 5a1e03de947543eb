"""Ewald electrostatics by smooth particle-mesh Ewald, with the
solute-solvent cross term scaled by lambda (FP64 reference).

TEST INFRASTRUCTURE (see the package docstring).

The paper treats long-range electrostatics with PME (Simulation Details,
citing Darden et al. 1993 and Essmann et al. 1995) and couples the solute
to the solvent through lambda-scaled slices of the nonbonded energy
(Linear Basis Function section, eq. 4): only the solute-solvent (S-W) part
of the Coulomb energy is scaled, by the schedule's electrostatic factor c
(le for the Beutler schedule, h_A for LBF).

Ewald sum of a periodic orthorhombic box (k_e = 332.06371, splitting
parameter a, m = (m1/L1, m2/L2, m3/L3) over integer triples m != 0):
    E_real  = sum over non-excluded pairs within r_c of k_e q_i q_j erfc(a r)/r
              (the C oracle with the Ewald flag)
    E_recip = k_e/(2 pi V) sum_m exp(-pi^2 |m|^2/a^2)/|m|^2 |S(m)|^2,
              S(m) = sum_j q_j exp(2 pi i m.r_j)
    E_self  = -k_e a/sqrt(pi) sum_i q_i^2
    E_excl  = -k_e sum over excluded pairs of q_i q_j erf(a r)/r (minimum image)
    E_bg    = -k_e pi Q^2/(2 V a^2), Q = sum_i q_i (neutralising background)
Every part is a sum over pairs of charges (self and background included),
so each splits into S-S, W-W and S-W parts; with S_S and S_W the structure
factors of the two groups, |S|^2 = |S_S|^2 + |S_W|^2 + 2 Re(S_S conj(S_W)).
The lambda-dependent energy is U = E^SS + E^WW + c(lambda) E^SW, so
dU/dlambda gains c'(lambda) E^SW and the forces are -grad U.

Smooth PME (Essmann et al. 1995) replaces S(m) by the discrete Fourier
transform of a charge grid built with cardinal B-splines M_n of order n:
    u_ia = K_a x_ia / L_a,  Q(k) = sum_i q_i prod_a M_n(u_ia - k_a), summed
    over periodic images of the grid;
    E_recip ~ 1/2 sum_m C(m) |F(Q)(m)|^2,
    C(m) = k_e/(pi V) exp(-pi^2 |m|^2/a^2)/|m|^2 B(m),  C(0) = 0,
    B(m) = prod_a |b_a(m_a)|^2,
    |b_a(m)|^2 = 1/|sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k/K_a)|^2,
with m_a taken in (-K_a/2, K_a/2] for |m|^2.  The grid potential
phi[Q] = K1 K2 K3 ifft(C fft(Q)) is dE/dQ; with two grids Q_S and Q_W,
U_recip = 1/2 Q_S.phi[Q_S] + 1/2 Q_W.phi[Q_W] + c Q_S.phi[Q_W], and an
atom of group X feels F_i = -sum_k dQ_X(k)/dx_i G_X(k) with
G_S = phi[Q_S] + c phi[Q_W], G_W = phi[Q_W] + c phi[Q_S].

Readings (the method's papers leave these points open):
- for an odd order on an even grid the denominator of b at m = K/2 is 0;
  its squared modulus is replaced by the mean of its two neighbours;
- the splitting parameter, grid and order are inputs (the paper states
  none of them); a cross-group exclusion is scaled by c like any S-W term.
"""
import math

import numpy as np

import oracle as O

KE = 332.06371


def bspline(u, n):
    """Cardinal B-spline M_n(u), support (0, n): M_2(u) = 1 - |u - 1| on
    [0, 2], M_n(u) = [u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)]/(n - 1)."""
    u = np.asarray(u, float)
    if n == 2:
        return np.where((u >= 0.0) & (u <= 2.0), 1.0 - np.abs(u - 1.0), 0.0)
    return (u * bspline(u, n - 1) + (n - u) * bspline(u - 1.0, n - 1)) / (n - 1)


def bspline_d(u, n):
    """dM_n/du = M_{n-1}(u) - M_{n-1}(u - 1)."""
    u = np.asarray(u, float)
    return bspline(u, n - 1) - bspline(u - 1.0, n - 1)


def bspline_moduli(K, n):
    """|b(m)|^2 for m = 0 .. K-1 (the reading above at a vanishing denominator)."""
    k = np.arange(n - 1)
    Mk = bspline(k + 1.0, n)
    m = np.arange(K)
    D = (Mk[None, :] * np.exp(2j * np.pi * np.outer(m, k) / K)).sum(axis=1)
    d2 = np.abs(D) ** 2
    for i in np.nonzero(d2 < 1e-10)[0]:
        d2[i] = 0.5 * (d2[i - 1] + d2[(i + 1) % K])
    return 1.0 / d2


def signed_index(K):
    """m in (-K/2, K/2] for the grid index 0 .. K-1."""
    m = np.arange(K)
    return np.where(m <= K // 2, m, m - K)


def influence(box, K, n, a):
    """C(m) on the K1 x K2 x K3 grid of reciprocal indices."""
    L = np.asarray(box, float)
    V = float(np.prod(L))
    mx, my, mz = [signed_index(k) / l for k, l in zip(K, L)]
    m2 = mx[:, None, None] ** 2 + my[None, :, None] ** 2 + mz[None, None, :] ** 2
    B = (bspline_moduli(K[0], n)[:, None, None] * bspline_moduli(K[1], n)[None, :, None]
         * bspline_moduli(K[2], n)[None, None, :])
    m2[0, 0, 0] = 1.0
    C = KE / (math.pi * V) * np.exp(-math.pi ** 2 * m2 / (a * a)) / m2 * B
    C[0, 0, 0] = 0.0
    return C


def spline_data(pos, box, K, n):
    """Per atom and axis: the n grid indices floor(u) - j (periodic), the
    weights M_n(u - floor(u) + j) and their x-derivatives, j = 0 .. n-1."""
    L = np.asarray(box, float)
    Ka = np.asarray(K, float)
    u = np.asarray(pos, float).reshape(-1, 3) / L * Ka
    u = u - Ka * np.floor(u / Ka)
    fl = np.floor(u)
    w = u - fl
    j = np.arange(n)
    idx = (fl[:, :, None].astype(np.int64) - j[None, None, :]) % np.asarray(K, np.int64)[None, :, None]
    arg = w[:, :, None] + j[None, None, :]
    th = bspline(arg, n)
    dth = bspline_d(arg, n) * (Ka / L)[None, :, None]
    return idx, th, dth


def charge_grid(idx, th, q, K):
    """Q(k): every atom's charge spread over its n^3 grid points."""
    Q = np.zeros(tuple(K))
    n = th.shape[2]
    for a in range(n):
        for b in range(n):
            for c in range(n):
                np.add.at(Q, (idx[:, 0, a], idx[:, 1, b], idx[:, 2, c]),
                          q * th[:, 0, a] * th[:, 1, b] * th[:, 2, c])
    return Q


def gather_forces(idx, th, dth, q, G):
    """F_i = -q_i sum_k grad_i(prod_a M_n) G(k)."""
    F = np.zeros((len(q), 3))
    n = th.shape[2]
    for a in range(n):
        for b in range(n):
            for c in range(n):
                g = q * G[idx[:, 0, a], idx[:, 1, b], idx[:, 2, c]]
                F[:, 0] -= g * dth[:, 0, a] * th[:, 1, b] * th[:, 2, c]
                F[:, 1] -= g * th[:, 0, a] * dth[:, 1, b] * th[:, 2, c]
                F[:, 2] -= g * th[:, 0, a] * th[:, 1, b] * dth[:, 2, c]
    return F


def gather_potential(idx, th, G):
    """sum_k prod_a M_n G(k) per atom (dU/dq_i divided by nothing: the potential)."""
    out = np.zeros(idx.shape[0])
    n = th.shape[2]
    for a in range(n):
        for b in range(n):
            for c in range(n):
                out += G[idx[:, 0, a], idx[:, 1, b], idx[:, 2, c]] * th[:, 0, a] * th[:, 1, b] * th[:, 2, c]
    return out


def pme_reciprocal(pos, q, solute, box, a, K, n, c=1.0):
    """Smooth-PME reciprocal energy parts (e_ss, e_ww, e_sw) and the forces of
    U = e_ss + e_ww + c e_sw."""
    K = tuple(int(k) for k in K)
    q = np.asarray(q, float)
    s = np.asarray(solute, bool)
    qs, qw = np.where(s, q, 0.0), np.where(s, 0.0, q)
    idx, th, dth = spline_data(pos, box, K, n)
    FS = np.fft.fftn(charge_grid(idx, th, qs, K))
    FW = np.fft.fftn(charge_grid(idx, th, qw, K))
    C = influence(box, K, n, a)
    e_ss = 0.5 * float(np.sum(C * np.abs(FS) ** 2))
    e_ww = 0.5 * float(np.sum(C * np.abs(FW) ** 2))
    e_sw = float(np.sum(C * (FS * np.conj(FW)).real))
    NK = K[0] * K[1] * K[2]
    phi_s = NK * np.fft.ifftn(C * FS).real
    phi_w = NK * np.fft.ifftn(C * FW).real
    GS, GW = phi_s + c * phi_w, phi_w + c * phi_s
    F = gather_forces(idx, th, dth, qs, GS) + gather_forces(idx, th, dth, qw, GW)
    pot = np.where(s, gather_potential(idx, th, GS), gather_potential(idx, th, GW))
    return dict(e_ss=e_ss, e_ww=e_ww, e_sw=e_sw, forces=F, potential=pot)


def ewald_reciprocal(pos, q, solute, box, a, mmax, c=1.0, chunk=2048):
    """The reciprocal sum by its definition over |m_i| <= mmax[i] (FP64):
    (e_ss, e_ww, e_sw) and the forces of e_ss + e_ww + c e_sw."""
    L = np.asarray(box, float)
    V = float(np.prod(L))
    pos = np.asarray(pos, float).reshape(-1, 3)
    q = np.asarray(q, float)
    s = np.asarray(solute, bool)
    qs, qw = np.where(s, q, 0.0), np.where(s, 0.0, q)
    axes = [np.arange(-int(m), int(m) + 1) for m in mmax]
    M = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    M = M[np.any(M != 0, axis=1)]
    e = np.zeros(3)
    F = np.zeros_like(pos)
    for b0 in range(0, len(M), chunk):
        mv = M[b0:b0 + chunk] / L
        m2 = (mv ** 2).sum(axis=1)
        f = np.exp(-math.pi ** 2 * m2 / (a * a)) / m2
        E = np.exp(2j * math.pi * (pos @ mv.T))
        SS, SW = qs @ E, qw @ E
        e[0] += KE / (2 * math.pi * V) * float(np.sum(f * np.abs(SS) ** 2))
        e[1] += KE / (2 * math.pi * V) * float(np.sum(f * np.abs(SW) ** 2))
        e[2] += KE / (math.pi * V) * float(np.sum(f * (SS * np.conj(SW)).real))
        GS, GW = SS + c * SW, SW + c * SS
        im = np.where(s[:, None], (E * np.conj(GS)[None, :]).imag, (E * np.conj(GW)[None, :]).imag)
        F += (2 * KE / V) * q[:, None] * ((im * f[None, :]) @ mv)
    return dict(e_ss=e[0], e_ww=e[1], e_sw=e[2], forces=F)


def ewald_corrections(pos, q, solute, exclusions, box, a, c=1.0):
    """Self, excluded-pair and background parts (e_ss, e_ww, e_sw) and the
    forces of e_ss + e_ww + c e_sw (the self and background parts have none)."""
    L = np.asarray(box, float)
    V = float(np.prod(L))
    pos = np.asarray(pos, float).reshape(-1, 3)
    q = np.asarray(q, float)
    s = np.asarray(solute, bool)
    e = dict(ss=0.0, ww=0.0, sw=0.0)
    e["ss"] -= KE * a / math.sqrt(math.pi) * float(np.sum(q[s] ** 2))
    e["ww"] -= KE * a / math.sqrt(math.pi) * float(np.sum(q[~s] ** 2))
    Qs, Qw = float(np.sum(q[s])), float(np.sum(q[~s]))
    e["ss"] -= KE * math.pi * Qs * Qs / (2 * V * a * a)
    e["ww"] -= KE * math.pi * Qw * Qw / (2 * V * a * a)
    e["sw"] -= KE * math.pi * Qs * Qw / (V * a * a)
    F = np.zeros_like(pos)
    for i, j in np.asarray(exclusions, np.int64).reshape(-1, 2):
        d = pos[j] - pos[i]
        d -= L * np.round(d / L)
        r = float(np.sqrt(d @ d))
        qq = q[i] * q[j]
        v = -KE * qq * math.erf(a * r) / r
        dv = -KE * qq * (2 * a / math.sqrt(math.pi) * math.exp(-a * a * r * r) / r - math.erf(a * r) / (r * r))
        key = "ss" if s[i] and s[j] else ("ww" if not s[i] and not s[j] else "sw")
        e[key] += v
        scale = c if key == "sw" else 1.0
        F[i] += scale * dv * d / r
        F[j] -= scale * dv * d / r
    return dict(e_ss=e["ss"], e_ww=e["ww"], e_sw=e["sw"], forces=F)


def elec_factor(schedule, lam):
    """c(lambda) and dc/dlambda of the S-W electrostatics (left derivative at the Beutler kink)."""
    if schedule == O.BEUTLER:
        return max(0.0, 2.0 * lam - 1.0), (2.0 if lam > 0.5 else 0.0)
    h = O.lbf_switches(lam)
    return float(h[0]), float(h[2])


def evaluate(positions, types, is_solute, exclusions, box, sigma, epsilon, charge, params, lam, grid, order,
             reciprocal=None, n_threads=0):
    """One box with Ewald electrostatics: the C oracle's short-range terms
    (params.ewald set: real space erfc(a r)/r) plus the PME reciprocal part
    and the corrections, assembled into the ten term slots:
        E_solv_solv += E^WW, E_solu_solu += E^SS, E_ss_elec += c X,
        U_A += X (LBF), dUdl_elec and dUdl += c' X, E_total += E^WW + E^SS + c X,
    X = E^SW.  reciprocal: None (PME on `grid` with `order`) or ('exact', mmax)."""
    assert params.ewald, "Ewald real space expected"
    r = O.evaluate(positions, types, is_solute, exclusions, box, sigma, epsilon, charge, params, lam,
                   forces=True, n_threads=n_threads)
    a = params.dsf_alpha
    c, dc = elec_factor(params.schedule, lam)
    q = np.asarray(charge, float)[np.asarray(types)]
    if reciprocal is None:
        rec = pme_reciprocal(positions, q, is_solute, box, a, grid, order, c)
    else:
        rec = ewald_reciprocal(positions, q, is_solute, box, a, reciprocal[1], c)
    cor = ewald_corrections(positions, q, is_solute, exclusions, box, a, c)
    e_ww = rec["e_ww"] + cor["e_ww"]
    e_ss = rec["e_ss"] + cor["e_ss"]
    X = rec["e_sw"] + cor["e_sw"]
    t = r["terms"].copy()
    t[0] += e_ww
    t[1] += e_ss
    t[3] += c * X
    if params.schedule == O.LBF:
        t[4] += X
    t[7] += dc * X
    t[8] += e_ww + e_ss + c * X
    t[9] += dc * X
    # magnitudes of what each slot sums (error scales): the pair oracle's sums of |u| plus the
    # magnitudes of the reciprocal and correction parts
    ab = r["abs_terms"].copy()
    p_ww = abs(rec["e_ww"]) + abs(cor["e_ww"])
    p_ss = abs(rec["e_ss"]) + abs(cor["e_ss"])
    p_x = abs(rec["e_sw"]) + abs(cor["e_sw"])
    ab[0] += p_ww
    ab[1] += p_ss
    ab[3] += abs(c) * p_x
    if params.schedule == O.LBF:
        ab[4] += p_x
    ab[7] += abs(dc) * p_x
    ab[8] += p_ww + p_ss + abs(c) * p_x
    ab[9] += abs(dc) * p_x
    return dict(terms=t, forces=r["forces"] + rec["forces"] + cor["forces"], n_pairs=r["n_pairs"],
                recip=rec, corr=cor, cross=X, abs_terms=ab)


def evaluate_system(system, ff, params, lam, grid, order, **kw):
    return evaluate(system.positions, system.types, system.is_solute, system.exclusions, system.box,
                    ff.sigma, ff.epsilon, ff.charge, params, lam, grid, order, **kw)
