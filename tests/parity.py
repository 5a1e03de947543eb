"""Error metrics and oracle/GPU comparison helpers shared by the GPU tests.

Metrics (forces, dU/dlambda, energies):
  e_F      = sqrt(sum_i |F_i - F_i^ref|^2 / sum_i |F_i^ref|^2)
  e_lambda = |d - d_ref| / |d_ref| when |d_ref| >= 1e-2 * S, else |d - d_ref| / S,
             S = sum over pairs of |du_ij/dlambda| (cancellation-safe fallback)
  e_E      = |E - E_ref| / sum over pairs of |u_ij| for the same term
"""
import numpy as np

import oracle as O

TOL = {
    # FP32 pair arithmetic with fixed-point forces
    0: dict(force=1e-5, dudl=1e-6, energy=1e-6),
    # FP64 path
    1: dict(force=1e-10, dudl=1e-10, energy=1e-11),
}


def force_error(F, Fref):
    den = np.sum(Fref * Fref)
    return float(np.sqrt(np.sum((F - Fref) ** 2) / den)) if den > 0 else float(np.abs(F).max())


def dudl_error(d, dref, scale):
    if scale <= 0:
        return abs(d - dref)
    if abs(dref) >= 1e-2 * scale:
        return abs(d - dref) / abs(dref)
    return abs(d - dref) / scale


def energy_error(E, Eref, scale):
    if scale <= 0:
        return abs(E - Eref)
    return abs(E - Eref) / scale


def oracle_for(workload, k, lam, schedule, positions=None, **kw):
    s = workload.systems[k]
    P = O.Params.of(workload, schedule)
    pos = s.positions if positions is None else positions
    return O.evaluate(pos, s.types, s.is_solute, s.exclusions, s.box, workload.ff.sigma, workload.ff.epsilon,
                      workload.ff.charge, P, lam, **kw)


def boundary_band(workload, k, positions, delta):
    """Number of pairs whose distance lies within delta of the cutoff."""
    s = workload.systems[k]
    hi = O.pair_set(positions, s.exclusions, s.box, workload.cutoff + delta).shape[0]
    lo = O.pair_set(positions, s.exclusions, s.box, workload.cutoff - delta).shape[0]
    return hi - lo


def compare(res, refs, workload, positions_per_box, precision, offsets, check_pairs=True, label="",
            energy_tol=None):
    """Compare one GPU result (dict of numpy arrays) with per-box oracle results.

    Returns a dict of the worst errors; asserts they are within TOL[precision]
    (energy_tol, when given, replaces the energy bar: energies carry no bar of
    their own in the targets, and a caller that sets one states its reason).
    """
    tol = dict(TOL[precision])
    if energy_tol is not None:
        tol["energy"] = energy_tol
    worst = dict(force=0.0, dudl=0.0, energy=0.0)
    for k, ref in enumerate(refs):
        a, b = offsets[k], offsets[k + 1]
        eF = force_error(res["forces"][a:b], ref["forces"]) if b > a else 0.0
        scale = ref["abs_terms"]
        ed = dudl_error(res["dudl"][k], ref["terms"][9], scale[9])
        eE = max(energy_error(res["terms"][k, j], ref["terms"][j], scale[j]) for j in range(10))
        worst["force"] = max(worst["force"], eF)
        worst["dudl"] = max(worst["dudl"], ed)
        worst["energy"] = max(worst["energy"], eE)
        assert eF <= tol["force"], "%s box %d force error %.3e" % (label, k, eF)
        assert ed <= tol["dudl"], "%s box %d dU/dlambda error %.3e (gpu %.12g ref %.12g)" % (
            label, k, ed, res["dudl"][k], ref["terms"][9])
        assert eE <= tol["energy"], "%s box %d energy error %.3e\n gpu %s\n ref %s" % (
            label, k, eE, res["terms"][k], ref["terms"])
        if check_pairs:
            dn = abs(int(res["n_pairs"][k]) - ref["n_pairs"])
            if dn:
                band = boundary_band(workload, k, positions_per_box[k], 1e-4)
                assert dn <= band, "%s box %d pair count %d vs %d" % (label, k, res["n_pairs"][k], ref["n_pairs"])
    return worst


def to_numpy(out):
    return {k: (v.detach().cpu().numpy() if hasattr(v, "detach") else v) for k, v in out.items() if v is not None}
