"""GPU parity at the large workloads: the octanol box (config 3, forward and
backward against the full oracle at three lambdas) and the 250k-atom slab
(config 5, sampled atoms against the per-atom oracle sums, the exact
dU/dlambda from the solute atoms, FP32 against FP64, backward and the four
dihedral CVs)."""
import numpy as np
import pytest

import oracle as O
from oracle import dihedral as OD

from conftest import workload
from parity import TOL, compare, force_error, oracle_for, to_numpy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ctx(w, precision):
    from paper_2608_12691_amd import alchnb
    return alchnb.from_workload(w, precision=precision, schedule=O.BEUTLER)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
def test_config3_forward_backward_three_lambdas(precision):
    """20-atom flexible solute in octanol: energies, forces, dU/dlambda and the
    per-type sigma / sqrt(eps) / charge gradients against the full oracle."""
    w = workload(3)
    s = w.systems[0]
    ctx = _ctx(w, precision)
    pos = ctx.positions(w.systems)
    T = ctx.n_types
    g = torch.ones(1, dtype=torch.float64, device=ctx.device)
    ptol = 1e-9 if precision == 1 else 3e-5
    for lam in w.info["fd_lambdas"]:
        print("config3 precision %d lambda %.2f atoms %d" % (precision, lam, s.n_atoms), flush=True)
        lt = ctx.lambdas([lam])
        res = to_numpy(ctx.compute_checked(pos, lt, flags=2))
        assert res["flags"] == 0
        ref = oracle_for(w, 0, lam, O.BEUTLER, param_grads=True)
        compare(res, [ref], w, [s.positions], precision, np.array([0, s.n_atoms]), label="cfg3 lam=%g" % lam)
        dsig, dse, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(3))
        dpos = torch.zeros_like(pos)
        dl = torch.zeros(1, dtype=torch.float64, device=ctx.device)
        ctx.backward(pos, lt, g, d_pos=dpos, d_lambda=dl, d_sigma=dsig, d_sqrt_eps=dse, d_charge=dq)
        torch.cuda.synchronize()
        assert force_error(-dpos.cpu().numpy(), ref["forces"]) <= TOL[precision]["force"]
        assert dl.item() == pytest.approx(ref["terms"][9], rel=max(TOL[precision]["dudl"], 1e-12))
        assert _rel(dsig.cpu().numpy(), ref["d_sigma"]) < ptol
        assert _rel(dse.cpu().numpy(), ref["d_sqrt_eps"]) < ptol
        assert _rel(dq.cpu().numpy(), ref["d_charge"]) < ptol


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
def test_config3_lbf_forward_and_parameter_pass(precision):
    """The LBF schedule on the octanol box (flexible solute with bond-graph exclusions) at lambdas on
    both sides of the h_A onset: forward and per-type gradients against the full oracle."""
    from paper_2608_12691_amd import alchnb
    w = workload(3)
    s = w.systems[0]
    ctx = alchnb.from_workload(w, precision=precision, schedule=O.LBF)
    pos = ctx.positions(w.systems)
    T = ctx.n_types
    g = torch.ones(1, dtype=torch.float64, device=ctx.device)
    ptol = 1e-9 if precision == 1 else 3e-5
    for lam in (0.25, 0.7):
        print("config3 lbf precision %d lambda %.2f" % (precision, lam), flush=True)
        lt = ctx.lambdas([lam])
        res = to_numpy(ctx.compute_checked(pos, lt, flags=2))
        assert res["flags"] == 0
        ref = oracle_for(w, 0, lam, O.LBF, param_grads=True)
        compare(res, [ref], w, [s.positions], precision, np.array([0, s.n_atoms]), label="cfg3 lbf lam=%g" % lam)
        dsig, dse, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(3))
        ctx.backward(pos, lt, g, d_sigma=dsig, d_sqrt_eps=dse, d_charge=dq)
        torch.cuda.synchronize()
        assert _rel(dsig.cpu().numpy(), ref["d_sigma"]) < ptol
        assert _rel(dse.cpu().numpy(), ref["d_sqrt_eps"]) < ptol
        assert _rel(dq.cpu().numpy(), ref["d_charge"]) < ptol


def test_config3_fp64_energy_fd_in_type_parameters():
    """Central differences (h = 1e-4) of the GPU FP64 energy in the parameters
    of the octanol carbon, the hydroxyl oxygen and two solute types."""
    from paper_2608_12691_amd import systems as S
    w = workload(3)
    lam, h = 0.7, 1e-4
    ctx = _ctx(w, 1)
    pos = ctx.positions(w.systems)
    T = ctx.n_types
    ctx.compute(pos, ctx.lambdas([lam]), flags=2)
    dsig, dse, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(3))
    ctx.backward(pos, ctx.lambdas([lam]), torch.ones(1, dtype=torch.float64, device=ctx.device),
                 d_sigma=dsig, d_sqrt_eps=dse, d_charge=dq)
    torch.cuda.synchronize()

    def energy(ff):
        w2 = S.Workload(w.name, w.systems, ff, w.cutoff, w.skin, w.switch_width, w.dsf_alpha, w.sc_alpha,
                        w.lambdas, w.seed)
        c = _ctx(w2, 1)
        o = c.compute(c.positions(w.systems), c.lambdas([lam]), flags=2)
        torch.cuda.synchronize()
        e = float(o["terms"][0, 8])
        c.close()
        return e

    names = list(w.ff.names)
    for t in (names.index("C"), names.index("O"), 6, 17):
        for arr, grad, tr in (("sigma", dsig, None), ("charge", dq, None), ("epsilon", dse, "sqrt")):
            fp = S.ForceField(w.ff.sigma.copy(), w.ff.epsilon.copy(), w.ff.charge.copy(), w.ff.names)
            fm = S.ForceField(w.ff.sigma.copy(), w.ff.epsilon.copy(), w.ff.charge.copy(), w.ff.names)
            if tr == "sqrt":
                if w.ff.epsilon[t] == 0:
                    continue
                e0 = np.sqrt(w.ff.epsilon[t])
                fp.epsilon[t], fm.epsilon[t] = (e0 + h) ** 2, (e0 - h) ** 2
            else:
                getattr(fp, arr)[t] += h
                getattr(fm, arr)[t] -= h
            fd = (energy(fp) - energy(fm)) / (2 * h)
            print("config3 FD type %d %s gpu %.10g fd %.10g" % (t, arr, float(grad[t]), fd), flush=True)
            assert float(grad[t]) == pytest.approx(fd, rel=1e-5, abs=1e-6), (arr, t)


def _slab():
    w = workload(5)
    return w, w.systems[0]


def test_config5_slab_sampled_oracle_fp32_fp64_and_cvs():
    w, s = _slab()
    lam = float(w.lambdas[0])
    print("config5 atoms %d lambda %.2f" % (s.n_atoms, lam), flush=True)
    res = {}
    for precision in (1, 0):
        ctx = _ctx(w, precision)
        pos = ctx.positions(w.systems)
        lt = ctx.lambdas([lam])
        r = to_numpy(ctx.compute_checked(pos, lt, flags=2))
        assert r["flags"] == 0
        T = ctx.n_types
        dsig, dse, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(3))
        dl = torch.zeros(1, dtype=torch.float64, device=ctx.device)
        ctx.backward(pos, lt, torch.ones(1, dtype=torch.float64, device=ctx.device), d_lambda=dl,
                     d_sigma=dsig, d_sqrt_eps=dse, d_charge=dq)
        torch.cuda.synchronize()
        r.update(d_sigma=dsig.cpu().numpy(), d_sqrt_eps=dse.cpu().numpy(), d_charge=dq.cpu().numpy(),
                 d_lambda=dl.item())
        if precision == 1:
            idx = torch.tensor(w.info["cv_atoms"], device=ctx.device)
            cv = ctx.dihedrals(pos, idx)
            torch.cuda.synchronize()
            ref_cv = OD.cvs(s.positions, w.info["cv_atoms"], s.box)
            assert np.allclose(cv["xi"].cpu().numpy(), ref_cv["xi"], rtol=0, atol=1e-12)
            assert _rel(cv["dxi"].cpu().numpy(), ref_cv["dxi"]) < 1e-11
        res[precision] = r
        ctx.close()
    # sampled atoms (1,200 random solvent atoms of both slabs and every solute atom) against the
    # per-atom oracle sums, which are O(N) each
    rng = np.random.Generator(np.random.PCG64(55))
    solu = np.nonzero(s.is_solute)[0]
    sel = np.concatenate([solu, rng.choice(np.nonzero(s.is_solute == 0)[0], 1200, replace=False)]).astype(np.int32)
    P = O.Params.of(w, O.BEUTLER)
    at = O.atoms_terms(sel, s, w.ff, P, lam)
    # dU/dlambda of the box is exactly the sum over the solute atoms
    dudl_ref = at["dudl"][: len(solu)].sum()
    for precision in (1, 0):
        r = res[precision]
        eF = force_error(r["forces"][sel], at["forces"])
        ed = abs(r["dudl"][0] - dudl_ref) / abs(dudl_ref)
        print("config5 precision %d sampled force error %.3e dudl error %.3e" % (precision, eF, ed), flush=True)
        assert eF <= TOL[precision]["force"]
        assert ed <= TOL[precision]["dudl"]
        assert r["d_lambda"] == pytest.approx(r["dudl"][0], rel=1e-12)
    # FP32 against FP64 on the whole slab
    r64, r32 = res[1], res[0]
    assert force_error(r32["forces"], r64["forces"]) <= TOL[0]["force"]
    assert int(r32["n_pairs"][0]) == pytest.approx(int(r64["n_pairs"][0]), abs=64)
    for j in range(10):
        assert abs(r32["terms"][0, j] - r64["terms"][0, j]) <= 1e-6 * max(abs(r64["terms"][0, 8]), 1.0)
    for key in ("d_sigma", "d_sqrt_eps", "d_charge"):
        assert _rel(r32[key], r64[key]) < 3e-5, key
