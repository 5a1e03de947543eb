"""GPU backward pass, dihedral CVs and the lambda/OPES update against the oracles."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import dihedral as OD
from oracle import opes as OO
from paper_2608_12691_amd import systems as S

from conftest import workload
from parity import oracle_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ctx(w, precision, schedule=O.BEUTLER):
    from paper_2608_12691_amd import alchnb
    return alchnb.from_workload(w, precision=precision, schedule=schedule)


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("precision,tol", [(1, 1e-9), (0, 2e-5)], ids=["fp64", "fp32"])
@pytest.mark.parametrize("schedule,lam", [(O.BEUTLER, 0.3), (O.BEUTLER, 0.7), (O.LBF, 0.45), (O.LBF, 0.9)])
def test_backward_against_oracle(precision, tol, schedule, lam):
    from paper_2608_12691_amd import autograd as AG
    w = workload(1)
    s = w.systems[0]
    ctx = _ctx(w, precision, schedule)
    dev = ctx.device
    pos = ctx.positions(w.systems).requires_grad_(True)
    lamt = ctx.lambdas([lam]).requires_grad_(True)
    sig = torch.tensor(w.ff.sigma, dtype=torch.float64, device=dev, requires_grad=True)
    eps = torch.tensor(w.ff.epsilon, dtype=torch.float64, device=dev, requires_grad=True)
    chg = torch.tensor(w.ff.charge, dtype=torch.float64, device=dev, requires_grad=True)
    E, F, dudl, terms = AG.AlchNonbonded.apply(ctx, pos, lamt, sig, eps, chg)
    (2.5 * E.sum()).backward()
    ref = oracle_for(w, 0, lam, schedule, param_grads=True)
    # dL/dx = -2.5 F, dL/dlambda = 2.5 dU/dlambda
    assert _rel(pos.grad.cpu().numpy(), -2.5 * ref["forces"]) < max(tol, 1e-6 if precision == 0 else tol)
    assert lamt.grad.item() == pytest.approx(2.5 * ref["terms"][9], rel=max(tol, 1e-6))
    assert _rel(sig.grad.cpu().numpy(), 2.5 * ref["d_sigma"]) < tol
    assert _rel(chg.grad.cpu().numpy(), 2.5 * ref["d_charge"]) < tol
    ge = eps.grad.cpu().numpy()
    pos_eps = w.ff.epsilon > 0
    assert np.all(np.isnan(ge[~pos_eps]))
    assert _rel(ge[pos_eps], 2.5 * ref["d_eps"][pos_eps]) < tol


def test_backward_fd_fp64_params_and_lambda():
    """Central differences (h = 1e-4) of the GPU FP64 energy in lambda and a few type parameters."""
    w = workload(1)
    lam, h = 0.3, 1e-4
    ctx = _ctx(w, 1)
    pos = ctx.positions(w.systems)
    g = torch.ones(1, dtype=torch.float64, device=ctx.device)
    out = ctx.compute(pos, ctx.lambdas([lam]), flags=2)
    T = ctx.n_types
    dsig = torch.zeros(T, dtype=torch.float64, device=ctx.device)
    dq = torch.zeros(T, dtype=torch.float64, device=ctx.device)
    ctx.backward(pos, ctx.lambdas([lam]), g, d_sigma=dsig, d_charge=dq)
    torch.cuda.synchronize()

    def energy(ff, l):
        w2 = S.Workload(w.name, w.systems, ff, w.cutoff, w.skin, w.switch_width, w.dsf_alpha, w.sc_alpha,
                        w.lambdas, w.seed)
        c = _ctx(w2, 1)
        o = c.compute(c.positions(w.systems), c.lambdas([l]), flags=2)
        torch.cuda.synchronize()
        return float(o["terms"][0, 8])

    fd_l = (energy(w.ff, lam + h) - energy(w.ff, lam - h)) / (2 * h)
    assert float(out["dudl"][0]) == pytest.approx(fd_l, rel=1e-6)
    for t in (0, 2, 7):
        for arr, grad in (("sigma", dsig), ("charge", dq)):
            fp = S.ForceField(w.ff.sigma.copy(), w.ff.epsilon.copy(), w.ff.charge.copy(), w.ff.names)
            fm = S.ForceField(w.ff.sigma.copy(), w.ff.epsilon.copy(), w.ff.charge.copy(), w.ff.names)
            getattr(fp, arr)[t] += h
            getattr(fm, arr)[t] -= h
            fd = (energy(fp, lam) - energy(fm, lam)) / (2 * h)
            assert float(grad[t]) == pytest.approx(fd, rel=1e-5, abs=1e-7), (arr, t)


def test_backward_batched_weights_per_box():
    """Upstream weights g_k scale each box's contribution separately."""
    rng = np.random.Generator(np.random.PCG64(4))
    w1 = workload(1)
    boxes = [S.random_tiny_system(rng, n, 22.0, n_solute=5, n_types=w1.ff.n_types, min_dist=2.0) for n in (120, 200)]
    w = S.Workload("two", boxes, w1.ff, 9.0, 1.0, 1.0, 0.2, 0.5, np.array([0.4, 0.8]), 4)
    ctx = _ctx(w, 1)
    pos = ctx.positions(w.systems)
    lam = ctx.lambdas(w.lambdas)
    ctx.compute(pos, lam, flags=2)
    g = torch.tensor([0.7, -1.3], dtype=torch.float64, device=ctx.device)
    T = ctx.n_types
    dsig, dse, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(3))
    dpos = torch.zeros_like(pos)
    dl = torch.zeros(2, dtype=torch.float64, device=ctx.device)
    ctx.backward(pos, lam, g, d_pos=dpos, d_lambda=dl, d_sigma=dsig, d_sqrt_eps=dse, d_charge=dq)
    torch.cuda.synchronize()
    refs = [oracle_for(w, k, w.lambdas[k], O.BEUTLER, param_grads=True) for k in range(2)]
    gk = [0.7, -1.3]
    want = sum(gk[k] * refs[k]["d_sigma"] for k in range(2))
    assert _rel(dsig.cpu().numpy(), want) < 1e-9
    want = sum(gk[k] * refs[k]["d_sqrt_eps"] for k in range(2))
    assert _rel(dse.cpu().numpy(), want) < 1e-9
    assert dl.cpu().numpy() == pytest.approx([gk[k] * refs[k]["terms"][9] for k in range(2)], rel=1e-10)
    n0 = boxes[0].n_atoms
    assert _rel(dpos.cpu().numpy()[:n0], -0.7 * refs[0]["forces"]) < 1e-9
    assert _rel(dpos.cpu().numpy()[n0:], 1.3 * refs[1]["forces"]) < 1e-9


def _peptide_box():
    """22-atom peptide-like solute in a small water box, with the four CVs."""
    rng = np.random.Generator(np.random.PCG64(77))
    x, bonds, _ = S.peptide_solute(rng)
    w1 = workload(1)
    s = S.solvated_rigid_solute(rng, 400, np.full(3, 26.0), x, np.arange(2, 14).repeat(2)[:22] % w1.ff.n_types)
    idx = np.array(list(S.PEPTIDE_CV.values()), np.int32)
    return S.Workload("pep", [s], w1.ff, 9.0, 1.0, 1.0, 0.2, 0.5, np.array([0.5]), 77), idx


def test_dihedrals_and_dafed_against_oracle():
    w, idx = _peptide_box()
    s = w.systems[0]
    ctx = _ctx(w, 1)
    pos = ctx.positions(w.systems)
    rng = np.random.default_rng(3)
    minv = torch.tensor(rng.uniform(0.05, 1.0, s.n_atoms), dtype=torch.float64, device=ctx.device)
    sv = torch.tensor([2.8, -2.9, 0.3, 3.1], dtype=torch.float64, device=ctx.device)
    kap = torch.tensor([400.0, 300.0, 200.0, 100.0], dtype=torch.float64, device=ctx.device)
    forces = torch.zeros_like(pos)
    r = ctx.dihedrals(pos, torch.tensor(idx, device=ctx.device), mass_inv=minv, s=sv, kappa=kap, forces=forces)
    torch.cuda.synchronize()
    ref = OD.cvs(s.positions, idx, s.box, minv.cpu().numpy(), sv.cpu().numpy(), kap.cpu().numpy())
    assert np.allclose(r["xi"].cpu().numpy(), ref["xi"], rtol=0, atol=1e-12)
    assert _rel(r["dxi"].cpu().numpy(), ref["dxi"]) < 1e-11
    assert _rel(r["msum"].cpu().numpy(), ref["msum"]) < 1e-12
    assert float(r["u_dafed"][0]) == pytest.approx(ref["u_dafed"], rel=1e-12)
    assert _rel(forces.cpu().numpy(), ref["forces"]) < 1e-11
    assert ctx.get_flags() == 0
    # an out-of-range index is reported, not followed
    bad = torch.tensor([[0, 1, 2, s.n_atoms + 5]], dtype=torch.int32, device=ctx.device)
    ctx.dihedrals(pos, bad)
    assert ctx.get_flags() & 64


def test_dihedrals_overlapping_many_cvs_against_oracle():
    """70 CVs over sliding windows of 8 solute atoms (each atom in up to 28
    entries, 70 > one block's 64-CV chunk): the coupling forces of atoms
    shared between CVs and chunks against the oracle."""
    w, _ = _peptide_box()
    s = w.systems[0]
    ctx = _ctx(w, 1)
    pos = ctx.positions(w.systems)
    sol = np.nonzero(s.is_solute)[0][:8]
    idx = np.array([[sol[(k + j) % 8] for j in range(4)] for k in range(70)], np.int32)
    rng = np.random.default_rng(11)
    sv = torch.tensor(rng.uniform(-np.pi, np.pi, 70), dtype=torch.float64, device=ctx.device)
    kap = torch.tensor(rng.uniform(50.0, 400.0, 70), dtype=torch.float64, device=ctx.device)
    forces = torch.zeros_like(pos)
    r = ctx.dihedrals(pos, torch.tensor(idx, device=ctx.device), s=sv, kappa=kap, forces=forces)
    torch.cuda.synchronize()
    ref = OD.cvs(s.positions, idx, s.box, None, sv.cpu().numpy(), kap.cpu().numpy())
    assert np.allclose(r["xi"].cpu().numpy(), ref["xi"], rtol=0, atol=1e-12)
    assert float(r["u_dafed"][0]) == pytest.approx(ref["u_dafed"], rel=1e-12)
    assert _rel(forces.cpu().numpy(), ref["forces"]) < 1e-11
    assert ctx.get_flags() == 0


def test_dihedral_cv_autograd_and_dafed():
    from paper_2608_12691_amd import autograd as AG
    w, idx = _peptide_box()
    s = w.systems[0]
    ctx = _ctx(w, 1)
    pos = ctx.positions(w.systems).requires_grad_(True)
    it = torch.tensor(idx, device=ctx.device)
    xi = AG.DihedralCV.apply(ctx, pos, it)
    sv = torch.tensor([0.1, 0.2, -3.0, 2.0], dtype=torch.float64, device=ctx.device)
    kap = torch.full((4,), 250.0, dtype=torch.float64, device=ctx.device)
    U = AG.dafed_energy(xi, sv, kap)
    U.backward()
    ref = OD.cvs(s.positions, idx, s.box, None, sv.cpu().numpy(), kap.cpu().numpy())
    assert float(U) == pytest.approx(ref["u_dafed"], rel=1e-12)
    assert _rel(pos.grad.cpu().numpy(), -ref["forces"]) < 1e-11


def test_opes_update_against_oracle():
    w = workload(1)
    ctx = _ctx(w, 1)
    kT = OO.KB_KCAL * 298.0
    st = ctx.opes_state(capacity=64, kT=kT, sigma=0.10, barrier_std=30.0, barrier_expl=5.0, theta0=0.15)
    ref = OO.DualOpes(kT, 0.10, 30.0, 5.0)
    lam_out = torch.zeros(1, dtype=torch.float64, device=ctx.device)
    dudl = torch.zeros(1, dtype=torch.float64, device=ctx.device)
    rng = np.random.default_rng(12)
    theta = 0.15
    for step in range(40):
        theta = theta + rng.normal(0, 0.12)          # a wandering theta, written by the caller
        st[0] = theta
        dd = float(rng.normal(0, 20.0))
        dudl.fill_(dd)
        dep = step % 3 == 0
        ctx.opes_update(st, dudl, lam_out, deposit=dep)
        torch.cuda.synchronize()
        r = ref.update(theta, dd, deposit=dep)
        h = st[:16].cpu().numpy()
        assert h[0] == pytest.approx(r["theta"], abs=1e-13)
        assert lam_out.item() == pytest.approx(r["lam"], abs=1e-13)
        assert h[2] == r["dlam_dtheta"]
        assert h[3] == pytest.approx(r["u_opes"], rel=1e-10, abs=1e-10)
        assert h[4] == pytest.approx(r["du_opes"], rel=1e-9, abs=1e-9)
        assert h[5] == pytest.approx(r["f_theta"], rel=1e-9, abs=1e-9)
        theta = r["theta"]
    assert int(st[10].item()) == len(ref.centers)
    gth, gu, gdu = ref.grid()
    assert np.allclose(st[16:16 + 101].cpu().numpy(), gu, rtol=1e-10, atol=1e-10)
    assert np.allclose(st[16 + 101:16 + 202].cpu().numpy(), gdu, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_backward_param_grads_repeat_bitwise(precision):
    """The per-type gradients are fixed-point slot sums added in a fixed order: repeats are identical."""
    w = workload(2)
    ctx = _ctx(w, precision)
    pos = ctx.positions(w.systems)
    lam = ctx.lambdas([0.55])
    g = torch.ones(1, dtype=torch.float64, device=ctx.device)
    T = ctx.n_types
    outs = []
    for rep in range(3):
        print("backward repeat %d precision %d" % (rep, precision), flush=True)
        ctx.compute(pos, lam, flags=2 if rep == 0 else 0)
        dsig, dse, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(3))
        ctx.backward(pos, lam, g, d_sigma=dsig, d_sqrt_eps=dse, d_charge=dq)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (dsig, dse, dq)])
    assert ctx.get_flags() == 0
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    assert np.any(outs[0][0] != 0.0) and np.any(outs[0][2] != 0.0)


@pytest.mark.parametrize("precision,tol", [(1, 1e-9), (0, 2e-5)], ids=["fp64", "fp32"])
def test_backward_many_types_reads_pair_table_from_hbm(precision, tol):
    """40 atom types: the parameter pass reads the type-pair table from HBM instead of LDS."""
    rng = np.random.Generator(np.random.PCG64(40))
    T = 40
    ff = S.ForceField(sigma=rng.uniform(2.5, 3.8, T), epsilon=rng.uniform(0.02, 0.25, T),
                      charge=rng.uniform(-0.6, 0.6, T), names=["t%d" % i for i in range(T)])
    box = S.random_tiny_system(rng, 700, 22.0, n_solute=12, n_types=T, min_dist=1.9)
    w = S.Workload("types40", [box], ff, 9.0, 1.0, 1.0, 0.2, 0.5, np.array([0.6]), 40)
    ctx = _ctx(w, precision)
    pos = ctx.positions(w.systems)
    lam = ctx.lambdas([0.6])
    print("many types precision %d" % precision, flush=True)
    ctx.compute(pos, lam, flags=2)
    g = torch.ones(1, dtype=torch.float64, device=ctx.device)
    dsig, dse, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(3))
    ctx.backward(pos, lam, g, d_sigma=dsig, d_sqrt_eps=dse, d_charge=dq)
    torch.cuda.synchronize()
    assert ctx.get_flags() == 0
    ref = oracle_for(w, 0, 0.6, O.BEUTLER, param_grads=True)
    assert _rel(dsig.cpu().numpy(), ref["d_sigma"]) < tol
    assert _rel(dse.cpu().numpy(), ref["d_sqrt_eps"]) < tol
    assert _rel(dq.cpu().numpy(), ref["d_charge"]) < tol


def test_dihedrals_reuse_outputs():
    """The binding's output reuse gives the same CVs as fresh outputs."""
    w, idx = _peptide_box()
    ctx = _ctx(w, 0)
    pos = ctx.positions(w.systems)
    it = torch.tensor(idx, device=ctx.device)
    minv = torch.ones(ctx.N, dtype=torch.float64, device=ctx.device)
    sv = torch.tensor([0.1, 0.2, -3.0, 2.0], dtype=torch.float64, device=ctx.device)
    kap = torch.full((4,), 250.0, dtype=torch.float64, device=ctx.device)
    a = ctx.dihedrals(pos, it, mass_inv=minv, s=sv, kappa=kap)
    b = ctx.dihedrals(pos + 0.01, it, mass_inv=minv, s=sv, kappa=kap)
    c = ctx.dihedrals(pos, it, mass_inv=minv, s=sv, kappa=kap, out=b)
    torch.cuda.synchronize()
    assert c["xi"] is b["xi"]
    for k in ("xi", "dxi", "msum", "u_dafed"):
        assert torch.equal(a[k], c[k]), k
