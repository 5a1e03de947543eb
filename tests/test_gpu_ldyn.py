"""GPU parity of lambda dynamics (theta BAOAB, dual OPES with compression,
binned dU/dlambda and TI) and of the d-AFED auxiliary variables against
the FP64 oracle (oracle/ldyn.py), through the C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import dihedral as D
from oracle import ldyn as L
from paper_2608_12691_amd import systems as S

from conftest import workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KT = L.KB_KCAL * 298.0
KT_S = L.KB_KCAL * 1000.0


def _params(n_cv, stride, compress, cap=96, bins=10):
    # the paper's theta mass, 1 Da nm^2 (a light theta makes the biased dynamics chaotic enough that
    # rounding differences grow past any tolerance within a few hundred steps)
    return dict(capacity=cap, stride=stride, ti_bins=bins, n_cv=n_cv, kT=KT, mass=L.DA_NM2_TO_KCAL_FS2, friction=0.025, dt=1.0,
                sigma=0.10, barrier_std=30.0, barrier_expl=5.0, compress=compress, kT_s=KT_S, friction_s=0.025)


def _oracle(p, theta0):
    return L.LambdaDynamics(p["kT"], p["mass"], p["friction"], p["dt"], p["sigma"], p["barrier_std"],
                            p["barrier_expl"], p["compress"], p["stride"], p["ti_bins"], theta0)


def _close(a, b, tol, what):
    a, b = np.asarray(a, float), np.asarray(b, float)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    scale = max(1.0, float(np.abs(b).max()) if b.size else 1.0)
    err = float(np.abs(a - b).max()) if b.size else 0.0
    assert err <= tol * scale, "%s: max error %.3e (scale %.3e)" % (what, err, scale)


def _compare_state(ctx, state, lay, ref_reps, ref_aux, tol):
    reps, aux = ctx.ld_view(state, lay)
    for r, (g, o) in enumerate(zip(reps, ref_reps)):
        assert g["n"] == o.n
        _close(g["theta"], o.theta, tol, "theta %d" % r)
        _close(g["p"], o.p, tol, "p %d" % r)
        for name, ks in (("std", o.opes.std), ("expl", o.opes.expl)):
            c, w, s = g[name]
            assert len(c) == len(ks.c), (r, name, len(c), len(ks.c))
            _close(c, ks.c, tol, "%s centres %d" % (name, r))
            _close(s, ks.s, tol, "%s widths %d" % (name, r))
            _close(np.log(w), np.log(ks.w), tol, "%s log weights %d" % (name, r))
        _close(g["ti_cnt"], o.ti_cnt, 0.0, "TI counts %d" % r)
        _close(g["ti_sum"], o.ti_sum, tol, "TI sums %d" % r)
    if ref_aux is not None:
        _close(aux["s"], ref_aux.s, tol, "s")
        _close(aux["p"], ref_aux.p, tol, "p_s")


@pytest.mark.parametrize("compress", [1.0, 0.0], ids=["compressed", "uncompressed"])
def test_ld_step_against_oracle_synthetic_drive(compress):
    """Three replicas and two auxiliary variables for 400 steps, a kernel
    every 5 steps (merging often when compressed), dU/dlambda a smooth
    function of each replica's own lambda, xi(t) given; every step's lambda,
    then theta, momenta, kernels, TI bins and s_k at the end."""
    from paper_2608_12691_amd import alchnb
    w = workload(1)
    # lambda dynamics runs one theta per box: a context of three copies of the box
    w3 = S.Workload("x3", [w.systems[0]] * 3, w.ff, w.cutoff, w.skin, w.switch_width, w.dsf_alpha, w.sc_alpha,
                    np.array([0.5] * 3), w.seed)
    ctx = alchnb.from_workload(w3, precision=alchnb.FP64, schedule=alchnb.LBF_DSF)
    K, n_cv, steps = 3, 2, 400
    p = _params(n_cv, 5, compress)
    rng = np.random.Generator(np.random.PCG64(2608))
    noise = rng.standard_normal((steps, K + n_cv))
    xi = np.array([[0.6 * math.sin(0.013 * t + k) + 2.9 * (k == 1) for k in range(n_cv)] for t in range(steps)])
    theta0 = np.array([0.15, 0.8, 1.7])
    coef = np.array([[3.0, -8.0, 1.5], [-2.0, 5.0, -0.7], [6.0, -1.0, 2.5]])
    dev = torch.device("cuda:0")
    state, lay = ctx.ld_init(p, theta0, s0=[0.2, -2.8], mass_s=[900.0, 1500.0], kappa=[239.0, 120.0])
    nz = torch.as_tensor(noise, device=dev)
    xs = torch.as_tensor(xi, device=dev)
    cf = torch.as_tensor(coef, device=dev)
    lam = torch.as_tensor([min(t, 2 - t) for t in theta0], dtype=torch.float64, device=dev)
    hist = torch.zeros((steps, K), dtype=torch.float64, device=dev)
    for t in range(steps):
        dudl = cf[:, 0] + cf[:, 1] * lam + cf[:, 2] * torch.sin(7.0 * lam)
        ctx.ld_step(state, dudl.contiguous(), nz, lam, xi=xs[t])
        hist[t] = lam
    torch.cuda.synchronize()
    assert ctx.get_flags() == 0
    refs = [_oracle(p, th) for th in theta0]
    aux = L.AuxiliaryDynamics(KT_S, [900.0, 1500.0], [239.0, 120.0], 0.025, 1.0, [0.2, -2.8])
    lam_ref = np.zeros((steps, K))
    for t in range(steps):
        for r in range(K):
            l = refs[r].lam()
            lam_ref[t, r] = refs[r].step(coef[r, 0] + coef[r, 1] * l + coef[r, 2] * math.sin(7.0 * l), noise[t, r])
        aux.step(xi[t], noise[t, K:])
    _close(hist.cpu().numpy(), lam_ref, 1e-9, "lambda history")
    _compare_state(ctx, state, lay, refs, aux, 1e-9)
    if compress > 0:
        assert all(len(o.opes.std.c) < 80 for o in refs)   # merging happened
    dG = ctx.ld_free_energy(state).cpu().numpy()
    for r in range(K):
        want = refs[r].free_energy()
        assert (math.isnan(want) and math.isnan(dG[r])) or dG[r] == pytest.approx(want, rel=1e-10)


def test_ld_end_to_end_with_the_nonbonded_path_and_dafed():
    """lambda-OPES-d-AFED on the 633-atom box: each step evaluates the FP64
    nonbonded path at the current lambda (LBF schedule), the two dihedral
    CVs at the current positions (coupled to s_k), and advances theta and
    s_k; the oracle does the same with its own evaluations."""
    from paper_2608_12691_amd import alchnb
    w = workload(1)
    s = w.systems[0]
    ctx = alchnb.from_workload(w, precision=alchnb.FP64, schedule=alchnb.LBF_DSF)
    steps, n_cv = 150, 2
    p = _params(n_cv, 10, 1.0, cap=32, bins=5)
    sol = np.nonzero(s.is_solute)[0]
    idx = np.array([sol[0:4], sol[4:8]], dtype=np.int32)
    walk = S.perturbation_walk(s, steps, 0.01, seed=2718)
    rng = np.random.Generator(np.random.PCG64(31415))
    noise = rng.standard_normal((steps, 1 + n_cv))
    kappa = [239.0, 239.0]
    mass_s = [50.0 * L.DA_NM2_TO_KCAL_FS2 * 1e-3, 50.0 * L.DA_NM2_TO_KCAL_FS2 * 1e-3]
    dev = torch.device("cuda:0")
    state, lay = ctx.ld_init(p, [0.3], s0=[0.0, 1.0], mass_s=mass_s, kappa=kappa)
    s_view = state[lay["cv_s"]:lay["cv_s"] + n_cv]
    nz = torch.as_tensor(noise, device=dev)
    lam = ctx.lambdas([0.3])
    out = ctx.new_outputs()
    di = torch.as_tensor(idx, device=dev)
    kap = torch.as_tensor(kappa, dtype=torch.float64, device=dev)
    cv = None
    hist = torch.zeros(steps, dtype=torch.float64, device=dev)
    for t in range(steps):
        x = ctx.positions(walk[t])
        ctx.compute(x, lam, flags=alchnb.AUTO_REBUILD, out=out)
        cv = ctx.dihedrals(x, di, s=s_view, kappa=kap, forces=out["forces"], out=cv)
        ctx.ld_step(state, out["dudl"], nz, lam, xi=cv["xi"])
        hist[t] = lam[0]
    torch.cuda.synchronize()
    assert ctx.get_flags() == 0
    ref = _oracle(p, 0.3)
    aux = L.AuxiliaryDynamics(KT_S, mass_s, kappa, 0.025, 1.0, [0.0, 1.0])
    P = O.Params.of(w, O.LBF)
    lam_ref = []
    for t in range(steps):
        r = O.evaluate(walk[t], s.types, s.is_solute, s.exclusions, s.box, w.ff.sigma, w.ff.epsilon, w.ff.charge, P,
                       ref.lam(), forces=False)
        xi = D.cvs(walk[t], idx, s.box)["xi"]
        lam_ref.append(ref.step(r["terms"][9], noise[t, 0]))
        aux.step(xi, noise[t, 1:])
    _close(hist.cpu().numpy(), np.array(lam_ref), 1e-9, "lambda history")
    _compare_state(ctx, state, lay, [ref], aux, 1e-9)
    dG = float(ctx.ld_free_energy(state)[0])
    want = ref.free_energy()
    assert (math.isnan(want) and math.isnan(dG)) or dG == pytest.approx(want, rel=1e-9)


@pytest.mark.parametrize("n_cv", [3, 70])
def test_ld_step_dafed_matches_the_two_call_step_bitwise(n_cv):
    """The fused step (CVs, coupling forces and the theta / s_k update in one
    launch) against alch_nb_dihedrals + alch_nb_ld_step on a 633-atom walk
    (FP32 evaluation, LBF schedule): forces, CVs, coupling energy, lambda
    and the whole state identical bit for bit every step; overlapping
    windows share atoms between CVs (and, with 70, between 64-CV chunks)."""
    from paper_2608_12691_amd import alchnb
    w = workload(1)
    s = w.systems[0]
    ctx = alchnb.from_workload(w, precision=alchnb.FP32_FIXED, schedule=alchnb.LBF_DSF)
    steps = 40
    p = _params(n_cv, 7, 1.0, cap=16, bins=5)
    sol = np.nonzero(s.is_solute)[0][:10]
    idx = np.array([[sol[(k + 2 * j) % 10] for j in range(4)] for k in range(n_cv)], dtype=np.int32)
    walk = S.perturbation_walk(s, steps, 0.01, seed=99)
    rng = np.random.Generator(np.random.PCG64(4242))
    s0 = rng.uniform(-np.pi, np.pi, n_cv)
    kappa = rng.uniform(100.0, 300.0, n_cv)
    mass_s = np.full(n_cv, 50.0 * L.DA_NM2_TO_KCAL_FS2 * 1e-3)
    dev = torch.device("cuda:0")
    nz = torch.as_tensor(rng.standard_normal((steps, 1 + n_cv)), device=dev)
    sa, lay = ctx.ld_init(p, [0.45], s0=s0, mass_s=mass_s, kappa=kappa)
    torch.cuda.synchronize()  # the binding keeps one init's inputs alive
    sb, _ = ctx.ld_init(p, [0.45], s0=s0, mass_s=mass_s, kappa=kappa)
    s_view = sa[lay["cv_s"]:lay["cv_s"] + n_cv]
    kap = torch.as_tensor(kappa, dtype=torch.float64, device=dev)
    di = torch.as_tensor(idx, device=dev)
    la, lb = ctx.lambdas([0.45]), ctx.lambdas([0.45])
    out = ctx.new_outputs()
    xb = torch.zeros(n_cv, dtype=torch.float64, device=dev)
    ub = torch.zeros(1, dtype=torch.float64, device=dev)
    cv = None
    for t in range(steps):
        x = ctx.positions(walk[t])
        ctx.compute(x, la, flags=alchnb.AUTO_REBUILD, out=out)
        fa, fb = out["forces"].clone(), out["forces"].clone()
        cv = ctx.dihedrals(x, di, s=s_view, kappa=kap, forces=fa, out=cv)
        ctx.ld_step(sa, out["dudl"], nz, la, xi=cv["xi"])
        ctx.ld_step_dafed(sb, out["dudl"], nz, lb, x, di, xi=xb, u_dafed=ub, forces=fb)
        torch.cuda.synchronize()
        assert torch.equal(fa, fb), t
        assert torch.equal(cv["xi"], xb) and torch.equal(cv["u_dafed"], ub), t
        assert torch.equal(la, lb) and torch.equal(sa, sb), t
    assert ctx.get_flags() == 0
    # an out-of-range index: flagged, no force, its CV value left as it was
    bad = di.clone()
    bad[0, 3] = ctx.N + 3
    xb.fill_(7.0)
    f0 = out["forces"].clone()
    fb = f0.clone()
    ctx.ld_step_dafed(sb, out["dudl"], nz, lb, ctx.positions(walk[0]), bad, xi=xb, u_dafed=ub, forces=fb)
    torch.cuda.synchronize()
    assert ctx.get_flags() & alchnb.FLAG_BAD_INDEX
    assert float(xb[0]) == 7.0 and bool(torch.isfinite(xb).all())
    moved = set(np.nonzero((fb != f0).any(dim=1).cpu().numpy())[0].tolist())
    assert moved <= set(idx[1:].ravel().tolist())


def test_ld_step_dafed_three_boxes_matches_the_two_call_step_bitwise():
    """Three boxes (one empty) with their own theta, and CVs in the first and
    the third box (global indices, each CV in its own box's minimum image):
    the fused step against alch_nb_dihedrals + alch_nb_ld_step, bit for bit
    over 25 steps of a small random walk."""
    from paper_2608_12691_amd import alchnb
    rng = np.random.Generator(np.random.PCG64(606))
    w1 = workload(1)
    boxes = [S.random_tiny_system(rng, 200, 20.0, n_solute=8, n_types=w1.ff.n_types, min_dist=2.0),
             S.System(positions=np.zeros((0, 3)), types=np.zeros(0, np.int32), is_solute=np.zeros(0, np.uint8),
                      exclusions=np.zeros((0, 2), np.int32), box=np.full(3, 20.0), molecule=np.zeros(0, np.int32)),
             S.random_tiny_system(rng, 300, 22.0, n_solute=8, n_types=w1.ff.n_types, min_dist=2.0)]
    w = S.Workload(name="three", systems=boxes, ff=w1.ff, cutoff=9.0, skin=1.0, switch_width=1.0, dsf_alpha=0.2,
                   sc_alpha=0.5, lambdas=np.array([0.2, 0.5, 0.8]), seed=606)
    off = np.concatenate([[0], np.cumsum([b.n_atoms for b in boxes])])
    s0 = np.nonzero(boxes[0].is_solute)[0] + off[0]
    s2 = np.nonzero(boxes[2].is_solute)[0] + off[2]
    idx = np.array([s0[0:4], s0[2:6], s2[0:4], s2[3:7], s2[[1, 3, 5, 7]]], dtype=np.int32)
    n_cv, steps = len(idx), 25
    ctx = alchnb.from_workload(w, precision=alchnb.FP64, schedule=alchnb.LBF_DSF)
    p = _params(n_cv, 6, 1.0, cap=16, bins=5)
    kappa = rng.uniform(100.0, 300.0, n_cv)
    mass_s = np.full(n_cv, 50.0 * L.DA_NM2_TO_KCAL_FS2 * 1e-3)
    th0 = [0.2, 0.5, 0.8]
    dev = torch.device("cuda:0")
    nz = torch.as_tensor(rng.standard_normal((steps, 3 + n_cv)), device=dev)
    sa, lay = ctx.ld_init(p, th0, s0=np.zeros(n_cv), mass_s=mass_s, kappa=kappa)
    torch.cuda.synchronize()  # the binding keeps one init's inputs alive
    sb, _ = ctx.ld_init(p, th0, s0=np.zeros(n_cv), mass_s=mass_s, kappa=kappa)
    s_view = sa[lay["cv_s"]:lay["cv_s"] + n_cv]
    kap = torch.as_tensor(kappa, dtype=torch.float64, device=dev)
    di = torch.as_tensor(idx, device=dev)
    la, lb = ctx.lambdas(th0), ctx.lambdas(th0)
    out = ctx.new_outputs()
    xb = torch.zeros(n_cv, dtype=torch.float64, device=dev)
    ub = torch.zeros(1, dtype=torch.float64, device=dev)
    x0 = np.concatenate([b.positions for b in boxes])
    walk = x0[None] + np.cumsum(np.concatenate([np.zeros((1,) + x0.shape), rng.normal(0.0, 0.01, (steps - 1,) + x0.shape)]), axis=0)
    cv = None
    for t in range(steps):
        x = ctx.positions(walk[t])
        ctx.compute(x, la, flags=alchnb.AUTO_REBUILD, out=out)
        fa, fb = out["forces"].clone(), out["forces"].clone()
        cv = ctx.dihedrals(x, di, s=s_view, kappa=kap, forces=fa, out=cv)
        ctx.ld_step(sa, out["dudl"], nz, la, xi=cv["xi"])
        ctx.ld_step_dafed(sb, out["dudl"], nz, lb, x, di, xi=xb, u_dafed=ub, forces=fb)
        torch.cuda.synchronize()
        assert torch.equal(fa, fb) and torch.equal(cv["xi"], xb) and torch.equal(cv["u_dafed"], ub), t
        assert torch.equal(la, lb) and torch.equal(sa, sb), t
    assert ctx.get_flags() == 0
    assert float(ub[0]) > 0.0


def test_ld_step_dafed_in_one_graph_matches_eager():
    """A whole lambda-OPES-d-AFED step (evaluation at the current lambda,
    CVs with their coupling forces and the theta / s_k update) captured once
    and replayed on a 633-atom walk, the positions copied into the captured
    buffer before each replay: every replay's lambda, and the final forces,
    CVs' coupling energy and state, equal the eager steps bit for bit."""
    from paper_2608_12691_amd import alchnb
    w = workload(1)
    s = w.systems[0]
    steps, n_cv = 30, 3
    p = _params(n_cv, 5, 1.0, cap=16, bins=5)
    sol = np.nonzero(s.is_solute)[0][:8]
    idx = np.array([sol[k:k + 4] for k in range(n_cv)], dtype=np.int32)
    walk = S.perturbation_walk(s, steps, 0.01, seed=1234)
    rng = np.random.Generator(np.random.PCG64(808))
    noise = rng.standard_normal((steps, 1 + n_cv))
    mass_s = np.full(n_cv, 50.0 * L.DA_NM2_TO_KCAL_FS2 * 1e-3)
    kappa = np.full(n_cv, 239.0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    runs = {}
    for mode in ("eager", "graph"):
        with torch.cuda.stream(stream):
            ctx = alchnb.from_workload(w, precision=alchnb.FP32_FIXED, schedule=alchnb.LBF_DSF)
            state, lay = ctx.ld_init(p, [0.35], s0=np.zeros(n_cv), mass_s=mass_s, kappa=kappa)
            nz = torch.as_tensor(noise, device=dev)
            di = torch.as_tensor(idx, device=dev)
            lam = ctx.lambdas([0.35])
            x = ctx.positions(walk[0])
            out = ctx.new_outputs()
            u = torch.zeros(1, dtype=torch.float64, device=dev)
            ctx.compute_checked(x, lam, flags=alchnb.FORCE_REBUILD, out=out)
            if mode == "graph":
                ctx.capture_begin()
                ctx.compute(x, lam, flags=alchnb.AUTO_REBUILD, out=out)
                ctx.ld_step_dafed(state, out["dudl"], nz, lam, x, di, u_dafed=u, forces=out["forces"])
                ctx.capture_end()
        hist = []
        for t in range(steps):
            with torch.cuda.stream(stream):
                x.copy_(torch.as_tensor(walk[t], device=dev))
                if mode == "graph":
                    ctx.launch_step()
                else:
                    ctx.compute(x, lam, flags=alchnb.AUTO_REBUILD, out=out)
                    ctx.ld_step_dafed(state, out["dudl"], nz, lam, x, di, u_dafed=u, forces=out["forces"])
            stream.synchronize()
            hist.append(float(lam[0]))
        print("%s: lambda %.6f" % (mode, hist[-1]), flush=True)
        assert ctx.get_flags() == 0
        runs[mode] = (hist, out["forces"].cpu(), u.cpu(), state.cpu())
    (ha, fa, ua, sa), (hb, fb, ub, sb) = runs["eager"], runs["graph"]
    assert ha == hb
    assert torch.equal(fa, fb) and torch.equal(ua, ub) and torch.equal(sa, sb)


def test_ld_capacity_flag_drops_kernels_without_fault():
    """A store of two kernels per variant with no merging: later depositions
    are dropped and raise the capacity flag; the dynamics continue."""
    from paper_2608_12691_amd import alchnb
    w = workload(1)
    ctx = alchnb.from_workload(w, precision=alchnb.FP64)
    p = _params(0, 1, 0.0, cap=2, bins=4)
    state, lay = ctx.ld_init(p, [0.4])
    nz = torch.zeros((8, 1), dtype=torch.float64, device="cuda:0")
    lam = ctx.lambdas([0.4])
    dudl = torch.ones(1, dtype=torch.float64, device="cuda:0")
    for _ in range(6):
        ctx.ld_step(state, dudl, nz, lam)
    assert ctx.get_flags() & alchnb.FLAG_LD_CAPACITY
    reps, _ = ctx.ld_view(state, lay)
    assert reps[0]["n"] == 6 and len(reps[0]["std"][0]) == 2
