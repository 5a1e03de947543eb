"""GPU parity of Ewald electrostatics by smooth PME (ALCH_NB_ELEC_PME)
against the FP64 oracle (oracle/pme.py with the pair oracle's Ewald real
space), through the C ABI: single boxes at several lambdas with both
schedules and precisions, a ragged batch with an empty box, the 8,973-atom
box, bit-identical repeats, graph replay and the gradients."""
import numpy as np
import pytest

import oracle as O
from oracle import pme as P
from paper_2608_12691_amd import systems as S

from conftest import workload
from parity import TOL, to_numpy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALPHA, ORDER, SPACING = 0.3, 5, 1.0


def _ctx(w, precision, schedule, order=ORDER, spacing=SPACING, **kw):
    from paper_2608_12691_amd import alchnb
    return alchnb.Context(w.ff, w.systems, w.cutoff, w.skin, w.switch_width, ALPHA, w.sc_alpha, schedule=schedule,
                          precision=precision, electrostatics=alchnb.ELEC_PME, pme_order=order, pme_spacing=spacing,
                          **kw)


def _oracle(w, k, lam, schedule, grid, order=ORDER):
    s = w.systems[k]
    prm = O.Params(w.cutoff, w.switch_width, ALPHA, w.sc_alpha, schedule, ewald=True)
    return P.evaluate_system(s, w.ff, prm, lam, grid, order)


def _check(res, ref, a, b, precision, label):
    """The parity bars of the short-range path (forces RMS, dU/dlambda and
    energies per term) with each term's scale taken over all its parts:
    the sum of |u_ij| of its pairs plus the magnitudes of its reciprocal and
    correction parts."""
    tol = TOL[precision]
    t, rt, ab = np.asarray(res["terms"]), ref["terms"], ref["abs_terms"]
    t = t[0] if t.ndim == 2 else t
    for j in (0, 1, 2, 3, 4, 5, 8):
        err = abs(t[j] - rt[j]) / max(ab[j], 1e-300)
        assert err <= tol["energy"], "%s term %d: %.6e vs %.6e (rel %.2e)" % (label, j, t[j], rt[j], err)
    dscale = abs(rt[9]) if abs(rt[9]) >= 1e-2 * ab[9] else ab[9]
    derr = abs(t[9] - rt[9]) / max(dscale, 1e-300)
    assert derr <= tol["dudl"], "%s dU/dlambda %.12e vs %.12e (rel %.2e)" % (label, t[9], rt[9], derr)
    f, rf = res["forces"][a:b], ref["forces"]
    ferr = np.sqrt(np.sum((f - rf) ** 2) / max(np.sum(rf ** 2), 1e-300))
    assert ferr <= tol["force"], "%s force RMS rel %.2e" % (label, ferr)
    print("%s: energy %.1e dudl %.1e force %.1e" % (label, max(abs(t[j] - rt[j]) / max(ab[j], 1e-300)
                                                              for j in (0, 1, 3, 8)), derr, ferr), flush=True)


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
@pytest.mark.parametrize("schedule", [O.BEUTLER, O.LBF], ids=["beutler", "lbf"])
def test_pme_config1_against_oracle(precision, schedule):
    """The 660-atom box (18.6 A, cutoff 9 A): 20^3 grid, order 5, a = 0.3 A^-1."""
    w = workload(1)
    ctx = _ctx(w, precision, schedule)
    grid = ctx.pme_grid(0)
    assert grid == (20, 20, 20)
    pos = ctx.positions(w.systems)
    for lam in (0.3, 0.62, 0.85, 1.0):
        print("pme cfg1 precision=%d schedule=%d lambda=%.2f" % (precision, schedule, lam), flush=True)
        res = to_numpy(ctx.compute_checked(pos, ctx.lambdas([lam]), flags=1))
        torch.cuda.synchronize()
        assert res["flags"] == 0
        ref = _oracle(w, 0, lam, schedule, grid)
        _check(res, ref, 0, w.systems[0].n_atoms, precision, "cfg1 lam=%g" % lam)


def _ortho_box(rng, n, box, n_solute, n_types, min_dist=2.0):
    """Random atoms in an orthorhombic box, at least min_dist apart (minimum image)."""
    box = np.asarray(box, float)
    pos = np.zeros((0, 3))
    while len(pos) < n:
        x = rng.uniform(0, 1, 3) * box
        d = pos - x
        d -= box * np.round(d / box)
        if len(pos) == 0 or np.min(np.sum(d * d, axis=1)) >= min_dist ** 2:
            pos = np.vstack([pos, x])
    sol = np.zeros(n, np.uint8)
    sol[:n_solute] = 1
    return S.System(positions=pos, types=rng.integers(0, n_types, n).astype(np.int32), is_solute=sol,
                    exclusions=np.zeros((0, 2), np.int32), box=box, molecule=np.arange(n, dtype=np.int32))


@pytest.mark.parametrize("order", [4, 6])
def test_pme_orders_and_anisotropic_grid(order):
    """Orders 4 and 6 in an orthorhombic 22 x 26 x 31 A box (grids of
    different sizes per axis, mixed radices), FP64."""
    rng = np.random.Generator(np.random.PCG64(314))
    w1 = workload(1)
    s = _ortho_box(rng, 900, (22.0, 26.0, 31.0), 9, w1.ff.n_types)
    w = S.Workload(name="ortho", systems=[s], ff=w1.ff, cutoff=9.0, skin=0.0, switch_width=1.0, dsf_alpha=ALPHA,
                   sc_alpha=0.5, lambdas=np.array([0.7]), seed=314)
    ctx = _ctx(w, 1, O.LBF, order=order, spacing=0.9)
    grid = ctx.pme_grid(0)
    assert grid[0] < grid[1] < grid[2]
    res = to_numpy(ctx.compute_checked(ctx.positions(w.systems), ctx.lambdas([0.7]), flags=1))
    ref = _oracle(w, 0, 0.7, O.LBF, grid, order)
    _check(res, ref, 0, s.n_atoms, 1, "ortho order %d" % order)


def test_pme_ragged_batch_with_empty_box():
    """Three boxes (one empty) of different sizes and grids at different lambdas."""
    rng = np.random.Generator(np.random.PCG64(99))
    w1 = workload(1)
    boxes = []
    for n, L in ((300, 22.0), (0, 22.0), (700, 27.0)):
        if n == 0:
            boxes.append(S.System(positions=np.zeros((0, 3)), types=np.zeros(0, np.int32),
                                  is_solute=np.zeros(0, np.uint8), exclusions=np.zeros((0, 2), np.int32),
                                  box=np.full(3, L), molecule=np.zeros(0, np.int32)))
        else:
            boxes.append(S.random_tiny_system(rng, n, L, n_solute=6, n_types=w1.ff.n_types, min_dist=2.0))
    lams = np.array([0.8, 0.45, 0.9])
    w = S.Workload(name="ragged", systems=boxes, ff=w1.ff, cutoff=9.0, skin=1.0, switch_width=1.0, dsf_alpha=ALPHA,
                   sc_alpha=0.5, lambdas=lams, seed=99)
    off = np.concatenate([[0], np.cumsum([s.n_atoms for s in boxes])])
    for precision in (1, 0):
        ctx = _ctx(w, precision, O.BEUTLER)
        res = to_numpy(ctx.compute_checked(ctx.positions(w.systems), ctx.lambdas(lams), flags=1))
        assert res["flags"] == 0
        for k, s in enumerate(boxes):
            rk = dict(terms=res["terms"][k], forces=res["forces"])
            if s.n_atoms == 0:
                assert np.all(res["terms"][k] == 0.0)
                continue
            ref = _oracle(w, k, lams[k], O.BEUTLER, ctx.pme_grid(k))
            _check(rk, ref, off[k], off[k + 1], precision, "ragged box %d p%d" % (k, precision))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_pme_water3000_box_against_oracle(precision):
    """The 8,973-atom box (44.85 A, cutoff 10 A, skin 1 A): 45^3 grid, full
    comparison after a short walk with a device-side rebuild."""
    w = workload(2)
    s = w.systems[0]
    ctx = _ctx(w, precision, O.BEUTLER)
    grid = ctx.pme_grid(0)
    assert grid == (45, 45, 45)
    # 30 steps of N(0, 0.03 A): atoms move up to 0.74 A (> skin/2), with no close contact
    walk = S.perturbation_walk(s, 30, 0.03, seed=5)
    out = ctx.new_outputs()
    lam = ctx.lambdas([0.8])
    for t in range(30):
        ctx.compute(ctx.positions(walk[t]), lam, flags=1, out=out)
    torch.cuda.synchronize()
    res = to_numpy(out)
    assert ctx.get_flags() == 0 and ctx.get_stats()["n_rebuilds"] >= 2
    ref = P.evaluate(walk[29], s.types, s.is_solute, s.exclusions, s.box, w.ff.sigma, w.ff.epsilon, w.ff.charge,
                     O.Params(w.cutoff, w.switch_width, ALPHA, w.sc_alpha, O.BEUTLER, ewald=True), 0.8, grid, ORDER)
    _check(res, ref, 0, s.n_atoms, precision, "water3000")


def test_pme_repeats_are_bit_identical_and_graph_replay_matches_eager():
    w = workload(2)
    s = w.systems[0]
    ctx = _ctx(w, 0, O.LBF)
    walk = S.perturbation_walk(s, 5, 0.05, seed=21)
    pos = ctx.positions(walk[0])
    lam = ctx.lambdas([0.6])
    outs = []
    for _ in range(3):
        outs.append(to_numpy(ctx.compute(pos, lam, flags=2)))
        torch.cuda.synchronize()
    for o in outs[1:]:
        for k in ("forces", "terms", "dudl"):
            assert np.array_equal(o[k], outs[0][k]), k
    out = ctx.new_outputs()
    ctx.compute(pos, lam, flags=1, out=out)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = _ctx(w, 0, O.LBF)
        gout = gctx.new_outputs()
        gpos = gctx.positions(walk[0])
        glam = gctx.lambdas([0.6])
        gctx.compute(gpos, glam, flags=1, out=gout)
        gctx.capture_step(gpos, glam, gout)
    for t in range(1, 5):
        x = torch.as_tensor(walk[t], device=pos.device)
        with torch.cuda.stream(stream):
            gpos.copy_(x)
            glam.fill_(0.15 * t)
            gctx.launch_step()
        stream.synchronize()
        pos.copy_(x)
        lam.fill_(0.15 * t)
        ctx.compute(pos, lam, flags=1, out=out)
        torch.cuda.synchronize()
        a, b = to_numpy(gout), to_numpy(out)
        for k in ("forces", "terms", "dudl", "n_pairs"):
            assert np.array_equal(a[k], b[k]), (t, k)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_pme_plane_transforms_match_line_tiles_bitwise(precision, monkeypatch):
    """The y and z transforms one y-z plane per block (the default where the
    planes fit in LDS) against the line tiles (ALCHNB_PME_FFT=lines): the
    8,973-atom box (45^3) and a ragged batch of two grids with an empty box
    give identical forces, terms and dU/dlambda."""
    rng = np.random.Generator(np.random.PCG64(4))
    w1 = workload(1)
    boxes = [S.random_tiny_system(rng, 300, 22.0, n_solute=6, n_types=w1.ff.n_types, min_dist=2.0),
             S.System(positions=np.zeros((0, 3)), types=np.zeros(0, np.int32), is_solute=np.zeros(0, np.uint8),
                      exclusions=np.zeros((0, 2), np.int32), box=np.full(3, 25.0), molecule=np.zeros(0, np.int32)),
             S.random_tiny_system(rng, 700, 27.0, n_solute=6, n_types=w1.ff.n_types, min_dist=2.0)]
    ragged = S.Workload(name="ragged", systems=boxes, ff=w1.ff, cutoff=9.0, skin=1.0, switch_width=1.0,
                        dsf_alpha=ALPHA, sc_alpha=0.5, lambdas=np.array([0.3, 0.5, 0.7]), seed=4)
    for w, schedule in ((workload(2), O.LBF), (ragged, O.BEUTLER)):
        res = []
        for mode in ("planes", "lines"):
            if mode == "lines":
                monkeypatch.setenv("ALCHNB_PME_FFT", "lines")
            else:
                monkeypatch.delenv("ALCHNB_PME_FFT", raising=False)
            ctx = _ctx(w, precision, schedule)
            r = to_numpy(ctx.compute_checked(ctx.positions(w.systems), ctx.lambdas(w.lambdas), flags=2))
            assert r["flags"] == 0
            res.append(r)
            print("%s %s: dU/dlambda %s" % (w.name, mode, r["dudl"]), flush=True)
        for k in ("forces", "terms", "dudl", "n_pairs"):
            assert np.array_equal(res[0][k], res[1][k]), (w.name, k)


def test_pme_backward_position_and_lambda_gradients():
    """dL/dx = sum_k g_k dU_k/dx = -g forces and dL/dlambda = g dU/dlambda
    come from the forward's state; the per-type gradients are refused."""
    from paper_2608_12691_amd import alchnb
    w = workload(1)
    ctx = _ctx(w, 1, O.BEUTLER)
    pos = ctx.positions(w.systems)
    lam = ctx.lambdas([0.7])
    res = to_numpy(ctx.compute(pos, lam, flags=1))
    g = torch.tensor([1.7], dtype=torch.float64, device=pos.device)
    d_pos = torch.zeros_like(pos)
    d_lam = torch.zeros_like(lam)
    ctx.backward(pos, lam, g, d_pos=d_pos, d_lambda=d_lam)
    torch.cuda.synchronize()
    assert np.allclose(d_pos.cpu().numpy(), -1.7 * res["forces"], rtol=1e-12, atol=1e-12)
    assert d_lam.cpu().numpy()[0] == pytest.approx(1.7 * res["dudl"][0], rel=1e-12)
    d_q = torch.zeros(w.ff.n_types, dtype=torch.float64, device=pos.device)
    with pytest.raises(alchnb.AlchNBError):
        ctx.backward(pos, lam, g, d_charge=d_q)


@pytest.mark.parametrize("schedule", [O.BEUTLER, O.LBF], ids=["beutler", "lbf"])
def test_cross_group_exclusions_dsf_and_pme(schedule):
    """Exclusions between solute and solvent atoms (besides solvent-solvent
    ones): the short-range pass skips them and PME scales their reciprocal
    correction by c(lambda) with the other solute-solvent parts; DSF and PME
    contexts, FP64, against the oracles at two lambdas."""
    from paper_2608_12691_amd import alchnb
    rng = np.random.Generator(np.random.PCG64(2718))
    w1 = workload(1)
    s = _ortho_box(rng, 600, (21.0, 23.0, 25.0), 8, w1.ff.n_types)
    ex = sorted({(0, 20), (1, 21), (2, 3), (3, 40), (30, 31), (30, 32), (55, 70)})
    s.exclusions = np.array(ex, np.int32)
    w = S.Workload(name="xexcl", systems=[s], ff=w1.ff, cutoff=9.0, skin=1.0, switch_width=1.0, dsf_alpha=ALPHA,
                   sc_alpha=0.5, lambdas=np.array([0.7]), seed=2718)
    for lam in (0.35, 0.8):
        # DSF
        ctx = alchnb.Context(w.ff, w.systems, w.cutoff, w.skin, w.switch_width, 0.2, w.sc_alpha, schedule=schedule,
                             precision=1)
        res = to_numpy(ctx.compute_checked(ctx.positions(w.systems), ctx.lambdas([lam]), flags=1))
        prm = O.Params(w.cutoff, w.switch_width, 0.2, w.sc_alpha, schedule)
        r0 = O.evaluate_system(s, w.ff, prm, lam)
        _check(res, r0, 0, s.n_atoms, 1, "dsf lam=%g" % lam)
        ctx.close()
        # PME
        ctx = _ctx(w, 1, schedule)
        res = to_numpy(ctx.compute_checked(ctx.positions(w.systems), ctx.lambdas([lam]), flags=1))
        ref = _oracle(w, 0, lam, schedule, ctx.pme_grid(0))
        assert ref["corr"]["e_sw"] != 0.0
        _check(res, ref, 0, s.n_atoms, 1, "pme lam=%g" % lam)
        ctx.close()


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
def test_pme_lbf_energies_are_linear_in_the_bases(precision):
    """Eq. 4 with PME: the solute-solvent Ewald part belongs to U_A, so the
    energy at any lambda follows from one evaluation's bases:
    U(l2) - U(l1) = (hA(l2) - hA(l1)) U_A + (hB(l2) - hB(l1)) U_B, which is
    what replica exchange relies on; and dU/dlambda = hA' U_A + hB' U_B."""
    w = workload(2)
    ctx = _ctx(w, precision, O.LBF)
    pos = ctx.positions(w.systems)
    rs = {}
    for lam in (0.42, 0.77):
        rs[lam] = to_numpy(ctx.compute_checked(pos, ctx.lambdas([lam]), flags=1))
    t1, t2 = rs[0.42]["terms"][0], rs[0.77]["terms"][0]
    h1, h2 = O.lbf_switches(0.42), O.lbf_switches(0.77)
    assert t1[4] == pytest.approx(t2[4], rel=1e-12) and t1[5] == pytest.approx(t2[5], rel=1e-12)
    want = (h2[0] - h1[0]) * t1[4] + (h2[1] - h1[1]) * t1[5]
    scale = abs(t1[4]) + abs(t1[5])
    assert abs((t2[8] - t1[8]) - want) <= 1e-9 * scale
    for t, h in ((t1, h1), (t2, h2)):
        assert t[9] == pytest.approx(h[2] * t[4] + h[3] * t[5], rel=1e-9, abs=1e-9 * scale)
