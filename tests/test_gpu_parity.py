"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2608_12691_amd import systems as S

from conftest import workload
from parity import TOL, compare, oracle_for, to_numpy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ctx(w, precision, schedule=O.BEUTLER, **kw):
    from paper_2608_12691_amd import alchnb
    return alchnb.from_workload(w, precision=precision, schedule=schedule, **kw)


def _offsets(w):
    return np.concatenate([[0], np.cumsum([s.n_atoms for s in w.systems])])


def _run(ctx, w, lam, positions=None, flags=1):
    pos_list = [s.positions for s in w.systems] if positions is None else positions
    pos = ctx.positions(np.concatenate(pos_list))
    res = ctx.compute_checked(pos, ctx.lambdas(lam), flags=flags)
    torch.cuda.synchronize()
    return to_numpy(res), pos_list


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
@pytest.mark.parametrize("schedule", [O.BEUTLER, O.LBF], ids=["beutler", "lbf"])
def test_config1_parity(precision, schedule):
    w = workload(1)
    ctx = _ctx(w, precision, schedule)
    for lam in (0.5, 0.0, 0.3, 0.75, 1.0):
        print("config1 precision=%d schedule=%d lambda=%.2f" % (precision, schedule, lam), flush=True)
        res, pos = _run(ctx, w, [lam])
        assert res["flags"] == 0
        ref = oracle_for(w, 0, lam, schedule)
        compare(res, [ref], w, pos, precision, _offsets(w), label="cfg1 lam=%g" % lam)


def test_config1_pair_set_bit_exact():
    w = workload(1)
    ctx = _ctx(w, 0)
    pos = ctx.positions(w.systems)
    ctx.build_list(pos)
    got = ctx.export_pairs()
    s = w.systems[0]
    ref = O.pair_set(s.positions, s.exclusions, s.box, w.cutoff + w.skin)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_deterministic_repeats(precision):
    w = workload(1)
    ctx = _ctx(w, precision)
    pos = ctx.positions(w.systems)
    lam = ctx.lambdas([0.62])
    outs = []
    for _ in range(5):
        o = ctx.compute(pos, lam, flags=2)
        torch.cuda.synchronize()
        outs.append(to_numpy(o))
    for o in outs[1:]:
        for k in ("forces", "terms", "dudl", "n_pairs"):
            assert np.array_equal(o[k], outs[0][k]), k


def test_ragged_batch_with_empty_box():
    """Three boxes of different sizes, one of them empty, at different lambdas."""
    rng = np.random.Generator(np.random.PCG64(99))
    w1 = workload(1)
    boxes = []
    for n, L in ((0, 22.0), (150, 22.0), (400, 27.0)):
        if n == 0:
            boxes.append(S.System(positions=np.zeros((0, 3)), types=np.zeros(0, np.int32),
                                  is_solute=np.zeros(0, np.uint8), exclusions=np.zeros((0, 2), np.int32),
                                  box=np.full(3, L), molecule=np.zeros(0, np.int32)))
        else:
            boxes.append(S.random_tiny_system(rng, n, L, n_solute=6, n_types=w1.ff.n_types, min_dist=2.0))
    w = S.Workload(name="ragged", systems=boxes, ff=w1.ff, cutoff=9.0, skin=1.0, switch_width=1.0, dsf_alpha=0.2,
                   sc_alpha=0.5, lambdas=np.array([0.2, 0.45, 0.9]), seed=99)
    for precision in (1, 0):
        ctx = _ctx(w, precision)
        res, pos = _run(ctx, w, w.lambdas)
        refs = [oracle_for(w, k, w.lambdas[k], O.BEUTLER) if s.n_atoms else
                dict(terms=np.zeros(10), forces=np.zeros((0, 3)), n_pairs=0, abs_terms=np.zeros(10))
                for k, s in enumerate(w.systems)]
        compare(res, refs, w, pos, precision, _offsets(w), label="ragged p%d" % precision)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_config2_protocol(precision):
    """24-atom solute in 3,000 waters, skin 1 A: the 1,000-call random walk with
    device-side rebuilds, checked against the oracle at calls 0, 99, ..., 999."""
    w = workload(2)
    s = w.systems[0]
    ctx = _ctx(w, precision)
    n_calls = 1000
    walk = S.perturbation_walk(s, n_calls, 0.01, seed=7)
    lams = S.lambda_draws(n_calls, seed=8)
    pos = ctx.positions(walk[0])
    lam = ctx.lambdas([lams[0]])
    out = ctx.new_outputs()
    checked = {0} | set(range(99, n_calls, 100))
    for t in range(n_calls):
        pos.copy_(torch.as_tensor(walk[t], device=pos.device))
        lam.fill_(float(lams[t]))
        ctx.compute(pos, lam, flags=1, out=out)
        if t in checked:
            torch.cuda.synchronize()
            res = to_numpy(out)
            ref = oracle_for(w, 0, lams[t], O.BEUTLER, positions=walk[t])
            print("config2 call %d lambda %.3f" % (t, lams[t]), flush=True)
            compare(res, [ref], w, [walk[t]], precision, _offsets(w), label="cfg2 t=%d" % t)
    st = ctx.get_stats()
    assert st["n_rebuilds"] >= 5  # the walk crosses skin/2 about every 100 calls
    assert ctx.get_flags() == 0


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_config2_lbf_walk(precision):
    """The LBF schedule on the 3,000-water box: 300 calls of the walk with device-side rebuilds, checked
    against the oracle at lambdas below the h_A onset (softened basis only), across it and near 1."""
    w = workload(2)
    s = w.systems[0]
    ctx = _ctx(w, precision, O.LBF)
    n_calls = 300
    walk = S.perturbation_walk(s, n_calls, 0.01, seed=17)
    checks = {0: 0.2, 120: 0.35, 180: 0.5, 299: 0.95}
    pos = ctx.positions(walk[0])
    lam = ctx.lambdas([0.1])
    out = ctx.new_outputs()
    for t in range(n_calls):
        pos.copy_(torch.as_tensor(walk[t], device=pos.device))
        lt = checks.get(t, 0.1 + 0.8 * t / n_calls)
        lam.fill_(lt)
        ctx.compute(pos, lam, flags=1, out=out)
        if t in checks:
            torch.cuda.synchronize()
            print("config2 lbf call %d lambda %.3f" % (t, lt), flush=True)
            ref = oracle_for(w, 0, lt, O.LBF, positions=walk[t])
            compare(to_numpy(out), [ref], w, [walk[t]], precision, _offsets(w), label="cfg2 lbf t=%d" % t)
    assert ctx.get_stats()["n_rebuilds"] >= 2
    assert ctx.get_flags() == 0


def test_config2_long_walk_many_rebuilds():
    """10,000 calls of a walk with N(0, 0.003 A) steps (about 0.3 A rms per coordinate at the end, as far
    as the 1,000-call protocol drifts; an uncorrelated walk of all atoms that goes much further brings
    non-bonded atoms into contact and overflows the fixed-point forces, as it should): no flags, the
    device-side rebuilds (eight for this seed), and the last call and the list built at its positions
    match the oracle."""
    w = workload(2)
    s = w.systems[0]
    ctx = _ctx(w, 0)
    n_calls = 10000
    rng = np.random.Generator(np.random.PCG64(2626))
    x = torch.as_tensor(s.positions, dtype=torch.float64, device="cuda")
    steps = torch.as_tensor(rng.normal(0.0, 0.003, (n_calls, s.n_atoms, 3)), device="cuda")
    lam = ctx.lambdas([0.6])
    out = ctx.new_outputs()
    print("config2 long walk: %d calls" % n_calls, flush=True)
    for t in range(n_calls):
        x += steps[t]
        ctx.compute(x, lam, flags=1, out=out)
    torch.cuda.synchronize()
    st = ctx.get_stats()
    assert ctx.get_flags() == 0
    assert st["n_rebuilds"] >= 5, st["n_rebuilds"]
    last = x.cpu().numpy()
    res = to_numpy(out)
    compare(res, [oracle_for(w, 0, 0.6, O.BEUTLER, positions=last)], w, [last], 0, _offsets(w), label="long walk")
    ctx.build_list(x)
    assert np.array_equal(ctx.export_pairs(), O.pair_set(last, s.exclusions, s.box, w.cutoff + w.skin))


def test_config2_pair_set_after_walk():
    w = workload(2)
    s = w.systems[0]
    ctx = _ctx(w, 0)
    walk = S.perturbation_walk(s, 40, 0.05, seed=3)
    pos = ctx.positions(walk[-1])
    ctx.build_list(pos)
    got = ctx.export_pairs()
    ref = O.pair_set(walk[-1], s.exclusions, s.box, w.cutoff + w.skin)
    assert np.array_equal(got, ref)


def test_flags_forced_from_host():
    w = workload(1)
    ctx = _ctx(w, 0)
    pos = ctx.positions(w.systems)
    ctx.compute(pos, ctx.lambdas([1.5]), flags=2)
    assert ctx.get_flags() & 8  # lambda clamped
    bad = pos.clone()
    bad[3, 1] = float("nan")
    ctx.compute(bad, ctx.lambdas([0.5]), flags=0)
    assert ctx.get_flags() & 4  # non-finite position
    # a skin violation without automatic rebuild (config 2 has skin 1 A)
    w2 = workload(2)
    c2 = _ctx(w2, 0)
    p2 = c2.positions(w2.systems)
    c2.compute(p2, c2.lambdas([0.5]), flags=2)
    assert c2.get_flags() == 0
    moved = p2.clone()
    moved[10, 0] += 0.8
    c2.compute(moved, c2.lambdas([0.5]), flags=0)
    assert c2.get_flags() & 2


def test_graph_replay_matches_eager():
    w = workload(2)
    s = w.systems[0]
    ctx = _ctx(w, 0)
    walk = S.perturbation_walk(s, 6, 0.05, seed=21)
    pos = ctx.positions(walk[0])
    lam = ctx.lambdas([0.4])
    out = ctx.new_outputs()
    ctx.compute(pos, lam, flags=1, out=out)  # builds the list before capture
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = _ctx(w, 0)
        gout = gctx.new_outputs()
        gpos = gctx.positions(walk[0])
        glam = gctx.lambdas([0.4])
        gctx.compute(gpos, glam, flags=1, out=gout)
        gctx.capture_step(gpos, glam, gout)
    for t in range(1, 6):
        x = torch.as_tensor(walk[t], device=pos.device)
        with torch.cuda.stream(stream):
            gpos.copy_(x)
            glam.fill_(0.1 * t)
            gctx.launch_step()
        stream.synchronize()
        pos.copy_(x)
        lam.fill_(0.1 * t)
        ctx.compute(pos, lam, flags=1, out=out)
        torch.cuda.synchronize()
        a, b = to_numpy(gout), to_numpy(out)
        for k in ("forces", "terms", "dudl", "n_pairs"):
            assert np.array_equal(a[k], b[k]), (t, k)


def test_autotune_keeps_parity_and_caches(tmp_path, monkeypatch):
    w = workload(2)
    monkeypatch.setenv("ALCHNB_TUNE_CACHE", str(tmp_path / "tune.json"))
    ctx = _ctx(w, 0)
    pos = ctx.positions(w.systems)
    lam = ctx.lambdas([0.37])
    ctx.autotune(pos, lam, reps=3)
    v = ctx.get_stats()["variant"]
    assert 0 <= v < ctx.lib.alch_nb_num_variants()
    assert (tmp_path / "tune.json").exists()
    res = to_numpy(ctx.compute_checked(pos, lam, flags=1))
    ref = oracle_for(w, 0, 0.37, O.BEUTLER)
    compare(res, [ref], w, [w.systems[0].positions], 0, _offsets(w), label="tuned")
    # a new context with the same key picks the cached variant
    ctx2 = _ctx(w, 0)
    assert ctx2.get_stats()["variant"] == v
    # every variant gives the same pair count and forces within tolerance
    for vv in range(ctx.lib.alch_nb_num_variants()):
        ctx.set_variant(vv)
        r = to_numpy(ctx.compute_checked(pos, lam, flags=0))
        compare(r, [ref], w, [w.systems[0].positions], 0, _offsets(w), label="variant %d" % vv)


_CFG4_REFS = {}


def _cfg4_refs(w, schedule, positions=None, lams=None):
    """Oracle results of every config-4 box (cached per schedule for the unperturbed boxes)."""
    key = (schedule,) if positions is None else None
    if key and key in _CFG4_REFS:
        return _CFG4_REFS[key]
    lams = w.lambdas if lams is None else lams
    refs = [oracle_for(w, k, lams[k], schedule, positions=None if positions is None else positions[k])
            for k in range(len(w.systems))]
    if key:
        _CFG4_REFS[key] = refs
    return refs


def _per_box(w, res, refs, positions, precision, label):
    off = _offsets(w)
    for k in range(len(w.systems)):
        sub = {kk: (v[off[k]:off[k + 1]] if kk == "forces" else v[k:k + 1]) for kk, v in res.items() if kk != "flags"}
        one = S.Workload(w.name, [w.systems[k]], w.ff, w.cutoff, w.skin, w.switch_width, w.dsf_alpha, w.sc_alpha,
                         w.lambdas[k:k + 1], w.seed)
        compare(sub, [refs[k]], one, [positions[k]], precision, np.array([0, off[k + 1] - off[k]]),
                label="%s box %d" % (label, k))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("schedule", [O.BEUTLER, O.LBF], ids=["beutler", "lbf"])
def test_config4_batched_replicas(precision, schedule):
    """16 boxes of 2,000-12,000 atoms at lambda_k = k/15 in one launch; every box vs the oracle
    (each box with its own lambda factors, for both schedules)."""
    w = workload(4)
    ctx = _ctx(w, precision, schedule)
    print("config4 precision=%d schedule=%d" % (precision, schedule), flush=True)
    res, pos = _run(ctx, w, w.lambdas, flags=2)
    assert res["flags"] == 0
    _per_box(w, res, _cfg4_refs(w, schedule), pos, precision, "cfg4")


def test_config4_graph_replay_batched():
    """The 16-box step captured as one hipGraph: every replay (new positions
    and lambdas copied into the captured buffers, eager work and syncs in
    between) is bit-identical to an eager call on the same inputs, and the
    last replay matches the oracle in every box."""
    w = workload(4)
    xs0 = np.concatenate([s.positions for s in w.systems])
    rng = np.random.Generator(np.random.PCG64(4040))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = _ctx(w, 0)
        gout = gctx.new_outputs()
        gpos = gctx.positions(xs0)
        glam = gctx.lambdas(w.lambdas)
        gctx.compute_checked(gpos, glam, flags=2, out=gout)
        gctx.capture_step(gpos, glam, gout)
    ctx = _ctx(w, 0)
    out = ctx.new_outputs()
    pos = ctx.positions(xs0)
    lam = ctx.lambdas(w.lambdas)
    ctx.compute_checked(pos, lam, flags=2, out=out)
    x = xs0.copy()
    lams = np.array(w.lambdas, dtype=np.float64)
    for t in range(1, 6):
        print("graph replay %d" % t, flush=True)
        x = x + rng.normal(0.0, 0.05, x.shape)
        lams = np.clip(lams + rng.normal(0.0, 0.02, lams.shape), 0.0, 1.0)
        xt = torch.as_tensor(x, device=pos.device)
        lt = torch.as_tensor(lams, device=pos.device)
        with torch.cuda.stream(stream):
            gpos.copy_(xt)
            glam.copy_(lt)
            gctx.launch_step()
        stream.synchronize()
        pos.copy_(xt)
        lam.copy_(lt)
        ctx.compute(pos, lam, flags=1, out=out)
        torch.cuda.synchronize()
        a, b = to_numpy(gout), to_numpy(out)
        for k in ("forces", "terms", "dudl", "n_pairs"):
            assert np.array_equal(a[k], b[k]), (t, k)
    assert gctx.get_flags() == 0 and ctx.get_flags() == 0
    off = _offsets(w)
    pos_k = [x[off[k]:off[k + 1]] for k in range(len(w.systems))]
    wl = S.Workload(w.name, w.systems, w.ff, w.cutoff, w.skin, w.switch_width, w.dsf_alpha, w.sc_alpha, lams, w.seed)
    refs = _cfg4_refs(wl, O.BEUTLER, positions=pos_k, lams=lams)
    _per_box(wl, to_numpy(gout), refs, pos_k, 0, "cfg4 graph")


@pytest.mark.parametrize("k", [1, 2])
def test_per_phase_list_build(k):
    """The list built by one kernel per phase (the fallback of the fused
    build) gives the oracle's pair set and parity, also after a walk with
    device-side rebuilds."""
    from paper_2608_12691_amd import alchnb
    w = workload(k)
    s = w.systems[0]
    ctx = _ctx(w, 0)
    ctx.set_list_mode(alchnb.LIST_PHASES)
    assert ctx.list_mode() == alchnb.LIST_PHASES
    pos = ctx.positions(w.systems)
    ctx.build_list(pos)
    assert np.array_equal(ctx.export_pairs(), O.pair_set(s.positions, s.exclusions, s.box, w.cutoff + w.skin))
    res, p = _run(ctx, w, [0.6], flags=2)
    assert res["flags"] == 0
    compare(res, [oracle_for(w, 0, 0.6, O.BEUTLER)], w, p, 0, _offsets(w), label="phases cfg%d" % k)
    if k == 2:
        walk = S.perturbation_walk(s, 200, 0.02, seed=77)
        lam = ctx.lambdas([0.3])
        out = ctx.new_outputs()
        n0 = ctx.get_stats()["n_rebuilds"]
        for t in range(200):
            ctx.compute(ctx.positions(walk[t]), lam, flags=1, out=out)
        assert ctx.get_stats()["n_rebuilds"] > n0
        assert ctx.get_flags() == 0
        res = to_numpy(out)
        compare(res, [oracle_for(w, 0, 0.3, O.BEUTLER, positions=walk[-1])], w, [walk[-1]], 0, _offsets(w),
                label="phases walk")
        ctx.build_list(ctx.positions(walk[-1]))
        assert np.array_equal(ctx.export_pairs(), O.pair_set(walk[-1], s.exclusions, s.box, w.cutoff + w.skin))
    ctx.set_list_mode(alchnb.LIST_AUTO)


def _squeezed_waters(w, d_oo):
    """Config 1 with one water moved rigidly so that its oxygen sits d_oo from
    another water's oxygen (every other atom pair stays >= 0.9 A apart)."""
    s = w.systems[0]
    x = s.positions.copy()
    L = s.box
    first = int(np.nonzero(s.is_solute == 0)[0][0])
    oxy = np.arange(first, s.n_atoms, 3)
    for a in oxy[:40]:
        for b in oxy:
            if b == a:
                continue
            v = x[b] - x[a]
            v -= L * np.rint(v / L)
            y = x.copy()
            y[b:b + 3] += (v / np.linalg.norm(v)) * d_oo - v
            dmin = np.inf
            for m in range(b, b + 3):
                dv = y - y[m]
                dv -= L * np.rint(dv / L)
                r = np.sqrt((dv * dv).sum(1))
                r[b:b + 3] = np.inf
                r[a] = np.inf if m == b else r[a]
                dmin = min(dmin, r.min())
            if dmin >= 0.9:
                return y, a, b
    raise AssertionError("no water pair to squeeze")


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
def test_large_pair_forces_fixed_point(precision):
    """An O-O contact at 1.2 A gives pair forces of ~6e5 kcal/mol/A: above
    2^51 fixed-point units in both precisions (the general conversion path of
    the force sums) and below the overflow limit (2^62 units)."""
    w = workload(1)
    y, a, b = _squeezed_waters(w, 1.2)
    ref = oracle_for(w, 0, 0.5, O.BEUTLER, positions=y)
    fmax = np.abs(ref["forces"]).max()
    scale = 2.0 ** 40 if precision == 1 else 2.0 ** 32
    assert 2.0 ** 51 < fmax * scale < 2.0 ** 62, fmax
    ctx = _ctx(w, precision)
    res, pos = _run(ctx, w, [0.5], positions=[y], flags=2)
    assert res["flags"] == 0
    compare(res, [ref], w, pos, precision, _offsets(w), label="squeezed O-O")


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
def test_config1_against_stored_oracle_values(precision):
    """The HIP path against the stored oracle results (tests/golden), no oracle call at run time."""
    import json
    import os
    from parity import dudl_error, energy_error, force_error
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config1_oracle.json")) as f:
        g = json.load(f)
    w = workload(1)
    atoms = g["force_atoms"]
    tol = TOL[precision]
    for name, sched in (("beutler", O.BEUTLER), ("lbf", O.LBF)):
        ctx = _ctx(w, precision, sched)
        for c in (c for c in g["cases"] if c["schedule"] == name):
            print("golden precision=%d schedule=%s lambda=%.2f" % (precision, name, c["lam"]), flush=True)
            res, _ = _run(ctx, w, [c["lam"]])
            assert res["flags"] == 0
            scale = c["abs_terms"]
            eF = force_error(res["forces"][atoms], np.asarray(c["forces"]))
            ed = dudl_error(res["dudl"][0], c["terms"][9], scale[9])
            eE = max(energy_error(res["terms"][0, j], c["terms"][j], scale[j]) for j in range(10))
            assert eF <= tol["force"], (name, c["lam"], eF)
            assert ed <= tol["dudl"], (name, c["lam"], ed)
            assert eE <= tol["energy"], (name, c["lam"], eE)
            # FP32 distances may put a pair within ~1e-6 A of the cutoff on the other side
            assert abs(int(res["n_pairs"][0]) - c["n_pairs"]) <= (0 if precision == 1 else 1)


def test_list_overflow_sets_flag_and_replan_recovers():
    """A list that outgrows its workspace evaluates nothing and says so; the re-plan gives the oracle's result."""
    w = workload(1)
    ctx = _ctx(w, 0, capacity_factor=0.005)
    pos = ctx.positions(w.systems)
    lam = ctx.lambdas([0.5])
    print("overflow: first build with 0.5% of the planned list capacity", flush=True)
    o = to_numpy(ctx.compute(pos, lam, flags=2))
    f = ctx.get_flags()
    assert f & 16, f
    assert int(o["n_pairs"][0]) == 0 and np.all(o["forces"] == 0.0) and np.all(o["terms"] == 0.0)
    print("overflow: compute_checked re-plans", flush=True)
    res = ctx.compute_checked(pos, lam, flags=2)
    torch.cuda.synchronize()
    assert res["flags"] == 0
    ref = oracle_for(w, 0, 0.5, O.BEUTLER)
    compare(to_numpy(res), [ref], w, [w.systems[0].positions], 0, _offsets(w), label="after re-plan")


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_coincident_atoms_flag_overflow(precision):
    """Two atoms of different molecules on the same point: the call completes, the force sums report
    FLAG_FIXED_OVERFLOW and the total energy is not finite (r = 0 has no finite LJ value)."""
    w = workload(1)
    s = w.systems[0]
    p = s.positions.copy()
    a, b = 20, 50
    assert s.molecule[a] != s.molecule[b]
    p[b] = p[a]
    ctx = _ctx(w, precision)
    pos = ctx.positions(p)
    print("coincident atoms precision %d" % precision, flush=True)
    out = to_numpy(ctx.compute(pos, ctx.lambdas([0.5]), flags=2))
    torch.cuda.synchronize()
    f = ctx.get_flags()
    assert f & 1, f
    assert not np.isfinite(out["terms"][0, 8])
    # the next call at valid positions is clean again
    res, _ = _run(ctx, w, [0.5], flags=2)
    assert res["flags"] == 0
    compare(res, [oracle_for(w, 0, 0.5, O.BEUTLER)], w, [s.positions], precision, _offsets(w), label="after")


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("schedule", [O.BEUTLER, O.LBF], ids=["beutler", "lbf"])
@pytest.mark.parametrize("alpha", [0.2, 0.0], ids=["dsf", "sf"])
def test_hard_truncation_and_plain_shifted_force(precision, schedule, alpha):
    """No LJ switch (the kernels without the switch) and, with alpha = 0, plain shifted-force Coulomb."""
    w1 = workload(1)
    w = S.Workload("cfg1-hard", w1.systems, w1.ff, w1.cutoff, w1.skin, 0.0, alpha, w1.sc_alpha, w1.lambdas, w1.seed)
    ctx = _ctx(w, precision, schedule)
    for lam in (0.3, 0.8):
        print("hard truncation precision=%d schedule=%d alpha=%.1f lambda=%.1f" % (precision, schedule, alpha, lam),
              flush=True)
        res, pos = _run(ctx, w, [lam], flags=2)
        assert res["flags"] == 0
        ref = oracle_for(w, 0, lam, schedule, param_grads=True)
        compare(res, [ref], w, pos, precision, _offsets(w), label="hard lam=%g" % lam)
        # the parameter pass without the switch
        T = ctx.n_types
        dsig, dq = (torch.zeros(T, dtype=torch.float64, device=ctx.device) for _ in range(2))
        ctx.backward(ctx.positions(pos[0]), ctx.lambdas([lam]), torch.ones(1, dtype=torch.float64, device=ctx.device),
                     d_sigma=dsig, d_charge=dq)
        torch.cuda.synchronize()
        tol = 1e-9 if precision == 1 else 2e-5
        for got, want in ((dsig, ref["d_sigma"]), (dq, ref["d_charge"])):
            g = got.cpu().numpy()
            assert np.abs(g - want).max() <= tol * np.abs(want).max()


def _orthorhombic_box(seed, L=(22.0, 26.0, 31.0)):
    """Atoms on a jittered grid (>= 2.6 A apart, liquid-like packing without bonded contacts) in an
    orthorhombic box with three different edges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.asarray(L)
    n = np.floor(L / 3.0).astype(int)
    g = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), -1).reshape(-1, 3).astype(float)
    pos = (g + 0.5) * (L / n) + rng.uniform(-0.2, 0.2, g.shape)
    w1 = workload(1)
    types = rng.integers(0, w1.ff.n_types, len(pos)).astype(np.int32)
    sol = np.zeros(len(pos), np.uint8)
    sol[rng.choice(len(pos), 10, replace=False)] = 1
    box = S.System(positions=pos, types=types, is_solute=sol, exclusions=np.zeros((0, 2), np.int32), box=L,
                   molecule=np.arange(len(pos), dtype=np.int32))
    return S.Workload("ortho", [box], w1.ff, 9.0, 1.0, 1.0, 0.2, 0.5, np.array([0.4]), seed)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_orthorhombic_box_pairs_and_parity(precision):
    """Edges 22 x 26 x 31 A: the exported pair set equals the oracle's and the results match it."""
    w = _orthorhombic_box(31)
    s = w.systems[0]
    ctx = _ctx(w, precision)
    pos = ctx.positions(w.systems)
    print("orthorhombic box precision %d atoms %d" % (precision, s.n_atoms), flush=True)
    ctx.build_list(pos)
    got = ctx.export_pairs()
    ref_pairs = O.pair_set(s.positions, s.exclusions, s.box, w.cutoff + w.skin)
    assert np.array_equal(got, ref_pairs)
    for lam in (0.4, 0.9):
        res, p = _run(ctx, w, [lam], flags=2)
        assert res["flags"] == 0
        compare(res, [oracle_for(w, 0, lam, O.BEUTLER)], w, p, precision, _offsets(w), label="ortho lam=%g" % lam)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_box_at_the_size_limit_and_many_boxes(precision):
    """A 20 A box with cutoff + skin = 10 A (exactly half the edge) and 40 small boxes in one call."""
    rng = np.random.Generator(np.random.PCG64(2020))
    w1 = workload(1)
    edge = S.random_tiny_system(rng, 260, 20.0, n_solute=6, n_types=w1.ff.n_types, min_dist=2.2)
    w = S.Workload("edge", [edge], w1.ff, 9.0, 1.0, 1.0, 0.2, 0.5, np.array([0.45]), 2020)
    ctx = _ctx(w, precision)
    pos = ctx.positions(w.systems)
    print("box at the limit precision %d" % precision, flush=True)
    ctx.build_list(pos)
    assert np.array_equal(ctx.export_pairs(), O.pair_set(edge.positions, edge.exclusions, edge.box, 10.0))
    res, p = _run(ctx, w, [0.45], flags=2)
    assert res["flags"] == 0
    compare(res, [oracle_for(w, 0, 0.45, O.BEUTLER)], w, p, precision, _offsets(w), label="edge")
    # 40 boxes of 30-90 atoms at lambda_k = k/39
    boxes = [S.random_tiny_system(rng, int(n), 20.0, n_solute=3, n_types=w1.ff.n_types, min_dist=2.6)
             for n in rng.integers(30, 90, 40)]
    lams = np.linspace(0.0, 1.0, 40)
    wm = S.Workload("many", boxes, w1.ff, 9.0, 1.0, 1.0, 0.2, 0.5, lams, 2021)
    cm = _ctx(wm, precision)
    print("40 boxes precision %d" % precision, flush=True)
    res, p = _run(cm, wm, list(lams), flags=2)
    assert res["flags"] == 0
    refs = [oracle_for(wm, k, lams[k], O.BEUTLER) for k in range(40)]
    # dU/dlambda cancels to 0.3-4% of sum |du/dlambda| in these boxes; the solute-solvent pairs are
    # evaluated in FP64 in both kernels, so the relative bar holds in both precisions.  Energies: a
    # box of 30-90 atoms has a few contact pairs at 2.6 A that dominate sum |u|; FP32 local
    # coordinates (up to ~8 A from the super-cluster origin, half an ulp = 2.4e-7 A) give r^2 a
    # relative error up to 2 x 2.4e-7 / 2.6 = 1.8e-7, which r^-12 = (r^2)^-6 multiplies by 6:
    # ~1.1e-6 of such a pair's energy.  The FP32 energy bar here is that floor, 2e-6 (measured
    # 1.0e-6); forces and dU/dlambda keep their bars
    compare(res, refs, wm, p, precision, _offsets(wm), label="many boxes",
            energy_tol=2e-6 if precision == 0 else None)
