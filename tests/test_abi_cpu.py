"""Host-side contract of the C ABI (no GPU needed): symbols, validation, planning."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2608_12691_amd import alchnb, build
    if not os.path.exists(alchnb.LIB_PATH):
        build.build(force=True)
    return alchnb.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "alch_nb.h")).read()
    pat = r"^\s*(?:alch_nb_status|void|const char\s*\*|int32_t|int64_t|double)\s*\*?\s*(alch_nb_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(pat, src, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    from paper_2608_12691_amd import alchnb
    assert sorted(alchnb.EXPORTED) == names


def _params(alchnb, ff, **kw):
    p = alchnb.Params_t()
    sig = np.ascontiguousarray(ff["sigma"], np.float64)
    eps = np.ascontiguousarray(ff["epsilon"], np.float64)
    chg = np.ascontiguousarray(ff["charge"], np.float64)
    p.n_types = len(sig)
    p.sigma, p.epsilon, p.charge = sig.ctypes.data, eps.ctypes.data, chg.ctypes.data
    p.cutoff, p.skin, p.switch_width, p.dsf_alpha, p.sc_alpha = 9.0, 0.0, 1.0, 0.2, 0.5
    p.schedule, p.precision, p.variant, p.list_capacity_factor = 0, 0, -1, 1.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p, (sig, eps, chg)


def _system(alchnb, n=4, box=20.0, types=None, sol=None, excl=None):
    s = alchnb.System_t()
    t = np.ascontiguousarray(types if types is not None else np.zeros(n), np.int32)
    so = np.ascontiguousarray(sol if sol is not None else np.zeros(n), np.uint8)
    ex = np.ascontiguousarray(excl if excl is not None else np.zeros((0, 2)), np.int32).reshape(-1, 2)
    s.n_atoms = len(t)
    s.type, s.is_solute = t.ctypes.data, so.ctypes.data
    s.n_excl = ex.shape[0]
    s.excl = ex.ctypes.data if ex.shape[0] else None
    for d in range(3):
        s.box[d] = box
    return s, (t, so, ex)


FF = dict(sigma=[3.0, 3.2], epsilon=[0.1, 0.0], charge=[0.4, -0.4])


def _create(lib, p, systems):
    from paper_2608_12691_amd import alchnb
    arr = (alchnb.System_t * len(systems))(*systems)
    ctx = ctypes.c_void_p()
    st = lib.alch_nb_create(ctypes.byref(p), arr, len(systems), ctypes.byref(ctx))
    return st, ctx


def test_create_plans_workspace(lib):
    from paper_2608_12691_amd import alchnb
    p, keep = _params(alchnb, FF)
    s, k2 = _system(alchnb, 6, 20.0, types=[0, 1, 0, 1, 0, 1], sol=[1, 0, 0, 0, 0, 0], excl=[[0, 1], [2, 3]])
    st, ctx = _create(lib, p, [s])
    assert st == 0 and ctx.value
    nb = ctypes.c_size_t()
    assert lib.alch_nb_workspace_size(ctx, ctypes.byref(nb)) == 0 and nb.value > 0
    stats = alchnb.Stats_t()
    assert lib.alch_nb_get_stats(ctx, ctypes.byref(stats)) == 0
    assert stats.n_atoms == 6 and stats.entry_capacity > 0
    # computing before binding is refused without touching the GPU
    assert lib.alch_nb_compute(ctx, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, None) == 6
    assert lib.alch_nb_build_list(ctx, ctypes.c_void_p(8)) == 6
    # the fused lambda-dynamics step: missing arguments first, then no binding
    v = ctypes.c_void_p(8)
    assert lib.alch_nb_ld_step_dafed(ctx, v, v, None, v, None, None, None, v, 1, None) == 1
    assert lib.alch_nb_ld_step_dafed(ctx, v, v, v, v, None, None, None, v, 0, None) == 1
    assert lib.alch_nb_ld_step_dafed(ctx, v, v, v, v, None, None, None, v, 1, None) == 6
    # timing: a negative stride is refused; 0 (off) creates no HIP object
    assert lib.alch_nb_set_timing(ctx, -1) == 1
    assert lib.alch_nb_set_timing(ctx, 0) == 0
    lib.alch_nb_destroy(ctx)


@pytest.mark.parametrize("field,value,code", [
    ("cutoff", -1.0, 1), ("skin", -0.5, 1), ("switch_width", 9.5, 1), ("schedule", 5, 1), ("precision", 3, 1),
    ("variant", 99, 1), ("cutoff", 10.5, 2), ("dsf_alpha", 0.6, 3),
])
def test_create_rejects_bad_params(lib, field, value, code):
    from paper_2608_12691_amd import alchnb
    p, keep = _params(alchnb, FF, **{field: value})
    s, k2 = _system(alchnb)
    st, ctx = _create(lib, p, [s])
    assert st == code
    assert not ctx.value


@pytest.mark.parametrize("kw", [
    dict(types=[0, 1, 2, 0]),                       # type out of range
    dict(sol=[0, 2, 0, 0]),                         # solute flag not 0/1
    dict(excl=[[1, 0]]),                            # i > j
    dict(excl=[[0, 2], [0, 1]]),                    # unsorted
    dict(excl=[[0, 1], [0, 1]]),                    # duplicate
    dict(excl=[[0, 7]]),                            # out of range
])
def test_create_rejects_bad_systems(lib, kw):
    from paper_2608_12691_amd import alchnb
    p, keep = _params(alchnb, FF)
    s, k2 = _system(alchnb, **kw)
    st, ctx = _create(lib, p, [s])
    assert st == 1


def test_create_rejects_null_and_empty(lib):
    from paper_2608_12691_amd import alchnb
    p, keep = _params(alchnb, FF)
    ctx = ctypes.c_void_p()
    assert lib.alch_nb_create(None, None, 1, ctypes.byref(ctx)) == 1
    assert lib.alch_nb_create(ctypes.byref(p), None, 1, ctypes.byref(ctx)) == 1
    s, k2 = _system(alchnb)
    arr = (alchnb.System_t * 1)(s)
    assert lib.alch_nb_create(ctypes.byref(p), arr, 0, ctypes.byref(ctx)) == 1
    assert lib.alch_nb_create(ctypes.byref(p), arr, 1, None) == 1


def test_empty_and_ragged_boxes_plan(lib):
    """Boxes with zero atoms and very different sizes are accepted."""
    from paper_2608_12691_amd import alchnb
    p, keep = _params(alchnb, FF, skin=1.0)
    s0, k0 = _system(alchnb, 0, 25.0, types=[], sol=[])
    s1, k1 = _system(alchnb, 5, 25.0)
    s2, k2 = _system(alchnb, 3, 40.0)
    st, ctx = _create(lib, p, [s0, s1, s2])
    assert st == 0
    lib.alch_nb_destroy(ctx)


def test_strerror_and_misc(lib):
    for code in range(8):
        assert lib.alch_nb_strerror(code)
    assert lib.alch_nb_num_variants() >= 4
    assert lib.alch_nb_flops_per_pair(0) > 50
    assert lib.alch_nb_flops_per_pair(1) > lib.alch_nb_flops_per_pair(0)
    offs = (ctypes.c_int32 * 18)()
    assert lib.alch_nb_opes_layout(offs, 18) == 0
    assert offs[0] == 0 and offs[15] == 16 and offs[17] == 16 + 2 * 101
    assert lib.alch_nb_opes_layout(offs, 3) == 1
    assert lib.alch_nb_opes_state_size(100) == 16 + 2 * 101 + 200
    assert lib.alch_nb_opes_state_size(0) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; there is no fallback path."""
    from paper_2608_12691_amd import alchnb
    monkeypatch.setattr(alchnb, "_lib", None)
    monkeypatch.setattr(alchnb, "LIB_PATH", str(tmp_path / "libalchnb.so"))
    with pytest.raises(ImportError):
        alchnb.load()


def test_compute_checked_reacts_to_barrier_timeout_and_capacity():
    """Host logic of the checked call (no GPU): a fused build that timed out
    is redone with one kernel per phase, a list overflow re-plans larger, and
    each retry forces a rebuild; other flags are returned to the caller."""
    from paper_2608_12691_amd import alchnb as A
    ctx = A.Context.__new__(A.Context)
    ctx.auto_capacity = True
    ctx._list_mode = A.LIST_AUTO
    ctx.generation = 0
    flags_seq = [A.FLAG_BARRIER_TIMEOUT, A.FLAG_CAPACITY, A.FLAG_LAMBDA_RANGE]
    calls = []
    ctx.compute = lambda pos, lam, flags, out: calls.append(("compute", flags)) or {}
    ctx.get_flags = lambda: flags_seq.pop(0)

    def set_mode(m):
        calls.append(("mode", m))
        ctx._list_mode = m
    ctx.set_list_mode = set_mode
    ctx.grow_capacity = lambda: calls.append(("grow",))
    res = A.Context.compute_checked(ctx, None, None, flags=A.AUTO_REBUILD)
    assert res["flags"] == A.FLAG_LAMBDA_RANGE
    assert calls == [("compute", A.AUTO_REBUILD), ("mode", A.LIST_PHASES), ("compute", A.FORCE_REBUILD),
                     ("grow",), ("compute", A.FORCE_REBUILD)]
    # a timeout on the per-phase path is not retried again: the flag is returned
    calls.clear()
    flags_seq[:] = [A.FLAG_BARRIER_TIMEOUT]
    assert A.Context.compute_checked(ctx, None, None)["flags"] == A.FLAG_BARRIER_TIMEOUT
    assert calls == [("compute", A.AUTO_REBUILD)]


def test_pme_grid_planning_and_rejections(lib):
    """PME contexts: per-box grids of 2^a 3^b 5^c points >= max(L/spacing, 2 order);
    bad orders, spacings and splitting parameters are refused, oversized grids unsupported."""
    from paper_2608_12691_amd import alchnb
    pme = dict(electrostatics=alchnb.ELEC_PME, pme_order=5, pme_spacing=1.0, dsf_alpha=0.3)
    p, keep = _params(alchnb, FF, **pme)
    s0, k0 = _system(alchnb, 4, 20.0)
    s1, k1 = _system(alchnb, 4, 44.85)
    s2, k2 = _system(alchnb, 0, 23.0, types=[], sol=[])
    st, ctx = _create(lib, p, [s0, s1, s2])
    assert st == 0
    dims = (ctypes.c_int32 * 3)()
    got = []
    for k in range(3):
        assert lib.alch_nb_pme_grid(ctx, k, dims) == 0
        got.append(tuple(dims))
    assert got == [(20, 20, 20), (45, 45, 45), (24, 24, 24)]
    assert lib.alch_nb_pme_grid(ctx, 3, dims) == 1
    nb_pme = ctypes.c_size_t()
    lib.alch_nb_workspace_size(ctx, ctypes.byref(nb_pme))
    lib.alch_nb_destroy(ctx)
    # the same boxes with DSF: no grid, a smaller workspace
    p, keep2 = _params(alchnb, FF)
    st, ctx = _create(lib, p, [s0, s1, s2])
    assert st == 0 and lib.alch_nb_pme_grid(ctx, 0, dims) == 3
    nb = ctypes.c_size_t()
    lib.alch_nb_workspace_size(ctx, ctypes.byref(nb))
    assert nb_pme.value > nb.value + 32 * (20 ** 3 + 45 ** 3)
    lib.alch_nb_destroy(ctx)
    # a coarse spacing still gives 2 order points per edge
    p, keep3 = _params(alchnb, FF, **dict(pme, pme_spacing=50.0, pme_order=6))
    st, ctx = _create(lib, p, [s0])
    assert st == 0 and lib.alch_nb_pme_grid(ctx, 0, dims) == 0 and tuple(dims) == (12, 12, 12)
    lib.alch_nb_destroy(ctx)
    for bad, code in ((dict(pme_order=3), 1), (dict(pme_order=7), 1), (dict(pme_spacing=0.0), 1),
                      (dict(dsf_alpha=0.0), 1), (dict(electrostatics=2), 1), (dict(pme_spacing=0.01), 3)):
        p, keep4 = _params(alchnb, FF, **dict(pme, **bad))
        st, ctx = _create(lib, p, [s0])
        assert st == code, bad
        assert not ctx.value
