"""The allocation-free binding (alch_nb_bind_static) against the workspace
binding: identical outputs on two calls in a row (the 8,973-atom box, then
the smaller 633-atom box), the evicted context refused, an oversized
context rejected."""
import ctypes

import numpy as np
import pytest

from conftest import workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(w, precision):
    from paper_2608_12691_amd import alchnb
    ref = alchnb.from_workload(w, precision=precision)
    sta = alchnb.from_workload(w, precision=precision, static_scratch=True)
    assert sta.ws is None and sta.get_stats()["n_atoms"] == w.n_atoms
    return ref, sta


def _run(ctx, pos, lam, flags):
    out = ctx.compute(pos, lam, flags=flags)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "fp64"])
def test_bind_static_matches_workspace_binding(precision):
    from paper_2608_12691_amd import alchnb
    from paper_2608_12691_amd import systems as S
    prev = None
    for k in (2, 1):  # the second call's input is the smaller box
        w = workload(k)
        print("bind_static precision %d config %d (%d atoms)" % (precision, k, w.n_atoms), flush=True)
        ref, sta = _pair(w, precision)
        if prev is not None:
            # the earlier static context lost the array to this one
            with pytest.raises(alchnb.AlchNBError) as ei:
                prev.compute(prev._last_pos, prev._last_lam)
            assert ei.value.status == 6
        s = w.systems[0]
        walk = S.perturbation_walk(s, 3, 0.02, seed=91 + k)
        for t, lamv in enumerate((0.3, 0.8, 0.55)):
            pos = ref.positions(walk[t])
            lam = ref.lambdas([lamv])
            flags = alchnb.FORCE_REBUILD if t == 0 else alchnb.AUTO_REBUILD
            a = _run(ref, pos, lam, flags)
            b = _run(sta, pos, lam, flags)
            for key in ("terms", "forces", "dudl", "n_pairs"):
                assert np.array_equal(a[key], b[key]), (k, t, key)
        assert ref.get_flags() == 0 and sta.get_flags() == 0
        sta._last_pos, sta._last_lam = pos, lam
        ref.close()
        if prev is not None:
            prev.close()
        prev = sta
    prev.close()


def test_bind_static_rejects_an_oversized_workspace():
    """The 39,548-atom octanol box needs ~97 MiB of workspace: beyond the array."""
    from paper_2608_12691_amd import alchnb
    w = workload(3)
    with pytest.raises(alchnb.AlchNBError) as ei:
        alchnb.from_workload(w, static_scratch=True)
    assert ei.value.status == 8
    lib = alchnb.load()
    assert lib.alch_nb_strerror(8).decode().startswith("workspace larger")
