"""GPU parity of the replica exchange (alch_nb_hrex_exchange) against the
FP64 oracle (oracle/hrex.py): the kernel alone on given basis energies, and
the 16-box HREX step (evaluation + exchange) captured as one graph."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import hrex as H
from paper_2608_12691_amd import systems as S

from conftest import workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KT = 0.0019872042586408316 * 298.0


def _margins_ok(log):
    """Every decision is determined far beyond rounding: |ln u + D| > 1e-7."""
    return all(abs(math.log(u) + D) > 1e-7 for _, _, D, u, _ in log if D > 0.0)


def test_exchange_kernel_against_oracle_on_given_energies():
    from paper_2608_12691_amd import alchnb
    w = workload(4)
    ctx = alchnb.from_workload(w, precision=alchnb.FP64, schedule=alchnb.LBF_DSF)
    K, n = len(w.systems), 200
    rng = np.random.Generator(np.random.PCG64(1661))
    terms = np.zeros((K, 10))
    terms[:, 4] = rng.normal(-300.0, 1.5, K)
    terms[:, 5] = rng.normal(40.0, 1.0, K)
    U = rng.uniform(0.0, 1.0, (n, K - 1))
    states = np.linspace(0.0, 1.0, K)
    dev = torch.device("cuda:0")
    so, stats = ctx.hrex_init()
    lam = torch.as_tensor(states, device=dev)
    tt, ls, uu = (torch.as_tensor(a, device=dev) for a in (terms, states, U))
    hist = torch.zeros((n, K), dtype=torch.float64, device=dev)
    for i in range(n):
        ctx.hrex_exchange(tt, ls, so, lam, uu, KT, stats)
        hist[i] = lam
    torch.cuda.synchronize()
    ref = H.Hrex(states, KT)
    want = np.array([ref.exchange(terms[:, 4], terms[:, 5], U[i]) for i in range(n)])
    assert _margins_ok(ref.log)
    assert np.array_equal(hist.cpu().numpy(), want)
    assert np.array_equal(so.cpu().numpy(), ref.state_of)
    st = stats.cpu().numpy()
    assert st[0] == n
    assert np.array_equal(st[1:K], ref.attempts) and np.array_equal(st[K:], ref.accepts)
    assert ref.accepts.sum() > 0 and (ref.accepts < ref.attempts).any()


@pytest.mark.parametrize("precision", [1, 0], ids=["fp64", "fp32"])
def test_hrex_step_in_one_graph(precision):
    """The 16 boxes at lambda_k = k/15 (LBF): evaluation and exchange captured
    once and replayed 30 times; every replay's lambdas equal the oracle's
    exchanges on the oracle's basis energies, and the last replay's outputs
    equal an eager evaluation at the final lambdas bit for bit."""
    from paper_2608_12691_amd import alchnb
    w = workload(4)
    K, n = len(w.systems), 30
    states = np.asarray(w.lambdas, float)
    rng = np.random.Generator(np.random.PCG64(777))
    U = rng.uniform(0.0, 1.0, (n, K - 1))
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = alchnb.from_workload(w, precision=precision, schedule=alchnb.LBF_DSF)
        pos = ctx.positions(w.systems)
        lam = ctx.lambdas(states)
        out = ctx.new_outputs()
        ls = torch.as_tensor(states, device=dev)
        uu = torch.as_tensor(U, device=dev)
        ctx.compute_checked(pos, lam, flags=alchnb.FORCE_REBUILD, out=out)
        so, stats = ctx.hrex_init()
        ctx.capture_begin()
        ctx.compute(pos, lam, flags=alchnb.AUTO_REBUILD, out=out)
        ctx.hrex_exchange(out["terms"], ls, so, lam, uu, KT, stats)
        ctx.capture_end()
    hist = []
    for i in range(n):
        with torch.cuda.stream(stream):
            ctx.launch_step()
        stream.synchronize()
        hist.append(lam.cpu().numpy().copy())
        print("replay %d accepted %d" % (i, int(stats[K:].sum())), flush=True)
    assert ctx.get_flags() == 0
    P = O.Params.of(w, O.LBF)
    bases = np.array([O.evaluate_system(s, w.ff, P, 0.5, forces=False)["terms"][4:6] for s in w.systems])
    ref = H.Hrex(states, KT)
    want = [ref.exchange(bases[:, 0], bases[:, 1], U[i]) for i in range(n)]
    assert _margins_ok(ref.log)
    assert np.array_equal(np.array(hist), np.array(want))
    assert ref.accepts.sum() > 0
    # the last replay's evaluation ran at the lambdas before its exchange
    with torch.cuda.stream(stream):
        eager = alchnb.from_workload(w, precision=precision, schedule=alchnb.LBF_DSF)
        lam_prev = eager.lambdas(hist[-2])
        e_out = eager.compute_checked(eager.positions(w.systems), lam_prev, flags=alchnb.FORCE_REBUILD)
    stream.synchronize()
    for key in ("forces", "terms", "dudl", "n_pairs"):
        assert np.array_equal(out[key].cpu().numpy(), e_out[key].cpu().numpy()), key
