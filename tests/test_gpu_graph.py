"""Captured steps (rzf_graph_*): replaying a captured step gives bit-identical
results to the eager calls it was captured from.

For each form (one track through rzf_update, a ragged batch through
rzf_update_batch, and the full-inversion calls) a twin set of tracks is
stepped eagerly while the graph's tracks are stepped by replays, with the
snapshots copied into the graph's fixed H buffers between replays and the
eager twin's launches interleaved on the same stream.  The reset period makes
the replays alternate between the Woodbury-step graph and the re-inversion
graph.  Every replay's W, sum rate and final A^-1 must equal the eager ones.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2512_16543_amd import rzf, workload as wl

pytestmark = pytest.mark.gpu

STEPS = 9
P, S2 = 1.0, 0.1


def walk(K, N, steps, seed):
    H = [wl.random_channel(K, N, seed)]
    for t in range(steps):
        H.append(wl.perturbed_channel(H[-1], seed * 1000 + t, rank=2, scale=0.02))
    return torch.from_numpy(np.asarray(H, dtype=np.complex64)).cuda()


@pytest.fixture(scope="module")
def ctx():
    c = rzf.Context(0, 256 << 20)
    yield c
    c.close()


def _pair(ctx, Hs, period):
    mk = lambda: [ctx.init(H[0], 0.3 + H.shape[1] / 25.0,
                           rzf.default_params(seed=3, track_id=i, reset_period=period))
                  for i, H in enumerate(Hs)]
    return mk(), mk()


@pytest.mark.parametrize("sizes,tol", [([(64, 256)], 0.999), ([(16, 64)], 0.9), ([(96, 128)], 0.95),
                                       ([(16, 64), (64, 256), (13, 37), (96, 128)], 0.95)])
def test_update_graph_replays_equal_eager(ctx, sizes, tol):
    Hs = [walk(K, N, STEPS, 40 + i) for i, (K, N) in enumerate(sizes)]
    torch.cuda.synchronize()
    eager, cap = _pair(ctx, Hs, period=4)
    n = len(sizes)
    Hbuf = [torch.empty_like(H[0]) for H in Hs]
    Wbuf = [torch.empty(N, K, dtype=torch.complex64, device="cuda") for K, N in sizes]
    sums = torch.zeros(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = ctx.graph_update(cap, Hbuf, Wbuf, tol, rate=(P, S2, sums))
    We = [torch.empty_like(w) for w in Wbuf]
    sums_e = torch.zeros(n, dtype=torch.float64, device="cuda")
    for t in range(1, STEPS + 1):
        for i in range(n):
            Hbuf[i].copy_(Hs[i][t])
        torch.cuda.synchronize()        # the library's stream does not follow torch's
        g.launch()
        if n == 1:
            eager[0].update(Hs[0][t], tol, We[0], want_info=False)
            ref = [ctx.sum_rate(Hs[0][t], We[0], P, S2)]
        else:
            ctx.update_batch(eager, [H[t] for H in Hs], We, tol)
            ctx.sum_rate_batch([H[t] for H in Hs], We, P, S2, sums=sums_e)
            ctx.sync()
            ref = sums_e.tolist()
        ctx.sync()
        for i in range(n):
            assert torch.equal(We[i], Wbuf[i]), (sizes[i], t)
        assert sums.tolist() == ref, t
    for a, b in zip(eager, cap):
        assert torch.equal(a.inverse(), b.inverse())
        assert a.query()["t"] == b.query()["t"] == STEPS
    # a track stepped outside the graph falls out of its reset schedule
    if n > 1:
        cap[0].update(Hs[0][STEPS], tol, Wbuf[0], want_info=False)
        with pytest.raises(rzf.RzfError):
            g.launch()
    # and cannot be destroyed while the graph exists
    with pytest.raises(rzf.RzfError):
        cap[0].destroy()
    g.destroy()
    for tr in eager + cap:
        tr.destroy()


@pytest.mark.parametrize("sizes,precision", [([(64, 256)], 0), ([(16, 64), (64, 1000), (96, 128)], 0),
                                             ([(40, 100)], rzf.PREC_BF16X3)])
def test_full_graph_replays_equal_eager(ctx, sizes, precision):
    Hs = [walk(K, N, 3, 60 + i) for i, (K, N) in enumerate(sizes)]
    alphas = [0.2 + K / 30.0 for K, _ in sizes]
    Hbuf = [torch.empty_like(H[0]) for H in Hs]
    Wbuf = [torch.empty(N, K, dtype=torch.complex64, device="cuda") for K, N in sizes]
    We = [torch.empty_like(w) for w in Wbuf]
    n = len(sizes)
    sums = torch.zeros(n, dtype=torch.float64, device="cuda")
    sums_e = torch.zeros(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = ctx.graph_full(Hbuf, alphas, 1.5, Wbuf, precision=precision, rate=(1.5, S2, sums))
    for t in range(4):
        for i in range(n):
            Hbuf[i].copy_(Hs[i][t])
        torch.cuda.synchronize()
        g.launch()
        if n == 1 and precision == 0:
            ctx.full(Hs[0][t], alphas[0], 1.5, We[0])
            ref = [ctx.sum_rate(Hs[0][t], We[0], 1.5, S2)]
        else:
            ctx.full_batch([H[t] for H in Hs], alphas, 1.5, We, precision=precision)
            ctx.sum_rate_batch([H[t] for H in Hs], We, 1.5, S2, sums=sums_e)
            ctx.sync()
            ref = sums_e.tolist()
        for i in range(n):
            assert torch.equal(We[i], Wbuf[i]), (sizes[i], t)
        assert sums.tolist() == ref, t
    g.destroy()


# ------------------------------------------------------------- launch tuning

def test_batched_precoder_rows_change_no_result(ctx):
    # a batch of K <= 64 tracks with 32, 64 and 256 precoder rows per workgroup
    # (a batch this small takes the single-track entry)
    sizes = [(64, 256), (16, 1000), (40, 520), (1, 8)]
    Hs = [walk(K, N, 0, 95 + i)[0] for i, (K, N) in enumerate(sizes)]
    outs = []
    for pb in (32, 64, 256):
        ctx.tune_table([{"K": K, "N": N, "precoder_rows": pb, "batch_precoder_rows": pb} for K, N in sizes])
        Ws = [torch.empty(N, K, dtype=torch.complex64, device="cuda") for K, N in sizes]
        ctx.full_batch(Hs, [0.4] * len(sizes), 1.0, Ws)
        ctx.sync()
        outs.append(Ws)
    ctx.tune_table([])
    for Ws in outs[1:]:
        for a, b in zip(Ws, outs[0]):
            assert torch.equal(a, b)


def test_batched_fused_normalisation(ctx):
    # a batch of >= 128 tracks with N <= 256 rows: with 256 precoder rows per
    # workgroup each workgroup holds a whole track and normalises W itself
    # (and advances the track's step); with 32 a second kernel does both.
    # Updates over three steps and a full-inversion batch must agree bit for bit.
    rng = np.random.default_rng(7)
    sizes = [(64, 256)] + [(int(rng.integers(1, 65)), int(rng.integers(8, 257))) for _ in range(135)]
    Hs = [walk(K, N, 3, 500 + i) for i, (K, N) in enumerate(sizes)]
    results = []
    for pb in (256, 32):
        ctx.tune_table([{"K": 64, "N": 256, "precoder_rows": pb, "batch_precoder_rows": pb}])
        trs = [ctx.init(H[0], 0.3 + H.shape[1] / 25.0, rzf.default_params(seed=3, track_id=i, reset_period=0))
               for i, H in enumerate(Hs)]
        Ws = [torch.empty(N, K, dtype=torch.complex64, device="cuda") for K, N in sizes]
        outs = []
        for t in range(1, 4):
            ctx.update_batch(trs, [H[t] for H in Hs], Ws, 0.95)
            ctx.sync()
            outs.append([w.clone() for w in Ws] + [tr.inverse() for tr in trs])
        Wf = [torch.empty_like(w) for w in Ws]
        ctx.full_batch([H[3] for H in Hs], [0.4] * len(Hs), 1.5, Wf)
        ctx.sync()
        outs.append(Wf)
        results.append(outs)
        for tr in trs:
            tr.destroy()
    ctx.tune_table([])
    for step_a, step_b in zip(*results):
        for a, b in zip(step_a, step_b):
            assert torch.equal(a, b)


def test_tuning_knobs_change_no_result(ctx):
    # the precoder's rows per workgroup and the single-track sum rate's
    # spread over workgroups are launch choices only
    for K, N in [(64, 256), (16, 1000), (40, 520), (96, 300)]:
        H = walk(K, N, 0, 90)[0]
        outs = []
        for pb, ns in [(64, 1), (32, 4), (256, 8), (64, 2)]:
            ctx.tune_table([{"K": K, "N": N, "precoder_rows": pb, "batch_precoder_rows": pb, "rate_splits": ns}])
            W = torch.empty(N, K, dtype=torch.complex64, device="cuda")
            r = torch.empty(K, dtype=torch.float32, device="cuda")
            ctx.full(H, 0.5, 1.0, W)
            R = ctx.sum_rate(H, W, 1.0, 0.1, r)
            outs.append((W, r, R))
        ctx.tune_table([])
        for W, r, R in outs[1:]:
            assert torch.equal(W, outs[0][0]) and torch.equal(r, outs[0][1]) and R == outs[0][2], (K, N)


def test_tuning_table_checks_entries(ctx):
    with pytest.raises(rzf.RzfError):
        ctx.tune_table([{"K": 64, "N": 256, "precoder_rows": 48}])
    with pytest.raises(rzf.RzfError):
        ctx.tune_table([{"K": 0, "N": 256}])
    with pytest.raises(rzf.RzfError):
        ctx.tune_table([{"K": 64, "N": 256, "rate_splits": 9}])
    ctx.tune_table([])
