"""BF16 and BF16x3 operand options of the Gram and precoder products.

Tolerances follow from the operand rounding: BF16 keeps 8 significant bits
(relative rounding error 2^-9 per operand, about 2^-8 per product), so the
Gram matrix, A^-1 and W carry relative errors of a few 1e-3, times the
condition number of the regularised Gram matrix (below 5 in these inputs):
TOL_BF16 = 2e-2.  BF16x3 (hi*hi + hi*lo + lo*hi) keeps about 16 bits
(2^-16 per product): TOL_BF16X3 = 1e-4.  Rank decisions taken on a
perturbed Delta A may part from the FP64 oracle's near eta; the one-step
parity replays the GPU's decision when a cumulative energy ratio lies within
the band of eta (1e-2 for BF16, the FP32 band for BF16x3).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.rzf as orz
from paper_2512_16543_amd import rzf, workload as wl
from tests.test_gpu_parity import TIE_BAND, _assert_recs, c64, dev, host, rel, run_snapshots

pytestmark = pytest.mark.gpu

TOL = {rzf.PREC_BF16: 2e-2, rzf.PREC_BF16X3: 1e-4}
BAND = {rzf.PREC_BF16: 1e-2, rzf.PREC_BF16X3: TIE_BAND}
# sigma_j^2 against the oracle's, relative to ||Delta A||_F^2: Delta A carries
# the operands' relative rounding (2^-8 per BF16 product, 2^-16 per BF16x3
# one), and sigma_j^2 moves by twice that times sigma_1 ||Delta A||_F
SIG = {rzf.PREC_BF16: 2e-2, rzf.PREC_BF16X3: 1e-4}
# relative sum rate of eq. (15) for the reduced-precision operand paths
TOL_RATE = 1e-3


@pytest.fixture(scope="module")
def ctx():
    c = rzf.Context(0, 512 << 20)
    yield c
    c.close()


@pytest.mark.parametrize("prec", [rzf.PREC_BF16, rzf.PREC_BF16X3])
@pytest.mark.parametrize("K,N", [(16, 64), (64, 256), (13, 37), (128, 1024), (256, 1024), (100, 70)])
def test_full_batch_precision(ctx, prec, K, N):
    H = c64(wl.random_channel(K, N, 90 + K)).astype(np.complex128)
    alpha, P = 0.5 + K / 40.0, 1.0
    W = torch.empty(N, K, dtype=torch.complex64, device="cuda")
    ctx.full_batch([dev(H)], [alpha], P, [W], precision=prec)
    ctx.sync()
    err = rel(host(W), orz.full_rzf(H, alpha, P))
    print(f"prec={prec} K={K} N={N} W rel err {err:.2e}", flush=True)
    assert err <= TOL[prec]
    # the FP32 operands give a strictly closer result
    W32 = torch.empty_like(W)
    ctx.full_batch([dev(H)], [alpha], P, [W32], precision=rzf.PREC_FP32)
    ctx.sync()
    assert rel(host(W32), orz.full_rzf(H, alpha, P)) < err


def _walk(K, N, steps, seed, rank=3, scale=0.02):
    H = [wl.random_channel(K, N, seed)]
    for t in range(steps):
        H.append(wl.perturbed_channel(H[-1], seed * 1000 + t, rank=rank, scale=scale))
    return c64(np.asarray(H)).astype(np.complex128)


@pytest.mark.parametrize("prec", [rzf.PREC_BF16, rzf.PREC_BF16X3])
@pytest.mark.parametrize("K,N", [(32, 128), (64, 256), (128, 256)])
def test_update_precision(ctx, prec, K, N):
    Hs = _walk(K, N, 5, 40 + K)
    d = dict(k_init=2, p=5, P=1.0, seed=7, track_id=K, reset_period=0, precision=prec)
    recs = run_snapshots(ctx, Hs, 0.4 + K / 40.0, d, 0.999, tie_band=BAND[prec])
    print([(r["path"], r["r"], round(r["ainv"], 7), round(r["w"], 7), round(r["e"], 7)) for r in recs], flush=True)
    _assert_recs(recs, tol=TOL[prec], max_forced=0.4, step_eps=TOL[prec], sig_tol=SIG[prec])
    # ||Delta A||_F^2 from the BF16 products stays within the operand precision
    assert all(r["e"] < 4 * TOL[prec] for r in recs)


def test_batch_mixed_precision_equals_alone(ctx):
    sizes = [(32, 64, rzf.PREC_BF16), (64, 256, rzf.PREC_BF16X3), (100, 128, rzf.PREC_FP32),
             (128, 256, rzf.PREC_BF16)]
    steps = 3
    Hs = [_walk(K, N, steps, 70 + i) for i, (K, N, _) in enumerate(sizes)]
    dv = [torch.from_numpy(c64(H)).cuda() for H in Hs]

    def make():
        return [ctx.init(d[0], 0.3 + K / 20.0, rzf.default_params(seed=5, track_id=i, precision=pr))
                for i, (d, (K, N, pr)) in enumerate(zip(dv, sizes))]

    alone, batch = make(), make()
    Wa = [torch.empty(N, K, dtype=torch.complex64, device="cuda") for K, N, _ in sizes]
    Wb = [torch.empty_like(w) for w in Wa]
    for t in range(1, steps + 1):
        for tr, d, w in zip(alone, dv, Wa):
            tr.update(d[t], 0.95, w)
        ctx.update_batch(batch, [d[t] for d in dv], Wb, 0.95)
        ctx.sync()
        for i in range(len(sizes)):
            assert torch.equal(Wa[i], Wb[i]), (t, sizes[i])
    for tr in alone + batch:
        tr.destroy()


def test_invalid_precision_rejected(ctx):
    H = dev(c64(wl.random_channel(8, 16, 1)))
    with pytest.raises(rzf.RzfError) as e:
        ctx.init(H, 1.0, rzf.default_params(precision=3))
    assert e.value.status == rzf.RZF_E_INVALID
    W = torch.empty(16, 8, dtype=torch.complex64, device="cuda")
    with pytest.raises(rzf.RzfError) as e:
        ctx.full_batch([H], [1.0], 1.0, [W], precision=-1)
    assert e.value.status == rzf.RZF_E_INVALID


@pytest.mark.parametrize("prec", [rzf.PREC_BF16, rzf.PREC_BF16X3])
def test_sum_rate_parity_precision(ctx, prec):
    # the K = 64, N = 256 pass with BF16 (or BF16x3) Gram and precoder
    # operands: each step's sum rate (eq. (15), scored on the snapshot itself)
    # within 1e-3 of the oracle's, from the GPU's own rzf_sum_rate and from
    # the GPU precoder scored in FP64; rank decisions replayed only at ties,
    # and not on most steps
    cfg = wl.CONFIGS["c2"]
    Hs = c64(wl.make_track(wl.with_overrides(cfg, steps=16)).snapshots()).astype(np.complex128)
    d = dict(k_init=cfg.k_init, p=cfg.p, P=cfg.P, seed=cfg.seed, track_id=0, reset_period=8, precision=prec)
    tr = ctx.init(dev(Hs[0]), cfg.alpha, rzf.default_params(**d))
    ot = orz.OracleTrack(Hs[0], orz.TrackParams(alpha=cfg.alpha, P=cfg.P, k_init=cfg.k_init, p=cfg.p,
                                                reset_period=8, seed=cfg.seed, track_id=0))
    W = torch.empty(cfg.N, cfg.K, dtype=torch.complex64, device="cuda")
    worst_gpu, worst_host, forced = 0.0, 0.0, 0
    for t in range(1, len(Hs)):
        st = ot.export_state()
        st["Ainv"] = host(tr.inverse())
        st["last_r"] = tr.query()["last_r"]
        ot.import_state(st)
        Ht = dev(Hs[t])
        info = tr.update(Ht, cfg.eta, W)
        R_gpu = ctx.sum_rate(Ht, W, cfg.P, cfg.sigma2)
        Wo, io = ot.update(Hs[t], cfg.eta)
        if (info.r, info.iters, info.path) != (io.r, io.iters, io.path):
            forced += 1
            ot.import_state(st)
            Wo, io = ot.update(Hs[t], cfg.eta, force_iters=info.iters, force_r=info.r)
        _, R_o = orz.sum_rate(Hs[t], Wo, cfg.P, cfg.sigma2)
        _, R_h = orz.sum_rate(Hs[t], host(W), cfg.P, cfg.sigma2)
        worst_gpu = max(worst_gpu, abs(R_gpu - R_o) / R_o)
        worst_host = max(worst_host, abs(R_h - R_o) / R_o)
    tr.destroy()
    print(f"prec={prec}: sum-rate rel err {worst_gpu:.2e} (rzf_sum_rate) {worst_host:.2e} (FP64 scoring), "
          f"forced {forced}/{len(Hs) - 1}", flush=True)
    assert worst_gpu <= TOL_RATE and worst_host <= TOL_RATE
    assert forced <= (len(Hs) - 1) // 4
