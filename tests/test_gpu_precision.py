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
    _assert_recs(recs, tol=TOL[prec], max_forced=1.0)
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
