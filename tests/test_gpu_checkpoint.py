"""Checkpoint / resume of a track: an imported track continues exactly as
the exported one (bit-identical precoders and inverses), in the same or in
another context; foreign or truncated blobs are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2512_16543_amd import rzf, workload as wl

pytestmark = pytest.mark.gpu


def walk(K, N, steps, seed, rank=3):
    H = [wl.random_channel(K, N, seed)]
    for t in range(steps):
        H.append(wl.perturbed_channel(H[-1], seed * 1000 + t, rank=rank, scale=0.02))
    return torch.from_numpy(np.asarray(H, dtype=np.complex64)).cuda()


# the last case changes in every direction, so its steps run to d = K and the
# blob carries a large track's full-width basis
@pytest.mark.parametrize("K,N,period,policy,rank", [(24, 80, 4, rzf.KINIT_FIXED, 3), (64, 256, 0, rzf.KINIT_WARM, 3),
                                                    (100, 128, 3, rzf.KINIT_WARM, 3),
                                                    (100, 128, 0, rzf.KINIT_FIXED, 100)])
def test_resume_is_bit_identical(K, N, period, policy, rank):
    Hs = walk(K, N, 9, 5 + K, rank)
    ctx = rzf.Context(0, 64 << 20)
    other = rzf.Context(0, 64 << 20)
    prm = rzf.default_params(seed=9, track_id=2, reset_period=period, kinit_policy=policy)
    a = ctx.init(Hs[0], 0.5 + K / 30.0, prm)
    Wa = torch.empty(N, K, dtype=torch.complex64, device="cuda")
    Wb = torch.empty_like(Wa)
    for t in range(1, 5):
        a.update(Hs[t], 0.95, Wa)
    ctx.sync()
    blob = a.export()
    b1 = ctx.import_track(blob)
    b2 = other.import_track(blob)
    assert (b1.K, b1.N) == (K, N) and b1.query()["t"] == 4
    assert b1.query() == a.query()
    assert torch.equal(b1.inverse(), a.inverse())
    for t in range(5, 10):
        ia = a.update(Hs[t], 0.95, Wa)
        ib = b1.update(Hs[t], 0.95, Wb)
        ctx.sync()
        assert (ia.r, ia.iters, ia.path) == (ib.r, ib.iters, ib.path), t
        assert torch.equal(Wa, Wb), t
        assert torch.equal(a.inverse(), b1.inverse()), t
        b2.update(Hs[t], 0.95, Wb)
        other.sync()
        assert torch.equal(Wa, Wb), t
    for tr in (a, b1, b2):
        tr.destroy()
    ctx.close()
    other.close()


def test_resume_keeps_full_width_basis():
    # the K = 64 track at eta = 0.999 ends every step at d = K, where the SVD
    # starts from the track's stored basis: the blob carries it, so the
    # resumed track (including its re-orthonormalisation schedule) continues
    # bit for bit
    cfg = wl.CONFIGS["c2"]
    Hs = torch.from_numpy(wl.make_track(wl.with_overrides(cfg, steps=14)).snapshots()
                          .astype(np.complex64)).cuda()
    ctx = rzf.Context(0, 64 << 20)
    prm = rzf.default_params(k_init=cfg.k_init, p=cfg.p, seed=cfg.seed, reset_period=0)
    a = ctx.init(Hs[0], cfg.alpha, prm)
    Wa = torch.empty(cfg.N, cfg.K, dtype=torch.complex64, device="cuda")
    Wb = torch.empty_like(Wa)
    for t in range(1, 6):
        a.update(Hs[t], 0.999, Wa)
    ctx.sync()
    b = ctx.import_track(a.export())
    for t in range(6, 15):
        ia = a.update(Hs[t], 0.999, Wa)
        ib = b.update(Hs[t], 0.999, Wb)
        ctx.sync()
        assert (ia.r, ia.iters, ia.path) == (ib.r, ib.iters, ib.path), t
        assert torch.equal(Wa, Wb), t
        assert torch.equal(a.inverse(), b.inverse()), t
        ca, cb = a.counters(), b.counters()
        assert ca["qr_columns"] == cb["qr_columns"], t
        if ia.iters == 6:
            assert ca["qr_columns"] == 7 + 9 + 13 + 21 + 37, t   # no QR at d = K
    a.destroy()
    b.destroy()
    ctx.close()

def test_resume_keeps_narrower_basis():
    # at eta = 0.99 the K = 64 track's steps decide at d = 37 < K: the Jacobi
    # there starts from the sketch's Q turned within its span towards the last
    # such SVD's directions, which the blob carries
    cfg = wl.CONFIGS["c2"]
    Hs = torch.from_numpy(wl.make_track(wl.with_overrides(cfg, steps=12)).snapshots()
                          .astype(np.complex64)).cuda()
    ctx = rzf.Context(0, 64 << 20)
    prm = rzf.default_params(k_init=cfg.k_init, p=cfg.p, seed=cfg.seed, reset_period=0)
    a = ctx.init(Hs[0], cfg.alpha, prm)
    Wa = torch.empty(cfg.N, cfg.K, dtype=torch.complex64, device="cuda")
    Wb = torch.empty_like(Wa)
    for t in range(1, 5):
        a.update(Hs[t], 0.99, Wa)
    ctx.sync()
    b = ctx.import_track(a.export())
    narrow = 0
    for t in range(5, 13):
        ia = a.update(Hs[t], 0.99, Wa)
        ib = b.update(Hs[t], 0.99, Wb)
        ctx.sync()
        assert (ia.r, ia.iters, ia.path) == (ib.r, ib.iters, ib.path), t
        assert torch.equal(Wa, Wb), t
        assert torch.equal(a.inverse(), b.inverse()), t
        ca, cb = a.counters(), b.counters()
        assert (ca["qr_columns"], ca["jacobi_sweeps"]) == (cb["qr_columns"], cb["jacobi_sweeps"]), t
        narrow += min(cfg.k_init * 2 ** (ia.iters - 1) + cfg.p, cfg.K) < cfg.K
    assert narrow > 0
    a.destroy()
    b.destroy()
    ctx.close()


def test_resume_keeps_large_full_width_basis():
    # a K = 256 track (the 32x32-array workload) at eta = 0.999 runs to d = K
    # every step; from its second step the full-width iteration starts from the
    # stored basis instead of a sketch and QR, and the blob carries that basis
    cfg = wl.CONFIGS["c5"]
    Hs = torch.from_numpy(wl.make_track(wl.with_overrides(cfg, steps=7)).snapshots()
                          .astype(np.complex64)).cuda()
    ctx = rzf.Context(0, 256 << 20)
    prm = rzf.default_params(k_init=cfg.k_init, p=cfg.p, seed=cfg.seed, reset_period=0)
    a = ctx.init(Hs[0], cfg.alpha, prm)
    Wa = torch.empty(cfg.N, cfg.K, dtype=torch.complex64, device="cuda")
    Wb = torch.empty_like(Wa)
    for t in range(1, 4):
        a.update(Hs[t], 0.999, Wa)
    ctx.sync()
    b = ctx.import_track(a.export())
    full = 0
    for t in range(4, 8):
        ia = a.update(Hs[t], 0.999, Wa)
        ib = b.update(Hs[t], 0.999, Wb)
        ctx.sync()
        assert (ia.r, ia.iters, ia.path) == (ib.r, ib.iters, ib.path), t
        assert torch.equal(Wa, Wb), t
        assert torch.equal(a.inverse(), b.inverse()), t
        ca, cb = a.counters(), b.counters()
        assert (ca["qr_columns"], ca["jacobi_sweeps"]) == (cb["qr_columns"], cb["jacobi_sweeps"]), t
        ds = [min(cfg.k_init * 2 ** i + cfg.p, cfg.K) for i in range(ia.iters)]
        if ds[-1] == cfg.K:
            # no QR at d = K (and none for the earlier iterations that the
            # full-width sigma_j rule out)
            full += 1
            assert ca["qr_columns"] <= sum(ds[:-1]), t
    assert full > 0
    a.destroy()
    b.destroy()
    ctx.close()


def test_import_rejects_bad_blobs():
    Hs = walk(8, 16, 1, 3)
    ctx = rzf.Context(0, 16 << 20)
    tr = ctx.init(Hs[0], 1.0, rzf.default_params())
    blob = tr.export()
    for bad in (blob[:40], blob[:-8], b"XXXXXXXX" + blob[8:]):
        with pytest.raises(rzf.RzfError) as e:
            ctx.import_track(bad)
        assert e.value.status == rzf.RZF_E_INVALID
    tr.destroy()
    ctx.close()
