"""GPU edge cases of Alg. 2 against the oracle: a singular Woodbury capacitance
(the nonsingularity assumption under eq. (12), Sec. III), non-finite
snapshots, and device errors of asynchronous work surviving synchronous calls.
"""
import struct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.rzf as orz
from paper_2512_16543_amd import rzf, workload as wl
from tests.test_gpu_parity import TOL_FP32, _oracle_params_a, c64, dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = rzf.Context(0, 128 << 20)
    yield c
    c.close()


def _blob_with_inverse(blob: bytes, M: np.ndarray) -> bytes:
    """A checkpoint blob whose stored inverse is replaced by M (the inverse
    follows the header, K x K complex64 row-major)."""
    hdr = struct.unpack_from("<I", blob, 12)[0]
    raw = c64(M).tobytes()
    return blob[:hdr] + raw + blob[hdr + len(raw):]


def test_singular_capacitance_falls_back(ctx):
    # H0 has a silent antenna n0; H1 lets user k hear it with gain 1, so
    # Delta A = e_k e_k^H exactly (also in FP32).  The stored inverse is set to
    # M = I - 2 e_k e_k^H: the rank-1 Woodbury capacitance
    # 1 / sigma + v^H M u = 1 - 1 vanishes (the matrix it would invert,
    # M^-1 + e_k e_k^H, is singular), so both sides must invert A' directly.
    K, N, k, n0, alpha = 8, 16, 2, 5, 1.0
    H0 = c64(wl.random_channel(K, N, 3, scale=1.0)).astype(np.complex128)
    H0[:, n0] = 0.0
    H1 = H0.copy()
    H1[k, n0] = 1.0
    M = np.eye(K, dtype=np.complex128)
    M[k, k] = -1.0
    d = dict(k_init=2, p=5, P=1.0, seed=9, track_id=0, reset_period=0)
    base = ctx.init(dev(H0), alpha, rzf.default_params(**d))
    tr = ctx.import_track(_blob_with_inverse(base.export(), M))
    base.destroy()
    np.testing.assert_array_equal(host(tr.inverse()), M)
    ot = orz.OracleTrack(H0, _oracle_params_a(alpha, d))
    st = ot.export_state()
    st["Ainv"] = M
    ot.import_state(st)
    W = torch.empty(N, K, dtype=torch.complex64, device="cuda")
    info = tr.update(dev(H1), 0.99, W)
    ctx.sync()
    Wo, io = ot.update(H1, 0.99)
    assert io.path == orz.PATH_FULL_SINGULAR and io.r == 1, io
    assert (info.path, info.r, info.iters) == (orz.PATH_FULL_SINGULAR, 1, 1), info.as_dict()
    assert rel(host(tr.inverse()), np.linalg.inv(orz.gram(H1, alpha))) <= TOL_FP32
    assert rel(host(W), Wo) <= TOL_FP32
    # the track goes on normally from the direct inverse
    H2 = c64(wl.perturbed_channel(H1, 4, 1, 0.05)).astype(np.complex128)
    info = tr.update(dev(H2), 0.99, W)
    ctx.sync()
    Wo, io = ot.update(H2, 0.99)
    assert (info.r, info.path) == (io.r, io.path) == (info.r, orz.PATH_WB)
    assert rel(host(W), Wo) <= TOL_FP32
    tr.destroy()


@pytest.mark.parametrize("K,N", [(16, 64), (96, 128)])
def test_nonfinite_snapshot_keeps_state(ctx, K, N):
    # NaN at step 2 (an update step) and at step 6 (a reset step, period 3):
    # each gives RZF_E_NONFINITE at sync and a NOOP record, and leaves the
    # track as it was, so the steps after it match the oracle, which skips such
    # a snapshot the same way
    H = [c64(wl.random_channel(K, N, 50 + K, scale=1.0)).astype(np.complex128)]
    for t in range(8):
        H.append(c64(wl.perturbed_channel(H[-1], 70 + t, 2, 0.02)).astype(np.complex128))
    bad = {2, 6}
    for t in bad:
        H[t] = H[t].copy()
        H[t][1, 3] = np.nan
    alpha = 0.5 + K / 40.0
    d = dict(k_init=2, p=5, P=1.0, seed=13, track_id=K, reset_period=3)
    tr = ctx.init(dev(H[0]), alpha, rzf.default_params(**d))
    ot = orz.OracleTrack(H[0], _oracle_params_a(alpha, d))
    W = torch.empty(N, K, dtype=torch.complex64, device="cuda")
    for t in range(1, 9):
        print(f"K={K} step {t}", flush=True)
        info = tr.update(dev(H[t]), 0.999, W)
        st = ctx.sync_status()
        Wo, io = ot.update(H[t], 0.999)
        if t in bad:
            assert st == rzf.RZF_E_NONFINITE, t
            assert info.path == rzf.PATH_NOOP and info.r == 0 and np.isnan(info.dA_fro2), info.as_dict()
            assert io.path == orz.PATH_NOOP
            continue
        assert st == rzf.RZF_OK, t
        assert (info.r, info.iters, info.path) == (io.r, io.iters, io.path), (t, info.as_dict(), io)
        assert rel(host(tr.inverse()), ot.Ainv) <= TOL_FP32, t
        assert rel(host(W), Wo) <= TOL_FP32, t
    q = tr.query()
    assert (q["t"], q["since_reset"]) == (8, ot.since_reset)
    tr.destroy()


def test_async_error_survives_synchronous_calls(ctx):
    # a NaN snapshot's error is recorded asynchronously; rzf_init of another
    # track (synchronous) succeeds and leaves it pending for rzf_sync
    K, N = 8, 16
    H0 = c64(wl.random_channel(K, N, 5, scale=1.0)).astype(np.complex128)
    tr = ctx.init(dev(H0), 1.0, rzf.default_params())
    bad = H0.copy()
    bad[0, 0] = np.inf
    W = torch.empty(N, K, dtype=torch.complex64, device="cuda")
    tr.update(dev(bad), 0.99, W)
    other = ctx.init(dev(H0), 1.0, rzf.default_params())
    blob = other.export()
    third = ctx.import_track(blob)
    assert ctx.sync_status() == rzf.RZF_E_NONFINITE
    assert ctx.sync_status() == rzf.RZF_OK
    for x in (tr, other, third):
        x.destroy()


def test_switch_beyond_workspace_refused(ctx):
    H = dev(c64(wl.random_channel(64, 80, 1)))
    with pytest.raises(rzf.RzfError) as e:
        ctx.init(H, 1.0, rzf.default_params(switch_ratio=0.75))
    assert e.value.status == rzf.RZF_E_INVALID
    with pytest.raises(rzf.RzfError) as e:
        ctx.init(H, 1.0, rzf.default_params(k_init=300))
    assert e.value.status == rzf.RZF_E_INVALID
    tr = ctx.init(H, 1.0, rzf.default_params(switch_ratio=0.5))
    tr.destroy()
