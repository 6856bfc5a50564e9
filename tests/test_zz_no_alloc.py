"""rzf_full_noalloc (the full-inversion RZF with the library's fixed device
scratch, for callers that cannot allocate) against rzf_full, through the C ABI:
two calls in a row, the second with a smaller input, on the same stream."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.rzf as orz
from paper_2512_16543_amd import rzf, workload as wl

pytestmark = pytest.mark.gpu


def c64(H):
    return np.asarray(H, dtype=np.complex64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_matches_full_twice():
    ctx = rzf.Context(0, 64 << 20)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    for K, N, seed in ((256, 1024, 1), (48, 100, 2), (64, 256, 3)):
        print(f"no-alloc K={K} N={N}", flush=True)
        H = torch.from_numpy(c64(wl.random_channel(K, N, seed, scale=1.0))).cuda()
        alpha, P = 0.5 + K / 40.0, 1.5
        Wa = torch.empty(N, K, dtype=torch.complex64, device="cuda")
        Wb = torch.full((N, K), 3 + 3j, dtype=torch.complex64, device="cuda")
        ctx.full(H, alpha, P, Wa)
        ctx.sync()
        rzf.full_noalloc(H, alpha, P, Wb, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        assert torch.equal(Wa, Wb), (K, N)       # the same kernels on the same inputs
        Wo = orz.full_rzf(H.cpu().numpy().astype(np.complex128), alpha, P)
        assert rel(Wb.cpu().numpy().astype(np.complex128), Wo) <= 1e-5
    ctx.close()


def test_noalloc_on_a_side_stream_and_errors():
    K, N = 8, 4
    H = torch.from_numpy(c64(wl.random_channel(K, N, 6, scale=1.0))).cuda()   # rank 4 < K
    W = torch.empty(N, K, dtype=torch.complex64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rzf.full_noalloc(H, 0.0, 1.0, W, err, stream=s)   # alpha = 0: singular Gram matrix
    s.synchronize()
    assert int(err.item()) == 1
    L = rzf.lib()
    hp, wp = ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(W.data_ptr())
    assert L.rzf_full_noalloc(None, 257, N, hp, N, 1.0, 1.0, wp, 257, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, K, 4097, hp, 4097, 1.0, 1.0, wp, K, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, K, N, hp, N - 1, 1.0, 1.0, wp, K, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, K, N, None, N, 1.0, 1.0, wp, K, None) == rzf.RZF_E_INVALID
    assert L.rzf_full_noalloc(None, K, N, hp, N, -1.0, 1.0, wp, K, None) == rzf.RZF_E_INVALID
    assert L.rzf_full_noalloc(None, K, N, hp, N, 1.0, 0.0, wp, K, None) == rzf.RZF_E_INVALID
    # a good call on the null stream after the failing one, no error word
    H2 = torch.from_numpy(c64(wl.random_channel(K, 16, 7, scale=1.0))).cuda()
    W2 = torch.empty(16, K, dtype=torch.complex64, device="cuda")
    assert L.rzf_full_noalloc(None, K, 16, ctypes.c_void_p(H2.data_ptr()), 16, 1.0, 1.0,
                              ctypes.c_void_p(W2.data_ptr()), K, None) == rzf.RZF_OK
    torch.cuda.synchronize()
    Wo = orz.full_rzf(H2.cpu().numpy().astype(np.complex128), 1.0, 1.0)
    assert rel(W2.cpu().numpy().astype(np.complex128), Wo) <= 1e-5
