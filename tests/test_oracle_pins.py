"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: a
brute-force loop on tiny inputs, a textbook identity, a closed form, a
different library routine, or a printed value.  `test_oracle_mutants.py`
plants plausible mistakes in copies of the oracle and checks that these pins
catch them.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import oracle.rzf as orz
from oracle import philox
from paper_2512_16543_amd import workload as wl


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------- sketch RNG

def _read_kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x64_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((tuple(w[0:4]), tuple(w[4:6]), tuple(w[6:10])))
    return rows


def test_philox_known_answers(golden_dir):
    rows = _read_kat(golden_dir)
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert philox.philox4x64_scalar(ctr, key) == out
        v = philox.philox4x64(np.array([ctr], dtype=np.uint64), key)[0]
        assert tuple(int(x) for x in v) == out


def _numpy_block(ctr, key):
    """numpy's Philox (an independent implementation) at one counter block."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)          # numpy increments before it generates
    cw = [(c >> (64 * i)) & philox.MASK64 for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(cw, dtype=np.uint64))
    return tuple(int(x) for x in bg.random_raw(4))


def test_philox_matches_numpy_bitgenerator():
    rng = np.random.default_rng(7)
    ctrs = rng.integers(0, 2 ** 63, size=(64, 4), dtype=np.uint64)
    key = (int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 2 ** 63)))
    vec = philox.philox4x64(ctrs, key)
    for c, v in zip(ctrs, vec):
        c = tuple(int(x) for x in c)
        assert tuple(int(x) for x in v) == _numpy_block(c, key)
        assert philox.philox4x64_scalar(c, key) == _numpy_block(c, key)


def test_sketch_addressing_independent_of_shape():
    big = philox.draw_sketch(3, 1, 17, 2, 40, 12)
    small = philox.draw_sketch(3, 1, 17, 2, 11, 5)
    np.testing.assert_array_equal(big[:11, :5], small)
    # a different iteration, step or track gives a different matrix
    assert not np.allclose(philox.draw_sketch(3, 1, 17, 3, 11, 5), small)
    assert not np.allclose(philox.draw_sketch(3, 1, 18, 2, 11, 5), small)
    assert not np.allclose(philox.draw_sketch(3, 2, 17, 2, 11, 5), small)


def test_sketch_entry_words():
    # entry (i, j) takes words 0,1 (even i) or 2,3 (odd i) of block q=(1024 j + i)>>1
    w = philox.sketch_words(5, 9, 4, 1, 6, 3)
    for i in range(6):
        for j in range(3):
            q = (1024 * j + i) >> 1
            blk = philox.philox4x64_scalar((q, 1, 4, 0), (5, 9))
            want = (blk[0], blk[1]) if i % 2 == 0 else (blk[2], blk[3])
            assert (int(w[i, j, 0]), int(w[i, j, 1])) == want


def test_sketch_is_standard_complex_gaussian():
    # Alg. 1 draws Omega with i.i.d. CN(0,1) entries
    z = np.concatenate([philox.draw_sketch(11, 0, t, 1, 1024, 8).ravel() for t in range(12)])
    n = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 5.0 / math.sqrt(n)
    assert abs(np.mean(z * z)) < 5.0 / math.sqrt(n)            # circular
    assert abs(np.var(z.real) - 0.5) < 5.0 / math.sqrt(n)
    assert abs(np.var(z.imag) - 0.5) < 5.0 / math.sqrt(n)
    # |z|^2 ~ Exp(1) and angle ~ U[0, 2 pi)
    assert scipy.stats.kstest(np.abs(z) ** 2, "expon").pvalue > 1e-3
    assert scipy.stats.kstest((np.angle(z) + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
    # neighbouring entries uncorrelated
    zz = philox.draw_sketch(11, 0, 0, 1, 1024, 64)
    c = np.mean(zz[:-1, :] * zz[1:, :].conj())
    assert abs(c) < 5.0 / math.sqrt(zz.size)


# ------------------------------------------------------------------- Gram

def test_gram_bruteforce():
    rng = np.random.default_rng(1)
    K, N, alpha = 3, 5, 0.7
    H = crandn(rng, K, N)
    A = orz.gram(H, alpha)
    for i in range(K):
        for j in range(K):
            s = sum(H[i, n] * H[j, n].conjugate() for n in range(N))
            if i == j:
                s += alpha
            assert abs(A[i, j] - s) < 1e-13


def test_gram_hermitian_positive_definite():
    rng = np.random.default_rng(2)
    for K, N, alpha in [(4, 2, 0.3), (8, 16, 1.0), (16, 8, 1e-3)]:
        A = orz.gram(crandn(rng, K, N), alpha)
        np.testing.assert_allclose(A, A.conj().T, atol=0)
        assert np.linalg.eigvalsh(A).min() >= alpha * (1 - 1e-10)
        np.linalg.cholesky(A)


def test_gram_correction_bruteforce():
    rng = np.random.default_rng(3)
    K, N = 3, 4
    H, dH = crandn(rng, K, N), crandn(rng, K, N)
    dA = orz.gram_correction(H, dH)
    for i in range(K):
        for j in range(K):
            s = 0j
            for n in range(N):
                s += H[i, n] * dH[j, n].conjugate()
                s += dH[i, n] * H[j, n].conjugate()
                s += dH[i, n] * dH[j, n].conjugate()
            assert abs(dA[i, j] - s) < 1e-13


def test_gram_correction_equals_gram_difference():
    # eq. (9): A' = A + Delta A
    rng = np.random.default_rng(4)
    for K, N in [(5, 9), (16, 64)]:
        H, dH = crandn(rng, K, N), 1e-2 * crandn(rng, K, N)
        lhs = orz.gram(H + dH, 0.4)
        rhs = orz.gram(H, 0.4) + orz.gram_correction(H, dH)
        assert rel(lhs, rhs) < 1e-14
        dA = orz.gram_correction(H, dH)
        np.testing.assert_allclose(dA, dA.conj().T, atol=1e-15)


# --------------------------------------------------------------- inversion

def test_direct_inverse():
    rng = np.random.default_rng(5)
    A = orz.gram(crandn(rng, 12, 20), 0.5)
    Ai = orz.direct_inverse(A)
    assert rel(A @ Ai, np.eye(12)) < 1e-14
    # Cholesky solve (a different LAPACK route) agrees
    c = scipy.linalg.cho_factor(A)
    assert rel(Ai, scipy.linalg.cho_solve(c, np.eye(12))) < 1e-13


# -------------------------------------------------------------------- arSVD

def _draw(seed, t=1):
    return lambda i, K, d: philox.draw_sketch(seed, 0, t, i, K, d)


def _hermitian_test_matrix(rng, K, spectrum):
    X = crandn(rng, K, K)
    Q, _ = np.linalg.qr(X)
    return (Q * spectrum) @ Q.conj().T


def test_arsvd_full_dimension_matches_eigenvalues():
    # with d = K the sketch spans everything: sigma(B) = |eig(Delta A)|
    rng = np.random.default_rng(6)
    K = 12
    dA = orz.gram_correction(crandn(rng, K, 30), 0.1 * crandn(rng, K, 30))
    res = orz.arsvd(dA, 0.9, k_init=K, p=0, i_max=1, draw=_draw(1))
    assert res.d == K
    ev = np.sort(np.abs(np.linalg.eigvalsh(dA)))[::-1]
    np.testing.assert_allclose(res.sigma, ev, rtol=1e-12, atol=1e-14 * ev[0])


def test_arsvd_eckart_young_residual():
    # truncation residual of the exact SVD is the discarded energy
    rng = np.random.default_rng(7)
    K = 10
    dA = _hermitian_test_matrix(rng, K, np.array([5, -4, 3, 2, -1, .5, .2, -.1, .05, .01]))
    for eta in (0.5, 0.9, 0.99):
        res = orz.arsvd(dA, eta, k_init=K, p=0, i_max=1, draw=_draw(2))
        approx = (res.U * res.s) @ res.V.conj().T
        resid = orz.fro2(dA - approx)
        tail = float(np.sum(res.sigma[res.r:] ** 2))
        assert abs(resid - tail) < 1e-12 * orz.fro2(dA)


def test_arsvd_rank_is_minimal():
    rng = np.random.default_rng(8)
    K = 20
    spec = np.array([1.0 / (1 + j) ** 1.5 for j in range(K)]) * np.where(np.arange(K) % 3, 1, -1)
    dA = _hermitian_test_matrix(rng, K, spec)
    E = orz.fro2(dA)
    for eta in (0.3, 0.6, 0.8, 0.95, 0.999):
        res = orz.arsvd(dA, eta, k_init=2, p=5, i_max=4, draw=_draw(3))
        c = np.cumsum(res.sigma ** 2)
        if res.r < res.d or c[-1] >= eta * E:
            assert c[res.r - 1] >= eta * E
            if res.r > 1:
                assert c[res.r - 2] < eta * E


def test_arsvd_exact_for_low_rank_perturbation():
    # a rank-1 dH gives rank(Delta A) <= 2 <= d: the sketch is exact
    rng = np.random.default_rng(9)
    K, N = 16, 40
    H = crandn(rng, K, N)
    dH = 1e-2 * np.outer(crandn(rng, K), crandn(rng, N))
    dA = orz.gram_correction(H, dH)
    assert np.linalg.matrix_rank(dA, tol=1e-12 * np.linalg.norm(dA)) == 2
    res = orz.arsvd(dA, 0.999999, k_init=2, p=5, i_max=4, draw=_draw(4))
    assert res.iters == 1 and res.r <= 2
    approx = (res.U * res.s) @ res.V.conj().T
    assert rel(approx, dA) < 1e-6


def test_arsvd_factors_orthonormal():
    rng = np.random.default_rng(10)
    K = 24
    dA = orz.gram_correction(crandn(rng, K, 64), 0.05 * crandn(rng, K, 64))
    res = orz.arsvd(dA, 0.95, k_init=2, p=5, i_max=5, draw=_draw(5))
    r = res.r
    assert rel(res.U.conj().T @ res.U, np.eye(r)) < 1e-12
    assert rel(res.V.conj().T @ res.V, np.eye(r)) < 1e-12
    assert np.all(np.diff(res.s) <= 0) and np.all(res.s > 0)


def test_arsvd_doubling_schedule():
    # Alg. 1: d = min(k0 + p, K), k0 doubling from k_init on each failure
    rng = np.random.default_rng(11)
    K = 64
    dA = _hermitian_test_matrix(rng, K, np.linspace(1, 0.5, K))   # flat: needs d = K
    seen = []

    def draw(i, KK, d):
        seen.append((i, d))
        return philox.draw_sketch(6, 0, 1, i, KK, d)
    res = orz.arsvd(dA, 0.999, k_init=2, p=5, i_max=orz.default_imax(K, 2, 5), draw=draw)
    assert seen == [(1, 7), (2, 9), (3, 13), (4, 21), (5, 37), (6, 64)]
    assert res.iters == 6 and res.d == 64


def test_arsvd_fall_through_returns_all_d():
    rng = np.random.default_rng(12)
    K = 32
    dA = _hermitian_test_matrix(rng, K, np.linspace(1, 0.9, K))
    res = orz.arsvd(dA, 0.99, k_init=2, p=1, i_max=2, draw=_draw(7))
    assert res.iters == 2 and res.d == 5 and res.r == 5 and res.U.shape == (K, 5)


def test_arsvd_zero_correction():
    res = orz.arsvd(np.zeros((8, 8), complex), 0.9, 2, 5, 3, _draw(8))
    assert res.r == 0 and res.iters == 0


def test_arsvd_halko_martinsson_tropp_bound():
    # E ||(I - Q Q^H) A||_F <= sqrt(1 + k/(p-1)) (sum_{j>k} sigma_j^2)^1/2
    # (Halko, Martinsson, Tropp 2011, Thm. 10.5), checked on the seed average.
    rng = np.random.default_rng(13)
    K, k, p = 48, 6, 4
    spec = 0.6 ** np.arange(K)
    A = _hermitian_test_matrix(rng, K, spec)
    errs = []
    for s in range(40):
        Om = philox.draw_sketch(100 + s, 0, 0, 1, K, k + p)
        Q, _ = np.linalg.qr(A @ Om)
        errs.append(np.linalg.norm(A - Q @ (Q.conj().T @ A)))
    bound = math.sqrt(1 + k / (p - 1)) * math.sqrt(np.sum(spec[k:] ** 2))
    assert np.mean(errs) <= bound


# ----------------------------------------------------------------- Woodbury

def _hpd(rng, K):
    return orz.gram(crandn(rng, K, 2 * K), 0.5)


def test_woodbury_exact_identity():
    # the output is the exact inverse of the rank-r corrected matrix
    rng = np.random.default_rng(14)
    K, r = 16, 5
    A = _hpd(rng, K)
    U, _ = np.linalg.qr(crandn(rng, K, r))
    V, _ = np.linalg.qr(crandn(rng, K, r))
    s = np.array([3.0, 1.0, 0.5, 0.2, 0.05])
    new, singular = orz.woodbury(np.linalg.inv(A), U, s, V)
    assert not singular
    Ap = A + (U * s) @ V.conj().T
    assert rel(Ap @ new, np.eye(K)) < 1e-13


def test_woodbury_sherman_morrison():
    rng = np.random.default_rng(15)
    K = 9
    A = _hpd(rng, K)
    Ai = np.linalg.inv(A)
    u = crandn(rng, K)
    v = crandn(rng, K)
    u /= np.linalg.norm(u)
    v /= np.linalg.norm(v)
    s = 0.8
    sm = Ai - s * np.outer(Ai @ u, v.conj() @ Ai) / (1 + s * (v.conj() @ Ai @ u))
    new, _ = orz.woodbury(Ai, u[:, None], np.array([s]), v[:, None])
    assert rel(new, sm) < 1e-13


def test_woodbury_full_rank_equals_inverse():
    rng = np.random.default_rng(16)
    K = 8
    A = _hpd(rng, K)
    dA = orz.gram_correction(crandn(rng, K, 16), 0.3 * crandn(rng, K, 16))
    Uf, s, Vh = np.linalg.svd(dA)
    new, _ = orz.woodbury(np.linalg.inv(A), Uf, s, Vh.conj().T)
    assert rel(new, np.linalg.inv(A + dA)) < 1e-12


def test_woodbury_singular_capacitance_flagged():
    rng = np.random.default_rng(17)
    K = 6
    A = _hpd(rng, K)
    Ai = np.linalg.inv(A)
    u = crandn(rng, K)
    s = 2.0
    # choose v so that 1/s + v^H A^-1 u = 0
    w = Ai.conj().T @ u
    beta = -1.0 / (s * (w.conj() @ Ai @ u))
    v = np.conj(beta) * w
    new, singular = orz.woodbury(Ai, u[:, None], np.array([s]), v[:, None])
    assert singular and new is None


def test_woodbury_drops_zero_singular_values():
    rng = np.random.default_rng(18)
    K = 7
    A = _hpd(rng, K)
    U, _ = np.linalg.qr(crandn(rng, K, 3))
    V, _ = np.linalg.qr(crandn(rng, K, 3))
    s = np.array([1.0, 0.3, 0.0])
    new, _ = orz.woodbury(np.linalg.inv(A), U, s, V)
    ref, _ = orz.woodbury(np.linalg.inv(A), U[:, :2], s[:2], V[:, :2])
    assert rel(new, ref) < 1e-15


# ---------------------------------------------------------------- precoder

def test_precoder_push_through_and_power():
    rng = np.random.default_rng(19)
    for K, N, alpha, P in [(4, 8, 0.3, 1.0), (16, 64, 1.6, 2.5), (8, 6, 0.9, 0.1)]:
        H = crandn(rng, K, N)
        W = orz.full_rzf(H, alpha, P)
        assert abs(orz.fro2(W) - P) < 1e-12 * P
        # push-through: H^H (H H^H + a I)^-1 = (H^H H + a I)^-1 H^H
        alt = np.linalg.solve(H.conj().T @ H + alpha * np.eye(N), H.conj().T)
        alt *= math.sqrt(P / orz.fro2(alt))
        assert rel(W, alt) < 1e-12


def test_precoder_bruteforce():
    rng = np.random.default_rng(20)
    K, N = 3, 4
    H = crandn(rng, K, N)
    Ai = np.linalg.inv(orz.gram(H, 0.5))
    W = orz.precoder(H, Ai, 1.0)
    raw = np.zeros((N, K), complex)
    for n in range(N):
        for k in range(K):
            raw[n, k] = sum(H[i, n].conjugate() * Ai[i, k] for i in range(K))
    raw /= math.sqrt(sum(abs(x) ** 2 for x in raw.ravel()))
    assert rel(W, raw) < 1e-13


# ---------------------------------------------------------------- sum rate

def test_sum_rate_single_user_closed_form():
    rng = np.random.default_rng(21)
    h = crandn(rng, 1, 10)
    for P, s2 in [(1.0, 0.1), (3.0, 2.0)]:
        W = orz.full_rzf(h, 0.2, P)
        _, R = orz.sum_rate(h, W, P, s2)
        assert abs(R - math.log2(1 + P * orz.fro2(h) / s2)) < 1e-12


def test_sum_rate_orthogonal_rows_closed_form():
    # H H^H = c I: R = K log2(1 + P c / (K sigma^2)) for every alpha
    K, N, c = 4, 8, 2.0
    F = np.exp(-2j * np.pi * np.outer(np.arange(N), np.arange(N)) / N) / math.sqrt(N)
    H = math.sqrt(c) * F[[0, 2, 5, 7], :]
    np.testing.assert_allclose(H @ H.conj().T, c * np.eye(K), atol=1e-14)
    for alpha in (0.01, 1.0, 5.0):
        W = orz.full_rzf(H, alpha, 1.5)
        _, R = orz.sum_rate(H, W, 1.5, 0.3)
        assert abs(R - K * math.log2(1 + 1.5 * c / (K * 0.3))) < 1e-12


def test_sum_rate_hand_example():
    # two users, explicit W: SINR_1 = |1|^2/(|0.5|^2+s), SINR_2 = |2|^2/(|1j|^2+s)
    H = np.array([[1.0, 0.0], [0.0, 1.0]], complex)
    W = np.array([[1.0, 0.5], [1j, 2.0]], complex)
    P = orz.fro2(W)
    rates, R = orz.sum_rate(H, W, P, 0.25)
    assert abs(rates[0] - math.log2(1 + 1.0 / (0.25 + 0.25))) < 1e-14
    assert abs(rates[1] - math.log2(1 + 4.0 / (1.0 + 0.25))) < 1e-14
    assert abs(R - rates.sum()) < 1e-14


def test_sum_rate_zero_forcing_nulls_interference():
    # alpha -> 0 with K <= N is zero forcing: row-n channel sees no interference
    rng = np.random.default_rng(22)
    K, N = 5, 12
    H = crandn(rng, K, N)
    W = orz.full_rzf(H, 1e-12, 1.0)
    E = H @ W
    off = E - np.diag(np.diag(E))
    assert np.abs(off).max() < 1e-9 * np.abs(np.diag(E)).max()
    rates, _ = orz.sum_rate(H, W, 1.0, 1e-3)
    g = np.abs(np.diag(E)) ** 2
    np.testing.assert_allclose(rates, np.log2(1 + g / 1e-3), rtol=1e-6)


# ------------------------------------------------------------ Alg. 2 track

def _track_inputs(K=16, N=64, steps=6, seed=0):
    cfg = wl.with_overrides(wl.CONFIGS["c1"], K=K, nx=int(math.isqrt(N)), steps=steps)
    tr = wl.make_track(cfg)
    return cfg, tr.snapshots()


def test_track_first_step_exact_identity():
    cfg, Hs = _track_inputs()
    prm = orz.TrackParams(alpha=cfg.alpha, switch_ratio=1.0, seed=1)
    ot = orz.OracleTrack(Hs[0], prm)
    A0 = orz.gram(Hs[0], cfg.alpha)
    dA = orz.gram_correction(Hs[0], Hs[1] - Hs[0])
    res = orz.arsvd(dA, 0.9, prm.k_init, prm.p, ot.i_max(), ot.draw(1))
    W, info = ot.update(Hs[1], 0.9)
    assert info.path == orz.PATH_WB and info.r == res.r
    Ap = A0 + (res.U * res.s) @ res.V.conj().T
    assert rel(Ap @ ot.Ainv, np.eye(cfg.K)) < 1e-12


def test_track_untruncated_update_equals_direct_inverse():
    cfg, Hs = _track_inputs(steps=4)
    K = cfg.K
    prm = orz.TrackParams(alpha=cfg.alpha, k_init=K, p=0, switch_ratio=1.0, seed=2)
    ot = orz.OracleTrack(Hs[0], prm)
    for t in range(1, 5):
        W, info = ot.update(Hs[t], 1.0 - 1e-13)
        assert info.path == orz.PATH_WB
        assert rel(ot.Ainv, np.linalg.inv(orz.gram(Hs[t], cfg.alpha))) < 1e-9
        assert rel(W, orz.full_rzf(Hs[t], cfg.alpha, 1.0)) < 1e-9


def test_track_switch_and_reset_paths():
    cfg, Hs = _track_inputs(steps=8)
    K = cfg.K
    # switch_ratio tiny: every nonzero rank goes to direct inversion
    ot = orz.OracleTrack(Hs[0], orz.TrackParams(alpha=cfg.alpha, switch_ratio=0.01))
    W, info = ot.update(Hs[1], 0.9)
    assert info.path == orz.PATH_FULL_RANK and info.r > 0.01 * K
    assert rel(ot.Ainv, np.linalg.inv(orz.gram(Hs[1], cfg.alpha))) < 1e-13
    # reset every 3 steps: steps 3 and 6 re-invert
    ot = orz.OracleTrack(Hs[0], orz.TrackParams(alpha=cfg.alpha, reset_period=3))
    paths = [ot.update(Hs[t], 0.9)[1].path for t in range(1, 8)]
    assert paths[2] == orz.PATH_RESET and paths[5] == orz.PATH_RESET
    assert orz.PATH_RESET not in paths[:2] + paths[3:5]


def test_track_nonfinite_snapshot_leaves_state():
    # a NaN snapshot changes nothing but the counters: the steps that follow
    # equal those of a track that never saw it (the same sketch draws, since
    # Omega is addressed by the step index, are taken from a twin whose step
    # counter skipped the same index)
    cfg, Hs = _track_inputs(steps=5)
    prm = orz.TrackParams(alpha=cfg.alpha, reset_period=3)
    a = orz.OracleTrack(Hs[0], prm)
    b = orz.OracleTrack(Hs[0], prm)
    a.update(Hs[1], 0.99)
    b.update(Hs[1], 0.99)
    bad = Hs[2].copy()
    bad[1, 3] = np.nan
    st = a.export_state()
    W, info = a.update(bad, 0.99)
    assert info.path == orz.PATH_NOOP and info.r == 0 and math.isnan(info.dA_fro2)
    assert not np.all(np.isfinite(W))
    after = a.export_state()
    for k in ("Ainv", "H_prev", "R"):
        assert np.array_equal(after[k], st[k]), k
    assert (after["t"], after["since_reset"], after["last_r"]) == (st["t"] + 1, st["since_reset"] + 1, st["last_r"])
    b.t += 1                        # the twin skips the same step index ...
    b.since_reset += 1              # ... and counts it towards the reset
    paths = []
    for t in (3, 4, 5):
        Wa, ia = a.update(Hs[t], 0.99)
        Wb, ib = b.update(Hs[t], 0.99)
        assert (ia.r, ia.iters, ia.path) == (ib.r, ib.iters, ib.path), t
        assert np.array_equal(Wa, Wb) and np.array_equal(a.Ainv, b.Ainv)
        paths.append(ia.path)
    # reset_period 3: step 2 (the NaN one) counted, so step 3 re-inverts
    assert paths[0] == orz.PATH_RESET and orz.PATH_RESET not in paths[1:]


def test_track_noop_when_channel_static():
    cfg, Hs = _track_inputs(steps=2)
    ot = orz.OracleTrack(Hs[0], orz.TrackParams(alpha=cfg.alpha))
    before = ot.Ainv.copy()
    W, info = ot.update(Hs[0], 0.9)
    assert info.path == orz.PATH_NOOP and info.r == 0
    np.testing.assert_array_equal(ot.Ainv, before)
    assert rel(W, orz.full_rzf(Hs[0], cfg.alpha, 1.0)) < 1e-13


def _recorded_sketch_sizes(ot):
    """Wrap ot.draw so that every sketch Alg. 1 draws is logged as (t, i, d)."""
    calls = []
    base = ot.draw

    def draw(t):
        f = base(t)

        def g(i, K, d):
            calls.append((t, i, d))
            return f(i, K, d)
        return g
    ot.draw = draw
    return calls


def test_track_warm_start_policy():
    # warm start: iteration 1 of step t draws d = min(max(k_init, r_{t-1}) + p, K)
    # and doubling goes on from that k0; the fixed policy starts at k_init
    cfg, Hs = _track_inputs(steps=6)
    for policy in (orz.KINIT_WARM, orz.KINIT_FIXED):
        prm = orz.TrackParams(alpha=cfg.alpha, kinit_policy=policy, p=3)
        ot = orz.OracleTrack(Hs[0], prm)
        calls = _recorded_sketch_sizes(ot)
        r_prev, grew = 0, False
        for t in range(1, 7):
            calls.clear()
            _, info = ot.update(Hs[t], 0.99)
            k0 = max(prm.k_init, r_prev) if policy == orz.KINIT_WARM else prm.k_init
            want = [min(k0 * 2 ** m + prm.p, cfg.K) for m in range(info.iters)]
            assert [c[2] for c in calls] == want, (policy, t, calls, r_prev)
            assert [(c[0], c[1]) for c in calls] == [(t, m + 1) for m in range(info.iters)]
            grew = grew or r_prev > prm.k_init
            r_prev = info.r
        assert grew     # some step started above k_init, so the policy mattered


def test_track_switch_is_algorithm_2_alone():
    # Alg. 2 takes Woodbury exactly when k_est <= floor(switch_ratio K), with no
    # other cap: at K = 16 a ratio of 1 sends every rank to Woodbury, and at
    # K = 64 a ratio of 0.75 sends a rank-40 step there too
    cfg, Hs = _track_inputs(steps=4)
    ot = orz.OracleTrack(Hs[0], orz.TrackParams(alpha=cfg.alpha, switch_ratio=1.0, k_init=16, p=0))
    for t in range(1, 4):
        _, info = ot.update(Hs[t], 1.0 - 1e-12)
        assert info.r == 16 and info.path == orz.PATH_WB
    K, N = 64, 80
    H0 = wl.random_channel(K, N, 31)
    H1 = wl.random_channel(K, N, 32)    # an i.i.d. redraw: Delta A of full rank
    for ratio, want in ((0.75, orz.PATH_WB), (0.5, orz.PATH_FULL_RANK)):
        ot = orz.OracleTrack(H0, orz.TrackParams(alpha=1.0, switch_ratio=ratio, k_init=40, p=0, i_max=1))
        _, info = ot.update(H1, 1.0)
        assert info.r == 40 and info.path == want, (ratio, info)
        assert rel(ot.Ainv, np.linalg.inv(orz.gram(H1, 1.0))) > 1e-8 or want != orz.PATH_WB


def test_track_early_fallback_policy():
    # an i.i.d. redraw makes Delta A full rank: no iteration reaches eta = 0.999
    # until d = K.  With the policy, the first iteration past the Woodbury
    # limit (K/2 = 8 for K = 16: d = 9, the second) ends Alg. 1 and the step
    # inverts directly; without it the loop runs on to d = K.
    K, N = 16, 64
    H0 = wl.random_channel(K, N, 1)
    H1 = wl.random_channel(K, N, 2)
    dA = orz.gram_correction(H0, H1 - H0)
    draw = lambda i, K_, d: orz.draw_sketch(3, 0, 1, i, K_, d)
    full = orz.arsvd(dA, 0.999, 2, 5, 4, draw)
    early = orz.arsvd(dA, 0.999, 2, 5, 4, draw, stop_d=8)
    assert (full.iters, full.d) == (4, 16) and full.r > 8
    assert (early.iters, early.d, early.r) == (2, 9, 9)
    # the first iteration is identical in both runs (same sketch), so the
    # policy only cuts the loop short
    assert early.energy == full.energy
    for pol, (it_exp, r_exp) in ((0, (full.iters, full.r)), (1, (2, 9))):
        ot = orz.OracleTrack(H0, orz.TrackParams(alpha=1.0, seed=3, early_fallback=pol))
        W, info = ot.update(H1, 0.999)
        assert info.path == orz.PATH_FULL_RANK and (info.iters, info.r) == (it_exp, r_exp)
        assert rel(ot.Ainv, np.linalg.inv(orz.gram(H1, 1.0))) < 1e-13


def test_track_error_feedback_bookkeeping():
    # R is A' of the step minus the Gram matrix whose inverse is stored, so it
    # equals A'_t - inv(A^-1_t) after every step; a truncated step leaves a
    # nonzero R, a direct inversion or a reset clears it
    cfg, Hs = _track_inputs(steps=12)
    prm = orz.TrackParams(alpha=cfg.alpha, seed=4, error_feedback=1, reset_period=9)
    ot = orz.OracleTrack(Hs[0], prm)
    seen_wb = False
    for t in range(1, 13):
        W, info = ot.update(Hs[t], 0.9)
        A_t = orz.gram(Hs[t], cfg.alpha)
        implied = np.linalg.inv(ot.Ainv)
        assert np.linalg.norm(ot.R - (A_t - implied)) <= 1e-9 * np.linalg.norm(A_t), t
        if info.path == orz.PATH_WB:
            seen_wb = True
            assert np.linalg.norm(ot.R) > 0.0
        else:
            assert np.linalg.norm(ot.R) == 0.0
    assert seen_wb


def test_track_error_feedback_bounds_drift():
    # without feedback the discarded energy of every truncated step stays in
    # the inverse; with it, each step re-sketches what is missing
    cfg, Hs = _track_inputs(steps=30)
    errs = {}
    for fb in (0, 1):
        ot = orz.OracleTrack(Hs[0], orz.TrackParams(alpha=cfg.alpha, seed=4, error_feedback=fb))
        for t in range(1, 31):
            ot.update(Hs[t], 0.9)
        ref = np.linalg.inv(orz.gram(Hs[30], cfg.alpha))
        errs[fb] = rel(ot.Ainv, ref)
    assert errs[1] < 0.5 * errs[0], errs


# ---------------------------------------------------------------- hybrid front end, eq. (4)

@pytest.mark.parametrize("nx,ny", [(1, 1), (4, 2), (3, 5), (16, 16)])
def test_dft_codebook_orthonormal(nx, ny):
    F = orz.dft_codebook(nx, ny)
    N = nx * ny
    assert F.shape == (N, N)
    assert rel(F.conj().T @ F, np.eye(N)) <= 1e-13
    assert np.allclose(np.abs(F), 1.0 / math.sqrt(N), rtol=0, atol=1e-15)


@pytest.mark.parametrize("nx,ny", [(4, 2), (3, 5), (16, 16)])
def test_dft_codebook_is_inverse_fft(nx, ny):
    # h F at beam b = q nx + p is N / sqrt(N) times numpy's inverse 2-D FFT of
    # h laid out as ny x nx (rows m_y, columns m_x), read at [q, p]
    rng = np.random.default_rng(41)
    K, N = 3, nx * ny
    H = crandn(rng, K, N)
    G = H @ orz.dft_codebook(nx, ny)
    ref = np.fft.ifft2(H.reshape(K, ny, nx), axes=(1, 2)) * (N / math.sqrt(N))
    assert rel(G, ref.reshape(K, N)) <= 1e-13


def _beamspace_bruteforce(H, nx, ny, n_rf):
    """Pure-Python loops over the definition: every beam's response by its
    sum, then the greedy choice with strict comparisons."""
    K, N = H.shape
    G = [[0j] * N for _ in range(K)]
    for n in range(K):
        for b in range(N):
            q, p = divmod(b, nx)
            acc = 0j
            for m in range(N):
                my, mx = divmod(m, nx)
                acc += H[n, m] * cmath.exp(2j * math.pi * (p * mx / nx + q * my / ny))
            G[n][b] = acc / math.sqrt(N)
    taken, beams = set(), []
    for c in range(n_rf):
        best, bi = -1.0, None
        for b in range(N):
            if b in taken:
                continue
            v = abs(G[c][b]) ** 2 if c < K else sum(abs(G[u][b]) ** 2 for u in range(K))
            if v > best:
                best, bi = v, b
        taken.add(bi)
        beams.append(bi)
    return beams, np.array([[G[n][b] for b in beams] for n in range(K)])


@pytest.mark.parametrize("K,nx,ny,n_rf,seed", [(3, 2, 2, 3, 1), (2, 3, 2, 5, 2), (4, 4, 2, 6, 3)])
def test_beamspace_bruteforce(K, nx, ny, n_rf, seed):
    rng = np.random.default_rng(seed)
    H = crandn(rng, K, nx * ny)
    beams, Heff = orz.beamspace(H, nx, ny, n_rf)
    bb, Hb = _beamspace_bruteforce(H, nx, ny, n_rf)
    assert list(beams) == bb
    assert rel(Heff, Hb) <= 1e-13
    assert rel(orz.beam_channel(H, nx, ny, beams), Heff) <= 1e-13


def test_beamspace_on_grid_users():
    # users whose channels are conjugate codebook beams see exactly one beam:
    # each takes its own beam and H_eff = I
    nx, ny = 8, 4
    F = orz.dft_codebook(nx, ny)
    own = [5, 17, 0, 30]
    H = F[:, own].conj().T
    beams, Heff = orz.beamspace(H, nx, ny, len(own))
    assert list(beams) == own
    assert rel(Heff, np.eye(len(own))) <= 1e-13


def test_beamspace_conflict_and_ties():
    nx, ny = 4, 2
    F = orz.dft_codebook(nx, ny)
    f = lambda b: F[:, b].conj()
    # user 1's strongest beam (5) is user 0's: it takes its second (2); the
    # extra chains then go by total power: beam 7 (0.09 + 0.09), then beam 0
    # (0.16, the larger single-user power)
    H = np.array([f(5) + 0.3 * f(7), 0.9 * f(5) + 0.5 * f(2) + 0.3 * f(7) + 0.4 * f(0)])
    beams, _ = orz.beamspace(H, nx, ny, 4)
    assert list(beams) == [5, 2, 7, 0]
    # an exact tie (two elements, h = [1, 0] sees both beams with power 1/2):
    # the lower index first, then the other one
    H2 = np.array([[1.0, 0.0], [1.0, 0.0]], dtype=complex)
    beams2, Heff2 = orz.beamspace(H2, 2, 1, 2)
    assert list(beams2) == [0, 1]
    assert np.allclose(np.abs(Heff2) ** 2, 0.5, rtol=0, atol=1e-15)


def test_hybrid_power_constraint():
    # eq. (4): the codebook columns are orthonormal, so scaling F_BB to
    # ||F_BB||_F^2 = P gives ||F_RF F_BB||_F^2 = P
    rng = np.random.default_rng(7)
    nx, ny, K, n_rf = 8, 8, 6, 10
    H = crandn(rng, K, nx * ny)
    beams, Heff = orz.beamspace(H, nx, ny, n_rf)
    Fbb = orz.full_rzf(Heff, 0.3, 2.0)
    Frf = orz.dft_codebook(nx, ny)[:, beams]
    assert abs(np.linalg.norm(Frf @ Fbb) ** 2 - 2.0) <= 1e-12
    # the sum rate through the analog stage equals the one on H F_RF
    _, R1 = orz.sum_rate(H @ Frf, Fbb, 2.0, 0.1)
    _, R2 = orz.sum_rate(orz.beam_channel(H, nx, ny, beams), Fbb, 2.0, 0.1)
    assert abs(R1 - R2) <= 1e-12 * abs(R1)
