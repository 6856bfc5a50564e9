"""Counter-based Gaussian sketch draws for the oracle (Alg. 1, the draw of Omega).

TEST INFRASTRUCTURE: part of the FP64 oracle.  Only tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the GPU path has its own,
independent implementation of the same published generator.

Algorithm 1 draws a fresh K x d matrix Omega with i.i.d. CN(0,1) entries in
every iteration.  The draw is made reproducible by addressing it with a
counter-based generator, Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11):

  * key     = (seed, track)
  * counter = (q, iteration, t, 0) with q = (j * 1024 + i) >> 1 for entry
    (row i, column j); the stride 1024 is the largest supported K, so an entry
    does not depend on K or d.
  * words (w0, w1) of a block serve the even row i, (w2, w3) the odd row.
  * u = ((w >> 11) + 0.5) 2^-53 in (0, 1); Box-Muller:
    z = sqrt(-2 ln u_a) (cos 2 pi u_b + j sin 2 pi u_b) / sqrt(2),
    so Re z, Im z ~ N(0, 1/2) and E|z|^2 = 1.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
# Philox4x64 round multipliers and Weyl key increments (SC'11, Sec. 4).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
ROUNDS = 10
KMAX_STRIDE = 1024


def philox4x64_scalar(ctr, key, rounds: int = ROUNDS):
    """Reference Philox4x64 on Python integers: obviously correct, slow."""
    x0, x1, x2, x3 = [c & MASK64 for c in ctr]
    k0, k1 = [k & MASK64 for k in key]
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0), lo1, (hi0 ^ x3 ^ k1), lo0
    return x0, x1, x2, x3


def _mulhilo64(a: int, b: np.ndarray):
    """(hi, lo) of the 128-bit product of constant a with uint64 array b."""
    mask32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo = np.uint64(a & 0xFFFFFFFF)
    a_hi = np.uint64(a >> 32)
    b_lo = b & mask32
    b_hi = b >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & mask32) + (hl & mask32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    lo = np.uint64(a) * b  # wraps mod 2^64
    return hi, lo


def philox4x64(ctr: np.ndarray, key, rounds: int = ROUNDS) -> np.ndarray:
    """Vectorised Philox4x64 over rows of ctr (n x 4 uint64) -> n x 4 uint64."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[:, i].copy() for i in range(4))
    k0 = int(key[0]) & MASK64
    k1 = int(key[1]) & MASK64
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = (k0 + PHILOX_W0) & MASK64
                k1 = (k1 + PHILOX_W1) & MASK64
            hi0, lo0 = _mulhilo64(PHILOX_M0, x0)
            hi1, lo1 = _mulhilo64(PHILOX_M1, x2)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0)), lo1, (hi0 ^ x3 ^ np.uint64(k1)), lo0
    return np.stack([x0, x1, x2, x3], axis=1)


def sketch_counters(t: int, it: int, K: int, d: int) -> np.ndarray:
    """Counter blocks (q, it, t, 0) for every (i, j) entry of a K x d sketch."""
    i = np.arange(K, dtype=np.uint64)[:, None]
    j = np.arange(d, dtype=np.uint64)[None, :]
    q = (j * np.uint64(KMAX_STRIDE) + i) >> np.uint64(1)
    ctr = np.zeros((K, d, 4), dtype=np.uint64)
    ctr[:, :, 0] = q
    ctr[:, :, 1] = np.uint64(it)
    ctr[:, :, 2] = np.uint64(t)
    return ctr


def sketch_words(seed: int, track: int, t: int, it: int, K: int, d: int) -> np.ndarray:
    """The two 64-bit words (w_a, w_b) behind each entry: K x d x 2 uint64."""
    ctr = sketch_counters(t, it, K, d).reshape(-1, 4)
    blocks = philox4x64(ctr, (seed, track)).reshape(K, d, 4)
    odd = (np.arange(K) & 1).astype(bool)[:, None]
    wa = np.where(odd, blocks[:, :, 2], blocks[:, :, 0])
    wb = np.where(odd, blocks[:, :, 3], blocks[:, :, 1])
    return np.stack([wa, wb], axis=2)


def words_to_cn(wa: np.ndarray, wb: np.ndarray) -> np.ndarray:
    """Box-Muller from two 53-bit uniforms to one CN(0,1) sample (complex128)."""
    ua = ((wa >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)
    ub = ((wb >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)
    rad = np.sqrt(-2.0 * np.log(ua)) / np.sqrt(2.0)
    ang = 2.0 * np.pi * ub
    return rad * np.cos(ang) + 1j * (rad * np.sin(ang))


def draw_sketch(seed: int, track: int, t: int, it: int, K: int, d: int) -> np.ndarray:
    """Omega in C^{K x d}, i.i.d. CN(0,1), for iteration `it` of step `t`."""
    w = sketch_words(seed, track, t, it, K, d)
    return words_to_cn(w[:, :, 0], w[:, :, 1])
