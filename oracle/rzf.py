"""Plain FP64 CPU oracle of WB-arSVD RZF precoding (complex128, NumPy/LAPACK).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU path:
the two meet only in the seeded input generator (the channel tracks) and in the
published definition of the sketch generator, which each side implements on
its own.

Each function follows one passage of the paper, in the paper's order and
notation (A is the Gram matrix, Delta A its per-step correction):

  gram               Sec. II, eq. (5):   A = H H^H + alpha I_K
  gram_correction    Sec. III, eq. (9):  Delta A = H dH^H + dH H^H + dH dH^H
  direct_inverse     Alg. 2, "direct matrix inversion"
  arsvd              Alg. 1 and the energy rule of eq. (14)
  woodbury           eq. (12), evaluated in the order of Sec. III-A steps 1-5
  precoder           eq. (5) with the power constraint ||W||_F^2 = P
  sum_rate           eq. (15)
  dft_codebook       eq. (4): the DFT codebook of the UPA
  beamspace          eq. (4): best-power beam choice and H_eff = H~ F_RF
  beam_channel       eq. (15): H F_RF for given beams
  OracleTrack        Alg. 2, with an optional periodic exact re-inversion

Readings taken where the paper is silent (each is also listed with the design
notes of the repository):
  * Delta A = 0 gives r = 0 and leaves the inverse unchanged.
  * A snapshot holding NaN or Inf leaves the track's state unchanged (the
    next one is taken against the last finite snapshot); the step counters
    advance as for any step.
  * "Non-zero singular values" (Sec. III): components with sigma_j == 0 are
    dropped from Sigma_r before eq. (12) inverts it.
  * The switch of Alg. 2 is inclusive: Woodbury when r <= 0.5 K.
  * The capacitance C is treated as singular when its smallest singular value
    is at most SINGULAR_RTOL (||Sigma_r^-1||_2 + ||V_r^H A^-1 U_r||_2); the
    step then inverts A' directly (path FULL_SINGULAR).
  * I_max (never given) defaults to the smallest I with
    k_init 2^(I-1) + p >= K, i.e. the doubling reaches d = K.
  * The row-n channel of eq. (15) is row n of H (H = [h_1 ... h_K]^T), so the
    received-signal matrix is E = H W.
  * The best-power criterion of eq. (4) (its rule is only cited): users in
    index order each take the strongest codebook beam not yet taken, lowest
    index on ties; chains beyond K take the untaken beams of largest total
    power.  The codebook sign is +j (the other sign only relabels beams).
  * The periodic exact re-inversion (reset_period) is not part of the paper; it
    bounds the drift of the stored inverse and is off unless asked for.  It
    fires once reset_period steps have passed since the last FP64 inversion
    (the initial one or a reset); inversions of A' taken by Alg. 2's own
    fallback do not restart the count.  A reset step skips Alg. 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

from .philox import draw_sketch

PATH_NOOP = 0
PATH_WB = 1
PATH_FULL_RANK = 2
PATH_FULL_SINGULAR = 3
PATH_RESET = 4
PATH_NAMES = {PATH_NOOP: "noop", PATH_WB: "wb", PATH_FULL_RANK: "full_rank",
              PATH_FULL_SINGULAR: "full_singular", PATH_RESET: "reset"}

KINIT_FIXED = 0
KINIT_WARM = 1

SINGULAR_RTOL = 1e-13


def fro2(X: np.ndarray) -> float:
    """Squared Frobenius norm."""
    return float(np.sum(X.real ** 2 + X.imag ** 2))


def hermitian(X: np.ndarray) -> np.ndarray:
    return X.conj().T


def gram(H: np.ndarray, alpha: float) -> np.ndarray:
    """A = H H^H + alpha I_K (Sec. II, eq. (5))."""
    K = H.shape[0]
    return H @ hermitian(H) + alpha * np.eye(K, dtype=np.complex128)


def gram_correction(H: np.ndarray, dH: np.ndarray) -> np.ndarray:
    """Delta A = H dH^H + dH H^H + dH dH^H (Sec. III, eq. (9))."""
    return H @ hermitian(dH) + dH @ hermitian(H) + dH @ hermitian(dH)


def direct_inverse(A: np.ndarray) -> np.ndarray:
    """A^{-1} by direct (LU) inversion (Alg. 2)."""
    return np.linalg.inv(A)


def default_imax(K: int, k_init: int, p: int) -> int:
    """Smallest I with k_init * 2^(I-1) + p >= K."""
    i, k0 = 1, k_init
    while k0 + p < K:
        k0 *= 2
        i += 1
    return i


@dataclasses.dataclass
class ArsvdResult:
    U: np.ndarray          # K x r, U_r
    s: np.ndarray          # r, diagonal of Sigma_r (descending)
    V: np.ndarray          # K x r, V_r
    r: int                 # k_est
    iters: int             # iterations run
    d: int                 # subspace dimension of the last iteration
    sigma: np.ndarray      # all d singular values of the last B
    energy: float          # ||Delta A||_F^2
    captured: float        # sum_{j<=r} sigma_j^2


def arsvd(dA: np.ndarray, eta: float, k_init: int, p: int, i_max: int,
          draw: Callable[[int, int, int], np.ndarray],
          force_iters: Optional[int] = None, force_r: Optional[int] = None,
          stop_d: Optional[int] = None) -> ArsvdResult:
    """Adaptive randomized SVD (Alg. 1).

    draw(i, K, d) returns the K x d CN(0,1) matrix Omega of iteration i.
    force_iters / force_r replay a run whose rank decisions were taken
    elsewhere (used only when another implementation's decision fell within
    rounding distance of the threshold): the loop then runs exactly
    force_iters iterations and returns rank force_r from the last one.
    stop_d (early-fallback policy, not in the paper): an iteration with
    d > stop_d that misses the target ends the loop like the last one does,
    returning all d components (k_est = d).
    """
    K = dA.shape[0]
    energy = fro2(dA)
    E_target = eta * energy
    if energy == 0.0:
        z = np.zeros((K, 0), dtype=np.complex128)
        return ArsvdResult(z, np.zeros(0), z, 0, 0, 0, np.zeros(0), 0.0, 0.0)
    k0 = k_init
    n_iter = i_max if force_iters is None else force_iters
    for i in range(1, n_iter + 1):
        d = min(k0 + p, K)
        Omega = draw(i, K, d)
        Y = dA @ Omega
        Q, _ = np.linalg.qr(Y, mode="reduced")          # Q = orth(Y)
        B = hermitian(Q) @ dA
        Uh, s, Vh = np.linalg.svd(B, full_matrices=False)
        U_approx = Q @ Uh
        V_hat = hermitian(Vh)
        csum = np.cumsum(s ** 2)
        last = (i == n_iter)
        if force_iters is not None:
            if last and force_r is not None:
                r = force_r
                return ArsvdResult(U_approx[:, :r], s[:r], V_hat[:, :r], r, i, d, s,
                                   energy, float(csum[r - 1]) if r > 0 else 0.0)
            hit = np.nonzero(csum >= E_target)[0]
            if last and hit.size:
                r = int(hit[0]) + 1
                return ArsvdResult(U_approx[:, :r], s[:r], V_hat[:, :r], r, i, d, s,
                                   energy, float(csum[r - 1]))
        else:
            hit = np.nonzero(csum >= E_target)[0]
            if hit.size:                                 # smallest r found
                r = int(hit[0]) + 1
                return ArsvdResult(U_approx[:, :r], s[:r], V_hat[:, :r], r, i, d, s,
                                   energy, float(csum[r - 1]))
            if stop_d is not None and d > stop_d:        # early fallback
                return ArsvdResult(U_approx[:, :d], s[:d], V_hat[:, :d], d, i, d, s,
                                   energy, float(csum[d - 1]))
        k0 = 2 * k0
    # no r met the target: return all d components (k_est = d)
    return ArsvdResult(U_approx[:, :d], s[:d], V_hat[:, :d], d, n_iter, d, s,
                       energy, float(csum[d - 1]))


def woodbury(Ainv: np.ndarray, U: np.ndarray, s: np.ndarray, V: np.ndarray):
    """(A + U Sigma V^H)^{-1} from A^{-1} by eq. (12), steps 1-5 of Sec. III-A.

    Returns (new inverse, singular) where singular flags a capacitance
    (Sigma^{-1} + V^H A^{-1} U) too close to singular to invert.
    """
    keep = s != 0.0                      # Sigma_r holds the non-zero sigma_j
    U, s, V = U[:, keep], s[keep], V[:, keep]
    if s.size == 0:
        return Ainv.copy(), False
    Vh = hermitian(V)
    AU = Ainv @ U                        # step 1: A^{-1} U_r
    C = np.diag(1.0 / s) + Vh @ AU       # step 2: Sigma_r^{-1} + V_r^H A^{-1} U_r
    # singular when the smallest singular value of C vanishes next to the
    # size of its two terms
    scale = 1.0 / s.min() + np.linalg.norm(Vh @ AU, 2)
    if np.linalg.svd(C, compute_uv=False).min() <= SINGULAR_RTOL * scale:
        return None, True
    Cinv = np.linalg.inv(C)              # step 3
    VA = Vh @ Ainv
    T = (AU @ Cinv) @ VA                 # step 4
    return Ainv - T, False               # step 5


def precoder(H: np.ndarray, Ainv: np.ndarray, P: float) -> np.ndarray:
    """W = H^H A^{-1} scaled so that ||W||_F^2 = P (eq. (5), Sec. II)."""
    W = hermitian(H) @ Ainv
    return W * math.sqrt(P / fro2(W))


def full_rzf(H: np.ndarray, alpha: float, P: float) -> np.ndarray:
    """Conventional RZF: full inversion of the Gram matrix every snapshot."""
    return precoder(H, direct_inverse(gram(H, alpha)), P)


def sum_rate(H: np.ndarray, W: np.ndarray, P: float, sigma2: float):
    """Per-user rates and the sum rate of eq. (15) after scaling ||W||_F^2 = P."""
    W = W * math.sqrt(P / fro2(W))
    E = H @ W
    K = H.shape[0]
    rates = np.empty(K)
    for n in range(K):
        sig = abs(E[n, n]) ** 2
        interf = sum(abs(E[n, i]) ** 2 for i in range(K) if i != n)
        rates[n] = math.log2(1.0 + sig / (interf + sigma2))
    return rates, float(np.sum(rates))


def dft_codebook(nx: int, ny: int) -> np.ndarray:
    """The N x N DFT codebook of an nx x ny UPA (N = nx ny, element index
    m_y nx + m_x): beam b = (q, p) = divmod(b, nx) has entries
    exp(+j 2 pi (p m_x / nx + q m_y / ny)) / sqrt(N) (eq. (4)'s analog beams;
    distinct beams are orthonormal)."""
    N = nx * ny
    mx = np.tile(np.arange(nx), ny)
    my = np.repeat(np.arange(ny), nx)
    b = np.arange(N)
    p, q = b % nx, b // nx
    ph = 2.0 * np.pi * (np.outer(mx, p) / nx + np.outer(my, q) / ny)
    return np.exp(1j * ph) / math.sqrt(N)


def beamspace(Ht: np.ndarray, nx: int, ny: int, n_rf: int):
    """Analog beam selection and H_eff = H~ F_RF of eq. (4).

    Best-power rule (reading: the cited rule is not available): user n in
    turn takes the codebook beam b maximising |(H~ F)_{n,b}|^2 among the beams
    not yet taken (lowest index on ties); the remaining n_rf - K chains take
    the untaken beams of largest total power sum_n |(H~ F)_{n,b}|^2.  Returns
    (beams, H_eff): the n_rf selected beam indices (users' beams first) and
    the K x n_rf matrix H~ F_RF."""
    K, N = Ht.shape
    assert N == nx * ny and K <= n_rf <= N
    G = Ht @ dft_codebook(nx, ny)                 # every beam's response, K x N
    pw = np.abs(G) ** 2
    taken = np.zeros(N, dtype=bool)
    beams = []
    for n in range(K):
        cand = np.where(taken, -1.0, pw[n])
        b = int(np.argmax(cand))                  # first index of the maximum
        taken[b] = True
        beams.append(b)
    tot = pw.sum(axis=0)
    for _ in range(n_rf - K):
        cand = np.where(taken, -1.0, tot)
        b = int(np.argmax(cand))
        taken[b] = True
        beams.append(b)
    beams = np.array(beams, dtype=np.int64)
    return beams, G[:, beams]


def beam_channel(H: np.ndarray, nx: int, ny: int, beams) -> np.ndarray:
    """H F_RF for given codebook beams: the channel seen through the analog
    stage, as in the numerator and interference terms of eq. (15)."""
    return H @ dft_codebook(nx, ny)[:, np.asarray(beams, dtype=np.int64)]


@dataclasses.dataclass
class TrackParams:
    alpha: float
    P: float = 1.0
    k_init: int = 2
    p: int = 5
    i_max: int = 0              # 0: default_imax
    switch_ratio: float = 0.5
    reset_period: int = 0
    seed: int = 0
    track_id: int = 0
    kinit_policy: int = KINIT_FIXED
    early_fallback: int = 0     # policy: stop Alg. 1 once d passes the Woodbury limit
    error_feedback: int = 0     # policy: sketch Delta A + R, R the residual not yet applied


@dataclasses.dataclass
class UpdateInfo:
    r: int
    iters: int
    path: int
    dA_fro2: float
    captured: float
    d: int

    @property
    def energy_ratio(self) -> float:
        return self.captured / self.dA_fro2 if self.dA_fro2 > 0 else 1.0


class OracleTrack:
    """Alg. 2 on one channel track: the inverse carried across snapshots."""

    def __init__(self, H0: np.ndarray, params: TrackParams):
        self.params = params
        self.K, self.N = H0.shape
        self.Ainv = direct_inverse(gram(H0, params.alpha))
        self.H_prev = np.array(H0, dtype=np.complex128)
        self.t = 0
        self.since_reset = 0
        self.last_r = 0
        # error feedback: R = A' of the last step minus the Gram matrix whose
        # inverse is stored (zero after every direct inversion)
        self.R = np.zeros((self.K, self.K), dtype=np.complex128)
        self.last_arsvd: Optional[ArsvdResult] = None   # Alg. 1's result of the last step

    def i_max(self) -> int:
        p = self.params
        return p.i_max if p.i_max > 0 else default_imax(self.K, p.k_init, p.p)

    def first_k0(self) -> int:
        """k0 of the first iteration of Alg. 1: k_init (the paper), or under
        the warm-start policy max(k_init, previous k_est)."""
        p = self.params
        if p.kinit_policy == KINIT_WARM:
            return max(p.k_init, self.last_r)
        return p.k_init

    def draw(self, t: int):
        p = self.params
        return lambda i, K, d: draw_sketch(p.seed, p.track_id, t, i, K, d)

    def update(self, H: np.ndarray, eta: float, force_iters: Optional[int] = None,
               force_r: Optional[int] = None):
        """One snapshot: returns (W, UpdateInfo)."""
        prm = self.params
        H = np.asarray(H, dtype=np.complex128)
        self.t += 1
        t = self.t
        if not np.all(np.isfinite(H)):
            # a snapshot with NaN or Inf has no Delta A: the state stays as
            # it was and the next snapshot is taken against the last finite
            # one; only the step counters advance (a reset step still
            # restarts the reset count)
            reset = prm.reset_period > 0 and self.since_reset + 1 >= prm.reset_period
            self.since_reset = 0 if reset else self.since_reset + 1
            self.last_arsvd = None
            with np.errstate(invalid="ignore", over="ignore"):
                W = hermitian(H) @ self.Ainv
            return W, UpdateInfo(0, 0, PATH_NOOP, float("nan"), 0.0, 0)
        dH = H - self.H_prev
        dA = gram_correction(self.H_prev, dH)            # eq. (9)
        if prm.error_feedback:
            dA = dA + self.R                             # the change the inverse still lacks
        A_new = gram(H, prm.alpha)                       # eq. (7)
        energy = fro2(dA)
        self.last_arsvd = None
        if prm.reset_period > 0 and self.since_reset + 1 >= prm.reset_period:
            self.Ainv = direct_inverse(A_new)
            info = UpdateInfo(0, 0, PATH_RESET, 0.0, 0.0, 0)
            self.since_reset = 0
            self.R[:] = 0.0
        else:
            k_init = self.first_k0()
            limit = math.floor(prm.switch_ratio * self.K)  # Alg. 2: k_est <= switch * K
            res = arsvd(dA, eta, k_init, prm.p, self.i_max(), self.draw(t),
                        force_iters=force_iters, force_r=force_r,
                        stop_d=limit if prm.early_fallback else None)
            self.last_arsvd = res
            info = UpdateInfo(res.r, res.iters, PATH_NOOP, energy, res.captured, res.d)
            if res.r == 0:
                info.path = PATH_NOOP
            elif res.r <= limit:                         # Alg. 2: k_est <= switch * K
                new, singular = woodbury(self.Ainv, res.U, res.s, res.V)
                if singular:
                    self.Ainv = direct_inverse(A_new)
                    info.path = PATH_FULL_SINGULAR
                else:
                    self.Ainv = new
                    info.path = PATH_WB
            else:
                self.Ainv = direct_inverse(A_new)
                info.path = PATH_FULL_RANK
            if prm.error_feedback:
                if info.path == PATH_WB:                 # what the rank-r update left out
                    self.R = dA - (res.U * res.s) @ hermitian(res.V)
                elif info.path == PATH_NOOP:             # nothing applied (dA is zero)
                    self.R = dA.copy()
                else:                                    # an exact inverse of A'
                    self.R[:] = 0.0
            self.since_reset += 1
            self.last_r = res.r
        self.H_prev = H
        W = precoder(H, self.Ainv, prm.P)
        return W, info

    def export_state(self):
        return dict(Ainv=self.Ainv.copy(), H_prev=self.H_prev.copy(), t=self.t,
                    since_reset=self.since_reset, last_r=self.last_r, R=self.R.copy())

    def import_state(self, st):
        self.Ainv = np.array(st["Ainv"], dtype=np.complex128)
        self.H_prev = np.array(st["H_prev"], dtype=np.complex128)
        self.t = int(st["t"])
        self.since_reset = int(st["since_reset"])
        self.last_r = int(st["last_r"])
        if "R" in st:
            self.R = np.array(st["R"], dtype=np.complex128)
