"""Seeded synthetic LEO channel tracks (system model of Sec. II, eqs. (1)-(3)).

This module only draws inputs: channel snapshots H(t) for a satellite pass, the
regularisation and the noise power.  It holds none of the precoding method's
arithmetic, so both the FP64 oracle and the GPU path consume the same inputs
without sharing any of the method's code.

Channel model (Sec. II):
  * H(t) = [h_1(t) ... h_K(t)]^T, K x N, rows are user channels (eq. (1)).
  * h_n = sqrt(K_R/(K_R+1)) h_n^LOS + sqrt(1/(K_R+1)) h_n^NLOS (eq. (2)).
  * h_n^LOS = gamma_n a(theta_n, phi_n) with the unit-norm array manifold of a
    planar array, a = N^-1/2 [exp(j kappa . r_m)]_m (eq. (3)).

Readings where the paper leaves the scenario open (the paper's link budget and
analog codebook are not given in full, so the pass is synthetic):
  * Fully digital array, N = N_t (the analog combiner F_RF of eq. (4) is the
    identity), except for configurations with n_rf > 0: those feed the
    manifolds H~(t) (`snapshots(manifold=True)`) to the hybrid front end and
    score eq. (15) on H(t) F_RF.
  * Square half-wavelength UPA in the satellite's x-y plane, boresight at
    nadir, so kappa . r_m = pi (m_x u + m_y v) with direction cosines
    u = (x_k - x_s)/d_k and v = y_k/d_k.
  * Flat ground, satellite at (x_s(t), 0, h) with x_s(t) = v_sat dt (t - T/2),
    overhead at mid-pass; v_sat = 7.6 km/s.
  * Users uniform in a disk of radius R around the sub-satellite track centre.
  * gamma_n = sqrt(beta_n) e^{j phi_n} with beta_n = (h/d_n)^2 (free-space loss
    relative to nadir) and a static phase phi_n ~ U[0, 2 pi).
  * NLOS term sqrt(beta_n) g_n / sqrt(N), g_n ~ CN(0, I_N) drawn once per track
    (static scatter), so K_R is the true LOS:NLOS power ratio.
  * P = 1, sigma^2 = P / SNR, alpha = K sigma^2 / P.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

V_SAT = 7.6e3  # m/s, LEO ground-track speed


@dataclasses.dataclass(frozen=True)
class TrackConfig:
    name: str
    seed: int            # first word of the SeedSequence and of the sketch key
    nx: int              # UPA side; N = nx * nx
    K: int               # users
    height_m: float
    radius_m: float
    dt_s: float
    steps: int           # number of updates after the initial snapshot
    kr_db: float         # Rician K-factor
    snr_db: float
    eta: float = 0.999   # retained-energy threshold of the rank rule
    p: int = 5           # oversampling
    k_init: int = 2
    reset_period: int = 0  # steps between FP64 re-inversions (0 = never)
    P: float = 1.0
    n_rf: int = 0        # RF chains of the hybrid front end of eq. (4) (0: fully digital)

    @property
    def N(self) -> int:
        return self.nx * self.nx

    @property
    def sigma2(self) -> float:
        return self.P / (10.0 ** (self.snr_db / 10.0))

    @property
    def alpha(self) -> float:
        return self.K * self.sigma2 / self.P


# Single-track workloads.  "c1" is small enough for the FP64 oracle to run in
# well under a second per pass; "c2" (K=64, N=256, 1000 steps of 10 ms, FP64
# drift reset every 100 steps) is the throughput/latency workload.
CONFIGS: Dict[str, TrackConfig] = {
    "c1": TrackConfig("c1", seed=1, nx=8, K=16, height_m=550e3, radius_m=50e3,
                      dt_s=0.1, steps=50, kr_db=10.0, snr_db=10.0, eta=0.999,
                      p=5, k_init=2, reset_period=0),
    "c2": TrackConfig("c2", seed=2, nx=16, K=64, height_m=550e3, radius_m=100e3,
                      dt_s=0.01, steps=1000, kr_db=10.0, snr_db=10.0, eta=0.999,
                      p=5, k_init=2, reset_period=100),
    "c5": TrackConfig("c5", seed=5, nx=32, K=256, height_m=550e3, radius_m=200e3,
                      dt_s=0.005, steps=500, kr_db=3.0, snr_db=10.0, eta=0.999,
                      p=5, k_init=2, reset_period=50),
    # Fully digital analog of the paper's Table V / Fig. 2 scenario: 16 x 16
    # array at 600 km, K = 16 users (a 16 x 16 Gram matrix, as after the
    # paper's 16 RF chains), 50 ms updates over a 120 s pass, p = 1,
    # k_init = 2, K-factor 10 dB; users in a 50 km disk at SNR 10 dB (the
    # paper's link budget is not given in full).
    "tv": TrackConfig("tv", seed=15, nx=16, K=16, height_m=600e3, radius_m=50e3,
                      dt_s=0.05, steps=2400, kr_db=10.0, snr_db=10.0, eta=0.9,
                      p=1, k_init=2, reset_period=0),
    # Hybrid front end (the paper's simulation table): 16 x 16 array, 16 RF
    # chains, 16 users, 600 km orbit, 50 ms updates over a 120 s pass, p = 1.
    # The users' disk (250 km) spreads them over about 36 beams of the 16 x 16
    # DFT grid, so most users get a beam of their own.
    "h1": TrackConfig("h1", seed=16, nx=16, K=16, height_m=600e3, radius_m=250e3,
                      dt_s=0.05, steps=2400, kr_db=10.0, snr_db=10.0, eta=0.9,
                      p=1, k_init=2, reset_period=0, n_rf=16),
}


def with_overrides(cfg: TrackConfig, **kw) -> TrackConfig:
    return dataclasses.replace(cfg, **kw)


# Multi-track mix: every track draws its own size and SNR.  The array side
# (8, 16 or 32 elements, N = 64, 256 or 1024) fixes the user-disk radius
# (50, 100 or 200 km); K is uniform on 16..128, the SNR uniform on 0..20 dB;
# K-factor 10 dB, 10 ms between snapshots, 200 steps, FP64 drift reset every
# 100 steps.
MIX_SIDES = (8, 16, 32)
MIX_RADIUS_M = {8: 50e3, 16: 100e3, 32: 200e3}


def mix_configs(n: int, seed: int = 3, k_range=(16, 128), eta: float = 0.999) -> list:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 777]))
    out = []
    for i in range(n):
        nx = int(MIX_SIDES[rng.integers(0, len(MIX_SIDES))])
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        snr = float(rng.uniform(0.0, 20.0))
        out.append(TrackConfig(f"mix{i}", seed=seed, nx=nx, K=K, height_m=550e3,
                               radius_m=MIX_RADIUS_M[nx], dt_s=0.01, steps=200, kr_db=10.0,
                               snr_db=snr, eta=eta, p=5, k_init=2, reset_period=100))
    return out


class Track:
    """Static geometry of one track; `snapshot(t)` returns H(t) (K x N)."""

    def __init__(self, cfg: TrackConfig, track: int = 0):
        self.cfg = cfg
        self.track = track
        rng = np.random.default_rng(np.random.SeedSequence([cfg.seed, track]))
        K, N = cfg.K, cfg.N
        rho = cfg.radius_m * np.sqrt(rng.random(K))
        ang = 2.0 * np.pi * rng.random(K)
        self.xk = rho * np.cos(ang)
        self.yk = rho * np.sin(ang)
        self.phase = 2.0 * np.pi * rng.random(K)
        self.g = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))) / np.sqrt(2.0)
        m = np.arange(cfg.nx) - (cfg.nx - 1) / 2.0
        # element (m_y, m_x) -> index m_y * nx + m_x
        self.mx = np.tile(m, cfg.nx)
        self.my = np.repeat(m, cfg.nx)

    def _snap(self, t: np.ndarray, manifold: bool = False) -> np.ndarray:
        """H(t) for a vector of step indices t (shape T x K x N); with
        manifold, the array manifolds a(theta_n, phi_n) alone (the rows of
        H~ in eq. (4), no gain and no NLOS term)."""
        cfg = self.cfg
        N = cfg.N
        t = np.asarray(t, dtype=np.float64)
        xs = V_SAT * cfg.dt_s * (t - cfg.steps / 2.0)                 # T
        dx = self.xk[None, :] - xs[:, None]                            # T x K
        dy = np.broadcast_to(self.yk[None, :], dx.shape)
        d = np.sqrt(dx * dx + dy * dy + cfg.height_m ** 2)
        u = dx / d
        v = dy / d
        beta = (cfg.height_m / d) ** 2
        a = np.exp(1j * np.pi * (u[:, :, None] * self.mx[None, None, :]
                                 + v[:, :, None] * self.my[None, None, :])) / math.sqrt(N)
        if manifold:
            return a.astype(np.complex128)
        kr = 10.0 ** (cfg.kr_db / 10.0)
        los = np.exp(1j * self.phase)[None, :, None] * a
        nlos = self.g[None, :, :] / math.sqrt(N)
        h = np.sqrt(beta)[:, :, None] * (math.sqrt(kr / (kr + 1.0)) * los
                                          + math.sqrt(1.0 / (kr + 1.0)) * nlos)
        return h.astype(np.complex128)

    def snapshot(self, t: int) -> np.ndarray:
        return self._snap(np.array([t]))[0]

    def snapshots(self, t0: int = 0, count: Optional[int] = None, manifold: bool = False) -> np.ndarray:
        """H(t) (or the manifolds H~(t)) for t = t0 .. t0+count-1 (default:
        the whole pass, steps+1)."""
        if count is None:
            count = self.cfg.steps + 1 - t0
        out = np.empty((count, self.cfg.K, self.cfg.N), dtype=np.complex128)
        for c0 in range(0, count, 64):
            c1 = min(count, c0 + 64)
            out[c0:c1] = self._snap(np.arange(t0 + c0, t0 + c1), manifold)
        return out


def make_track(cfg: TrackConfig, track: int = 0) -> Track:
    return Track(cfg, track)


def random_channel(K: int, N: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """i.i.d. CN(0, scale^2/N) K x N matrix, for unstructured test inputs."""
    rng = np.random.default_rng(np.random.SeedSequence([9000, seed, K, N]))
    g = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))) / np.sqrt(2.0)
    return scale * g / math.sqrt(N)


def perturbed_channel(H: np.ndarray, seed: int, rank: int, scale: float) -> np.ndarray:
    """H + dH where dH = X Y^H has the given rank (structured test inputs)."""
    K, N = H.shape
    rng = np.random.default_rng(np.random.SeedSequence([9100, seed, K, N, rank]))
    X = (rng.standard_normal((K, rank)) + 1j * rng.standard_normal((K, rank))) / np.sqrt(2.0)
    Y = (rng.standard_normal((N, rank)) + 1j * rng.standard_normal((N, rank))) / np.sqrt(2.0)
    return H + scale * (X @ Y.conj().T) / math.sqrt(N * max(rank, 1))
