"""Plant plausible mistakes in the oracle (on the CPU) and check a pin fails.

Each mutant replaces one oracle function (or constant) with a copy carrying a
dropped term, a wrong sign or index, or a transposed operand.  The pins in
`test_oracle_pins.py` must reject every one of them; a mutant that survives
means the pins leave that part of the oracle unchecked.
"""
import math

import numpy as np
import pytest

import oracle.rzf as orz
from oracle import philox
import tests.test_oracle_pins as pins


def H_(X):
    return X.conj().T


def m_gram_no_alpha(H, alpha):
    return H @ H_(H)


def m_gram_transposed(H, alpha):
    return H @ H.T + alpha * np.eye(H.shape[0])


def m_corr_no_quadratic(H, dH):
    return H @ H_(dH) + dH @ H_(H)


def m_corr_sign(H, dH):
    return H @ H_(dH) - dH @ H_(H) + dH @ H_(dH)


def _arsvd_variant(kind):
    def f(dA, eta, k_init, p, i_max, draw, force_iters=None, force_r=None):
        K = dA.shape[0]
        energy = orz.fro2(dA)
        k0 = k_init
        for i in range(1, i_max + 1):
            d = min(k0 + p, K)
            Y = dA @ draw(i, K, d)
            Q, _ = np.linalg.qr(Y)
            B = (Q.T if kind == "no_conj" else H_(Q)) @ dA
            Uh, s, Vh = np.linalg.svd(B, full_matrices=False)
            U = Q @ Uh
            V = Vh.T if kind == "v_transpose" else H_(Vh)
            c = np.cumsum(s ** 2)
            hit = np.nonzero(c >= eta * energy)[0]
            if hit.size:
                r = int(hit[0]) + (0 if kind == "off_by_one" else 1)
                r = max(r, 1)
                return orz.ArsvdResult(U[:, :r], s[:r], V[:, :r], r, i, d, s, energy, float(c[r - 1]))
            k0 = k0 + 1 if kind == "no_doubling" else 2 * k0
        return orz.ArsvdResult(U, s, V, d, i_max, d, s, energy, float(c[-1]))
    return f


def _woodbury_variant(kind):
    def f(Ainv, U, s, V):
        if kind == "swap_uv":
            U, V = V, U
        Vh = H_(V)
        AU = Ainv @ U
        core = np.diag(s) if kind == "sigma_not_inverted" else np.diag(1.0 / s)
        C = core + Vh @ AU
        T = AU @ np.linalg.inv(C) @ (Vh @ Ainv)
        return (Ainv + T if kind == "plus" else Ainv - T), False
    return f


def m_precoder_unscaled(H, Ainv, P):
    return H_(H) @ Ainv


def m_precoder_transpose(H, Ainv, P):
    W = H.T @ Ainv
    return W * math.sqrt(P / orz.fro2(W))


def _sum_rate_variant(kind):
    def f(H, W, P, sigma2):
        W = W * math.sqrt(P / orz.fro2(W))
        E = (H.conj() if kind == "conj_rows" else H) @ W
        K = H.shape[0]
        rates = np.empty(K)
        for n in range(K):
            sig = abs(E[n, n]) ** 2
            intf = sum(abs(E[n, i]) ** 2 for i in range(K) if i != n)
            rates[n] = math.log2(1 + sig / (intf + (0.0 if kind == "no_noise" else sigma2)))
        return rates, float(rates.sum())
    return f


def m_words_to_cn_unscaled(wa, wb):
    ua = ((wa >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    ub = ((wb >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(ua))
    return rad * np.exp(2j * np.pi * ub)


def _codebook_variant(kind):
    def f(nx, ny):
        N = nx * ny
        mx = np.tile(np.arange(nx), ny)
        my = np.repeat(np.arange(ny), nx)
        b = np.arange(N)
        p, q = b % nx, b // nx
        if kind == "swap_axes":
            p, q = b // ny, b % ny
        sgn = -1.0 if kind == "minus_j" else 1.0
        ph = sgn * 2.0 * np.pi * (np.outer(mx, p) / nx + np.outer(my, q) / ny)
        return np.exp(1j * ph) / (1.0 if kind == "unnormalised" else math.sqrt(N))
    return f


def _beamspace_variant(kind):
    def f(Ht, nx, ny, n_rf):
        K, N = Ht.shape
        G = Ht @ orz.dft_codebook(nx, ny)
        pw = np.abs(G) ** 2
        taken = np.zeros(N, dtype=bool)
        beams = []
        for n in range(K):
            cand = pw[n] if kind == "no_exclusion" else np.where(taken, -1.0, pw[n])
            b = int(N - 1 - np.argmax(cand[::-1])) if kind == "last_on_tie" else int(np.argmax(cand))
            taken[b] = True
            beams.append(b)
        score = pw.max(axis=0) if kind == "extra_by_max" else pw.sum(axis=0)
        for _ in range(n_rf - K):
            b = int(np.argmax(np.where(taken, -1.0, score)))
            taken[b] = True
            beams.append(b)
        beams = np.array(beams, dtype=np.int64)
        return beams, G[:, beams]
    return f


def m_first_k0_plus_one(self):
    p = self.params
    return max(p.k_init, self.last_r + 1) if p.kinit_policy == orz.KINIT_WARM else p.k_init


def m_first_k0_always_warm(self):
    return max(self.params.k_init, self.last_r)


MUTANTS = [
    ("gram_no_alpha", orz, "gram", m_gram_no_alpha, ["test_gram_bruteforce", "test_gram_hermitian_positive_definite"]),
    ("gram_transposed", orz, "gram", m_gram_transposed, ["test_gram_bruteforce"]),
    ("corr_no_quadratic", orz, "gram_correction", m_corr_no_quadratic, ["test_gram_correction_bruteforce", "test_gram_correction_equals_gram_difference"]),
    ("corr_sign", orz, "gram_correction", m_corr_sign, ["test_gram_correction_bruteforce"]),
    ("arsvd_no_conj", orz, "arsvd", _arsvd_variant("no_conj"), ["test_arsvd_eckart_young_residual"]),
    ("arsvd_off_by_one", orz, "arsvd", _arsvd_variant("off_by_one"), ["test_arsvd_rank_is_minimal"]),
    ("arsvd_no_doubling", orz, "arsvd", _arsvd_variant("no_doubling"), ["test_arsvd_doubling_schedule"]),
    ("arsvd_v_transpose", orz, "arsvd", _arsvd_variant("v_transpose"), ["test_arsvd_eckart_young_residual"]),
    ("woodbury_plus", orz, "woodbury", _woodbury_variant("plus"), ["test_woodbury_exact_identity"]),
    ("woodbury_swap_uv", orz, "woodbury", _woodbury_variant("swap_uv"), ["test_woodbury_exact_identity"]),
    ("woodbury_sigma", orz, "woodbury", _woodbury_variant("sigma_not_inverted"), ["test_woodbury_exact_identity"]),
    ("precoder_unscaled", orz, "precoder", m_precoder_unscaled, ["test_precoder_push_through_and_power"]),
    ("precoder_transpose", orz, "precoder", m_precoder_transpose, ["test_precoder_bruteforce"]),
    ("sum_rate_conj_rows", orz, "sum_rate", _sum_rate_variant("conj_rows"), ["test_sum_rate_zero_forcing_nulls_interference"]),
    ("sum_rate_no_noise", orz, "sum_rate", _sum_rate_variant("no_noise"), ["test_sum_rate_hand_example"]),
    ("philox_m0", philox, "PHILOX_M0", philox.PHILOX_M0 ^ 1, ["test_philox_known_answers"]),
    ("philox_w1", philox, "PHILOX_W1", philox.PHILOX_W1 + 2, ["test_philox_known_answers"]),
    ("box_muller_unscaled", philox, "words_to_cn", m_words_to_cn_unscaled, ["test_sketch_is_standard_complex_gaussian"]),
    ("codebook_minus_j", orz, "dft_codebook", _codebook_variant("minus_j"),
     [("test_dft_codebook_is_inverse_fft", dict(nx=4, ny=2))]),
    ("codebook_swap_axes", orz, "dft_codebook", _codebook_variant("swap_axes"),
     [("test_dft_codebook_is_inverse_fft", dict(nx=3, ny=5))]),
    ("codebook_unnormalised", orz, "dft_codebook", _codebook_variant("unnormalised"),
     [("test_dft_codebook_orthonormal", dict(nx=4, ny=2))]),
    ("beamspace_no_exclusion", orz, "beamspace", _beamspace_variant("no_exclusion"), ["test_beamspace_conflict_and_ties"]),
    ("beamspace_last_on_tie", orz, "beamspace", _beamspace_variant("last_on_tie"), ["test_beamspace_conflict_and_ties"]),
    ("beamspace_extra_by_max", orz, "beamspace", _beamspace_variant("extra_by_max"), ["test_beamspace_conflict_and_ties"]),
    ("warm_k0_plus_one", orz.OracleTrack, "first_k0", m_first_k0_plus_one, ["test_track_warm_start_policy"]),
    ("warm_k0_always", orz.OracleTrack, "first_k0", m_first_k0_always_warm, ["test_track_warm_start_policy"]),
]


@pytest.mark.parametrize("name,mod,attr,repl,pin_names", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_mutant(name, mod, attr, repl, pin_names, monkeypatch, golden_dir):
    monkeypatch.setattr(mod, attr, repl)
    caught = False
    for pn in pin_names:
        pn, kw = pn if isinstance(pn, tuple) else (pn, {})
        fn = getattr(pins, pn)
        try:
            if "golden_dir" in fn.__code__.co_varnames[:fn.__code__.co_argcount]:
                fn(golden_dir, **kw)
            else:
                fn(**kw)
        except (AssertionError, ValueError, np.linalg.LinAlgError, IndexError):
            caught = True
    assert caught, f"mutant {name} survived pins {pin_names}"
