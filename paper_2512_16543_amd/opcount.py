"""Operation-count model of Tables I-III, used to report the paper's savings.

The paper counts only the inverse maintenance: a full inversion costs K^3,
the WB-arSVD update K^2 + K^2 r + r^3 + r^2 K (Table III; Table I for WB
alone, Table II for arSVD), with the arSVD iterations and the oversampling
left out (Sec. IV-A).  This is a reporting model, not part of the computation.
"""


def full_inverse_ops(K: int) -> float:
    """Table I / Table III, full matrix inversion: K^3."""
    return float(K) ** 3


def wb_arsvd_ops(K: int, r: int) -> float:
    """Table III, WB-arSVD: K^2 + K^2 r + r^3 + r^2 K."""
    K, r = float(K), float(r)
    return K * K + K * K * r + r ** 3 + r * r * K


def normalized_complexity(K: int, r: int) -> float:
    """The quantity plotted in Fig. 1: WB-arSVD cost over full-inversion cost."""
    return wb_arsvd_ops(K, r) / full_inverse_ops(K)


def savings(K: int, r: float) -> float:
    """Fractional saving of Table V for a mean retained rank r (r may be fractional)."""
    K = float(K)
    return 1.0 - (K * K + K * K * r + r ** 3 + r * r * K) / K ** 3
