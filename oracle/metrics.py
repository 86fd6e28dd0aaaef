"""Embedding-quality measures from the paper's definitions (oracle; tests only)."""
import numpy as np


def distortion(SQ):
    """Injectivity and dilation of a sketch on range(Q).

    Prop. 1.9: for orthonormal Q, alpha = sigma_min^2(S Q) (the OSI
    injectivity of Def. 1.2) and, for the OSE of Def. 1.1, beta =
    sigma_max^2(S Q). Returns (alpha, beta, eps) with
    eps = max(1 - alpha, beta - 1).
    """
    s = np.linalg.svd(np.asarray(SQ, dtype=np.float64), compute_uv=False)
    a, b = s[-1] ** 2, s[0] ** 2
    return a, b, max(1.0 - a, b - 1.0)


def coherence(Q):
    """mu(Q) = max_i ||e_i^T Q||^2 for orthonormal Q (notation, Sec. 1.6)."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.max(np.sum(Q * Q, axis=1)))


def orth(A):
    """Orthonormal basis of range(A) (Householder QR)."""
    Q, _ = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    return Q
