"""Randomized SVD (Alg. 1) and its error measures (oracle; test infrastructure only).

Readings where the paper is silent: orth() is Householder QR (numpy/LAPACK);
svd_econ(B) is LAPACK's SVD; there is no oversampling and no power iteration
(Alg. 1 has none).
"""
import numpy as np


def rsvd_from_sketch(A, Y):
    """Alg. 1 after the sketch Y = A Omega: Q = orth(Y); B = Q^T A; [Uh, s, V] = svd_econ(B); U = Q Uh."""
    A = np.asarray(A, dtype=np.float64)
    Q, _ = np.linalg.qr(np.asarray(Y, dtype=np.float64), mode="reduced")
    B = Q.T @ A
    Uh, s, Vt = np.linalg.svd(B, full_matrices=False)
    return Q @ Uh, s, Vt, Q


def spectral_residual(A, Q, iters=50, seed=0):
    """||A - Q Q^T A||_2 by power iteration on (I - QQ^T) A, float64."""
    A = np.asarray(A, dtype=np.float64)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(A.shape[1])
    x /= np.linalg.norm(x)
    est = 0.0
    for _ in range(iters):
        # y = (I - QQ^T) A x lies in range(I - QQ^T), so (I - QQ^T)^T y = y
        # and M^T y = A^T y for M = (I - QQ^T) A.
        y = A @ x
        y -= Q @ (Q.T @ y)
        z = A.T @ y
        nz = np.linalg.norm(z)
        if nz == 0:
            return 0.0
        est = np.sqrt(nz)
        x = z / nz
    return est


def frobenius_residual(A, Q):
    """||A - Q Q^T A||_F."""
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.norm(A - Q @ (Q.T @ A))
