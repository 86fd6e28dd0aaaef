"""Randomized SVD (Alg. 1), Nystrom (Alg. 2), generalized Nystrom (Alg. 4 and
5) and their error measures (oracle; test infrastructure only).

Readings where the paper is silent: orth() and qr_econ() are Householder QR
(numpy/LAPACK); svd_econ() is LAPACK's SVD; there is no oversampling and no
power iteration (Alg. 1 has none); eps_mach in the rank rule of Alg. 4 and 5
is the FP64 unit roundoff 2^-52; in Alg. 2, ||Y|| is the spectral norm and
chol() factors the symmetrized Omega^T Y_nu (its upper factor C, B = C^T C).
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


EPS_MACH = 2.0 ** -52


def _numerical_rank(s, eps):
    """r = #{i : s_i > 5 eps s_1} (the rank rule of Alg. 4 and 5; s descending)."""
    return int(np.count_nonzero(s > 5.0 * eps * s[0])) if s.size and s[0] > 0 else 0


def gen_nystrom_outer(A, Omega, Psi, eps=EPS_MACH):
    """Alg. 4 (outer-product form): A ~ F G^T.

    Y = A Omega, X = A^T Psi; [U, S, V] = svd_econ(X^T Omega); r from S;
    F = Y V(:, :r) S(:r)^-1, G = X U(:, :r). Returns (F, G, r).
    """
    A = np.asarray(A, dtype=np.float64)
    Y = A @ Omega
    X = A.T @ Psi
    U, s, Vt = np.linalg.svd(X.T @ Omega, full_matrices=False)
    r = _numerical_rank(s, eps)
    F = Y @ (Vt[:r].T / s[:r])
    G = X @ U[:, :r]
    return F, G, r


def gen_nystrom_svd(A, Omega, Psi, eps=EPS_MACH):
    """Alg. 5 (SVD form): A ~ U diag(sigma) V^T.

    Y = A Omega, X = A^T Psi; [Q, ~] = qr_econ(Y), [P, T] = qr_econ(X);
    [U1, S1, V1] = svd_econ(Psi^T Q); r from S1; C = V1_r S1_r^-1 U1_r^T T^T;
    [Uh, sigma, Vh] = svd_econ(C); U = Q Uh, V = P Vh. Returns (U, sigma, V, r).
    """
    A = np.asarray(A, dtype=np.float64)
    Y = A @ Omega
    X = A.T @ Psi
    Q, _ = np.linalg.qr(Y, mode="reduced")
    P, T = np.linalg.qr(X, mode="reduced")
    U1, s1, V1t = np.linalg.svd(Psi.T @ Q, full_matrices=False)
    r = _numerical_rank(s1, eps)
    C = V1t[:r].T @ ((U1[:, :r].T @ T.T) / s1[:r, None])
    Uh, sig, Vht = np.linalg.svd(C, full_matrices=False)
    return Q @ Uh, sig, P @ Vht.T, r


def nystrom_psd(A, Omega, eps=EPS_MACH):
    """Alg. 2: A ~ U diag(lam) U^T for a psd A (n x n).

    Y = A Omega; nu = sqrt(n) eps ||Y||_2; Y_nu = Y + nu Omega;
    C = chol(Omega^T Y_nu) (upper, symmetrized input); B = Y_nu C^-1;
    [U, S, ~] = svd_econ(B); lam = max(0, S^2 - nu). Returns (U, lam, nu).
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Y = A @ Omega
    nu = np.sqrt(n) * eps * np.linalg.norm(Y, 2)
    Ynu = Y + nu * Omega
    M = Omega.T @ Ynu
    M = 0.5 * (M + M.T)
    C = np.linalg.cholesky(M).T  # upper: M = C^T C
    B = np.linalg.solve(C.T, Ynu.T).T  # B C = Y_nu
    U, s, _ = np.linalg.svd(B, full_matrices=False)
    lam = np.maximum(0.0, s * s - nu)
    return U, lam, nu
