"""Least-squares drivers written from the paper (oracle; test infrastructure only).

  sketch_and_solve        Alg. 3 (sketch-and-solve with a structured sketch)
  exact_lstsq_tsqr        the plain definition x* = argmin ||Ax - b||, by
                          Householder QR of [A | b] over row chunks (TSQR)
  lsqr                    Paige & Saunders, ACM TOMS 8 (1982), the Krylov
                          solver used by sketch-and-precondition
  sketch_and_precondition the method the paper names as the standard
                          high-accuracy least-squares solver (Sec. 1.4,
                          remark after Thm. 1.4), in the form of its
                          references: QR of the sketch, then LSQR on A R^-1.

Readings where the paper is silent (shared with the GPU library):
  * eps_mach in Alg. 3 is the spacing of doubles at 1, 2^-52, and the rank
    test is strict: sigma_i > 5 eps sigma_1;
  * sketch-and-precondition warm-starts from the sketch-and-solve point
    x0 = R^-1 Q^T (S b) and stops on LSQR's least-squares test
    ||M^T r|| <= tol * ||M||_F(est) * ||r|| for M = A R^-1, or on
    ||r|| <= tol * ||r0|| (a consistent system).
"""
import numpy as np
import scipy.linalg as sla

EPS_MACH = 2.0 ** -52


def sketch_and_solve(SA, Sb, eps=EPS_MACH):
    """Alg. 3 given the sketched data SA (p x d) and Sb (p [x m]).

    [U, s, V] = svd_econ(SA); r = #{i : s_i > 5 eps s_1};
    x = V_r (s_r^-1 (U_r^T Sb)). Returns (x, r, s).
    """
    U, s, Vt = np.linalg.svd(np.asarray(SA, dtype=np.float64), full_matrices=False)
    r = int(np.count_nonzero(s > 5.0 * eps * s[0])) if s.size else 0
    Ub = U[:, :r].T @ np.asarray(Sb, dtype=np.float64)
    z = Ub / (s[:r] if np.ndim(Ub) == 1 else s[:r, None])
    return Vt[:r].T @ z, r, s


def exact_lstsq_tsqr(A, b, chunk=1 << 16):
    """x* = argmin ||A x - b||_2 and ||A x* - b|| from the R factor of [A | b].

    Each row chunk of the augmented matrix is reduced by Householder QR
    (LAPACK via numpy.linalg.qr, mode='r'); the stacked triangular factors are
    reduced again. With Rhat = R([A b]) ((m+1) x (m+1)),
    x* = Rhat[:m,:m]^-1 Rhat[:m, m] and ||r*|| = |Rhat[m, m]|.
    Returns (x*, ||r*||, Rhat).
    """
    n, m = A.shape
    R = np.zeros((0, m + 1))
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        blk = np.empty((r1 - r0, m + 1))
        blk[:, :m] = A[r0:r1]
        blk[:, m] = b[r0:r1]
        Rc = np.linalg.qr(blk, mode="r")
        R = np.linalg.qr(np.vstack([R, Rc]), mode="r")
    if R.shape[0] < m + 1:
        R = np.vstack([R, np.zeros((m + 1 - R.shape[0], m + 1))])
    x = sla.solve_triangular(R[:m, :m], R[:m, m])
    return x, abs(R[m, m]), R


def lsqr(matvec, rmatvec, b, n_cols, atol=1e-10, btol=1e-10, maxit=200):
    """LSQR (Paige & Saunders 1982): min ||M y - b|| by Golub-Kahan bidiagonalization.

    matvec(v) = M v, rmatvec(u) = M^T u. Returns (y, info) where info has
    iters, converged, rnorm (the recurrence estimate of ||b - M y||),
    arnorm (estimate of ||M^T (b - M y)||) and anorm (estimate of ||M||_F).
    Stopping: arnorm <= atol * anorm * rnorm (least-squares test), or
    rnorm <= btol * ||b|| (compatible system).
    """
    y = np.zeros(n_cols)
    beta = np.linalg.norm(b)
    info = dict(iters=0, converged=False, rnorm=beta, arnorm=0.0, anorm=0.0)
    if beta == 0.0:
        info["converged"] = True
        return y, info
    u = b / beta
    v = rmatvec(u)
    alpha = np.linalg.norm(v)
    if alpha == 0.0:
        info["converged"] = True
        return y, info
    v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    anorm2 = 0.0
    bnorm = beta
    for k in range(1, maxit + 1):
        # bidiagonalization step
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u = u / beta
        anorm2 += alpha * alpha + beta * beta
        v = rmatvec(u) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0:
            v = v / alpha
        # plane rotation eliminating the subdiagonal beta
        rho = np.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        # update the solution and the search direction
        y = y + (phi / rho) * w
        w = v - (theta / rho) * w
        rnorm = phibar
        arnorm = phibar * alpha * abs(c)
        anorm = np.sqrt(anorm2)
        info.update(iters=k, rnorm=rnorm, arnorm=arnorm, anorm=anorm)
        if rnorm <= btol * bnorm or arnorm <= atol * anorm * rnorm:
            info["converged"] = True
            break
    return y, info


def householder_qr(X):
    """Economy QR of a tall X in float64 (LAPACK geqrf/orgqr via numpy)."""
    return np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")


def sketch_and_precondition(A, b, SA, Sb, tol=1e-10, maxit=200, warm_start=True):
    """QR of the sketch, warm start, LSQR on A R^-1, back-substitution.

    SA, Sb are the sketched data (any sketch kind or precision, promoted to
    float64 here). Returns (x, info) with info from lsqr plus the warm start.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    Qs, R = householder_qr(SA)
    m = A.shape[1]
    if warm_start:
        x0 = sla.solve_triangular(R, Qs.T @ np.asarray(Sb, dtype=np.float64))
    else:
        x0 = np.zeros(m)
    r0 = b - A @ x0

    def matvec(v):
        return A @ sla.solve_triangular(R, v)

    def rmatvec(u):
        return sla.solve_triangular(R, A.T @ u, trans="T")

    y, info = lsqr(matvec, rmatvec, r0, m, atol=tol, btol=tol, maxit=maxit)
    x = x0 + sla.solve_triangular(R, y)
    info["x0"] = x0
    return x, info
