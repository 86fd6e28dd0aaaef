"""Pins for the oracle's least-squares and low-rank drivers.

  * sketch-and-solve (Alg. 3): exact on consistent systems; the identity
    sketch reduces to LAPACK's least squares; Lemma 2.5's error formula and
    the Pythagorean split used in the proof of Thm. 2.6 hold to rounding;
    the 5 eps rank test removes an exactly dependent column and returns the
    minimum-norm solution; closed form for one column;
  * the TSQR exact solver agrees with LAPACK's least squares and its
    residual is orthogonal to range(A);
  * LSQR agrees with scipy's independent implementation;
  * sketch-and-precondition reaches the exact solution;
  * RSVD (Alg. 1): exact on rank <= k inputs; error bounded below by the
    Eckart-Young floor and above by the HMT decomposition (Thm. 9.1 of
    Halko et al., quoted before the proof of Thm. 2.2).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import lowrank, lstsq, metrics
from oracle import sketches as sk


def _problem(n=2000, m=20, noise=1e-3, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m))
    xt = rng.standard_normal(m)
    b = A @ xt + noise * rng.standard_normal(n)
    return A, b, xt


def test_sketch_and_solve_consistent_system_exact():
    A, b, xt = _problem(noise=0.0)
    SA = sk.sparsestack_apply(A, 80, 4, seed=1)
    Sb = sk.sparsestack_apply(b[:, None], 80, 4, seed=1)[:, 0]
    x, r, _ = lstsq.sketch_and_solve(SA, Sb)
    assert r == A.shape[1]
    np.testing.assert_allclose(x, xt, rtol=1e-12, atol=1e-12)


def test_identity_sketch_is_lapack_lstsq():
    A, b, _ = _problem()
    x, r, _ = lstsq.sketch_and_solve(A, b)
    np.testing.assert_allclose(x, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-11, atol=1e-12)


def test_lemma_2_5_and_pythagorean_split():
    A, b, _ = _problem(n=600, m=8, noise=0.3, seed=4)
    d, zeta = 40, 4
    Q, Rq = np.linalg.qr(A)
    Qfull, _ = np.linalg.qr(A, mode="complete")
    Qp = Qfull[:, A.shape[1]:]
    S = sk.sparsestack_dense(A.shape[0], d, zeta, seed=3)
    Psi1, Psi2 = S @ Q, S @ Qp
    z_star = Q.T @ b
    z_tilde = np.linalg.pinv(Psi1) @ (S @ b)
    np.testing.assert_allclose(z_tilde - z_star, np.linalg.pinv(Psi1) @ Psi2 @ (Qp.T @ b), rtol=1e-9, atol=1e-11)
    # the oracle's x maps to z_tilde through z = R x
    x, _, _ = lstsq.sketch_and_solve(S @ A, S @ b)
    np.testing.assert_allclose(Rq @ x, z_tilde, rtol=1e-9, atol=1e-11)
    r_tilde = np.linalg.norm(A @ x - b) ** 2
    r_star = np.linalg.norm(Q @ z_star - b) ** 2
    assert abs(r_tilde - (r_star + np.linalg.norm(z_tilde - z_star) ** 2)) < 1e-10 * r_tilde


def test_rank_truncation_minimum_norm():
    A, b, _ = _problem(n=500, m=6, seed=2)
    A = np.hstack([A, A[:, :1]])  # exactly dependent column
    x, r, s = lstsq.sketch_and_solve(A, b)
    assert r == 6 and s[-1] <= 5 * lstsq.EPS_MACH * s[0]
    np.testing.assert_allclose(x, np.linalg.pinv(A) @ b, rtol=1e-9, atol=1e-10)
    assert abs(x[0] - x[-1]) < 1e-10  # minimum norm splits the weight evenly


def test_single_column_closed_form():
    rng = np.random.default_rng(9)
    a, b = rng.standard_normal(12), rng.standard_normal(12)
    x, r, _ = lstsq.sketch_and_solve(a[:, None], b)
    assert abs(x[0] - np.dot(a, b) / np.dot(a, a)) < 1e-14


def test_tsqr_matches_lapack_and_orthogonality():
    A, b, _ = _problem(n=5000, m=15, noise=0.5, seed=3)
    x, rn, R = lstsq.exact_lstsq_tsqr(A, b, chunk=777)
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    np.testing.assert_allclose(x, xl, rtol=1e-12, atol=1e-13)
    r = b - A @ x
    assert abs(rn - np.linalg.norm(r)) < 1e-12 * np.linalg.norm(r)
    assert np.linalg.norm(A.T @ r) < 1e-10 * np.linalg.norm(A) * np.linalg.norm(r)


def test_lsqr_against_scipy():
    A, b, _ = _problem(n=3000, m=30, noise=0.1, seed=5)
    A = A * np.logspace(0, 2, 30)
    y, info = lstsq.lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 30, atol=1e-12, btol=1e-12, maxit=500)
    ys = spla.lsqr(A, b, atol=1e-12, btol=1e-12, iter_lim=500)[0]
    np.testing.assert_allclose(y, ys, rtol=1e-8, atol=1e-10)
    assert info["converged"]


def test_sketch_and_precondition_reaches_exact_solution():
    rng = np.random.default_rng(6)
    n, m = 20000, 40
    A = rng.standard_normal((n, m)) * np.logspace(0, -8, m)  # kappa ~ 1e8 from column scaling
    b = A @ rng.standard_normal(m) + 1e-3 * rng.standard_normal(n)
    SA = sk.sparsestack_apply(A, 160, 8, seed=2)
    Sb = sk.sparsestack_apply(b[:, None], 160, 8, seed=2)[:, 0]
    x, info = lstsq.sketch_and_precondition(A, b, SA, Sb, tol=1e-12)
    xs, rs, _ = lstsq.exact_lstsq_tsqr(A, b)
    assert info["converged"] and info["iters"] < 80
    assert abs(np.linalg.norm(A @ x - b) - rs) <= 1e-10 * rs
    assert np.linalg.norm(A @ (x - xs)) <= 1e-10 * np.linalg.norm(b)


def test_rsvd_exact_for_low_rank():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((300, 12)) @ rng.standard_normal((12, 200))
    Y = sk.sparsestack_apply_T(A, 32, 8, seed=1)
    U, s, Vt, Q = lowrank.rsvd_from_sketch(A, Y)
    np.testing.assert_allclose((U * s) @ Vt, A, rtol=0, atol=1e-10 * np.linalg.norm(A))
    np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)


def test_rsvd_error_between_eckart_young_and_hmt():
    rng = np.random.default_rng(8)
    n, dcols, k, r = 200, 150, 40, 20
    Uo = metrics.orth(rng.standard_normal((n, dcols)))
    Vo = metrics.orth(rng.standard_normal((dcols, dcols)))
    sig = np.arange(1, dcols + 1, dtype=float) ** -2.0
    A = (Uo * sig) @ Vo.T
    Om = sk.sparsestack_dense(dcols, k, 4, seed=5).T  # dcols x k
    _, _, _, Q = lowrank.rsvd_from_sketch(A, A @ Om)
    err2 = lowrank.frobenius_residual(A, Q) ** 2
    floor = np.sum(sig[k:] ** 2)
    V1, V2 = Vo[:, :r], Vo[:, r:]
    S2 = sig[r:]
    hmt = np.sum(S2 ** 2) + np.linalg.norm((S2[:, None] * (V2.T @ Om)) @ np.linalg.pinv(V1.T @ Om)) ** 2
    assert floor * (1 - 1e-9) <= err2 <= hmt * (1 + 1e-9)
    spec = lowrank.spectral_residual(A, Q, iters=200)
    assert abs(spec - np.linalg.norm(A - Q @ (Q.T @ A), 2)) < 1e-6 * spec
