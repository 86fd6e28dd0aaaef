"""Pins of the generalized Nystrom oracle (Alg. 4 and Alg. 5) to facts the
paper and linear algebra fix, independent of the oracle's own steps:

  * exact recovery: if rank(A) <= k and Psi^T A Omega keeps that rank, the
    approximation Y (Psi^T Y)^+ Psi^T A equals A (the identity behind
    eq. (generalized-nystrom): Y spans range(A));
  * the defining formula, eq. (generalized-nystrom), A_hat = Y (Psi^T Y)^+ X^T,
    evaluated by a least-squares solve instead of the SVD route;
  * the two algorithms return the same approximation, the SVD form with
    orthonormal factors and a nonnegative descending spectrum;
  * the rank rule of Alg. 4 counts the numerical rank of Psi^T Y.
The test matrices are SparseStack sketches (Def. 1.5) from the oracle.
"""
import numpy as np
import pytest

from oracle import lowrank as lr
from oracle import sketches as sk


def _tests(rows, cols, k, p, zeta, seed):
    Omega = sk.sparsestack_dense(cols, k, zeta, seed).T  # cols x k
    Psi = sk.sparsestack_dense(rows, p, zeta, seed + 1).T  # rows x p
    return Omega, Psi


def _lowrank_plus_noise(rows, cols, rank, noise, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((rows, rank)))
    V, _ = np.linalg.qr(rng.standard_normal((cols, rank)))
    s = np.logspace(0, -3, rank)
    return (U * s) @ V.T + noise * rng.standard_normal((rows, cols))


@pytest.mark.parametrize("rows,cols,rank,k,p", [(80, 60, 6, 8, 12), (120, 90, 10, 12, 20)])
def test_exact_recovery_low_rank(rows, cols, rank, k, p):
    A = _lowrank_plus_noise(rows, cols, rank, 0.0, seed=rank)
    Omega, Psi = _tests(rows, cols, k, p, 4, seed=7)
    F, G, r = lr.gen_nystrom_outer(A, Omega, Psi)
    assert r == rank
    assert np.linalg.norm(F @ G.T - A) <= 1e-10 * np.linalg.norm(A)
    U, s, V, r5 = lr.gen_nystrom_svd(A, Omega, Psi)
    assert r5 == k  # Psi^T Q has full column rank k: Q is orthonormal
    assert np.linalg.norm((U * s) @ V.T - A) <= 1e-10 * np.linalg.norm(A)


def test_matches_defining_formula():
    rows, cols, k, p = 150, 110, 16, 24
    A = _lowrank_plus_noise(rows, cols, 12, 1e-4, seed=3)
    Omega, Psi = _tests(rows, cols, k, p, 4, seed=11)
    F, G, r = lr.gen_nystrom_outer(A, Omega, Psi)
    assert r == k
    Y = A @ Omega
    Z, *_ = np.linalg.lstsq(Psi.T @ Y, Psi.T @ A, rcond=None)  # (Psi^T Y)^+ Psi^T A
    ref = Y @ Z
    assert np.linalg.norm(F @ G.T - ref) <= 1e-9 * np.linalg.norm(ref)


def test_forms_agree_and_svd_form_is_orthonormal():
    rows, cols, k, p = 160, 100, 20, 30
    A = _lowrank_plus_noise(rows, cols, 15, 1e-3, seed=5)
    Omega, Psi = _tests(rows, cols, k, p, 2, seed=13)
    F, G, _ = lr.gen_nystrom_outer(A, Omega, Psi)
    U, s, V, _ = lr.gen_nystrom_svd(A, Omega, Psi)
    assert np.linalg.norm(F @ G.T - (U * s) @ V.T) <= 1e-10 * np.linalg.norm(A)
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= 1e-12 * k
    assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-12 * k
    assert np.all(s >= 0) and np.all(np.diff(s) <= 0)


def test_rank_rule_counts_numerical_rank():
    rows, cols, k, p = 100, 70, 12, 16
    A = _lowrank_plus_noise(rows, cols, 4, 0.0, seed=9)
    Omega, Psi = _tests(rows, cols, k, p, 4, seed=21)
    _, _, r = lr.gen_nystrom_outer(A, Omega, Psi)
    assert r == np.linalg.matrix_rank(Psi.T @ (A @ Omega), tol=5 * 2.0 ** -52 *
                                      np.linalg.norm(Psi.T @ (A @ Omega), 2))
    assert r == 4
