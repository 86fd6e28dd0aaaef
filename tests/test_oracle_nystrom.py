"""Pins of the Nystrom oracle (Alg. 2) to facts fixed by the paper and linear
algebra, independent of the oracle's steps:

  * the defining formula, eq. (nystrom-approx): A_hat = Y (Omega^T Y)^+ Y^T,
    evaluated by a pseudo-inverse, matches U diag(lam) U^T up to the shift
    (nu ~ sqrt(n) 2^-52 ||Y||);
  * exact for a psd A of rank <= k: the eigenvalues are recovered;
  * U is orthonormal and lam is nonnegative and descending;
  * the Gram correspondence (Thm. "Gram correspondence"): Nystrom on A equals
    the RSVD projection of A^{1/2}: A_hat = A^{1/2} P A^{1/2}, P the
    orthogonal projector onto range(A^{1/2} Omega).
"""
import numpy as np
import pytest

from oracle import lowrank as lr
from oracle import sketches as sk


def _psd(n, rank, seed, decay=2.0):
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((n, rank)))
    lam = np.arange(1, rank + 1, dtype=np.float64) ** -decay
    return (V * lam) @ V.T, lam, V


def _omega(n, k, zeta, seed):
    return sk.sparsestack_dense(n, k, zeta, seed).T


def test_matches_defining_formula():
    n, k = 300, 40
    A, _, _ = _psd(n, n, seed=1)
    Om = _omega(n, k, 4, 3)
    U, lam, nu = lr.nystrom_psd(A, Om)
    Y = A @ Om
    ref = Y @ np.linalg.pinv(Om.T @ Y) @ Y.T
    assert np.linalg.norm((U * lam) @ U.T - ref) <= 1e-8 * np.linalg.norm(A)
    assert nu < 1e-12 * np.linalg.norm(A, 2) * np.sqrt(n)


@pytest.mark.parametrize("n,rank,k", [(200, 10, 16), (256, 24, 32)])
def test_exact_for_low_rank(n, rank, k):
    A, lam_true, _ = _psd(n, rank, seed=rank)
    Om = _omega(n, k, 4, 5)
    U, lam, _ = lr.nystrom_psd(A, Om)
    assert np.max(np.abs(lam[:rank] - lam_true) / lam_true) <= 1e-8
    assert np.all(lam[rank:] <= 1e-10)
    assert np.linalg.norm((U * lam) @ U.T - A) <= 1e-9 * np.linalg.norm(A)


def test_orthonormal_nonnegative_descending():
    n, k = 250, 48
    A, _, _ = _psd(n, n, seed=7, decay=1.0)
    U, lam, _ = lr.nystrom_psd(A, _omega(n, k, 8, 9))
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= 1e-12 * k
    assert np.all(lam >= 0) and np.all(np.diff(lam) <= 0)


def test_gram_correspondence():
    n, k = 220, 30
    A, lam_all, V = _psd(n, n, seed=11)
    Om = _omega(n, k, 2, 13)
    U, lam, _ = lr.nystrom_psd(A, Om)
    Ahalf = (V * np.sqrt(lam_all)) @ V.T
    Q, _ = np.linalg.qr(Ahalf @ Om)
    ref = Ahalf @ Q @ Q.T @ Ahalf
    assert np.linalg.norm((U * lam) @ U.T - ref) <= 1e-8 * np.linalg.norm(A)
