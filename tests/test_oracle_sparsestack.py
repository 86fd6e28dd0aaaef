"""Pins for the oracle's SparseStack (Def. 1.5) against what the paper fixes.

  * structure: exactly zeta nonzeros per column of S, one in each block of
    nb rows, values +-1/sqrt(zeta) (Def. 1.5); unit column norms;
  * zeta = 1 is a CountSketch (eq. B.1; Sec. 3.3);
  * isotropy E[S^T S] = I (Def. 1.2, eq. for isotropy; Lemma B.1);
  * the exact second moment of Lemma B.1 gives, for real x,
    Var ||S x||^2 = (2/d) (||x||_2^4 - ||x||_4^4);
  * the bucket law is uniform and the signs are balanced (Def. 1.5);
  * the scipy product equals a dense product and a chunked row-streaming sum.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import sketches as sk


@pytest.mark.parametrize("n,d,zeta", [(257, 40, 4), (100, 24, 8), (64, 7, 1), (33, 5, 5)])
def test_structure(n, d, zeta):
    S = sk.sparsestack_dense(n, d, zeta, seed=11)
    nb = d // zeta
    assert S.shape == (d, n)
    v = sk.inv_sqrt(zeta)
    nz = S != 0
    assert np.all(nz.sum(axis=0) == zeta)
    for t in range(zeta):
        assert np.all(nz[t * nb:(t + 1) * nb].sum(axis=0) == 1)
    assert set(np.unique(np.abs(S[nz]))) == {v}
    np.testing.assert_allclose(np.linalg.norm(S, axis=0), 1.0, rtol=0, atol=4e-16)


def test_countsketch_special_case():
    S = sk.sparsestack_dense(500, 16, 1, seed=3)
    assert np.all((S != 0).sum(axis=0) == 1)
    assert set(np.unique(S[S != 0])) == {-1.0, 1.0}


def test_scale_is_exact_for_powers_of_four():
    assert sk.inv_sqrt(4) == 0.5 and sk.inv_sqrt(1) == 1.0 and sk.inv_sqrt(16) == 0.25


def test_seeds_and_streams_differ():
    b1, s1 = sk.sparsestack_pattern(1000, 64, 8, seed=1)
    b2, s2 = sk.sparsestack_pattern(1000, 64, 8, seed=2)
    assert np.mean(b1 == b2) < 0.3
    # blocks within one column are independent draws (different words)
    assert np.mean(b1[:, 0] == b1[:, 1]) < 0.3
    assert np.mean(b1[:, 3] == b1[:, 4]) < 0.3  # across the Philox call boundary


def test_bucket_law_uniform_and_signs_balanced():
    n, d, zeta = 200_000, 400, 8
    nb = d // zeta
    b, s = sk.sparsestack_pattern(n, d, zeta, seed=12345)
    assert b.min() >= 0 and b.max() < nb
    for t in range(zeta):
        counts = np.bincount(b[:, t], minlength=nb)
        chi2 = np.sum((counts - n / nb) ** 2 / (n / nb))
        assert stats.chi2.sf(chi2, nb - 1) > 1e-6
        plus = np.count_nonzero(s[:, t] == 1)
        assert stats.binomtest(plus, n, 0.5).pvalue > 1e-6
    # pairwise: block t bucket vs block t' bucket independent (collision rate 1/nb)
    coll = np.mean(b[:, 0] == b[:, 5])
    assert abs(coll - 1 / nb) < 5 * np.sqrt((1 / nb) * (1 - 1 / nb) / n)


def test_isotropy():
    """E[S^T S] = I: diag is exactly 1 for every draw; off-diagonals average to 0."""
    n, d, zeta, T = 64, 32, 4, 2000
    acc = np.zeros((n, n))
    for seed in range(T):
        S = sk.sparsestack_dense(n, d, zeta, seed=1000 + seed)
        G = S.T @ S
        assert np.allclose(np.diag(G), 1.0, atol=1e-15, rtol=0)
        acc += G
    acc /= T
    off = acc[~np.eye(n, dtype=bool)]
    # each off-diagonal entry has mean 0 and variance exactly 1/d per draw
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(d * T)
    # and the spread matches that variance
    assert abs(np.var(off) * d * T - 1.0) < 0.15


def test_variance_closed_form():
    """Var ||Sx||^2 = (2/d)(||x||_2^4 - ||x||_4^4) from Lemma B.1 and eq. (B.2)."""
    n, d, zeta, T = 48, 24, 4, 6000
    rng = np.random.default_rng(5)
    x = rng.standard_normal(n)
    vals = np.empty(T)
    for k in range(T):
        vals[k] = np.sum(sk.sparsestack_apply(x[:, None], d, zeta, seed=50_000 + k) ** 2)
    want_mean = np.sum(x ** 2)
    want_var = 2.0 / d * (np.sum(x ** 2) ** 2 - np.sum(x ** 4))
    assert abs(vals.mean() - want_mean) < 5 * np.sqrt(want_var / T)
    assert abs(vals.var() / want_var - 1.0) < 0.12


def test_unit_vector_norm_exact():
    """||S e_i|| = 1 exactly for every i (x = e_i makes the variance zero)."""
    n = 50
    SA = sk.sparsestack_apply(np.eye(n), 20, 4, seed=9)
    np.testing.assert_allclose(np.sum(SA ** 2, axis=0), 1.0, rtol=0, atol=1e-15)


def test_sparse_dense_and_chunked_paths_agree():
    rng = np.random.default_rng(0)
    n, m, d, zeta = 1000, 7, 64, 8
    A = rng.standard_normal((n, m))
    SA = sk.sparsestack_apply(A, d, zeta, seed=77)
    S = sk.sparsestack_dense(n, d, zeta, seed=77)
    np.testing.assert_allclose(SA, S @ A, rtol=1e-13, atol=1e-13)
    part = sum(sk.sparsestack_apply_rows(A[r:r + 300], np.arange(r, min(n, r + 300)), d, zeta, 77)
               for r in range(0, n, 300)) * sk.inv_sqrt(zeta)
    np.testing.assert_allclose(SA, part, rtol=1e-13, atol=1e-13)


def test_right_apply_and_adjoint():
    rng = np.random.default_rng(1)
    n, d, zeta = 300, 40, 4
    S = sk.sparsestack_dense(n, d, zeta, seed=5)
    A = rng.standard_normal((9, n))
    np.testing.assert_allclose(sk.sparsestack_apply_T(A, d, zeta, 5), A @ S.T, rtol=1e-13, atol=1e-13)
    Y = rng.standard_normal((d, 3))
    np.testing.assert_allclose(sk.sparsestack_adjoint(Y, n, zeta, 5), S.T @ Y, rtol=1e-13, atol=1e-13)
    # <S X, Y> = <X, S^T Y>
    X = rng.standard_normal((n, 3))
    lhs = np.sum(sk.sparsestack_apply(X, d, zeta, 5) * Y)
    rhs = np.sum(X * sk.sparsestack_adjoint(Y, n, zeta, 5))
    assert abs(lhs - rhs) < 1e-12 * max(1, abs(lhs))


def test_planted_shared_word_is_caught(monkeypatch):
    """If every block reused one Philox word, Var||Sx||^2 would grow by zeta."""
    from oracle import philox as px
    real = px.philox4x32_10

    def same_word(*a, **k):
        w = real(*a, **k)
        return (w[0], w[0], w[0], w[0])

    monkeypatch.setattr(px, "philox4x32_10", same_word)
    n, d, zeta, T = 48, 24, 4, 1500
    x = np.random.default_rng(5).standard_normal(n)
    vals = [np.sum(sk.sparsestack_apply(x[:, None], d, zeta, seed=9000 + k) ** 2) for k in range(T)]
    want_var = 2.0 / d * (np.sum(x ** 2) ** 2 - np.sum(x ** 4))
    assert np.var(vals) / want_var > 2.0
