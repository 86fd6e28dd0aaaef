"""Pins for the oracle's SRTT (eq. 1.1) and Gaussian (Def. 1.4) sketches.

SRTT: the transform is pinned to scipy's Sylvester Hadamard matrix (a
library routine), to H H = npad I and Parseval; the sample is a set of d
distinct sorted rows; each column of S has norm exactly 1; the sketch is
isotropic (E[S^T S] = I, the scaling rule of Sec. 1.4.2).
Gaussian: entries are iid N(0, 1/d) (mean, variance, Kolmogorov-Smirnov,
lag correlation) and the squared singular values of G Q sit inside the
Marchenko-Pastur edges (1 -+ sqrt(r/d))^2 (the Gaussian law quoted with
Fig. 2 at r/d = 1/2).
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy import stats

from oracle import metrics
from oracle import sketches as sk


@pytest.mark.parametrize("N", [1, 2, 8, 64, 1024])
def test_fwht_matches_sylvester_hadamard(N):
    rng = np.random.default_rng(N)
    X = rng.standard_normal((N, 3))
    np.testing.assert_allclose(sk.fwht_rows(X), sla.hadamard(N) @ X, rtol=1e-12, atol=1e-12)


def test_fwht_involution_and_parseval():
    rng = np.random.default_rng(2)
    N = 4096
    x = rng.standard_normal(N)
    hx = sk.fwht_rows(x)
    np.testing.assert_allclose(sk.fwht_rows(hx), N * x, rtol=1e-12, atol=1e-9)
    assert abs(np.dot(hx, hx) - N * np.dot(x, x)) < 1e-9 * N * np.dot(x, x)


def test_padding_length():
    assert [sk.srtt_padded_length(n) for n in (1, 2, 3, 20000, 1 << 22)] == [1, 2, 4, 32768, 1 << 22]


@pytest.mark.parametrize("npad,d", [(16, 16), (1024, 100), (32768, 200), (1 << 22, 800)])
def test_sample_distinct_sorted(npad, d):
    R = sk.srtt_sample(npad, d, seed=4)
    assert R.size == d and np.all(np.diff(R) > 0) and R[0] >= 0 and R[-1] < npad


def test_sample_is_uniform():
    """Floyd's algorithm gives each index probability d/npad."""
    npad, d, T = 64, 8, 4000
    hits = np.zeros(npad)
    for s in range(T):
        hits[sk.srtt_sample(npad, d, seed=s)] += 1
    chi2 = np.sum((hits - T * d / npad) ** 2 / (T * d / npad))
    assert stats.chi2.sf(chi2, npad - 1) > 1e-6


def test_srtt_columns_unit_norm_and_values():
    n, d = 100, 24
    S = sk.srtt_dense(n, d, seed=3)
    np.testing.assert_allclose(np.linalg.norm(S, axis=0), 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(np.abs(S), 1 / np.sqrt(d), rtol=0, atol=1e-15)


def test_srtt_isotropy():
    n, d, T = 32, 16, 1500
    acc = np.zeros((n, n))
    for s in range(T):
        S = sk.srtt_dense(n, d, seed=s)
        acc += S.T @ S
    acc /= T
    np.testing.assert_allclose(np.diag(acc), 1.0, atol=1e-12)
    assert np.max(np.abs(acc[~np.eye(n, dtype=bool)])) < 5.0 * np.sqrt(1.0 / (d * T)) * 1.5


def test_srtt_signs_balanced():
    D = sk.srtt_signs(1 << 16, seed=8)
    assert set(np.unique(D)) == {-1.0, 1.0}
    assert stats.binomtest(int(np.sum(D > 0)), D.size, 0.5).pvalue > 1e-6


def test_gaussian_entries_distribution():
    d, n = 64, 4000
    G = sk.gaussian_dense(n, d, seed=21)
    z = (G * np.sqrt(d)).ravel()
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # cos/sin partners of one Box-Muller pair are uncorrelated
    c = np.corrcoef(G[0::2].ravel(), G[1::2].ravel())[0, 1]
    assert abs(c) < 5 / np.sqrt(G.size / 2)


def test_gaussian_apply_chunked_equals_dense():
    rng = np.random.default_rng(3)
    n, d = 700, 20
    A = rng.standard_normal((n, 4))
    np.testing.assert_allclose(sk.gaussian_apply(A, d, 5, chunk=128), sk.gaussian_dense(n, d, 5) @ A,
                               rtol=1e-12, atol=1e-12)


def test_gaussian_marchenko_pastur_edges():
    n, d, r = 4000, 800, 200
    rng = np.random.default_rng(0)
    Q = metrics.orth(rng.standard_normal((n, r)))
    a, b, _ = metrics.distortion(sk.gaussian_apply(Q, d, seed=1))
    lo, hi = (1 - np.sqrt(r / d)) ** 2, (1 + np.sqrt(r / d)) ** 2
    assert lo * 0.85 < a < lo * 1.25 and hi * 0.9 < b < hi * 1.1


def test_sparsestack_distortion_near_gaussian_edges():
    """SparseStack with zeta = 8 on a generic subspace: alpha close to the MP edge."""
    n, d, r = 4000, 800, 200
    rng = np.random.default_rng(0)
    Q = metrics.orth(rng.standard_normal((n, r)))
    a, b, _ = metrics.distortion(sk.sparsestack_apply(Q, d, 8, seed=1))
    lo, hi = (1 - np.sqrt(r / d)) ** 2, (1 + np.sqrt(r / d)) ** 2
    assert lo * 0.8 < a and b < hi * 1.2
