"""Pins for the oracle's SparseRTT (Def. 1.7) and its SparseCol factor (Def. 4.1).

The sketch is pinned to the definition Omega = D F S written with scipy's
Sylvester Hadamard matrix (a library routine, not the oracle's FWHT) and to
explicit products; the SparseCol factor to its structure (exactly xi distinct
nonzeros of magnitude sqrt(npad/xi)/sqrt(d) per column) and to uniform
selection (chi-square); the whole sketch to isotropy, E ||S x||^2 = ||x||^2,
which fixes the 1/sqrt(d xi) scale; and to the embedding property the paper
proves (Thm. 4.2) on the adversarial basis Q = [e_1 ... e_r] at k = 2r.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy import stats

from oracle import sketches as sk


@pytest.mark.parametrize("npad,d,xi,seed", [(8, 3, 1, 0), (32, 16, 5, 1), (64, 40, 64, 2), (1024, 7, 11, 3)])
def test_sparsecol_structure(npad, d, xi, seed):
    sel, sgn = sk.sparsecol_selectors(npad, d, xi, seed)
    assert sel.shape == (d, xi) and sgn.shape == (d, xi)
    for j in range(d):
        assert len(set(sel[j].tolist())) == xi
        assert np.all(np.diff(sel[j]) > 0)
        assert sel[j].min() >= 0 and sel[j].max() < npad
    assert set(np.unique(sgn).tolist()) <= {-1.0, 1.0}
    M = sk.sparsecol_dense(npad, d, xi, seed)
    assert np.all((M != 0).sum(axis=0) == xi)
    np.testing.assert_allclose(np.abs(M[M != 0]), math.sqrt(npad / xi) / math.sqrt(d), rtol=1e-15)


@pytest.mark.parametrize("n,d,xi,seed", [(1, 1, 1, 0), (5, 3, 2, 4), (20, 8, 3, 5), (64, 24, 7, 6), (100, 40, 9, 7)])
def test_sparsertt_matches_definition(n, d, xi, seed):
    npad = sk.srtt_padded_length(n)
    D = np.diag(sk.srtt_signs(npad, seed))
    F = sla.hadamard(npad) / math.sqrt(npad)
    Omega = D @ F @ sk.sparsecol_dense(npad, d, xi, seed)
    S_def = Omega[:n].T  # rows n..npad-1 of Omega only meet the zero padding
    np.testing.assert_allclose(sk.sparsertt_dense(n, d, xi, seed), S_def, rtol=0, atol=1e-13)


def test_sparsecol_selection_uniform():
    npad, d, xi = 64, 3000, 8
    sel, _ = sk.sparsecol_selectors(npad, d, xi, seed=11)
    counts = np.bincount(sel.ravel(), minlength=npad)
    _, p = stats.chisquare(counts)
    assert p > 1e-3
    # the signs are fair
    _, sgn = sk.sparsecol_selectors(npad, d, xi, seed=12)
    assert abs(sgn.mean()) < 4.0 / math.sqrt(sgn.size)


def test_sparsertt_isotropy():
    n, d, xi, trials = 48, 32, 4, 400
    rng = np.random.default_rng(5)
    xs = [np.eye(n)[0], rng.standard_normal(n)]
    for x in xs:
        vals = [np.sum((sk.sparsertt_apply(x[:, None], d, xi, seed=s)) ** 2) for s in range(trials)]
        mean, se = np.mean(vals), np.std(vals) / math.sqrt(trials)
        assert abs(mean - x @ x) < 5 * se + 1e-12 * (x @ x)


def test_default_column_sparsity():
    assert sk.sparsertt_default_xi(800, 1 << 22) == 11  # 1.5 ln 800 = 10.03
    assert sk.sparsertt_default_xi(64, 1 << 10) == 7
    assert sk.sparsertt_default_xi(1, 4) == 1
    assert sk.sparsertt_default_xi(100, 4) == 4


def test_sparsertt_embeds_coordinate_basis():
    # Thm. 4.2: an (r, 1/2)-OSI at k = O(r), xi = O(log r). The coordinate
    # basis is the input that defeats plain subsampling (Sec. 4.1).
    n, r = 1024, 32
    d = 2 * r
    xi = sk.sparsertt_default_xi(d, n)
    Q = np.eye(n)[:, :r]
    for seed in range(5):
        s = np.linalg.svd(sk.sparsertt_apply(Q, d, xi, seed), compute_uv=False)
        assert s[-1] ** 2 > 0.02 and s[0] ** 2 < 4.0
