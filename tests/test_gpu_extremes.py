"""GPU injectivity / dilation estimates of a SparseStack on Q = [e_1 ... e_r] (Fig. 2).

  * at sizes where the oracle can take the SVD of S Q, the Lanczos extremes
    match the exact alpha = sigma_min(S Q)^2 and beta = sigma_max(S Q)^2
    (oracle.metrics.distortion, Prop. 1.9) for zeta in {1, 2, 4, 8}, k = 2r;
  * the estimate is bitwise reproducible;
  * at a large r (beyond the oracle) the estimates satisfy what holds at any
    size: alpha <= 1 <= beta (the mean eigenvalue of S^T S is exactly 1 since
    every column of S has unit norm), the 3/4-step values are no better than
    the final ones (Cauchy interlacing of the Lanczos tridiagonals), and the
    values sit where the paper reports them for zeta = 8: alpha near the
    Gaussian limit (1 - 1/sqrt 2)^2 and beta above (1 + 1/sqrt 2)^2;
  * invalid arguments are refused.
"""
import math

import numpy as np
import pytest
import torch

from oracle import metrics
from oracle import sketches as sk

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lib():
    from paper_2508_21189_amd import libsketch
    libsketch.load()
    return libsketch


@pytest.mark.parametrize("r,zeta,seed", [(100, 1, 1), (100, 8, 2), (500, 4, 3), (1000, 2, 4), (2000, 8, 5),
                                         (64, 2, 6), (1, 1, 7)])
def test_extremes_match_exact_svd(lib, r, zeta, seed):
    d = 2 * r
    if d % zeta:
        pytest.skip("d must be a multiple of zeta")
    S = lib.Sketch("sparsestack", d, r, zeta, seed)
    a, b, rc, info = lib.sv_extremes(S, steps=min(r, 800), start_seed=9)
    assert rc == 0
    ae, be, _ = metrics.distortion(sk.sparsestack_dense(r, d, zeta, seed))
    assert abs(b - be) <= 1e-9 * be
    assert abs(a - ae) <= 1e-9 * be
    assert info["steps"] <= min(r, 800)


def test_extremes_reproducible(lib):
    S = lib.Sketch("sparsestack", 20000, 10000, 4, 3)
    r1 = lib.sv_extremes(S, steps=150, start_seed=1)
    r2 = lib.sv_extremes(S, steps=150, start_seed=1)
    assert r1[0] == r2[0] and r1[1] == r2[1]


def test_extremes_large_r_properties(lib):
    r = 1 << 20
    S = lib.Sketch("sparsestack", 2 * r, r, 8, 11)
    a, b, rc, info = lib.sv_extremes(S, steps=300, start_seed=2)
    assert rc == 0 and info["steps"] == 300
    assert 0.0 <= a <= 1.0 <= b
    assert info["alpha_at_3_4"] >= a and info["beta_at_3_4"] <= b
    ga, gb = (1 - 1 / math.sqrt(2)) ** 2, (1 + 1 / math.sqrt(2)) ** 2
    assert 0.5 * ga <= a <= 1.5 * ga
    assert b >= gb


def test_extremes_invalid(lib):
    G = lib.Sketch("gaussian", 20, 10, 1, 1)
    with pytest.raises(lib.SketchError):
        lib.sv_extremes(G, steps=10)
    S = lib.Sketch("sparsestack", 20, 10, 2, 1)
    with pytest.raises(lib.SketchError):
        lib.sv_extremes(S, steps=0)
