"""GPU parity of the SRTT sketch (eq. 1.1 with the Walsh-Hadamard transform).

  * S recovered by applying the sketch to identity columns equals the
    oracle's matrix bit for bit (every entry is +-1/sqrt(d) or 0, and each
    output of an identity column is one signed term);
  * SA matches the oracle within (p + 2^a + 2) u sum_i |A_ic| / sqrt(d)
    (p butterfly stages, a of them summed directly at the sampled rows) on
    paddings with zero, one, two and three full passes, several column slabs
    and ragged heights;
  * the least-squares drivers reach the exact solution with an SRTT sketch.
"""
import numpy as np
import pytest
import torch

from oracle import lstsq as ol
from oracle import sketches as sk

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lib():
    from paper_2508_21189_amd import libsketch
    libsketch.load()
    return libsketch


@pytest.mark.parametrize("n,d,seed", [(100, 40, 1), (300, 64, 2), (256, 256, 3), (257, 10, 4)])
def test_identity_recovers_S(lib, n, d, seed):
    S = lib.Sketch("srtt", d, n, 1, seed)
    got = S.apply(torch.eye(n, dtype=torch.float64, device="cuda")).cpu().numpy()
    ref = sk.srtt_dense(n, d, seed)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,m,d,seed", [(20000, 50, 200, 11), (70000, 37, 300, 2), (4096, 8, 64, 3),
                                        (3000, 130, 100, 4), (200, 3, 20, 5), (1 << 20, 20, 80, 6),
                                        (1 << 25, 1, 16, 7)])
def test_apply_parity(lib, n, m, d, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m)) * np.logspace(0, -3, m)
    S = lib.Sketch("srtt", d, n, 1, seed)
    got = S.apply(torch.from_numpy(A).cuda()).cpu().numpy()
    ref = sk.srtt_apply(A, d, seed)
    p = int(np.ceil(np.log2(n)))
    npass = (p - 1) // 8 if p > 8 else 0
    a = p - 8 * npass
    bound = (p + 2 ** a + 2) * 2.0 ** -53 * np.abs(A).sum(axis=0)[None, :] / np.sqrt(d)
    err = np.abs(got - ref)
    assert np.all(err <= bound), "max err/bound %g" % np.max(err / bound)


def test_lstsq_with_srtt_sketch(lib):
    from paper_2508_21189_amd import inputs
    n, m, d = 30011, 60, 240
    A, b, _ = inputs.small_gaussian(n, m, seed=22)
    Ag, bg = torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()
    S = lib.Sketch("srtt", d, n, 1, 22)
    x, rc, info = S.lstsq_precond(Ag, bg, tol=1e-12, maxit=200)
    assert rc == 0
    xs, rs, _ = ol.exact_lstsq_tsqr(A, b)
    assert np.linalg.norm(A @ (x.cpu().numpy() - xs)) <= 1e-10 * np.linalg.norm(b)
    x2, rc2, info2 = S.lstsq_solve(Ag, bg)
    xr, r, _ = ol.sketch_and_solve(sk.srtt_apply(A, d, 22), sk.srtt_apply(b[:, None], d, 22)[:, 0])
    assert info2["rank"] == r == m
    assert np.linalg.norm(x2.cpu().numpy() - xr) <= 1e-11 * np.linalg.norm(xr)
