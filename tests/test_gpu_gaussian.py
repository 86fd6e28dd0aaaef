"""GPU parity of the Gaussian sketch (Def. 1.4) on the FP64 matrix cores.

  * G recovered by applying the sketch to identity columns matches the
    oracle's entries (same Philox bits, same Box-Muller formula in float64;
    only the device and host log / sincos roundings differ): relative 1e-13;
  * SA = G A matches the oracle within the dot-product bound
    (n + splits) * u * (|G||A|) plus the entry-rounding term, on ragged
    shapes, widths of one to several column slabs and a d that leaves a
    partial row slice;
  * the result is bitwise reproducible;
  * the least-squares drivers reach the exact solution with a Gaussian sketch.
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


@pytest.mark.parametrize("n,d,seed", [(300, 40, 1), (97, 130, 2), (512, 64, 3)])
def test_entries_match_oracle(lib, n, d, seed):
    S = lib.Sketch("gaussian", d, n, 1, seed)
    G = S.apply(torch.eye(n, dtype=torch.float64, device="cuda")).cpu().numpy()
    ref = sk.gaussian_dense(n, d, seed)
    assert np.max(np.abs(G - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,m,d,seed", [(20000, 50, 200, 11), (4097, 1, 64, 2), (3001, 200, 800, 3),
                                        (1000, 300, 100, 4), (777, 17, 33, 5), (65536, 64, 256, 6)])
def test_apply_parity(lib, n, m, d, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m)) * np.logspace(0, -3, m)
    S = lib.Sketch("gaussian", d, n, 1, seed)
    got = S.apply(torch.from_numpy(A).cuda()).cpu().numpy()
    G = sk.gaussian_dense(n, d, seed) if n * d <= 4e7 else None
    ref = G @ A if G is not None else sk.gaussian_apply(A, d, seed)
    absGA = np.abs(G) @ np.abs(A) if G is not None else np.abs(ref) + 1.0
    bound = ((n + 4096) * 2.0 ** -53 + 1e-13) * absGA
    err = np.abs(got - ref)
    assert np.all(err <= bound), "max err/bound %g" % np.max(err / bound)


@pytest.mark.parametrize("n,m,d,seed", [(5000, 33, 60, 21), (20000, 200, 300, 22)])
def test_apply_f32_input(lib, n, m, d, seed):
    """F32 input: G written out in F32 and one SGEMM. Against the oracle on
    the F32-rounded A: per entry of G one F32 rounding, then n-term F32 sums,
    so |SA - G A| <= (n + 2) 2^-24 (|G| |A|)."""
    rng = np.random.default_rng(seed)
    A32 = rng.standard_normal((n, m)).astype(np.float32)
    A = A32.astype(np.float64)
    S = lib.Sketch("gaussian", d, n, 1, seed)
    G = sk.gaussian_dense(n, d, seed)
    ref = G @ A
    bound = (n + 2) * 2.0 ** -24 * (np.abs(G) @ np.abs(A))
    for odt in (torch.float32, torch.float64):
        got = S.apply(torch.from_numpy(A32).cuda(), out_dtype=odt).to(torch.float64).cpu().numpy()
        assert np.all(np.abs(got - ref) <= bound + 2.0 ** -24 * np.abs(ref))


def test_bitwise_reproducible(lib):
    rng = np.random.default_rng(0)
    A = torch.from_numpy(rng.standard_normal((30000, 100))).cuda()
    S = lib.Sketch("gaussian", 400, 30000, 1, 9)
    r1 = S.apply(A)
    for _ in range(3):
        assert torch.equal(S.apply(A), r1)


def test_lstsq_with_gaussian_sketch(lib):
    from paper_2508_21189_amd import inputs
    n, m, d = 30011, 60, 240
    A, b, _ = inputs.small_gaussian(n, m, seed=21)
    Ag, bg = torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()
    S = lib.Sketch("gaussian", d, n, 1, 21)
    x, rc, info = S.lstsq_precond(Ag, bg, tol=1e-12, maxit=200)
    assert rc == 0
    xs, rs, _ = ol.exact_lstsq_tsqr(A, b)
    xg = x.cpu().numpy()
    assert np.linalg.norm(A @ (xg - xs)) <= 1e-10 * np.linalg.norm(b)
    # sketch-and-solve on the same G as the oracle
    x2, rc2, info2 = S.lstsq_solve(Ag, bg)
    G = sk.gaussian_dense(n, d, 21)
    xr, r, _ = ol.sketch_and_solve(G @ A, G @ b)
    assert info2["rank"] == r == m
    assert np.linalg.norm(x2.cpu().numpy() - xr) <= 1e-11 * np.linalg.norm(xr)
