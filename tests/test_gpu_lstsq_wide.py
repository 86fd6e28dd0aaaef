"""GPU parity of the least-squares drivers at every width their kernels
specialise on, against the oracle (through the C-ABI).

Sketch-and-precondition (the high-accuracy solver of Sec. 1.4: QR of the
sketch, then LSQR on A R^-1) at the mixed-precision workload's width, m = 500
and the odd m = 499, n = 2^20, kappa(D) = 1e10, SparseStack d = 2000,
zeta = 8, tol 1e-10, with the sketch reading A itself, its float32 copy and
(m even) its bfloat16 copy: each solution meets both gates against the
oracle's exact solution x* (Householder TSQR of [A b] on the host),
||A (x - x*)|| <= 1e-10 ||b|| and | ||r|| - ||r*|| | <= 1e-10 ||r*||.
Together with the narrower cases here (m = 101, 201, 250, 257, 384) every
instantiation of the fused LSQR pass (16 lanes a row for even m <= 256: 1,
2, 4, 7, 8 column pairs a lane; 64 lanes a row otherwise: 1, 2, 4, 8 columns
a lane) and the wide Householder panel (m > 256) is checked against the
oracle.

Sketch-and-solve (Alg. 3) at m = 200, 500 and 1024 (its largest width):
the device solution equals the oracle's sketch-and-solve on the oracle's own
S A and S b for the same S to 1e-11 relative, with the same rank.
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


def _gates(A, b, x, xs, rs, tol=1e-10):
    r = np.linalg.norm(A @ x - b)
    dA = np.linalg.norm(A @ (x - xs))
    nb = np.linalg.norm(b)
    assert dA <= tol * nb, "||A(x-x*)||/||b|| = %g" % (dA / nb)
    assert abs(r - rs) <= tol * rs, "residual rel diff = %g" % (abs(r - rs) / rs)


@pytest.fixture(scope="module", params=[500, 499])
def wide(request):
    from paper_2508_21189_amd import inputs
    m = request.param
    n = 1 << 20
    print("wide system n=%d m=%d kappa=1e10" % (n, m), flush=True)
    A, b, _ = inputs.scaled_gaussian(n, m, exponent=10.0, seed=300 + m)
    Ah, bh = A.cpu().numpy(), b.cpu().numpy()
    xs, rs, _ = ol.exact_lstsq_tsqr(Ah, bh)
    return m, A, b, Ah, bh, xs, rs


@pytest.mark.parametrize("sketch_dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_precond_wide_vs_exact(lib, wide, sketch_dtype):
    m, A, b, Ah, bh, xs, rs = wide
    if sketch_dtype == torch.bfloat16 and m % 2:
        pytest.skip("bfloat16 rows of odd width are not 4-byte multiples; the apply refuses them")
    n = A.shape[0]
    S = lib.Sketch("sparsestack", 2000, n, 8, 3000 + m)
    As = None if sketch_dtype == torch.float64 else A.to(sketch_dtype)
    x, rc, info = S.lstsq_precond(A, b, tol=1e-10, maxit=300, A_sketch=As)
    assert rc == 0 and info["converged"] == 1
    _gates(Ah, bh, x.cpu().numpy(), xs, rs)


def test_precond_wide_bf16_odd_width_refused(lib):
    n, m = 4096, 499
    A = torch.randn((n, m), dtype=torch.float64, device="cuda")
    b = torch.randn((n,), dtype=torch.float64, device="cuda")
    S = lib.Sketch("sparsestack", 2000, n, 8, 1)
    with pytest.raises(lib.SketchError):
        S.lstsq_precond(A, b, tol=1e-10, maxit=10, A_sketch=A.to(torch.bfloat16))


@pytest.mark.parametrize("m", [101, 201, 250, 257, 384])
def test_precond_every_pass_width_vs_exact(lib, m):
    from paper_2508_21189_amd import inputs
    n = 100003
    A, b, _ = inputs.scaled_gaussian(n, m, exponent=8.0, seed=400 + m)
    Ah, bh = A.cpu().numpy(), b.cpu().numpy()
    xs, rs, _ = ol.exact_lstsq_tsqr(Ah, bh)
    S = lib.Sketch("sparsestack", 4 * m, n, 8 if (4 * m) % 8 == 0 else 4, 500 + m)
    x, rc, info = S.lstsq_precond(A, b, tol=1e-10, maxit=300)
    assert rc == 0 and info["converged"] == 1
    _gates(Ah, bh, x.cpu().numpy(), xs, rs)


@pytest.mark.parametrize("m", [200, 500, 1024])
def test_sketch_and_solve_wide_matches_oracle(lib, m):
    from paper_2508_21189_amd import inputs
    d, zeta = 2 * m, 4
    n = 4 * d + 3
    A, b, _ = inputs.small_gaussian(n, m, seed=m)
    S = lib.Sketch("sparsestack", d, n, zeta, 600 + m)
    x, rc, info = S.lstsq_solve(torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda())
    SA = sk.sparsestack_apply(A, d, zeta, 600 + m)
    Sb = sk.sparsestack_apply(b[:, None], d, zeta, 600 + m)[:, 0]
    xr, r, s = ol.sketch_and_solve(SA, Sb)
    assert rc == 0 and info["rank"] == r == m
    assert abs(info["sigma_max"] - s[0]) <= 1e-12 * s[0]
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-11 * np.linalg.norm(xr)
