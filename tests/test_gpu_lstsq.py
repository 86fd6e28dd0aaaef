"""GPU parity of the least-squares drivers against the oracle (through the C-ABI).

Sketch-and-solve (Alg. 3): the device solution equals the oracle's
sketch_and_solve on the oracle's own S A and S b (same seed, same S) to a
tolerance of 1e-11 relative (both are backward stable solves of the same
d x m problem with kappa(S A) ~ 1), with the same numerical rank; on a
rank-deficient A both sides truncate the same singular values.

Sketch-and-precondition: the device solution matches the exact least-squares
solution x* of the oracle (Householder TSQR of [A b] in float64):
||A (x - x*)|| <= 1e-10 ||b|| and | ||r|| - ||r*|| | <= 1e-10 ||r*||, for the
float64 sketch and for float32 and bfloat16 sketch copies of A, on Gaussian,
coherent (Pareto rows, spikes, kappa = 1e8) and kappa = 1e10 column-scaled
inputs, including the benchmark's full 4,194,304 x 200 coherent solve at
tol 1e-10; at the full 8,388,608 x 500 mixed-precision size the float32 and
bfloat16 sketch variants reach the float64 variant's solution; the run is
bitwise reproducible; the iteration cap and the cold
start behave as documented.
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


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _coherent_cpu(n, m, exponent, seed):
    from paper_2508_21189_amd import inputs
    A, b, _, _ = inputs.coherent(n, m, exponent=exponent, seed=seed, device="cpu")
    return A.numpy(), b.numpy()


def _scaled_cpu(n, m, exponent, seed):
    from paper_2508_21189_amd import inputs
    A, b, _ = inputs.scaled_gaussian(n, m, exponent=exponent, seed=seed, device="cpu")
    return A.numpy(), b.numpy()


def _check_vs_exact(A, b, x, tol=1e-10):
    xs, rs, _ = ol.exact_lstsq_tsqr(A, b)
    r = np.linalg.norm(A @ x - b)
    dA = np.linalg.norm(A @ (x - xs))
    nb = np.linalg.norm(b)
    assert dA <= tol * nb, "||A(x-x*)||/||b|| = %g" % (dA / nb)
    assert abs(r - rs) <= tol * rs, "residual rel diff = %g" % (abs(r - rs) / rs)
    return dA / nb, abs(r - rs) / rs


# ---------------------------------------------------------------- sketch-and-solve
@pytest.mark.parametrize("n,m,d,zeta,seed", [(20000, 50, 200, 4, 11), (5001, 37, 160, 8, 2), (3000, 1, 8, 2, 5),
                                            (9000, 64, 64, 4, 3)])
def test_sketch_and_solve_matches_oracle(lib, n, m, d, zeta, seed):
    from paper_2508_21189_amd import inputs
    A, b, _ = inputs.small_gaussian(n, m, seed=seed)
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    x, rc, info = S.lstsq_solve(_gpu(A), _gpu(b))
    SA = sk.sparsestack_apply(A, d, zeta, seed)
    Sb = sk.sparsestack_apply(b[:, None], d, zeta, seed)[:, 0]
    xr, r, s = ol.sketch_and_solve(SA, Sb)
    assert rc == 0 and info["rank"] == r == m
    assert abs(info["sigma_max"] - s[0]) <= 1e-12 * s[0]
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - xr) <= 1e-11 * np.linalg.norm(xr)
    # residual ratio against the exact solve agrees with the oracle's
    xs, rs, _ = ol.exact_lstsq_tsqr(A, b)
    q_gpu = np.linalg.norm(A @ xg - b) / rs
    q_ref = np.linalg.norm(A @ xr - b) / rs
    assert q_gpu >= 1.0 - 1e-12 and abs(q_gpu - q_ref) <= 1e-10 * q_ref


def test_sketch_and_solve_config_distortion(lib):
    """The 20000 x 50 sketch-and-solve configuration (d = 200, zeta = 4): the
    distortion of S on range(A) (Prop. 1.9: alpha = sigma_min(SQ)^2,
    beta = sigma_max(SQ)^2 for an orthonormal basis Q) from the GPU sketch of Q
    equals the oracle's to 1e-12, and it is an embedding (0 < alpha <= 1 <= beta)."""
    from oracle import metrics
    from paper_2508_21189_amd import inputs
    n, m, d, zeta, seed = 20000, 50, 200, 4, 11
    A, _, _ = inputs.small_gaussian(n, m, seed=seed)
    Q = np.linalg.qr(A)[0]
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    ag, bg, eg = metrics.distortion(S.apply(_gpu(Q)).cpu().numpy())
    ar, br, er = metrics.distortion(sk.sparsestack_apply(Q, d, zeta, seed))
    assert abs(ag - ar) <= 1e-12 and abs(bg - br) <= 1e-12
    assert 0.0 < ag <= 1.0 <= bg


def test_sketch_and_solve_rank_deficient(lib):
    from paper_2508_21189_amd import inputs
    n, m, d, zeta, seed = 6000, 24, 96, 4, 8
    A, b, _ = inputs.small_gaussian(n, m, seed=seed)
    A[:, 5] = 2.0 * A[:, 0]   # exact dependencies (scaling by 2 is exact in S A)
    A[:, 17] = -4.0 * A[:, 3]
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    x, rc, info = S.lstsq_solve(_gpu(A), _gpu(b))
    SA = sk.sparsestack_apply(A, d, zeta, seed)
    Sb = sk.sparsestack_apply(b[:, None], d, zeta, seed)[:, 0]
    xr, r, _ = ol.sketch_and_solve(SA, Sb)
    assert r == m - 2 and info["rank"] == r and rc == lib.SK_W_RANKDEF
    # the truncated solution is unique: minimum norm on the kept subspace
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-9 * np.linalg.norm(xr)


def test_sketch_and_solve_identity_is_exact(lib):
    from paper_2508_21189_amd import inputs
    n, m = 2500, 30
    A, b, _ = inputs.small_gaussian(n, m, seed=4)
    S = lib.Sketch("identity", n, n, 1, 0)
    x, rc, _ = S.lstsq_solve(_gpu(A), _gpu(b))
    assert rc == 0
    _check_vs_exact(A, b, x.cpu().numpy(), tol=1e-13)


# ---------------------------------------------------------- sketch-and-precondition
@pytest.mark.parametrize("n,m,d,zeta,seed", [(20000, 50, 200, 4, 1), (30011, 200, 800, 8, 2), (777, 1, 4, 2, 3),
                                            (4096, 64, 64, 8, 4), (100003, 130, 520, 8, 5)])
def test_precond_gaussian_matches_exact(lib, n, m, d, zeta, seed):
    from paper_2508_21189_amd import inputs
    A, b, _ = inputs.small_gaussian(n, m, seed=seed)
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    x, rc, info = S.lstsq_precond(_gpu(A), _gpu(b), tol=1e-12, maxit=200)
    assert rc == 0 and info["converged"] == 1
    _check_vs_exact(A, b, x.cpu().numpy())


def test_precond_identity_converges_at_once(lib):
    from paper_2508_21189_amd import inputs
    n, m = 3000, 20
    A, b, _ = inputs.small_gaussian(n, m, seed=9)
    S = lib.Sketch("identity", n, n, 1, 0)
    x, rc, info = S.lstsq_precond(_gpu(A), _gpu(b), tol=1e-12, maxit=20)
    # A R^-1 has orthonormal columns: the warm start is already the solution
    assert rc == 0 and info["iters"] <= 2
    _check_vs_exact(A, b, x.cpu().numpy(), tol=1e-12)


@pytest.mark.parametrize("exponent", [4.0, 8.0])
def test_precond_coherent(lib, exponent):
    n, m, d, zeta = 200000, 200, 800, 8
    A, b = _coherent_cpu(n, m, exponent, seed=21)
    S = lib.Sketch("sparsestack", d, n, zeta, 77)
    x, rc, info = S.lstsq_precond(_gpu(A), _gpu(b), tol=1e-12, maxit=300)
    assert rc == 0
    _check_vs_exact(A, b, x.cpu().numpy())


def test_precond_full_size_coherent(lib):
    """The solve the benchmark times, at its full size: coherent 4,194,304 x 200
    (Pareto rows, spikes, kappa(D) = 1e8; the same generator and seeds),
    SparseStack d = 800, zeta = 8, tol 1e-10, against the oracle's exact
    solution (Householder TSQR of [A b] on the host, about half a minute)."""
    from paper_2508_21189_amd import inputs
    n, m, d, zeta = 1 << 22, 200, 800, 8
    A, b, _, _ = inputs.coherent(n, m, exponent=8.0, seed=200)
    S = lib.Sketch("sparsestack", d, n, zeta, 2000)
    x, rc, info = S.lstsq_precond(A, b, tol=1e-10, maxit=300)
    assert rc == 0 and info["converged"] == 1
    _check_vs_exact(A.cpu().numpy(), b.cpu().numpy(), x.cpu().numpy())


def test_precond_full_size_mixed_precision(lib):
    """The benchmark's mixed-precision system at its full size: 8,388,608 x 500,
    kappa(D) = 1e10 (same generator and seeds), SparseStack d = 2000, zeta = 8,
    tol 1e-10, with the sketch reading A itself, its float32 copy and its
    bfloat16 copy. A property that holds at any size: all three converge to the
    same least-squares solution, so ||A (x_lo - x_64)|| <= 2e-10 ||b|| and the
    residual norms agree to 2e-10 (A x is formed by torch in float64)."""
    from paper_2508_21189_amd import inputs
    n, m, d = 1 << 23, 500, 2000
    A, b, _ = inputs.scaled_gaussian(n, m, exponent=10.0, seed=201)
    S = lib.Sketch("sparsestack", d, n, 8, 2001)
    x64, rc, info = S.lstsq_precond(A, b, tol=1e-10, maxit=300)
    assert rc == 0 and info["converged"] == 1
    nb = float(b.norm())
    r64 = float((A @ x64 - b).norm())
    for dt in (torch.float32, torch.bfloat16):
        As = A.to(dt)
        x, rc, info = S.lstsq_precond(A, b, tol=1e-10, maxit=300, A_sketch=As)
        del As
        assert rc == 0 and info["converged"] == 1
        assert float((A @ (x - x64)).norm()) <= 2e-10 * nb
        assert abs(float((A @ x - b).norm()) - r64) <= 2e-10 * r64


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16])
def test_precond_low_precision_sketch(lib, dt):
    n, m, d, zeta = 120000, 100, 400, 8
    A, b = _scaled_cpu(n, m, 10.0, seed=31)
    Ag = _gpu(A)
    S = lib.Sketch("sparsestack", d, n, zeta, 5)
    x, rc, info = S.lstsq_precond(Ag, _gpu(b), tol=1e-12, maxit=300, A_sketch=Ag.to(dt))
    assert rc == 0 and info["converged"] == 1
    _check_vs_exact(A, b, x.cpu().numpy())


def test_precond_cold_start_and_reproducible(lib):
    from paper_2508_21189_amd import inputs
    n, m, d, zeta = 50000, 80, 320, 8
    A, b, _ = inputs.small_gaussian(n, m, seed=12)
    Ag, bg = _gpu(A), _gpu(b)
    S = lib.Sketch("sparsestack", d, n, zeta, 12)
    x1, rc1, i1 = S.lstsq_precond(Ag, bg, tol=1e-12, maxit=200)
    x2, rc2, i2 = S.lstsq_precond(Ag, bg, tol=1e-12, maxit=200)
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]
    x3, rc3, i3 = S.lstsq_precond(Ag, bg, tol=1e-12, maxit=200, warm_start=False)
    assert rc3 == 0
    _check_vs_exact(A, b, x3.cpu().numpy())


def test_precond_iteration_cap(lib):
    from paper_2508_21189_amd import inputs
    n, m, d, zeta = 20000, 40, 160, 4
    A, b, _ = inputs.small_gaussian(n, m, seed=13)
    Ag, bg = _gpu(A), _gpu(b)
    S = lib.Sketch("sparsestack", d, n, zeta, 13)
    x, rc, info = S.lstsq_precond(Ag, bg, tol=1e-14, maxit=3)
    assert rc == lib.SK_W_NOCONV and info["iters"] == 3 and info["converged"] == 0
    x0, rc0, info0 = S.lstsq_precond(Ag, bg, tol=1e-12, maxit=0)
    assert rc0 == lib.SK_W_NOCONV and info0["iters"] == 0
    # maxit = 0 returns the warm start: the sketch-and-solve solution of the same S
    xs, rcs, _ = S.lstsq_solve(Ag, bg)
    assert torch.allclose(x0, xs, rtol=0, atol=1e-10 * float(xs.abs().max()))


def test_residual(lib):
    from paper_2508_21189_amd import inputs
    n, m = 70001, 33
    A, b, xt = inputs.small_gaussian(n, m, seed=14)
    S = lib.Sketch("sparsestack", 4 * m, n, 4, 1)
    r = S.residual(_gpu(A), _gpu(b), _gpu(xt))
    ref = np.linalg.norm(b - A @ xt)
    assert abs(r - ref) <= 1e-12 * ref


def test_invalid_arguments(lib):
    S = lib.Sketch("sparsestack", 8, 100, 2, 1)
    A = torch.zeros((100, 9), dtype=torch.float64, device="cuda")
    b = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SketchError):
        S.lstsq_precond(A, b)  # d < m
    with pytest.raises(lib.SketchError):
        S.lstsq_solve(A, b)
