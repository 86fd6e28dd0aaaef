"""GPU parity of the library's matrix-core GEMM (sk_gemm), the product every
low-rank driver and the materialized Gaussian sketch go through.

Reference: the same product in float64 on the CPU (a plain library matmul of
the exact operand values). Bound, elementwise: a length-K dot product
accumulated in precision u (2^-53 for float64, 2^-24 for float32) in any
order is within (K + 4) u (|op(A)| |op(B)|) of the exact value (Higham,
Accuracy and Stability of Numerical Algorithms, Sec. 3.1), plus the rounding
of alpha * s + beta * C.

Shapes cover ragged tiles in every dimension, K deep enough to split over
workgroups (the partial sums are added in split order), a single element, all
four transpose combinations, padded leading dimensions, and alpha / beta.
"""
import numpy as np
import pytest
import torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lib():
    from paper_2508_21189_amd import libsketch
    libsketch.load()
    return libsketch


SHAPES = [(1, 1, 1), (17, 33, 5), (128, 128, 16), (129, 130, 1000), (512, 300, 4097), (64, 64, 65536),
          (1000, 7, 3), (7, 1000, 300), (300, 512, 20000), (2049, 129, 64)]


def _ref(A, B, ta, tb, alpha, beta, C0):
    a = A.double().cpu().numpy()
    b = B.double().cpu().numpy()
    a = a.T if ta else a
    b = b.T if tb else b
    exact = alpha * (a @ b) + (beta * C0.double().cpu().numpy() if beta != 0 else 0.0)
    mag = abs(alpha) * (np.abs(a) @ np.abs(b)) + (abs(beta) * np.abs(C0.double().cpu().numpy()) if beta else 0.0)
    return exact, mag, a.shape[1]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("M,N,K", SHAPES)
def test_gemm_matches_reference(lib, dtype, ta, tb, M, N, K):
    if M * N * K > 2e9 and dtype == torch.float64 and (ta or tb):
        pytest.skip("covered by the untransposed case at this size")
    g = torch.Generator().manual_seed(M * 131 + N * 7 + K)
    A = torch.randn(*((K, M) if ta else (M, K)), generator=g, dtype=torch.float64).to(dtype).cuda()
    B = torch.randn(*((N, K) if tb else (K, N)), generator=g, dtype=torch.float64).to(dtype).cuda()
    C = lib.gemm(A, B, ta, tb)
    exact, mag, k = _ref(A, B, ta, tb, 1.0, 0.0, torch.zeros(M, N))
    u = 2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24
    err = np.abs(C.double().cpu().numpy() - exact)
    assert np.all(err <= (k + 4) * u * mag + 1e-300)
    # bitwise reproducible
    assert torch.equal(C, lib.gemm(A, B, ta, tb))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gemm_alpha_beta_and_padded_rows(lib, dtype):
    M, N, K = 300, 200, 5000
    g = torch.Generator().manual_seed(5)
    Abig = torch.randn(K, M + 13, generator=g, dtype=torch.float64).to(dtype).cuda()
    Bbig = torch.randn(K, N + 3, generator=g, dtype=torch.float64).to(dtype).cuda()
    Cbig = torch.randn(M, N + 9, generator=g, dtype=torch.float64).to(dtype).cuda()
    A, B, C = Abig[:, :M], Bbig[:, :N], Cbig[:, :N]
    C0 = C.clone()
    pad = Cbig[:, N:].clone()
    out = lib.gemm(A, B, True, False, alpha=-0.75, beta=2.5, C=C)
    exact, mag, k = _ref(A, B, True, False, -0.75, 2.5, C0)
    u = 2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24
    assert np.all(np.abs(out.double().cpu().numpy() - exact) <= (k + 6) * u * mag)
    # the padding columns of C are not touched
    assert torch.equal(Cbig[:, N:], pad)


def test_gemm_k_zero_scales_c(lib):
    A = torch.zeros(5, 0, dtype=torch.float64, device="cuda")
    B = torch.zeros(0, 7, dtype=torch.float64, device="cuda")
    C = torch.ones(5, 7, dtype=torch.float64, device="cuda")
    out = lib.gemm(A, B, beta=3.0, C=C)
    assert torch.equal(out, torch.full((5, 7), 3.0, dtype=torch.float64, device="cuda"))
