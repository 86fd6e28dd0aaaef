"""GPU parity of generalized Nystrom (Alg. 4 and 5) against the oracle.

The approximation A_hat is unique (the factors are not: singular vectors
carry signs), so the tests compare A_hat = F G^T (Alg. 4) and U diag(s) V^T
(Alg. 5) with the oracle's, plus the numerical rank, the singular values of
the SVD form and its orthonormality. Both test matrices are SparseStack
sketches (Omega^T = S_omega, Psi^T = S_psi); the oracle builds the same ones
from the same seeds. Tolerances: A_hat passes through (Psi^T Y)^+, whose
conditioning kappa multiplies rounding, so the bound is a few times
kappa(Psi^T Y) * 2^-53 * ||A|| (F64) or * 2^-24 (F32 input, accumulated in
F32 by the applies).
"""
import numpy as np
import pytest
import torch

from oracle import lowrank as lr
from oracle import sketches as sk

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lib():
    from paper_2508_21189_amd import libsketch
    libsketch.load()
    return libsketch


def _lowrank_plus_noise(rows, cols, rank, noise, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((rows, rank)))
    V, _ = np.linalg.qr(rng.standard_normal((cols, rank)))
    s = np.logspace(0, -2, rank)
    return (U * s) @ V.T + noise * rng.standard_normal((rows, cols))


def _setup(lib, rows, cols, k, p, zeta, seed):
    So = lib.Sketch("sparsestack", k, cols, zeta, seed)
    Sp = lib.Sketch("sparsestack", p, rows, zeta, seed + 1)
    Omega = sk.sparsestack_dense(cols, k, zeta, seed).T
    Psi = sk.sparsestack_dense(rows, p, zeta, seed + 1).T
    return So, Sp, Omega, Psi


def _kappa(A, Omega, Psi):
    s = np.linalg.svd(Psi.T @ (A @ Omega), compute_uv=False)
    return s[0] / s[-1]


@pytest.mark.parametrize("rows,cols,k,p,zeta", [(3000, 2000, 40, 60, 4), (1500, 2500, 32, 48, 8),
                                                (4001, 777, 24, 36, 4)])
def test_outer_matches_oracle_f64(lib, rows, cols, k, p, zeta):
    A = _lowrank_plus_noise(rows, cols, 30, 1e-4, seed=k)
    So, Sp, Omega, Psi = _setup(lib, rows, cols, k, p, zeta, 100 + k)
    F, G, rc, info = lib.gen_nystrom(So, Sp, torch.from_numpy(A).cuda(), form="outer")
    assert rc == 0
    Fr, Gr, r = lr.gen_nystrom_outer(A, Omega, Psi)
    assert info["rank"] == r == k
    got = F.cpu().numpy() @ G.cpu().numpy().T
    ref = Fr @ Gr.T
    tol = 50 * _kappa(A, Omega, Psi) * 2.0 ** -53 * np.linalg.norm(A)
    assert np.linalg.norm(got - ref) <= tol, (np.linalg.norm(got - ref), tol)


def test_outer_exact_for_low_rank(lib):
    rows, cols, k, p = 2000, 1200, 16, 24
    A = _lowrank_plus_noise(rows, cols, 10, 0.0, seed=1)
    So, Sp, Omega, Psi = _setup(lib, rows, cols, k, p, 4, 7)
    F, G, rc, info = lib.gen_nystrom(So, Sp, torch.from_numpy(A).cuda(), form="outer")
    assert rc == 0 and info["rank"] == 10
    got = F.cpu().numpy() @ G.cpu().numpy().T
    assert np.linalg.norm(got - A) <= 1e-9 * np.linalg.norm(A)
    # the columns past the rank are zero
    assert torch.all(F[:, 10:] == 0) and torch.all(G[:, 10:] == 0)


@pytest.mark.parametrize("rows,cols,k,p,zeta", [(3000, 2000, 40, 60, 4), (2500, 1500, 32, 48, 2)])
def test_svd_form_matches_oracle_f64(lib, rows, cols, k, p, zeta):
    A = _lowrank_plus_noise(rows, cols, 30, 1e-4, seed=k + 1)
    So, Sp, Omega, Psi = _setup(lib, rows, cols, k, p, zeta, 200 + k)
    U, s, V, rc, info = lib.gen_nystrom(So, Sp, torch.from_numpy(A).cuda(), form="svd")
    assert rc == 0
    Ur, sr, Vr, r = lr.gen_nystrom_svd(A, Omega, Psi)
    assert info["rank"] == r
    U, s, V = U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy()
    kap = _kappa(A, Omega, Psi)
    assert np.max(np.abs(s - sr)) <= 50 * kap * 2.0 ** -53 * sr[0]
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= 1e-10 * k
    assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-10 * k
    got = (U * s) @ V.T
    ref = (Ur * sr) @ Vr.T
    assert np.linalg.norm(got - ref) <= 50 * kap * 2.0 ** -53 * np.linalg.norm(A)


def test_outer_f32_input(lib):
    rows, cols, k, p = 3000, 2000, 40, 60
    A = _lowrank_plus_noise(rows, cols, 30, 1e-3, seed=4).astype(np.float32)
    A64 = A.astype(np.float64)
    So, Sp, Omega, Psi = _setup(lib, rows, cols, k, p, 4, 300)
    F, G, rc, info = lib.gen_nystrom(So, Sp, torch.from_numpy(A).cuda(), form="outer")
    assert rc == 0
    Fr, Gr, r = lr.gen_nystrom_outer(A64, Omega, Psi)
    assert info["rank"] == r
    got = F.cpu().numpy() @ G.cpu().numpy().T
    ref = Fr @ Gr.T
    tol = 50 * _kappa(A64, Omega, Psi) * (rows + cols) * 2.0 ** -24 * np.linalg.norm(A64)
    assert np.linalg.norm(got - ref) <= tol, (np.linalg.norm(got - ref), tol)


def test_forms_agree_on_gpu(lib):
    rows, cols, k, p = 2000, 1600, 24, 36
    A = torch.from_numpy(_lowrank_plus_noise(rows, cols, 20, 1e-4, seed=8)).cuda()
    So = lib.Sketch("sparsestack", k, cols, 4, 55)
    Sp = lib.Sketch("sparsestack", p, rows, 4, 56)
    F, G, _, _ = lib.gen_nystrom(So, Sp, A, form="outer")
    U, s, V, _, _ = lib.gen_nystrom(So, Sp, A, form="svd")
    d = torch.linalg.norm(F @ G.T - (U * s) @ V.T) / torch.linalg.norm(A)
    assert d.item() <= 1e-8


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_outer_with_gaussian_tests(lib, dtype):
    """The comparison in the paper's compression experiment: Gaussian Omega
    and Psi (Def. 1.4; Psi^T A through the F64 MFMA kernel or, for F32 input,
    G written out and one SGEMM)."""
    rows, cols, k, p = 2500, 1800, 32, 48
    A = _lowrank_plus_noise(rows, cols, 24, 1e-3, seed=12).astype(dtype)
    A64 = A.astype(np.float64)
    So = lib.Sketch("gaussian", k, cols, 1, 400)
    Sp = lib.Sketch("gaussian", p, rows, 1, 401)
    Omega = sk.gaussian_dense(cols, k, 400).T
    Psi = sk.gaussian_dense(rows, p, 401).T
    F, G, rc, info = lib.gen_nystrom(So, Sp, torch.from_numpy(A).cuda(), form="outer")
    assert rc == 0
    Fr, Gr, r = lr.gen_nystrom_outer(A64, Omega, Psi)
    assert info["rank"] == r
    got = F.cpu().numpy() @ G.cpu().numpy().T
    u = 2.0 ** -53 if dtype == np.float64 else (rows + cols) * 2.0 ** -24
    tol = 50 * _kappa(A64, Omega, Psi) * u * np.linalg.norm(A64)
    assert np.linalg.norm(got - Fr @ Gr.T) <= tol


def test_invalid_shapes_fail_cleanly(lib):
    A = torch.zeros((100, 80), dtype=torch.float64, device="cuda")
    So = lib.Sketch("sparsestack", 16, 80, 4, 1)
    Sp = lib.Sketch("sparsestack", 12, 100, 4, 2)  # p < k
    with pytest.raises(lib.SketchError):
        lib.gen_nystrom(So, Sp, A, form="outer")
