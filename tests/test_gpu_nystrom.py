"""GPU parity of the Nystrom approximation (Alg. 2) against the oracle.

U diag(lam) U^T is unique where the eigenvalues are simple, so the tests
compare the approximation, the eigenvalues (relative to lam_1: entries near
the shift nu carry errors of order nu), the shift, and U's orthonormality.
The shift uses ||Y||_2 from 100 power iterations on the device and the exact
norm in the oracle; both are ~sqrt(n) 2^-52 ||Y||, so their difference moves
lam by far less than the tolerance.
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


def _psd(n, rank, seed, decay=2.0):
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((n, rank)))
    lam = np.arange(1, rank + 1, dtype=np.float64) ** -decay
    A = (V * lam) @ V.T
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("n,k,zeta,decay", [(2000, 64, 4, 2.0), (3001, 96, 8, 1.0), (1024, 40, 2, 3.0)])
def test_matches_oracle_f64(lib, n, k, zeta, decay):
    A = _psd(n, n, seed=k, decay=decay)
    S = lib.Sketch("sparsestack", k, n, zeta, 500 + k)
    U, lam, rc, info = lib.nystrom_psd(S, torch.from_numpy(A).cuda())
    assert rc == 0
    Ur, lr_, nu = lr.nystrom_psd(A, sk.sparsestack_dense(n, k, zeta, 500 + k).T)
    U, lam = U.cpu().numpy(), lam.cpu().numpy()
    assert abs(info["nu"] - nu) <= 1e-3 * nu
    assert np.max(np.abs(lam - lr_)) <= 1e-9 * lr_[0]
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= 1e-10 * k
    got = (U * lam) @ U.T
    ref = (Ur * lr_) @ Ur.T
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(A)


def test_exact_for_low_rank(lib):
    n, rank, k = 1500, 20, 32
    A = _psd(n, rank, seed=3)
    S = lib.Sketch("sparsestack", k, n, 4, 77)
    U, lam, rc, _ = lib.nystrom_psd(S, torch.from_numpy(A).cuda())
    assert rc == 0
    lam = lam.cpu().numpy()
    true = np.arange(1, rank + 1, dtype=np.float64) ** -2.0
    assert np.max(np.abs(lam[:rank] - true) / true) <= 1e-8
    U = U.cpu().numpy()
    assert np.linalg.norm((U * lam) @ U.T - A) <= 1e-9 * np.linalg.norm(A)


@pytest.mark.parametrize("kind", ["gaussian", "sparsestack"])
def test_f32_input_and_gaussian(lib, kind):
    n, k = 2048, 64
    A64 = _psd(n, n, seed=5)
    A32 = A64.astype(np.float32)
    zeta = 4 if kind == "sparsestack" else 1
    S = lib.Sketch(kind, k, n, zeta, 91)
    U, lam, rc, _ = lib.nystrom_psd(S, torch.from_numpy(A32).cuda())
    assert rc == 0
    Om = (sk.sparsestack_dense(n, k, zeta, 91) if kind == "sparsestack" else sk.gaussian_dense(n, k, 91)).T
    Ur, lr_, _ = lr.nystrom_psd(A32.astype(np.float64), Om)
    lam = lam.cpu().numpy()
    # F32 accumulation in the sketch: n-term sums, relative 2^-24 each
    assert np.max(np.abs(lam - lr_)) <= n * 2.0 ** -24 * lr_[0]
