"""Seeded synthetic inputs for the benchmark workloads (shared by tests and bench).

This module only draws random test data; it contains none of the sketching or
solver arithmetic. Recipes (the workload shapes of the benchmark configs):

  small_gaussian  A: n x m iid N(0,1); b = A x_true + noise * g, x_true, g ~ N(0, I)
  coherent        A = P G D (n x m): G iid N(0,1); P = diag of Pareto(alpha=1.5)
                  row factors (classical Pareto with x_m = 1), each row further
                  multiplied by 1e3 with probability 0.01 (spikes); D =
                  diag(10^(-e j/(m-1))), j = 0..m-1, so kappa(D) = 10^e exactly.
  scaled_gaussian A = G D with the same column scaling D.
  lowrank_decay   A = U diag(i^-2) V^T with Haar-random orthonormal U (rows x k)
                  and V (cols x k), k = min(rows, cols) (QR of Gaussians).
"""
import numpy as np
import torch


def small_gaussian(n, m, noise=1e-3, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m))
    x = rng.standard_normal(m)
    b = A @ x + noise * rng.standard_normal(n)
    return A, b, x


def _gen(device, seed):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def column_scaling(m, exponent, device="cpu", dtype=torch.float64):
    j = torch.arange(m, device=device, dtype=dtype)
    return torch.pow(torch.tensor(10.0, dtype=dtype, device=device), -exponent * j / max(1, m - 1))


def coherent(n, m, exponent=8.0, alpha=1.5, spike_prob=0.01, spike=1e3, noise=1e-3, seed=0, device="cuda",
             chunk=1 << 20):
    """A = P G D in float64 on `device`, plus b = A x_true + noise g. Returns (A, b, x_true, n_spikes)."""
    g = _gen(device, seed)
    A = torch.empty((n, m), dtype=torch.float64, device=device)
    D = column_scaling(m, exponent, device)
    nspk = 0
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        G = torch.randn((r1 - r0, m), generator=g, dtype=torch.float64, device=device)
        U = torch.rand((r1 - r0,), generator=g, dtype=torch.float64, device=device)
        P = torch.pow(1.0 - U, -1.0 / alpha)  # classical Pareto(alpha), x_m = 1
        S = torch.rand((r1 - r0,), generator=g, dtype=torch.float64, device=device) < spike_prob
        nspk += int(S.sum().item())
        P = torch.where(S, P * spike, P)
        A[r0:r1] = G * P[:, None] * D[None, :]
    x = torch.randn((m,), generator=g, dtype=torch.float64, device=device)
    b = A @ x + noise * torch.randn((n,), generator=g, dtype=torch.float64, device=device)
    return A, b, x, nspk


def scaled_gaussian(n, m, exponent=10.0, noise=1e-3, seed=0, device="cuda", chunk=1 << 20):
    """A = G D in float64 on `device`, plus b. Returns (A, b, x_true)."""
    g = _gen(device, seed)
    A = torch.empty((n, m), dtype=torch.float64, device=device)
    D = column_scaling(m, exponent, device)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        A[r0:r1] = torch.randn((r1 - r0, m), generator=g, dtype=torch.float64, device=device) * D[None, :]
    x = torch.randn((m,), generator=g, dtype=torch.float64, device=device)
    b = A @ x + noise * torch.randn((n,), generator=g, dtype=torch.float64, device=device)
    return A, b, x


def lowrank_decay(rows, cols, seed=0, device="cuda", dtype=torch.float32):
    """A = U diag(i^-2) V^T (rows x cols), U and V Haar-orthonormal; float64 build, cast to dtype."""
    g = _gen(device, seed)
    k = min(rows, cols)
    U, _ = torch.linalg.qr(torch.randn((rows, k), generator=g, dtype=torch.float64, device=device))
    V, _ = torch.linalg.qr(torch.randn((cols, k), generator=g, dtype=torch.float64, device=device))
    sig = torch.arange(1, k + 1, dtype=torch.float64, device=device) ** -2.0
    A = (U * sig[None, :]) @ V.T
    return A.to(dtype), sig


def snapshots_stand_in(rows=131072, cols=40000, rank=300, noise=1e-6, seed=0, device="cuda", dtype=torch.float32):
    """Synthetic stand-in for a matrix of simulation snapshots (the paper's
    compression experiment uses 131072 x 40000 real-ified Gross-Pitaevskii
    snapshots, which are not available): A = U diag(s) V^T + noise * N with
    U, V Haar-orthonormal (rows x rank, cols x rank), s_i = i^-2, N iid
    N(0, 1) scaled by 1/sqrt(cols); then every column is centred to zero mean,
    as the paper does with the snapshots. Built in F32 on the device in
    blocks of rows."""
    g = _gen(device, seed)
    U, _ = torch.linalg.qr(torch.randn((rows, rank), generator=g, dtype=torch.float64, device=device))
    V, _ = torch.linalg.qr(torch.randn((cols, rank), generator=g, dtype=torch.float64, device=device))
    s = torch.arange(1, rank + 1, dtype=torch.float64, device=device) ** -2.0
    Us = (U * s[None, :]).to(dtype)
    Vt = V.T.contiguous().to(dtype)
    del U, V
    A = torch.empty((rows, cols), dtype=dtype, device=device)
    blk = 16384
    for r0 in range(0, rows, blk):
        r1 = min(rows, r0 + blk)
        torch.matmul(Us[r0:r1], Vt, out=A[r0:r1])
        A[r0:r1].add_(torch.randn((r1 - r0, cols), generator=g, dtype=dtype, device=device),
                      alpha=noise / cols ** 0.5)
    A -= A.mean(dim=0, keepdim=True)
    return A


def psd_stand_in(n=32768, rank=1000, delta=1e-6, seed=0, device="cuda", dtype=torch.float32):
    """Synthetic psd matrix (kernel/covariance stand-in): A = V diag(i^-2) V^T +
    delta I with V Haar-orthonormal (n x rank), built in F64 in row blocks
    and cast to dtype."""
    g = _gen(device, seed)
    V, _ = torch.linalg.qr(torch.randn((n, rank), generator=g, dtype=torch.float64, device=device))
    lam = torch.arange(1, rank + 1, dtype=torch.float64, device=device) ** -2.0
    Vl = V * lam[None, :]
    A = torch.empty((n, n), dtype=dtype, device=device)
    blk = 4096
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        B = Vl[r0:r1] @ V.T
        B[:, r0:r1].diagonal().add_(delta)
        A[r0:r1] = B.to(dtype)
    return A
