"""Pins for metrics.coherence (the notation paragraph of Sec. 1.6:
mu(Q) = max_i ||e_i^* Q||^2 for an orthonormal basis Q).

  * a basis containing a coordinate vector has mu = 1 (the largest value
    any orthonormal Q can have: each row norm of Q is at most 1);
  * m orthonormal columns of a normalized Hadamard matrix have every row
    norm equal to m/n, the smallest value (the row norms of an n x m
    orthonormal Q sum to m);
  * mu is invariant under a change of basis of the same subspace, Q -> Q U;
  * the coherent generator of the benchmark's sketch-and-precondition
    workload (Pareto rows with spikes) is coherent, the plain Gaussian one
    is not: mu sits far above, respectively close to, the floor m/n.
"""
import numpy as np
import scipy.linalg as sla

from oracle import metrics


def test_coordinate_vector_gives_one():
    rng = np.random.default_rng(0)
    n, m = 300, 7
    X = rng.standard_normal((n, m))
    X[:, 0] = 0.0
    X[17, 0] = 1.0
    X[17, 1:] = 0.0
    Q = metrics.orth(X)
    assert abs(metrics.coherence(Q) - 1.0) <= 1e-14


def test_hadamard_columns_give_floor():
    n = 256
    H = sla.hadamard(n) / np.sqrt(n)
    for m in (1, 5, 64, 200):
        Q = H[:, 3:3 + m]
        assert abs(metrics.coherence(Q) - m / n) <= 1e-14


def test_basis_invariance_and_bounds():
    rng = np.random.default_rng(1)
    n, m = 500, 12
    Q = metrics.orth(rng.standard_normal((n, m)) * np.exp(3 * rng.standard_normal((n, 1))))
    U = np.linalg.qr(rng.standard_normal((m, m)))[0]
    mu = metrics.coherence(Q)
    assert abs(metrics.coherence(Q @ U) - mu) <= 1e-13
    assert m / n - 1e-15 <= mu <= 1.0 + 1e-15


def test_benchmark_generators_coherent_vs_incoherent():
    from paper_2508_21189_amd import inputs
    n, m = 1 << 16, 20
    A, _, _, nspk = inputs.coherent(n, m, exponent=8.0, seed=3, device="cpu")
    G, _, _ = inputs.scaled_gaussian(n, m, exponent=8.0, seed=3, device="cpu")
    mu_c = metrics.coherence(metrics.orth(A.numpy()))
    mu_g = metrics.coherence(metrics.orth(G.numpy()))
    floor = m / n
    assert nspk > 0
    assert mu_c >= 100.0 * floor
    assert mu_g <= 4.0 * floor
