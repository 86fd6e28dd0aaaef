"""GPU parity of the batched sketch-and-solve (lstsq_sketch_solve_batched).

Every problem is solved with its own SparseStack (d = 4k, zeta = 4, its own
seed) and compared with the oracle's sketch-and-solve (Alg. 3) on the
oracle's own S A and S b for the same sketch:
  * float64 problems to 1e-11 relative, as the single-problem driver;
  * float32 and bfloat16 problems (the sketch accumulates in float32) within
    the first-order perturbation bound of the small least-squares problem,
    (||E|| ||x|| + ||e||) / s_min + ||E|| ||r|| / s_min^2 (doubled), where
    |E| <= (c_j + 8) 2^-24 (|S||A|) and |e| <= (c_j + 8) 2^-24 (|S||b|)
    bound the sketch's rounding entrywise (the oracle reads the same rounded
    values);
  * a rank-deficient problem (which the full-rank certificate cannot pass, so
    it is redone with the SVD of R) is reported as such, with the oracle's
    truncated solution, while the others succeed;
  * a batch is bitwise reproducible, and a caller workspace gives the same
    results as the internal one.
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


def _problem(n, k, dtype, seed, dependent=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, k))
    if dependent:
        A[:, k - 1] = 2.0 * A[:, 0]
    b = A @ rng.standard_normal(k) + 1e-4 * rng.standard_normal(n)
    At = torch.from_numpy(A).to(dtype).cuda()
    bt = torch.from_numpy(b).to(dtype).cuda()
    return At, bt


def _oracle(A64, b64, k, seed, u):
    d = 4 * k
    SA = sk.sparsestack_apply(A64, d, 4, seed)
    Sb = sk.sparsestack_apply(b64[:, None], d, 4, seed)[:, 0]
    x, r, s = ol.sketch_and_solve(SA, Sb)
    Sabs = abs(sk.sparsestack_csr(A64.shape[0], d, 4, seed))
    cnt = np.asarray((Sabs != 0).sum(axis=1)).ravel()[:, None]
    E = np.linalg.norm((cnt + 8.0) * u * (Sabs @ np.abs(A64)))
    e = np.linalg.norm((cnt[:, 0] + 8.0) * u * (Sabs @ np.abs(b64)))
    res = np.linalg.norm(SA @ x - Sb)
    smin = s[r - 1]
    tol = 2.0 * ((E * np.linalg.norm(x) + e) / smin + E * res / smin ** 2)
    return x, r, tol


CASES = [(3000, 16, torch.float64), (12000, 33, torch.float32), (40001, 64, torch.float32),
         (5000, 100, torch.bfloat16), (20000, 48, torch.float64), (7000, 20, torch.float32)]


def test_batched_matches_oracle(lib):
    problems = []
    for i, (n, k, dt) in enumerate(CASES):
        A, b = _problem(n, k, dt, 10 + i)
        problems.append((A, b, 1000 + i))
    xs, status, ranks, t_ms, rc = lib.solve_batched(problems)
    assert rc == 0 and status == [0] * len(CASES)
    for (A, b, seed), x, rank, t, (n, k, dt) in zip(problems, xs, ranks, t_ms, CASES):
        A64 = A.to(torch.float64).cpu().numpy()
        b64 = b.to(torch.float64).cpu().numpy()
        xg = x.cpu().numpy()
        if dt == torch.float64:
            xr, r, _ = _oracle(A64, b64, k, seed, 2.0 ** -53)
            assert np.linalg.norm(xg - xr) <= 1e-11 * np.linalg.norm(xr)
        else:
            xr, r, tol = _oracle(A64, b64, k, seed, 2.0 ** -24)
            assert np.linalg.norm(xg - xr) <= tol
        assert rank == r == k and t > 0.0


def test_batched_rank_deficient_problem(lib):
    problems = [(*_problem(4000, 12, torch.float64, 1), 5), (*_problem(4000, 12, torch.float64, 2, True), 6)]
    xs, status, ranks, t_ms, rc = lib.solve_batched(problems)
    assert rc == lib.SK_W_RANKDEF
    assert status == [0, lib.SK_W_RANKDEF] and ranks == [12, 11]
    A64 = problems[1][0].cpu().numpy()
    b64 = problems[1][1].cpu().numpy()
    xr, r, _ = _oracle(A64, b64, 12, 6, 2.0 ** -53)
    assert r == 11 and np.linalg.norm(xs[1].cpu().numpy() - xr) <= 1e-9 * np.linalg.norm(xr)


def test_batched_reproducible_and_caller_workspace(lib):
    problems = []
    for i, (n, k, dt) in enumerate(CASES[:4]):
        A, b = _problem(n, k, dt, 40 + i)
        problems.append((A, b, 77 + i))
    x1 = lib.solve_batched(problems)[0]
    x2 = lib.solve_batched(problems)[0]
    ws = torch.empty(lib.batched_workspace_size(problems), dtype=torch.uint8, device="cuda")
    x3 = lib.solve_batched(problems, ws=ws)[0]
    for a, b, c in zip(x1, x2, x3):
        assert torch.equal(a, b) and torch.equal(a, c)
    with pytest.raises(lib.SketchError):
        lib.solve_batched(problems, ws=ws[:16])


def test_batched_refuses_unsupported_layout_before_any_work(lib):
    """BF16 data with an odd number of columns (> 4) has rows that are not 4-byte
    multiples, which the apply does not take: that problem's status and the
    call's result are SK_E_NOTSUP, and no solution is written."""
    good = _problem(3000, 16, torch.float32, 1)
    odd = _problem(3000, 17, torch.bfloat16, 2)
    arr, xs = lib._batched_array([(*good, 1), (*odd, 2)])
    for x in xs:
        x.fill_(7.0)
    rc = lib.load().lstsq_sketch_solve_batched(arr, 2, 4, 4, None, 0, None)
    assert rc == lib.SK_E_NOTSUP
    assert [p.status for p in arr] == [0, lib.SK_E_NOTSUP]
    torch.cuda.synchronize()
    assert all(bool((x == 7.0).all()) for x in xs)


WIDE = [(30011, 128, torch.float32), (50000, 200, torch.float32), (70001, 256, torch.float32),
        (20000, 256, torch.float64), (40000, 160, torch.bfloat16)]


def test_batched_wide_problems_match_oracle(lib):
    """The benchmark batch draws k up to 256 (d = 4k = 1024): problems at
    k = 128, 200 and 256 (float32, the benchmark's type), one at k = 256 in
    float64 and one at k = 160 in bfloat16, each against the oracle's
    sketch-and-solve on the same S."""
    problems = []
    for i, (n, k, dt) in enumerate(WIDE):
        A, b = _problem(n, k, dt, 60 + i)
        problems.append((A, b, 2000 + i))
    xs, status, ranks, t_ms, rc = lib.solve_batched(problems)
    assert rc == 0 and status == [0] * len(WIDE)
    for (A, b, seed), x, rank, (n, k, dt) in zip(problems, xs, ranks, WIDE):
        A64 = A.to(torch.float64).cpu().numpy()
        b64 = b.to(torch.float64).cpu().numpy()
        xg = x.cpu().numpy()
        if dt == torch.float64:
            xr, r, _ = _oracle(A64, b64, k, seed, 2.0 ** -53)
            assert np.linalg.norm(xg - xr) <= 1e-11 * np.linalg.norm(xr)
        else:
            xr, r, tol = _oracle(A64, b64, k, seed, 2.0 ** -24)
            assert np.linalg.norm(xg - xr) <= tol
        assert rank == r == k


def test_batched_mixes_batch_factored_and_per_problem_steps(lib):
    """Problems with d = 4k <= 1024 are factored together in the batched launches, the others (here k = 300, d =
    1200) on their own stream; both kinds in one call match the oracle, and the batch is bitwise reproducible."""
    shapes = [(9000, 300, torch.float64), (3000, 40, torch.float64), (8000, 256, torch.float32),
              (6000, 290, torch.float32), (2500, 1, torch.float64)]
    problems = []
    for i, (n, k, dt) in enumerate(shapes):
        A, b = _problem(n, k, dt, 80 + i)
        problems.append((A, b, 3000 + i))
    xs, status, ranks, t_ms, rc = lib.solve_batched(problems)
    assert rc == 0 and status == [0] * len(shapes)
    for (A, b, seed), x, rank, t, (n, k, dt) in zip(problems, xs, ranks, t_ms, shapes):
        A64 = A.to(torch.float64).cpu().numpy()
        b64 = b.to(torch.float64).cpu().numpy()
        xg = x.cpu().numpy()
        if dt == torch.float64:
            xr, r, _ = _oracle(A64, b64, k, seed, 2.0 ** -53)
            assert np.linalg.norm(xg - xr) <= 1e-11 * np.linalg.norm(xr)
        else:
            xr, r, tol = _oracle(A64, b64, k, seed, 2.0 ** -24)
            assert np.linalg.norm(xg - xr) <= tol
        assert rank == r == k and t > 0.0
    again = lib.solve_batched(problems)[0]
    for a, b in zip(xs, again):
        assert torch.equal(a, b)


VARIANTS = [(20000, 150, torch.float64, 0), (9000, 201, torch.float32, 0), (30000, 255, torch.float32, 0),
            (5000, 200, torch.float32, 0), (3000, 63, torch.float64, 0), (4000, 64, torch.bfloat16, 0),
            (100, 8, torch.float32, 0), (70001, 16, torch.float32, 0), (2000, 3, torch.float32, 0),
            (6000, 4, torch.float64, 0), (8000, 37, torch.float32, 3), (2500, 96, torch.bfloat16, 2)]


def test_batched_sketch_variants_match_oracle(lib):
    """The batched sketch (one launch per kernel variant for all problems, b as the column after A's last) across its
    variants: FP64 and FP32 bucket parts (k = 150; k = 201 and 255), the 200-slot file without parts (k = 200), the
    b column alone in the last lane of a slab (k = 63) and in a slab of its own lane range (k = 64), n below one tile
    (n = 100), many row chunks with a ragged last tile (n = 70001), k = 4, rows with a stride and an offset of one or
    three elements (so only 4-byte loads), beside a problem the batched sketch does not take (k = 3, sketched on its
    own), in one call; every solution matches the oracle, and the batch is bitwise reproducible."""
    problems = []
    for i, (n, k, dt, pad) in enumerate(VARIANTS):
        A, b = _problem(n, k, dt, 200 + i)
        if pad:
            wide = torch.zeros((n, k + 2 * pad), dtype=dt, device="cuda")
            wide[:, pad:pad + k] = A
            A = wide[:, pad:pad + k]
        problems.append((A, b, 5000 + i))
    xs, status, ranks, t_ms, rc = lib.solve_batched(problems)
    assert rc == 0 and status == [0] * len(VARIANTS)
    for (A, b, seed), x, rank, t, (n, k, dt, _) in zip(problems, xs, ranks, t_ms, VARIANTS):
        A64 = A.to(torch.float64).cpu().numpy()
        b64 = b.to(torch.float64).cpu().numpy()
        xg = x.cpu().numpy()
        if dt == torch.float64:
            xr, r, _ = _oracle(A64, b64, k, seed, 2.0 ** -53)
            assert np.linalg.norm(xg - xr) <= 1e-11 * np.linalg.norm(xr), (n, k, dt)
        else:
            xr, r, tol = _oracle(A64, b64, k, seed, 2.0 ** -24)
            assert np.linalg.norm(xg - xr) <= tol, (n, k, dt)
        assert rank == r == k and t > 0.0
    again = lib.solve_batched(problems)[0]
    for a, b in zip(xs, again):
        assert torch.equal(a, b)


def test_batched_sketch_groups_do_not_change_results(lib, monkeypatch):
    """A batch whose codes and partials do not fit one area is sketched in several launch groups (here one problem
    a group, through SKETCH_BATCH_AREA_MB); every problem's plan and arithmetic are its own, so the solutions are
    bitwise those of the one-group run."""
    problems = []
    for i, (n, k, dt, pad) in enumerate(VARIANTS[:8]):
        A, b = _problem(n, k, dt, 300 + i)
        problems.append((A, b, 6000 + i))
    one = lib.solve_batched(problems)
    assert one[4] == 0
    monkeypatch.setenv("SKETCH_BATCH_AREA_MB", "1")
    split = lib.solve_batched(problems)
    assert split[4] == 0 and split[1] == one[1] and split[2] == one[2]
    for a, b in zip(one[0], split[0]):
        assert torch.equal(a, b)
