"""GPU parity of the SparseStack hot path against the oracle (through the C-ABI).

  * the device hash reproduces the oracle's (bucket, sign) pattern bit for bit;
  * applying S to identity columns recovers every entry of S bit for bit;
  * SA matches the oracle element by element within the summation bound
    |SA_gpu - SA_ref| <= (c_j + 8) * u * (|S||A|)_jc, where c_j is the number
    of rows in bucket j and u the unit roundoff of the accumulation type
    (2^-53 for float64, 2^-24 for float32), on ragged shapes, several tiles,
    zeta in {1, 2, 4, 8, 64}, one bucket per block (d = zeta), blocks of more
    buckets than one workgroup holds (up to 16384), and float32 / bfloat16
    inputs (compared with the oracle applied to the same rounded values);
  * edge cases: one row of A, d = 1, zeta = 100 blocks of one bucket, 1000
    columns, a tile exactly full and a one-row tail;
  * results are bitwise reproducible run to run;
  * S^T (adjoint) matches the oracle and satisfies <SA, Y> = <A, S^T Y>;
  * at the full 4,194,304 x 200 float64 shape, sampled columns match the
    oracle computed column by column.
"""
import numpy as np
import pytest
import torch

from oracle import sketches as sk

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lib():
    from paper_2508_21189_amd import libsketch
    libsketch.load()
    return libsketch


def _bound(A64, d, zeta, seed, u):
    """(c_j + 8) * u * (|S||A|) from the oracle's pattern."""
    n = A64.shape[0]
    Sabs = abs(sk.sparsestack_csr(n, d, zeta, seed))
    SA_abs = Sabs @ np.abs(A64)
    cnt = np.asarray((Sabs != 0).sum(axis=1)).ravel()
    return (cnt[:, None] + 8.0) * u * SA_abs


def _check(gpu, ref, bound):
    err = np.abs(gpu - ref)
    ratio = np.max(err / np.maximum(bound, 1e-300))
    assert np.all(err <= bound), "max err/bound = %g" % ratio
    return ratio


@pytest.mark.parametrize("n,d,zeta,seed", [(1000, 40, 4, 1), (4099, 800, 8, 7), (70000, 200, 4, 3),
                                          (12345, 17, 1, 5), (3000, 5, 5, 9)])
def test_pattern_bit_exact(lib, n, d, zeta, seed):
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    b, s = S.pattern()
    rb, rs = sk.sparsestack_pattern(n, d, zeta, seed)
    assert np.array_equal(b.cpu().numpy(), rb.astype(np.int32))
    assert np.array_equal(s.cpu().numpy(), rs)


@pytest.mark.parametrize("n,d,zeta", [(300, 40, 4), (1024, 64, 8), (777, 16, 1), (513, 6, 6)])
def test_apply_identity_recovers_S_bitwise(lib, n, d, zeta):
    S = lib.Sketch("sparsestack", d, n, zeta, 42)
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    got = S.apply(I).cpu().numpy()
    want = sk.sparsestack_dense(n, d, zeta, 42)
    assert np.array_equal(got, want)


CASES = [
    (20000, 50, 200, 4, 11),   # workload 1 shape
    (1037, 7, 40, 4, 2),       # ragged rows, narrow
    (5000, 65, 96, 8, 3),      # two column slabs (64 + 1)
    (3001, 129, 800, 8, 4),    # three slabs, 100 buckets per block
    (2500, 33, 8, 8, 5),       # one bucket per block (d = zeta)
    (4096, 20, 64, 1, 6),      # CountSketch
    (300, 1, 30, 3, 7),        # single column (the right-hand side)
    (9000, 200, 800, 8, 8),    # workload 2 column count, several row tiles
    (200000, 50, 200, 4, 9),   # many sub-tiles per row chunk (both LDS buffers in use)
    (50000, 3, 400, 8, 10),    # narrow input: lanes over buckets, several tiles per chunk
    (70001, 2, 2000, 8, 12),   # narrow input, two buckets per lane, ragged last tile
    (9000, 4, 4096, 4, 13),    # narrow input at its largest d (four buckets per lane)
    (1000003, 1, 800, 8, 15),  # narrow input, the right-hand side at scale (many tiles per chunk)
    (4000, 5, 64, 4, 14),      # the narrowest input of the wide kernel
    (5003, 70, 1602, 2, 17),   # 801 buckets per block: one more than 16 waves hold, two bucket ranges
    (30011, 40, 8000, 2, 16),  # 4000 buckets per block: five bucket ranges per block
    (20000, 16, 16384, 1, 18), # the largest block of the row apply (16384 buckets, 21 ranges)
    (4000, 5, 640, 64, 19),    # 64 blocks: the plan kernel's tile shrinks to fit its LDS
    (20011, 100, 1200, 8, 29), # 150 buckets per block: two bucket parts of the register file
    (12007, 500, 2000, 8, 30), # 250 buckets (the mixed-precision shape): three parts, eight slabs
    (9001, 70, 1600, 4, 31),   # 400 buckets: four parts, one block per workgroup group
    (20011, 33, 500, 5, 32),   # zeta = 5, FP64 rows of 264 bytes (4-byte loads): 1.5 tile rows a load step
    (9001, 51, 700, 7, 33),    # zeta = 7, the same with seven waves a workgroup
]


@pytest.mark.parametrize("n,m,d,zeta,seed", CASES)
def test_apply_f64_parity(lib, n, m, d, zeta, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m)) * np.logspace(0, -3, m)
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    got = S.apply(torch.from_numpy(A).cuda()).cpu().numpy()
    ref = sk.sparsestack_apply(A, d, zeta, seed)
    _check(got, ref, _bound(A, d, zeta, seed, 2.0 ** -53))


EDGE_CASES = [
    (1, 5, 8, 8, 21),          # one row of A: one partial tile, every other chunk empty
    (1, 1, 3, 3, 22),          # one row, one column (narrow kernel)
    (7, 64, 1, 1, 23),         # d = 1: a single bucket, every row lands in it
    (500, 130, 100, 100, 24),  # zeta = 100 > 16 blocks: several block groups, plan waves loop over blocks
    (300, 3, 100, 100, 25),    # zeta = 100 on the narrow kernel
    (2000, 1000, 40, 4, 26),   # 1000 columns: 16 column slabs
    (163, 50, 800, 8, 27),     # exactly one full tile of the coherent layout
    (164, 50, 800, 8, 28),     # one full tile and a one-row tail
]


@pytest.mark.parametrize("n,m,d,zeta,seed", EDGE_CASES)
def test_apply_edge_cases(lib, n, m, d, zeta, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m))
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    got = S.apply(torch.from_numpy(A).cuda()).cpu().numpy()
    ref = sk.sparsestack_apply(A, d, zeta, seed)
    _check(got, ref, _bound(A, d, zeta, seed, 2.0 ** -53))
    # float32 with an odd column count takes the 4-byte load path
    A32 = torch.from_numpy(A).to(torch.float32)
    got32 = S.apply(A32.cuda(), out_dtype=torch.float64).cpu().numpy()
    A64 = A32.double().numpy()
    ref32 = sk.sparsestack_apply(A64, d, zeta, seed)
    _check(got32, ref32, _bound(A64, d, zeta, seed, 2.0 ** -24))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n,m,d,zeta,seed", [(20000, 64, 200, 4, 1), (6007, 100, 2000, 8, 2),
                                             (3000, 16, 64, 8, 3), (1000, 500, 400, 8, 4),
                                             (100000, 64, 400, 8, 5), (30000, 1, 200, 4, 6),
                                             (20011, 3, 96, 8, 7), (20000, 64, 2048, 1, 8),
                                             (7001, 24, 6000, 2, 9), (9000, 130, 3200, 8, 10),
                                             (15013, 64, 3200, 4, 11)])
def test_apply_lowprec_parity(lib, dtype, n, m, d, zeta, seed):
    rng = np.random.default_rng(seed)
    A = torch.from_numpy(rng.standard_normal((n, m))).cuda().to(torch.float32).to(dtype)
    A64 = A.to(torch.float64).cpu().numpy()  # the exact values the kernel reads
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    for odt in (torch.float32, torch.float64):
        got = S.apply(A, out_dtype=odt).to(torch.float64).cpu().numpy()
        ref = sk.sparsestack_apply(A64, d, zeta, seed)
        # float32 accumulation, plus the final rounding to float32 output
        _check(got, ref, _bound(A64, d, zeta, seed, 2.0 ** -24) + 2.0 ** -24 * np.abs(ref))


def test_bitwise_reproducible(lib):
    rng = np.random.default_rng(0)
    A = torch.from_numpy(rng.standard_normal((50000, 200))).cuda()
    S = lib.Sketch("sparsestack", 800, 50000, 8, 123)
    r1 = S.apply(A)
    for _ in range(5):
        assert torch.equal(S.apply(A), r1)


def test_adjoint(lib):
    rng = np.random.default_rng(1)
    n, d, zeta, m = 3000, 96, 8, 5
    S = lib.Sketch("sparsestack", d, n, zeta, 77)
    Y = torch.from_numpy(rng.standard_normal((d, m))).cuda()
    Z = S.adjoint(Y).cpu().numpy()
    np.testing.assert_allclose(Z, sk.sparsestack_adjoint(Y.cpu().numpy(), n, zeta, 77), rtol=1e-14, atol=1e-14)
    X = torch.from_numpy(rng.standard_normal((n, m))).cuda()
    lhs = float((S.apply(X) * Y).sum())
    rhs = float((X.cpu() * torch.from_numpy(Z)).sum())
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


def test_full_size_sampled_columns(lib):
    """4,194,304 x 200 float64 (the coherent workload), d = 800, zeta = 8."""
    from paper_2508_21189_amd import inputs
    n, m, d, zeta, seed = 1 << 22, 200, 800, 8, 2000
    A, b, _, _ = inputs.coherent(n, m, exponent=8.0, seed=200)
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    SA = S.apply(A).cpu().numpy()
    for c in (0, 57, 199):
        col = A[:, c].cpu().numpy()[:, None]
        ref = sk.sparsestack_apply(col, d, zeta, seed)
        _check(SA[:, c:c + 1], ref, _bound(col, d, zeta, seed, 2.0 ** -53))
    Sb = S.apply(b[:, None].contiguous()).cpu().numpy()
    ref = sk.sparsestack_apply(b.cpu().numpy()[:, None], d, zeta, seed)
    _check(Sb, ref, _bound(b.cpu().numpy()[:, None], d, zeta, seed, 2.0 ** -53))


@pytest.mark.parametrize("kind,dtype,n,m,d,zeta", [("sparsestack", torch.float64, 20000, 50, 200, 4),
                                                   ("sparsestack", torch.float32, 7001, 130, 96, 8),
                                                   ("sparsestack", torch.bfloat16, 3000, 34, 64, 4),
                                                   ("sparsestack", torch.float64, 5000, 3, 40, 4),
                                                   ("gaussian", torch.float64, 3000, 20, 64, 1),
                                                   ("srtt", torch.float64, 4096, 17, 64, 1),
                                                   ("sparsertt", torch.float64, 3000, 9, 48, 0)])
def test_apply_column_major_equals_row_major(lib, kind, dtype, n, m, d, zeta):
    """Column-major A (a transposed view, and one with lda > n) gives SA bitwise
    equal to the same matrix in row-major order."""
    g = torch.Generator().manual_seed(n + m)
    A = torch.randn((n, m), generator=g, dtype=torch.float64).to(dtype).cuda()
    S = lib.Sketch(kind, d, n, zeta, 5)
    ref = S.apply(A.contiguous())
    At = A.t().contiguous().t()  # column-major view: stride (1, n)
    assert At.stride() == (1, n)
    got = S.apply(At)
    assert torch.equal(got, ref)
    pad = torch.zeros((m, n + 7), dtype=dtype, device="cuda")
    pad[:, :n] = A.t()
    Ap = pad[:, :n].t()  # column-major with lda = n + 7
    assert Ap.stride() == (1, n + 7)
    assert torch.equal(S.apply(Ap), ref)
    # a caller workspace of exactly the queried size (op 2) gives the same result
    ws = torch.empty(S.workspace_size(2, dtype, m), dtype=torch.uint8, device="cuda")
    assert torch.equal(S.apply(At, ws=ws), ref)
