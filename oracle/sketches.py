"""Test matrices and their application, written from the definitions (oracle).

Test infrastructure only (see the package docstring).

Orientation. The paper writes a test matrix Omega (ambient x embedding) and
applies it on the right, A -> A Omega, or as Psi^T on the left. This module
works with the short-fat matrix S = Omega^T (d x n, d = embedding dimension)
and computes SA = S @ A for a tall A (n x m), the paper's Psi^T A in Alg. 3.

Readings of points the paper leaves open (each applies to both the oracle and
the GPU library):
  * random source: Philox4x32-10 (oracle.philox); entry (i, t) of a
    SparseStack uses counter (i mod 2^32, i >> 32, t // 4, TAG) and output
    word t mod 4;
  * sign = +1 if bit 0 of the word is 0, else -1;
  * bucket = ((word >> 1) * nb) >> 31 (a multiply-shift map of 31 random
    bits onto [0, nb); its bias is below nb / 2^31);
  * indices are 0-based and row t*nb + s of S belongs to block t, bucket s,
    i.e. the blocks of Def. 1.5 are stacked in order;
  * the 1/sqrt(zeta) scale is applied once, after the signed sum.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import philox as px


# ----------------------------------------------------------------------------
# SparseStack (Def. 1.5; restated in Sec. 3.1) and CountSketch (eq. B.1)
# ----------------------------------------------------------------------------
def sparsestack_pattern(n, d, zeta, seed, rows=None):
    """Bucket indices s_it in [0, d/zeta) and Rademacher signs rho_it.

    Def. 1.5: each column of S (each row of Omega) holds, in every one of the
    zeta blocks of b = d/zeta rows, exactly one entry rho/sqrt(zeta), at a
    uniformly random position; all draws are independent.

    Returns (buckets int64 [len(rows), zeta], signs int8 [len(rows), zeta]).
    `rows` selects a subset of column indices i of S (default: all n).
    """
    if zeta < 1 or d % zeta != 0:
        raise ValueError("SparseStack needs 1 <= zeta and zeta | d")
    nb = d // zeta
    i = np.arange(n, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    k0, k1 = px.key_of_seed(seed)
    buckets = np.empty((i.size, zeta), dtype=np.int64)
    signs = np.empty((i.size, zeta), dtype=np.int8)
    lo = i & np.uint64(0xFFFFFFFF)
    hi = i >> np.uint64(32)
    for g in range((zeta + 3) // 4):
        words = px.philox4x32_10(lo, hi, g, px.TAG_SPARSESTACK, k0, k1)
        for j in range(4):
            t = 4 * g + j
            if t >= zeta:
                break
            w = words[j].astype(np.uint64)
            signs[:, t] = np.where((w & np.uint64(1)) == 0, 1, -1)
            buckets[:, t] = ((w >> np.uint64(1)) * np.uint64(nb)) >> np.uint64(31)
    return buckets, signs


def inv_sqrt(x):
    """fl(1 / fl(sqrt(x))) in IEEE double, the scale used by both sides."""
    return 1.0 / math.sqrt(float(x))


def sparsestack_csr(n, d, zeta, seed, scaled=True):
    """S as a scipy CSR matrix (d x n). Entry (t*nb + s_it, i) = rho_it [/sqrt(zeta)]."""
    nb = d // zeta
    buckets, signs = sparsestack_pattern(n, d, zeta, seed)
    rows = (np.arange(zeta)[None, :] * nb + buckets).ravel()
    cols = np.repeat(np.arange(n), zeta)
    vals = signs.astype(np.float64).ravel()
    if scaled:
        vals = vals * inv_sqrt(zeta)
    return sp.csr_matrix((vals, (rows, cols)), shape=(d, n))


def sparsestack_dense(n, d, zeta, seed):
    """S as a dense float64 array (small n only)."""
    return sparsestack_csr(n, d, zeta, seed).toarray()


def sparsestack_apply(A, d, zeta, seed):
    """SA = S @ A for a tall A (n x m), promoted to float64.

    SA[t*nb + s, c] = (1/sqrt(zeta)) * sum_{i : s_it = s} rho_it * A[i, c].
    The signed sums use scipy's sparse product; the scale is applied after.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Spm = sparsestack_csr(n, d, zeta, seed, scaled=False)
    return (Spm @ A) * inv_sqrt(zeta)


def sparsestack_apply_rows(A_rows, row_ids, d, zeta, seed):
    """Contribution of a subset of rows of A to SA (for chunked/streamed use)."""
    A_rows = np.asarray(A_rows, dtype=np.float64)
    nb = d // zeta
    buckets, signs = sparsestack_pattern(None, d, zeta, seed, rows=row_ids)
    out = np.zeros((d, A_rows.shape[1]))
    for t in range(zeta):
        np.add.at(out, t * nb + buckets[:, t], signs[:, t, None] * A_rows)
    return out


def sparsestack_apply_T(A, d, zeta, seed):
    """Y = A @ S^T for a wide A (rows x n): the paper's A Omega (the sketching step of Alg. 1)."""
    A = np.asarray(A, dtype=np.float64)
    Spm = sparsestack_csr(A.shape[1], d, zeta, seed, scaled=False)
    return (Spm @ A.T).T * inv_sqrt(zeta)


def sparsestack_adjoint(Y, n, zeta, seed):
    """S^T @ Y for Y (d x m): out[i, :] = sum_t rho_it/sqrt(zeta) * Y[t*nb + s_it, :]."""
    Y = np.asarray(Y, dtype=np.float64)
    d = Y.shape[0]
    S = sparsestack_csr(n, d, zeta, seed)
    return S.T @ Y


# ----------------------------------------------------------------------------
# Subsampled randomized trigonometric transform (eq. 1.1 with a restriction S)
# ----------------------------------------------------------------------------
def srtt_padded_length(n):
    """Smallest power of two >= n: the WHT is only defined for 2^p (Sec. 4.2)."""
    p = 0
    while (1 << p) < n:
        p += 1
    return 1 << p


def srtt_signs(npad, seed):
    """Rademacher diagonal D (eq. 1.1): bit (i mod 128) of Philox block i // 128."""
    k0, k1 = px.key_of_seed(seed)
    nblk = (npad + 127) // 128
    b = np.arange(nblk, dtype=np.uint64)
    words = px.philox4x32_10(b & np.uint64(0xFFFFFFFF), b >> np.uint64(32), 0, px.TAG_SRTT_SIGN, k0, k1)
    W = np.stack(words, axis=1)  # [nblk, 4]
    i = np.arange(npad)
    bits = (W[i // 128, (i % 128) // 32] >> (i % 32).astype(np.uint32)) & 1
    return np.where(bits == 0, 1.0, -1.0)


def srtt_sample(npad, d, seed):
    """d distinct row indices of [0, npad), sorted ascending.

    The paper's restriction selects coordinates uniformly at random (Sec. 1.4.2)
    without saying whether repeats are allowed; it is sampled here without
    replacement (as SparseCol does, Def. 4.1) using Floyd's algorithm: for
    j = npad-d .. npad-1 draw u uniform on {0..j}; insert u, or j if u is
    already chosen. u = (w * (j+1)) >> 32 with w the first Philox word of
    counter (j, 0, TAG_SRTT_SAMPLE).
    """
    if d > npad:
        raise ValueError("SRTT needs d <= padded length")
    k0, k1 = px.key_of_seed(seed)
    chosen = set()
    for j in range(npad - d, npad):
        w = px.philox4x32_10(j & 0xFFFFFFFF, j >> 32, 0, px.TAG_SRTT_SAMPLE, k0, k1)[0]
        u = (int(w) * (j + 1)) >> 32
        chosen.add(j if u in chosen else u)
    return np.array(sorted(chosen), dtype=np.int64)


def fwht_rows(X):
    """Unnormalized Walsh-Hadamard transform along axis 0, Sylvester ordering.

    H_1 = [1], H_{2h} = [[H_h, H_h], [H_h, -H_h]]; returns H @ X.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    N = X.shape[0]
    rest = X.shape[1:]
    h = 1
    while h < N:
        Y = X.reshape((N // (2 * h), 2, h) + rest)
        top = Y[:, 0].copy()
        bot = Y[:, 1]
        Y[:, 0] = top + bot
        Y[:, 1] = top - bot
        X = Y.reshape((N,) + rest)
        h *= 2
    return X


def srtt_apply(A, d, seed):
    """Y = (1/sqrt(d)) * R H D A_pad (eq. 1.1 as S = Omega^T, applied on the left).

    A is padded with zero rows to npad = 2^ceil(log2 n); D is the Rademacher
    diagonal, H the unnormalized Sylvester Hadamard matrix (so H/sqrt(npad)
    is the unitary F), R restricts to the sampled rows; the factor
    sqrt(npad/d) * (1/sqrt(npad)) = 1/sqrt(d) makes the sketch isotropic.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    npad = srtt_padded_length(n)
    Dsig = srtt_signs(npad, seed)
    Ap = np.zeros((npad,) + A.shape[1:])
    Ap[:n] = A * Dsig[:n].reshape((n,) + (1,) * (A.ndim - 1))
    HA = fwht_rows(Ap)
    R = srtt_sample(npad, d, seed)
    return HA[R] * inv_sqrt(d)


def srtt_dense(n, d, seed):
    """The SRTT matrix S (d x n) formed explicitly (small n only)."""
    return srtt_apply(np.eye(n), d, seed)


# ----------------------------------------------------------------------------
# SparseRTT (Def. 1.7) with a SparseCol sparse factor (Def. 4.1)
# ----------------------------------------------------------------------------
def sparsertt_default_xi(d, npad):
    """Column sparsity xi = ceil(1.5 log k) at embedding dimension k = d (Sec. 4.3).

    Reading: log is the natural logarithm; xi is clamped to [1, npad].
    """
    return int(min(max(1, math.ceil(1.5 * math.log(d))), npad))


def sparsecol_selectors(npad, d, xi, seed):
    """Selectors and signs of the SparseCol matrix (Def. 4.1): for each column j < d,
    xi distinct indices of [0, npad) and xi Rademacher signs.

    Column j draws its selectors without replacement by Floyd's algorithm: for
    t = npad-xi .. npad-1, the Philox words of counter (t mod 2^32, t >> 32, j,
    TAG_SPARSECOL) give u = (w0 * (t+1)) >> 32, uniform on {0..t}; the index
    taken at this step is u, or t if u was taken before, and its sign is -1
    iff bit 0 of w1 is 1. Returns (sel, sgn), each d x xi, every row sorted by
    index (the order in which the sketch adds the selected rows).
    """
    if not 1 <= xi <= npad:
        raise ValueError("SparseCol needs 1 <= xi <= npad")
    k0, k1 = px.key_of_seed(seed)
    t = np.arange(npad - xi, npad, dtype=np.uint64)
    sel = np.zeros((d, xi), dtype=np.int64)
    sgn = np.zeros((d, xi))
    for j in range(d):
        w0, w1, _, _ = px.philox4x32_10(t & np.uint64(0xFFFFFFFF), t >> np.uint64(32), j, px.TAG_SPARSECOL, k0, k1)
        taken = {}
        for q in range(xi):
            tq = int(t[q])
            u = (int(w0[q]) * (tq + 1)) >> 32
            idx = tq if u in taken else u
            taken[idx] = -1.0 if (int(w1[q]) & 1) else 1.0
        order = sorted(taken)
        sel[j] = order
        sgn[j] = [taken[i] for i in order]
    return sel, sgn


def sparsecol_dense(npad, d, xi, seed):
    """The SparseCol matrix (npad x d) of Def. 4.1: column j is
    (1/sqrt(d)) sqrt(npad/xi) sum_i rho_ji e_{s_ji}."""
    sel, sgn = sparsecol_selectors(npad, d, xi, seed)
    M = np.zeros((npad, d))
    for j in range(d):
        M[sel[j], j] = sgn[j] * math.sqrt(npad / xi) / math.sqrt(d)
    return M


def sparsertt_apply(A, d, xi, seed):
    """SA = Omega^T A for the SparseRTT Omega = D F S (Def. 1.7), S = SparseCol.

    A is padded with zero rows to npad = 2^ceil(log2 n) (the WHT needs a power
    of two); D is the SRTT's Rademacher diagonal, F = H/sqrt(npad) the unitary
    WHT. Since F and D are symmetric, row j of Omega^T A_pad is
    (1/sqrt(d)) sqrt(npad/xi) (1/sqrt(npad)) sum_i rho_ji (H D A_pad)[s_ji]
    = (1/sqrt(d xi)) sum_i rho_ji (H D A_pad)[s_ji]; the selected rows are
    added in increasing index order and the sum is scaled once.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    npad = srtt_padded_length(n)
    Dsig = srtt_signs(npad, seed)
    Ap = np.zeros((npad,) + A.shape[1:])
    Ap[:n] = A * Dsig[:n].reshape((n,) + (1,) * (A.ndim - 1))
    HA = fwht_rows(Ap)
    sel, sgn = sparsecol_selectors(npad, d, xi, seed)
    out = np.zeros((d,) + A.shape[1:])
    for j in range(d):
        acc = np.zeros(A.shape[1:])
        for q in range(xi):
            acc = acc + sgn[j, q] * HA[sel[j, q]]
        out[j] = acc
    return out * inv_sqrt(d * xi)


def sparsertt_dense(n, d, xi, seed):
    """The SparseRTT sketch S = Omega^T (d x n) formed explicitly (small n only)."""
    return sparsertt_apply(np.eye(n), d, xi, seed)


# ----------------------------------------------------------------------------
# Gaussian test matrix (Def. 1.4): iid N(0, 1/d) entries for S (d x n)
# ----------------------------------------------------------------------------
TWO_PI = 2.0 * math.pi


def gaussian_entries(rows_j, cols_i, d, seed):
    """G[j, i] for index arrays (broadcast together), float64.

    Pair q = j // 2 of column i uses Philox counter (i, q, TAG_GAUSS) -> four
    words; u1 and u2 take 52 bits from words (0, 1) and (2, 3):
    u = (x + 1/2) 2^-52 in (0, 1). The Box-Muller transform (Box & Muller,
    1958) gives r = sqrt(-2 ln u1), theta = 2 pi u2, and
    z = r cos(theta) for even j, r sin(theta) for odd j. G = z * fl(1/sqrt(d)).
    """
    j = np.asarray(rows_j, dtype=np.int64)
    i = np.asarray(cols_i, dtype=np.int64)
    j, i = np.broadcast_arrays(j, i)
    iu = i.astype(np.uint64)
    k0, k1 = px.key_of_seed(seed)
    w0, w1, w2, w3 = px.philox4x32_10(iu & np.uint64(0xFFFFFFFF), iu >> np.uint64(32),
                                      (j // 2).astype(np.uint64), px.TAG_GAUSS, k0, k1)

    def unif(a, b):
        x = (a.astype(np.uint64) << np.uint64(20)) | (b.astype(np.uint64) >> np.uint64(12))
        return (x.astype(np.float64) + 0.5) * (2.0 ** -52)

    u1 = unif(w0, w1)
    u2 = unif(w2, w3)
    r = np.sqrt(-2.0 * np.log(u1))
    th = TWO_PI * u2
    z = np.where(j % 2 == 0, r * np.cos(th), r * np.sin(th))
    return z * inv_sqrt(d)


def gaussian_dense(n, d, seed):
    """G (d x n), small n only."""
    J, I = np.meshgrid(np.arange(d), np.arange(n), indexing="ij")
    return gaussian_entries(J, I, d, seed)


def gaussian_apply(A, d, seed, chunk=1 << 16):
    """SA = G @ A, accumulating G[:, chunk] @ A[chunk] over row chunks of A."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    out = np.zeros((d,) + A.shape[1:])
    jj = np.arange(d)[:, None]
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        G = gaussian_entries(jj, np.arange(r0, r1)[None, :], d, seed)
        out += G @ A[r0:r1]
    return out


# ----------------------------------------------------------------------------
# Dispatch by kind (the same integer codes as the C library's enum)
# ----------------------------------------------------------------------------
KIND_SPARSESTACK = 0
KIND_GAUSSIAN = 1
KIND_SRTT = 2
KIND_SPARSERTT = 3
KIND_IDENTITY = 99


def apply(kind, A, d, zeta, seed):
    """SA for any supported kind (A tall, n x m)."""
    if kind == KIND_SPARSESTACK:
        return sparsestack_apply(A, d, zeta, seed)
    if kind == KIND_GAUSSIAN:
        return gaussian_apply(A, d, seed)
    if kind == KIND_SRTT:
        return srtt_apply(A, d, seed)
    if kind == KIND_SPARSERTT:
        npad = srtt_padded_length(np.asarray(A).shape[0])
        return sparsertt_apply(A, d, zeta if zeta else sparsertt_default_xi(d, npad), seed)
    if kind == KIND_IDENTITY:
        return np.asarray(A, dtype=np.float64).copy()
    raise ValueError(kind)


def dense(kind, n, d, zeta, seed):
    if kind == KIND_SPARSESTACK:
        return sparsestack_dense(n, d, zeta, seed)
    if kind == KIND_GAUSSIAN:
        return gaussian_dense(n, d, seed)
    if kind == KIND_SRTT:
        return srtt_dense(n, d, seed)
    if kind == KIND_SPARSERTT:
        return sparsertt_dense(n, d, zeta if zeta else sparsertt_default_xi(d, srtt_padded_length(n)), seed)
    if kind == KIND_IDENTITY:
        return np.eye(n)
    raise ValueError(kind)
