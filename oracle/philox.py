"""Philox4x32-10 in NumPy (oracle side; test infrastructure only).

The paper only asks for iid uniform bucket indices and Rademacher signs
(Def. 1.5). They are drawn here from Philox4x32-10, the counter-based
generator of Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as
easy as 1, 2, 3", SC'11), so that entry (i, t) of the sketch is a pure
function of (seed, i, t) and either side can produce any entry on demand.

Definition used (from the SC'11 paper):
  state: four 32-bit counter words (c0, c1, c2, c3) and a two-word key (k0, k1)
  one round:  (hi0, lo0) = mulhilo(M0, c0); (hi1, lo1) = mulhilo(M1, c2)
              c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
  key bump between rounds: k0 += W0, k1 += W1 (mod 2^32)
  ten rounds, with M0 = 0xD2511F53, M1 = 0xCD9E8D57, W0 = 0x9E3779B9,
  W1 = 0xBB67AE85.

Pins: the published known-answer vectors of the Random123 distribution and
rocRAND's independent host implementation (tests/test_oracle_philox.py).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

# Stream tags: the fourth counter word separates independent uses of one seed.
TAG_SPARSESTACK = 1
TAG_SRTT_SIGN = 2
TAG_SRTT_SAMPLE = 3
TAG_GAUSS = 4
TAG_SPARSECOL = 5


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on broadcastable uint32 arrays.

    Returns a tuple of four uint32 arrays (the output block).
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    ka = int(k0) & 0xFFFFFFFF
    kb = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(ka)), lo1, (hi0 ^ c3 ^ np.uint64(kb)), lo0
        if rnd < 9:
            ka = (ka + W0) & 0xFFFFFFFF
            kb = (kb + W1) & 0xFFFFFFFF
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def key_of_seed(seed):
    """Key words (k0, k1) = (low 32 bits, high 32 bits) of a 64-bit seed."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32
