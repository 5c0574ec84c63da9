"""Philox4x32-10 counter-based generator and the maps from its words to
uniforms and Gaussian normals.  Test infrastructure only (see package doc).

The paper asks only for "independent, zero mean Gaussian Fourier modes"
(Sec. 2, eq. Papos2) and names no generator.  The generator used here is
Philox4x32 with 10 rounds from Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11), restated from that paper's description:

* state: four 32-bit words (c0, c1, c2, c3); key: two 32-bit words (k0, k1);
* one round multiplies c0 and c2 by two fixed odd constants, keeping both the
  high and low 32-bit halves of each 64-bit product; the high halves are
  XOR-ed with the other two state words and with the round key, and the four
  words are permuted;
* between rounds the key is advanced by two Weyl increments (the golden ratio
  and sqrt(3)-1 scaled to 2**32).

Parity: the word stream is pinned against an independent library
implementation (rocRAND's host Philox4x32-10 generator) in a GPU-box test,
because that library cannot initialise without a device.  On the CPU it is
pinned by statistical properties only (uniformity, independence of words).

Uniform maps (our convention, fixed for parity):

* ``u32_to_unit(x)``  = (x + 1/2) 2**-32                 -- in (0, 1), exact in FP64
* ``u52_to_unit(x0, x1)`` = (((x0 << 20) | (x1 >> 12)) + 1/2) 2**-52 -- exact in FP64

Box-Muller (Box & Muller 1958): for uniforms u1, u2 in (0, 1],
r = sqrt(-2 ln u1), a = r cos(2 pi u2), b = r sin(2 pi u2) are independent N(0, 1).
"""

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# Round multipliers and Weyl key increments of Philox4x32 (Salmon et al. 2011).
MUL_A = np.uint64(0xD2511F53)
MUL_B = np.uint64(0xCD9E8D57)
WEYL_A = np.uint64(0x9E3779B9)
WEYL_B = np.uint64(0xBB67AE85)
ROUNDS = 10


def key_from_seed(seed):
    """Split a 64-bit seed into the two key words (low word first)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def philox4x32_10(c0, c1, c2, c3, key):
    """Apply ten Philox rounds to counters (arrays broadcastable together).

    ``key`` is a pair of 32-bit ints.  Returns four uint32 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for rnd in range(ROUNDS):
        if rnd > 0:
            k0 = (k0 + WEYL_A) & MASK32
            k1 = (k1 + WEYL_B) & MASK32
        prod_a = c0 * MUL_A          # < 2**64: exact in uint64
        prod_b = c2 * MUL_B
        hi_a, lo_a = prod_a >> np.uint64(32), prod_a & MASK32
        hi_b, lo_b = prod_b >> np.uint64(32), prod_b & MASK32
        c0, c1, c2, c3 = (hi_b ^ c1 ^ k0), lo_b, (hi_a ^ c3 ^ k1), lo_a
    return tuple(np.asarray(c, dtype=np.uint32) for c in (c0, c1, c2, c3))


def u32_to_unit(x):
    """(x + 1/2) * 2**-32 as float64 (exact)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * 2.0 ** -32


def u52_to_unit(x0, x1):
    """52-bit uniform from two words: ((x0 << 20) | (x1 >> 12)) + 1/2, times 2**-52 (exact)."""
    v = (np.asarray(x0, dtype=np.uint64) << np.uint64(20)) | (
        np.asarray(x1, dtype=np.uint64) >> np.uint64(12))
    return (v.astype(np.float64) + 0.5) * 2.0 ** -52


def box_muller(u1, u2):
    """Two independent standard normals from two uniforms (Box & Muller 1958)."""
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return r * np.cos(ang), r * np.sin(ang)
