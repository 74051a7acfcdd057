"""Philox4x32-10 and the counter contract of the walker (oracle side).

The paper only asks for i.i.d. uniforms (Sec. "Monte Carlo estimators":
i.i.d. copies of the chain and of Y, Y~ per walk).  Both the oracle and the
GPU path draw them from one counter-based generator, Philox4x32-10
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC 2011), implemented independently on each side from that published
definition, so that identical seeds give identical walks up to rounding.

Philox4x32-10: a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1).
One round multiplies c0 and c2 by two fixed odd constants, takes the high and
low 32-bit halves of the 64-bit products, and permutes/XORs them with c1, c3
and the key.  The key is advanced by two Weyl constants between rounds; ten
rounds are applied.

Counter contract (shared by both sides, defined here for the oracle):

* key = (seed mod 2^32, seed >> 32)
* counter = (l, i, block, tag) with l the walk index, i the site index,
  tag 0 for walks, 1 for the cell-volume points.
* walk blocks: 0 -> (u1, u2, u3, u4): R = median(u1,u2,u3), S = 1 - sqrt(u4);
  d = 2: block 1 -> (a_Z, a_Zs, a_U1, -) angles in revolutions;
  d = 3: block 1 -> (Z: 2 uniforms, Zs: 2 uniforms), block 2 -> (U1: 2, -, -);
  step k >= 1 (the move X_k -> X_{k+1}) draws d-1 uniforms from block
  STEP_BLOCK0 + (k-1) // q, lanes ((k-1) % q) * (d-1) .. , q = 4 // (d-1).
* uniform(x) = ((x >> 9) + 0.5) * 2^-23 = (2k + 1) * 2^-24 with k < 2^23:
  in (0, 1), 24 significant bits, so exact in FP32 and FP64 (and so is 1 - u).

Pinned by: tests/test_oracle_philox.py (known-answer vectors of the
published generator, and agreement with the rocRAND Philox4x32-10 engine on
random counters and keys).
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

TAG_WALK = 0
TAG_VOLUME = 1
STEP_BLOCK0 = 4


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All inputs broadcast to uint32 arrays.

    Returns a tuple of four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    sh = np.uint64(32)
    msk = np.uint64(MASK32)
    for _ in range(10):
        p0 = m0 * c0                      # < 2^64: no overflow in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & msk
        hi1, lo1 = p1 >> sh, p1 & msk
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def to_uniform(x):
    """uint32 -> float64 uniform on (0,1): ((x >> 9) + 1/2) * 2^-23."""
    x = np.asarray(x, dtype=np.uint32)
    return ((x >> np.uint32(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK32, seed >> 32


def walk_block(seed, walk, site, block):
    """Four uniforms of block `block` for walks `walk` (array) of site `site`."""
    k0, k1 = seed_key(seed)
    out = philox4x32_10(walk, site, block, TAG_WALK, k0, k1)
    return [to_uniform(o) for o in out]


def step_uniforms(seed, walk, site, k, dim):
    """The d-1 uniforms that move step k (k >= 1) of each walk.

    `walk` and `k` are arrays of equal length (one entry per walk still
    alive); returns a list of d-1 float64 arrays.
    """
    q = 4 // (dim - 1)
    k = np.asarray(k, dtype=np.int64)
    block = STEP_BLOCK0 + (k - 1) // q
    lane0 = ((k - 1) % q) * (dim - 1)
    k0, k1 = seed_key(seed)
    words = np.stack(philox4x32_10(walk, site, block, TAG_WALK, k0, k1))
    idx = np.arange(words.shape[1])
    return [to_uniform(words[lane0 + t, idx]) for t in range(dim - 1)]
