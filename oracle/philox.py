"""Philox-4xW-10 counter-based generator (test infrastructure, oracle side).

Definition followed: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3" (SC'11), section 4 (the Philox S-box: two W x W -> 2W
multiplications per round, the "hi" halves xored with the other two counter
words and the round key, the key bumped by a Weyl sequence each round).

Two implementations of the same definition live here:

* ``philox_scalar``  -- Python integers, any word width W (32 or 64).  At W=64
  it is checked against numpy's own Philox bit generator (a 4x64-10
  implementation), at W=32 against the publication's known-answer vectors.
* ``philox4x32``     -- numpy-vectorised W=32 version used by the oracle; it is
  checked against ``philox_scalar`` on random counters and keys.

The paper being implemented leaves its generator R() unspecified; this module
is the shared noise contract that both the oracle and the GPU library follow.
"""
import numpy as np

# Round multipliers and Weyl key increments of the SC'11 publication.
PHILOX_CONST = {
    32: dict(M0=0xD2511F53, M1=0xCD9E8D57, W0=0x9E3779B9, W1=0xBB67AE85),
    64: dict(M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
             W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B),
}
ROUNDS = 10


def philox_scalar(ctr, key, width=32, rounds=ROUNDS):
    """Philox-4xW over Python ints.  ctr: 4 words, key: 2 words."""
    k = PHILOX_CONST[width]
    mask = (1 << width) - 1
    c = [int(v) & mask for v in ctr]
    kk = [int(v) & mask for v in key]
    for _ in range(rounds):
        p0 = k["M0"] * c[0]
        p1 = k["M1"] * c[2]
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c = [hi1 ^ c[1] ^ kk[0], lo1, hi0 ^ c[3] ^ kk[1], lo0]
        kk = [(kk[0] + k["W0"]) & mask, (kk[1] + k["W1"]) & mask]
    return c


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Vectorised Philox-4x32.

    c0..c3: integer arrays (broadcastable) holding 32-bit counter words.
    k0, k1: 32-bit key words (scalars).  Returns four uint32 arrays.
    """
    K = PHILOX_CONST[32]
    m32 = np.uint64(0xFFFFFFFF)
    c = [np.asarray(v, dtype=np.uint64) & m32 for v in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    kk0, kk1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    M0, M1 = np.uint64(K["M0"]), np.uint64(K["M1"])
    sh = np.uint64(32)
    for _ in range(rounds):
        p0 = M0 * c[0]              # < 2^64, exact in uint64
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> sh, p0 & m32
        hi1, lo1 = p1 >> sh, p1 & m32
        c = [hi1 ^ c[1] ^ np.uint64(kk0), lo1, hi0 ^ c[3] ^ np.uint64(kk1), lo0]
        kk0 = (kk0 + K["W0"]) & 0xFFFFFFFF
        kk1 = (kk1 + K["W1"]) & 0xFFFFFFFF
    return [v.astype(np.uint32) for v in c]


def key_of(seed):
    """64-bit seed -> (k0, k1) = (low word, high word)."""
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    return s & 0xFFFFFFFF, s >> 32
