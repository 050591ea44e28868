"""Noise contract: seed -> i.i.d. standard normals (test infrastructure).

The paper's algorithms only ask for a generator R() of independent centred
normals (Section 3, the Input lists of the three algorithms).  To make a GPU
sample comparable element by element with this oracle, both follow one
contract:

* field b of a batch uses the 64-bit Philox key ``seed + b``;
* a field's noise is a real array z with the field's own shape
  [N_1, ..., N_d].  "row" is the linear index over the leading d-1 axes,
  s the index along the last axis;
* z[row, s] is lane (s mod 4) of the Philox-4x32-10 block with counter
  (s div 4, row, tag, 0); tag 0 is the white noise of the two-FFT algorithm,
  tag 1 the Fourier-space noise of the one-FFT (Hermitian) algorithm, tag 2
  the slot coefficients of the cosine / sine transforms (reflecting
  boundaries), tag 3 the sequential stream of the recursive algorithm (its
  j-th draw is z in row-major order);
* the 32-bit outputs x become uniforms u = (x + 1/2) 2^-32 in (0, 1);
* Box and Muller (1958): lanes (0,1) and (2,3) of a block are pairs
  (u_a, u_b) -> sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b).
"""
import numpy as np

from .philox import philox4x32, key_of

TAG_ALG1 = 0
TAG_ALG2 = 1
TAG_REFLECT = 2
TAG_RECURSIVE = 3


def uniforms(x):
    """uint32 -> float64 uniforms (x + 1/2) 2^-32 (exact in float64)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * 2.0 ** -32


def box_muller(ua, ub):
    """Pair of uniforms -> pair of independent N(0,1) (Box & Muller 1958)."""
    r = np.sqrt(-2.0 * np.log(ua))
    t = 2.0 * np.pi * ub
    return r * np.cos(t), r * np.sin(t)


def block_normals(q, row, tag, seed):
    """Four normals of the blocks with counters (q, row, tag, 0).

    Returns an array of shape broadcast(q, row) + (4,).
    """
    k0, k1 = key_of(seed)
    x = philox4x32(q, row, tag, 0, k0, k1)
    u = [uniforms(v) for v in x]
    n0, n1 = box_muller(u[0], u[1])
    n2, n3 = box_muller(u[2], u[3])
    return np.stack([n0, n1, n2, n3], axis=-1)


def field_noise(dims, seed, tag):
    """z for one field: float64 array of shape dims (N_d must be even)."""
    dims = tuple(int(n) for n in dims)
    rows = int(np.prod(dims[:-1], dtype=np.int64)) if len(dims) > 1 else 1
    nd = dims[-1]
    nq = (nd + 3) // 4
    q = np.arange(nq, dtype=np.uint64)[None, :]
    r = np.arange(rows, dtype=np.uint64)[:, None]
    nb = block_normals(q, r, tag, seed)            # [rows, nq, 4]
    z = nb.reshape(rows, nq * 4)[:, :nd]
    return z.reshape(dims)


def batch_noise(dims, seed, batch, tag):
    """Noise of fields seed, seed+1, ..., seed+batch-1 stacked on axis 0."""
    return np.stack([field_noise(dims, (int(seed) + b) & 0xFFFFFFFFFFFFFFFF, tag)
                     for b in range(batch)])


def philox_raw(seed, counters):
    """Raw uint32 output for explicit counters [n, 4] (the bit-exact check)."""
    c = np.asarray(counters, dtype=np.uint64)
    k0, k1 = key_of(seed)
    out = philox4x32(c[:, 0], c[:, 1], c[:, 2], c[:, 3], k0, k1)
    return np.stack(out, axis=-1)
