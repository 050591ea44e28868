"""Algorithm 3 of Section 3: the recursive one-FFT sampler that draws exactly
P = prod N_i normals (test infrastructure).

create_random_field fills the full complex spectrum A by set_array over all
d axes and transforms it back.  set_array over the axes 1..j (the axes after
j fixed at given values) first sets every entry whose axis-j index lies in
1 .. N_j/2 - 1 (any index on the axes before j), drawing two normals for the
real and imaginary part (each times 2^{-1/2} h) and writing the conjugate at
the mirrored entry; then it handles the two hyperplanes k_j = 0 and
k_j = N_j/2 by the same procedure one dimension lower, and for j = 1 those
planes are the two real entries k_1 = 0 and k_1 = N_1/2, one normal each.

Readings (the typeset listing is ambiguous there): the recursion into the two
hyperplanes runs once, after the loop (it is printed inside the loop body);
the loop over the axes before j runs 0 .. N_i - 1 (printed as 0 .. N_i); the
loop nest is row-major, the axis-1 index outermost and the axis-j index
innermost.  With these readings exactly P normals are drawn.

Scaling as in the other algorithms of this package: z ~ N(0, 1), h the
filter sqrt(S(p)/|D|), output F*[A] (inverse DFT without normalisation).  The
normals are taken from a sequential stream: the j-th draw is the j-th value
of the field-shaped noise of the contract with tag 3, in row-major order.
"""
import numpy as np

from . import noise as _noise
from .spectra import filter_h

TAG = _noise.TAG_RECURSIVE


def spectrum_from_stream(stream, dims, h_full):
    """A (full complex spectrum) by the recursion; `stream` yields normals.
    Returns (A, number of draws)."""
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    A = np.full(dims, np.nan + 1j * np.nan)
    it = iter(stream)
    count = [0]

    def R():
        count[0] += 1
        return float(next(it))

    s = 2.0 ** -0.5

    def set_array(j, tail):
        # axes 0 .. j-1 (0-based) free; axes j .. d-1 fixed at `tail`
        lead = [range(dims[i]) for i in range(j - 1)]
        Mj = dims[j - 1] // 2
        for kk in np.ndindex(*[len(r) for r in lead], Mj - 1):
            k = tuple(kk[:-1]) + (kk[-1] + 1,) + tuple(tail)
            re = s * R() * h_full[k]
            im = s * R() * h_full[k]
            A[k] = re + 1j * im
            km = tuple((-ki) % n for ki, n in zip(k, dims))
            A[km] = re - 1j * im
        if j == 1:
            for a in (0, Mj):
                k = (a,) + tuple(tail)
                A[k] = R() * h_full[k]
        else:
            set_array(j - 1, (0,) + tuple(tail))
            set_array(j - 1, (Mj,) + tuple(tail))

    set_array(d, ())
    return A, count[0]


def alg3_from_stream(stream, dims, lengths, kind, sigma, ell, nu=0.5, h_full=None):
    dims = tuple(int(n) for n in dims)
    P = int(np.prod(dims, dtype=np.int64))
    if h_full is None:
        h_full = filter_h(dims, lengths, kind, sigma, ell, nu, half=False)
    A, _ = spectrum_from_stream(stream, dims, h_full)
    return np.real(np.fft.ifftn(A)) * P


def sample(dims, lengths, kind, sigma, ell, nu=0.5, seed=0, batch=1, h_full=None):
    """Fields seed .. seed + batch - 1, each from its own sequential stream."""
    dims = tuple(int(n) for n in dims)
    out = np.empty((batch,) + dims)
    for b in range(batch):
        z = _noise.field_noise(dims, (int(seed) + b) & 0xFFFFFFFFFFFFFFFF, TAG).ravel()
        out[b] = alg3_from_stream(z, dims, lengths, kind, sigma, ell, nu, h_full=h_full)
    return out
