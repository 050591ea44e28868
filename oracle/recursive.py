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


def draw_order(dims):
    """The entries in the order in which the recursion draws for them:
    (k, 2) for an entry that takes a real and an imaginary part (its mirror
    -k gets the conjugate), (k, 1) for a real entry."""
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    out = []

    def set_array(j, tail):
        # axes 0 .. j-1 (0-based) free; axes j .. d-1 fixed at `tail`
        Mj = dims[j - 1] // 2
        for kk in np.ndindex(*[dims[i] for i in range(j - 1)], Mj - 1):
            out.append((tuple(kk[:-1]) + (kk[-1] + 1,) + tuple(tail), 2))
        if j == 1:
            for a in (0, Mj):
                out.append(((a,) + tuple(tail), 1))
        else:
            set_array(j - 1, (0,) + tuple(tail))
            set_array(j - 1, (Mj,) + tuple(tail))

    set_array(d, ())
    return out


def spectrum_from_stream(stream, dims, h_full):
    """A (full complex spectrum) by the recursion; `stream` yields normals.
    Returns (A, number of draws)."""
    dims = tuple(int(n) for n in dims)
    A = np.full(dims, np.nan + 1j * np.nan)
    it = iter(stream)
    count = 0
    s = 2.0 ** -0.5
    for k, nd in draw_order(dims):
        if nd == 2:
            re = s * float(next(it)) * h_full[k]
            im = s * float(next(it)) * h_full[k]
            A[k] = re + 1j * im
            A[tuple((-ki) % n for ki, n in zip(k, dims))] = re - 1j * im
        else:
            A[k] = float(next(it)) * h_full[k]
        count += nd
    return A, count


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


# ---------------------------------------------------------------------------
# Adjoint (the sampler is linear in the stream): for phi = F*[A] and an
# upstream gradient g, dL = sum_{k full} Re(dA_k conj G_k) with G = F[g].

def grad_theta(stream, g, lengths, kind, sigma, ell, nu=0.5):
    """(dL/dsigma, dL/dell, dL/dnu): sum over the full spectrum of
    (h_k / 2) d log S / d theta Re(xi_k conj G_k), xi = A / h."""
    from .spectra import dlog_spectral_density, freq2_grid
    g = np.asarray(g, dtype=np.float64)
    dims = g.shape
    xi, _ = spectrum_from_stream(stream, dims, np.ones(dims))
    G = np.fft.fftn(g)
    h = filter_h(dims, lengths, kind, sigma, ell, nu, half=False)
    p2 = freq2_grid(dims, lengths, half=False)
    core = 0.5 * h * np.real(xi * np.conj(G))
    return np.array([np.sum(core * dl) for dl in dlog_spectral_density(kind, p2, len(dims), sigma, ell, nu)])


def grad_stream(g, lengths, kind, sigma, ell, nu=0.5, h_full=None):
    """dL/d(draw j) for every draw of the sequence (row-major field shape):
    an entry with two draws gives sqrt(2) h (Re G, Im G) (it and its mirror
    both carry them), a real entry h Re G."""
    g = np.asarray(g, dtype=np.float64)
    dims = g.shape
    G = np.fft.fftn(g)
    h = filter_h(dims, lengths, kind, sigma, ell, nu, half=False) if h_full is None else h_full
    out = np.empty(int(np.prod(dims)))
    j = 0
    for k, nd in draw_order(dims):
        if nd == 2:
            out[j] = np.sqrt(2.0) * h[k] * G[k].real
            out[j + 1] = np.sqrt(2.0) * h[k] * G[k].imag
        else:
            out[j] = h[k] * G[k].real
        j += nd
    return out.reshape(dims)
