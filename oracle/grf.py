"""The two sampling algorithms of Section 3, in float64 (test infrastructure).

Notation: dims N = (N_1, ..., N_d), all even; lengths l; P = prod N_i;
|D| = prod l_i.  Discrete transforms (numpy's): forward
F[z]_k = sum_j z_j e^{-2 pi i k.j/N}; inverse without normalisation
F*[A]_j = sum_k A_k e^{+2 pi i k.j/N}.

Scaling (the paper leaves it to "FFT includes all necessary rescaling"): with
R() ~ N(0, |Delta|^-1), FFT = |Delta| F (Riemann sum of FW, Section 2) and
FFT^-1 = F*, the two-FFT algorithm becomes phi = F*[h F[z] / sqrt(P)] with
z ~ N(0, 1) and h_k = sqrt(S(p_k) / |D|).  Both algorithms then give
Cov(phi_j, phi_j') = (1/|D|) sum_k S(p_k) e^{2 pi i k.(j-j')/N}, the Riemann
sum of the covariance integral.

The frequency of index k is p_k = kappa(k)/l with kappa the wrapped index
(k, or k - N_i from N_i/2 on); the algorithms' printed (k_i - N_i/2)/l_i is
that grid written in centred order.

Half-spectrum: entries k_d = 0..N_d/2 of the last axis; the rest follows from
A_{-k} = conj(A_k) (eq. (3)).
"""
import numpy as np

from . import noise as _noise
from .spectra import filter_h


def _rows_shape(dims):
    return tuple(int(n) for n in dims[:-1])


def neg_row_index(dims):
    """For each row (linear index over the leading d-1 axes) the row of -k."""
    lead = _rows_shape(dims)
    if not lead:
        return np.zeros(1, dtype=np.int64)
    idx = np.indices(lead).reshape(len(lead), -1)
    neg = [(-idx[i]) % lead[i] for i in range(len(lead))]
    return np.ravel_multi_index(neg, lead).astype(np.int64)


def hermitian_noise(z):
    """Fourier-space noise xi on the half-spectrum from real normals z.

    The Hermitian data arrangement of the one-FFT algorithm (Section 3, with
    Lemma 1, eq. (3) and rules b-d of Section 2): entries with K = -K are real
    with variance 1, the others are (a + i b)/sqrt(2) with a, b independent
    N(0,1), and a mirrored entry is the conjugate of its partner.

    z has the field's shape [..., N_d]; the map uses every z exactly once:
    * interior k_d (0 < k_d < N_d/2): xi[row, k_d] = (z[row, 2k_d] + i z[row, 2k_d+1]) / sqrt(2);
    * the planes k_d = 0 and k_d = N_d/2 use slots 0 and 1 of each row.  With
      c(r) = (z[r, 0] + i z[r, 1]) / sqrt(2) and -r the mirrored row:
        row = -row (self-conjugate): xi[row, 0] = z[row, 0],  xi[row, N_d/2] = z[row, 1];
        row < -row (representative): xi[row, 0] = c(row),     xi[row, N_d/2] = c(-row);
        row > -row:                  xi[row, 0] = conj c(-row), xi[row, N_d/2] = conj c(row).
    Returns complex128 array of shape [..., N_d/2 + 1].
    """
    z = np.asarray(z, dtype=np.float64)
    dims = z.shape
    nd = dims[-1]
    m = nd // 2
    rows = int(np.prod(dims[:-1], dtype=np.int64)) if len(dims) > 1 else 1
    zz = z.reshape(rows, nd)
    xi = np.zeros((rows, m + 1), dtype=np.complex128)
    s2 = np.sqrt(0.5)
    if m > 1:
        xi[:, 1:m] = (zz[:, 2:2 * m:2] + 1j * zz[:, 3:2 * m:2]) * s2
    neg = neg_row_index(dims)
    r = np.arange(rows)
    c = (zz[:, 0] + 1j * zz[:, 1]) * s2
    selfc = neg == r
    rep = r < neg
    other = r > neg
    xi[selfc, 0] = zz[selfc, 0]
    xi[selfc, m] = zz[selfc, 1]
    xi[rep, 0] = c[rep]
    xi[rep, m] = c[neg[rep]]
    xi[other, 0] = np.conj(c[neg[other]])
    xi[other, m] = np.conj(c[other])
    return xi.reshape(dims[:-1] + (m + 1,))


def hermitian_extend(half, dims):
    """Full spectrum from the half-spectrum via A_{-k} = conj(A_k)."""
    dims = tuple(int(n) for n in dims)
    nd = dims[-1]
    m = nd // 2
    full = np.zeros(dims, dtype=np.complex128)
    full[..., : m + 1] = half
    for kd in range(m + 1, nd):
        # -k: negate every index mod N
        src = half[..., nd - kd]
        for ax in range(len(dims) - 1):
            src = np.roll(np.flip(src, axis=ax), 1, axis=ax)
        full[..., kd] = np.conj(src)
    return full


def alg2_from_noise(z, lengths, kind, sigma, ell, nu=0.5, return_parts=False, h=None):
    """One-FFT (Hermitian) algorithm on given normals z (field-shaped).  h: the
    half-spectrum filter, instead of the family (kind, sigma, ell, nu)."""
    z = np.asarray(z, dtype=np.float64)
    dims = z.shape
    P = int(np.prod(dims, dtype=np.int64))
    xi = hermitian_noise(z)
    if h is None:
        h = filter_h(dims, lengths, kind, sigma, ell, nu, half=True)
    A = h * xi
    phi = P * np.fft.irfftn(A, s=dims, axes=tuple(range(len(dims))))
    if return_parts:
        return phi, dict(xi=xi, h=h, A=A)
    return phi


def alg1_from_noise(z, lengths, kind, sigma, ell, nu=0.5, return_parts=False, h=None):
    """Two-FFT algorithm on given white noise z (field-shaped); h as above."""
    z = np.asarray(z, dtype=np.float64)
    dims = z.shape
    P = int(np.prod(dims, dtype=np.int64))
    Z = np.fft.rfftn(z)
    if h is None:
        h = filter_h(dims, lengths, kind, sigma, ell, nu, half=True)
    A = h * Z / np.sqrt(P)
    phi = P * np.fft.irfftn(A, s=dims, axes=tuple(range(len(dims))))
    if return_parts:
        return phi, dict(Z=Z, h=h, A=A)
    return phi


def alg2_full_complex(z, lengths, kind, sigma, ell, nu=0.5):
    """The paper's literal path: full complex array, complex inverse FFT."""
    z = np.asarray(z, dtype=np.float64)
    dims = z.shape
    P = int(np.prod(dims, dtype=np.int64))
    xi = hermitian_noise(z)
    h = filter_h(dims, lengths, kind, sigma, ell, nu, half=True)
    full = hermitian_extend(h * xi, dims)
    return P * np.fft.ifftn(full)


def sample(dims, lengths, kind, sigma, ell, nu=0.5, seed=0, batch=1, alg=2, h=None):
    """Fields seed..seed+batch-1 of algorithm ``alg`` (1 or 2), float64; h: an
    explicit half-spectrum filter instead of the family."""
    dims = tuple(int(n) for n in dims)
    tag = _noise.TAG_ALG2 if alg == 2 else _noise.TAG_ALG1
    f = alg2_from_noise if alg == 2 else alg1_from_noise
    out = np.empty((batch,) + dims)
    for b in range(batch):
        z = _noise.field_noise(dims, (int(seed) + b) & 0xFFFFFFFFFFFFFFFF, tag)
        out[b] = f(z, lengths, kind, sigma, ell, nu, h=h)
    return out


def discrete_covariance(dims, lengths, kind, sigma, ell, nu=0.5, h_full=None):
    """C_N(j) = (1/|D|) sum_k S(p_k) e^{2 pi i k.j/N}: the exact covariance of
    both algorithms' output between grid points 0 and j (field-shaped).
    h_full: an explicit filter on the full spectrum instead of the family."""
    dims = tuple(int(n) for n in dims)
    P = int(np.prod(dims, dtype=np.int64))
    hf = filter_h(dims, lengths, kind, sigma, ell, nu, half=False) if h_full is None else h_full
    return np.real(np.fft.ifftn(hf ** 2)) * P
