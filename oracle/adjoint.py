"""Gradients of a loss through the samplers (test infrastructure).

The sampler is linear in the noise: phi = F*[A] with A = h_theta * xi(z)
(one-FFT algorithm) or A = h_theta * F[z] / sqrt(P) (two-FFT algorithm).
For a loss L with upstream gradient g = dL/dphi (real, field-shaped):

    dL = sum_{k full} Re(dA_k conj(G_k)),   G = F[g]  (forward transform),

because sum_j g_j e^{+2 pi i k.j/N} = conj(G_k) for real g.  Hence

* dL/dtheta = sum_{k full} dh_k/dtheta Re(xi_k conj(G_k)),
  dh/dtheta = (h/2) d log S/dtheta.  On the half-spectrum every interior
  entry (0 < k_d < N_d/2) stands for itself and its mirror: weight 2; the
  planes k_d in {0, N_d/2} hold both members of each pair: weight 1.
* dL/dz for the one-FFT algorithm follows the Hermitian arrangement back to
  the normals: interior entries give sqrt(2) h (Re G, Im G) to their two
  slots; in the planes a representative row r gives sqrt(2) h (Re G, Im G) of
  (r, 0) to slots (r, 0..1) and of (r, N_d/2) to slots (-r, 0..1); a
  self-conjugate row gives h Re G of (r, 0) and of (r, N_d/2) to slots
  (r, 0) and (r, 1).  (The mirrored rows hold the conjugates, so they add
  nothing new.)
* dL/dz for the two-FFT algorithm: phi = F*[h F[z]]/sqrt(P) with h real and
  even (h_{-k} = h_k) is a symmetric operator, so dL/dz = F*[h F[g]]/sqrt(P).
"""
import numpy as np

from .grf import hermitian_noise, neg_row_index
from .spectra import freq2_grid, filter_h, dlog_spectral_density


def half_weights(dims):
    nd = int(dims[-1])
    m = nd // 2
    w = np.full(m + 1, 2.0)
    w[0] = 1.0
    w[m] = 1.0
    return w


def grad_theta_alg2(z, g, lengths, kind, sigma, ell, nu=0.5):
    """(dL/dsigma, dL/dell, dL/dnu) for the one-FFT algorithm, float64."""
    z = np.asarray(z, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    dims = z.shape
    xi = hermitian_noise(z)
    G = np.fft.rfftn(g)
    p2 = freq2_grid(dims, lengths, half=True)
    h = filter_h(dims, lengths, kind, sigma, ell, nu, half=True)
    dlog = dlog_spectral_density(kind, p2, len(dims), sigma, ell, nu)
    w = half_weights(dims)
    core = w * np.real(xi * np.conj(G))
    return np.array([np.sum(0.5 * h * dl * core) for dl in dlog])


def grad_theta_alg1(z, g, lengths, kind, sigma, ell, nu=0.5):
    """(dL/dsigma, dL/dell, dL/dnu) for the two-FFT algorithm, float64."""
    z = np.asarray(z, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    dims = z.shape
    P = int(np.prod(dims, dtype=np.int64))
    xi = np.fft.rfftn(z) / np.sqrt(P)
    G = np.fft.rfftn(g)
    p2 = freq2_grid(dims, lengths, half=True)
    h = filter_h(dims, lengths, kind, sigma, ell, nu, half=True)
    dlog = dlog_spectral_density(kind, p2, len(dims), sigma, ell, nu)
    w = half_weights(dims)
    core = w * np.real(xi * np.conj(G))
    return np.array([np.sum(0.5 * h * dl * core) for dl in dlog])


def grad_noise_alg2(g, lengths, kind, sigma, ell, nu=0.5, h=None):
    """dL/dz (field-shaped) for the one-FFT algorithm."""
    g = np.asarray(g, dtype=np.float64)
    dims = g.shape
    nd = dims[-1]
    m = nd // 2
    rows = int(np.prod(dims[:-1], dtype=np.int64)) if len(dims) > 1 else 1
    G = np.fft.rfftn(g).reshape(rows, m + 1)
    if h is None:
        h = filter_h(dims, lengths, kind, sigma, ell, nu, half=True)
    h = np.asarray(h).reshape(rows, m + 1)
    gz = np.zeros((rows, nd))
    s2 = np.sqrt(2.0)
    if m > 1:
        gz[:, 2:2 * m:2] = s2 * h[:, 1:m] * G[:, 1:m].real
        gz[:, 3:2 * m:2] = s2 * h[:, 1:m] * G[:, 1:m].imag
    neg = neg_row_index(dims)
    r = np.arange(rows)
    selfc = neg == r
    rep = r < neg
    gz[selfc, 0] = h[selfc, 0] * G[selfc, 0].real
    gz[selfc, 1] = h[selfc, m] * G[selfc, m].real
    gz[rep, 0] = s2 * h[rep, 0] * G[rep, 0].real
    gz[rep, 1] = s2 * h[rep, 0] * G[rep, 0].imag
    nr = neg[rep]
    gz[nr, 0] = s2 * h[rep, m] * G[rep, m].real
    gz[nr, 1] = s2 * h[rep, m] * G[rep, m].imag
    return gz.reshape(dims)


def grad_noise_alg1(g, lengths, kind, sigma, ell, nu=0.5):
    """dL/dz (field-shaped) for the two-FFT algorithm.

    phi = F*[h F[z]]/sqrt(P) is a real symmetric-filter convolution, so its
    transpose is the same operator: dL/dz = F*[h F[g]] / sqrt(P).
    """
    g = np.asarray(g, dtype=np.float64)
    dims = g.shape
    P = int(np.prod(dims, dtype=np.int64))
    h = filter_h(dims, lengths, kind, sigma, ell, nu, half=True)
    return P * np.fft.irfftn(h * np.fft.rfftn(g), s=dims, axes=tuple(range(len(dims)))) / np.sqrt(P)
