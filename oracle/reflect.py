"""Reflecting boundaries: Neumann and Dirichlet fields by cosine and sine
transforms (test infrastructure).

The introduction and the remark that opens Section 3 say that the FFT makes
the fields periodic and that discrete cosine and sine transforms in its place
give Neumann and Dirichlet boundaries; the paper gives no further detail.
The reading written out here (one boundary kind per axis):

* grid: cell centres x_j = (j + 1/2) l / N, j = 0..N-1, on [0, l];
* slot n = 0..N-1 of an axis carries the mode
      cosine axis (Neumann):   b(n, j) = cos(pi n (j + 1/2) / N),        k = n
      sine axis (Dirichlet):   b(n, j) = sin(pi (N - n) (j + 1/2) / N),  k = N - n
  of frequency p = k / (2 l) (cycles): the modes of the periodic grid of 2N
  points on [-l, l) that are even (cosine) or odd (sine) about x = 0;
* slot weight c(0) = 1, c(n) = 2 for n >= 1, and
      phi_j = sum_n a_n z_n prod_i b_i(n_i, j_i),
      a_n = sigma sqrt(S(p_n) prod_i c(n_i) / |D|),   |D| = prod l_i,
  with z the noise contract's normals (tag 2) indexed by slot.

Then Cov(phi_j, phi_j') = sum_r s_r C2(j - r(j')): the method of images,
over the 2^d reflections r_i(j') in {j'_i, -j'_i - 1} (mod 2 N_i) of the
doubled grid, s_r = -1 to the number of reflected sine axes, and C2 the
exact covariance of the periodic algorithms on the doubled grid (2 N_i
points, lengths 2 l_i).  A slot-0 mode of a sine axis is the Nyquist mode
k = N of the doubled grid, which that grid holds once; hence its weight 1.

Every step is the definition, with the per-axis basis as an explicit matrix:
O(N^2) per axis, for small grids only.
"""
import numpy as np

from . import noise as _noise
from .spectra import spectral_density

TAG = _noise.TAG_REFLECT


def axis_basis(n, sine):
    """B[j, slot] of one axis (n points)."""
    j = np.arange(n, dtype=np.float64)[:, None] + 0.5
    s = np.arange(n, dtype=np.float64)[None, :]
    if sine:
        return np.sin(np.pi * (n - s) * j / n)
    return np.cos(np.pi * s * j / n)


def slot_frequencies(n, l, sine):
    """p (cycles) of the slots of one axis."""
    s = np.arange(n, dtype=np.float64)
    return ((n - s) if sine else s) / (2.0 * float(l))


def slot_weights(n):
    c = np.full(n, 2.0)
    c[0] = 1.0
    return c


def _grid(dims, per_axis):
    d = len(dims)
    out = []
    for i, v in enumerate(per_axis):
        shape = [1] * d
        shape[i] = dims[i]
        out.append(np.asarray(v, dtype=np.float64).reshape(shape))
    return out


def slot_components(dims, lengths, sine_axes):
    """Per-axis frequency components on the slot grid (broadcastable)."""
    dims = tuple(int(n) for n in dims)
    return _grid(dims, [slot_frequencies(n, l, s) for n, l, s in zip(dims, lengths, sine_axes)])


def coefficients(dims, lengths, sine_axes, kind=None, sigma=1.0, ell=1.0, nu=0.5, density=None, S=None):
    """a_n over the slot grid for a family (kind, sigma, ell, nu), a density
    given as a function of the per-axis frequencies (times sigma^2), or S
    tabulated on the slot grid (times sigma^2)."""
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    comps = slot_components(dims, lengths, sine_axes)
    if S is not None:
        Sg = float(sigma) ** 2 * np.asarray(S, dtype=np.float64)
    elif density is not None:
        Sg = float(sigma) ** 2 * np.asarray(density(comps), dtype=np.float64)
    else:
        p2 = sum(c ** 2 for c in comps)
        Sg = spectral_density(kind, p2, d, sigma, ell, nu)
    c = 1.0
    for w in _grid(dims, [slot_weights(n) for n in dims]):
        c = c * w
    vol = float(np.prod(lengths))
    return np.broadcast_to(np.sqrt(Sg * c / vol), dims).copy()


def apply_basis(coef, sine_axes):
    """sum_n coef_n prod_i b_i(n_i, j_i): the basis matrix of each axis applied
    along that axis."""
    out = np.asarray(coef, dtype=np.float64)
    for i, s in enumerate(sine_axes):
        B = axis_basis(out.shape[i], s)
        out = np.moveaxis(np.tensordot(B, out, axes=([1], [i])), 0, i)
    return out


def field_from_noise(z, a, sine_axes):
    return apply_basis(np.asarray(a) * np.asarray(z, dtype=np.float64), sine_axes)


def sample(dims, lengths, sine_axes, seed=0, batch=1, a=None, **family):
    """Fields seed .. seed + batch - 1 (float64); a: explicit coefficients."""
    dims = tuple(int(n) for n in dims)
    if a is None:
        a = coefficients(dims, lengths, sine_axes, **family)
    out = np.empty((batch,) + dims)
    for b in range(batch):
        z = _noise.field_noise(dims, (int(seed) + b) & 0xFFFFFFFFFFFFFFFF, TAG)
        out[b] = field_from_noise(z, a, sine_axes)
    return out


def covariance_with(a, sine_axes, jp):
    """Cov(phi_j, phi_jp) for every j: sum_n a_n^2 prod_i b_i(n_i, j_i) b_i(n_i, jp_i)."""
    a = np.asarray(a, dtype=np.float64)
    w = a ** 2
    for i, s in enumerate(sine_axes):
        bj = axis_basis(a.shape[i], s)[jp[i]]
        shape = [1] * a.ndim
        shape[i] = a.shape[i]
        w = w * bj.reshape(shape)
    return apply_basis(w, sine_axes)


# ---------------------------------------------------------------------------
# Adjoint.  phi = B (a * z) with B the product of the axis bases, so for an
# upstream gradient g = dL/dphi:
#   dL/dz     = a * B^T g,
#   dL/dtheta = sum_n (B^T g)_n z_n da_n/dtheta,  da/dtheta = (a/2) d log S/dtheta.
# B^T along an axis is the transposed basis matrix: sum_j g_j b(n, j).

def apply_basis_transpose(v, sine_axes):
    """sum_j v_j prod_i b_i(n_i, j_i) for every slot n."""
    out = np.asarray(v, dtype=np.float64)
    for i, s in enumerate(sine_axes):
        B = axis_basis(out.shape[i], s)
        out = np.moveaxis(np.tensordot(B.T, out, axes=([1], [i])), 0, i)
    return out


def grad_theta(z, g, lengths, sine_axes, kind=None, sigma=1.0, ell=1.0, nu=0.5, density=None, S=None):
    """(dL/dsigma, dL/dell, dL/dnu); a family given by a density or a table
    has only sigma (the other two are 0)."""
    from .spectra import dlog_spectral_density
    dims = np.shape(z)
    a = coefficients(dims, lengths, sine_axes, kind, sigma, ell, nu, density=density, S=S)
    G = apply_basis_transpose(g, sine_axes)
    core = 0.5 * a * np.asarray(z, dtype=np.float64) * G
    if density is not None or S is not None:
        return np.array([np.sum(core) * 2.0 / float(sigma), 0.0, 0.0])
    p2 = sum(c ** 2 for c in slot_components(dims, lengths, sine_axes))
    dl = dlog_spectral_density(kind, np.broadcast_to(p2, dims), len(dims), sigma, ell, nu)
    return np.array([np.sum(core * d) for d in dl])


def grad_noise(g, a, sine_axes):
    return np.asarray(a) * apply_basis_transpose(g, sine_axes)
