"""Covariance families and their spectral densities (test infrastructure).

Convention (Section 2 of the paper, Bochner's theorem): C(x) = \\int S(p)
e^{-2 pi i p.x} dp, i.e. S is the Fourier transform of C in "cycles"
frequency p.  The paper calls the density gamma; S here is that gamma.

Families (sigma = marginal standard deviation, ell = length scale):
* Gaussian   C(r) = sigma^2 exp(-r^2 / (2 ell^2))
             S(p) = sigma^2 (2 pi ell^2)^{d/2} exp(-2 pi^2 ell^2 |p|^2)
* Matern     C(r) = sigma^2 2^{1-nu}/Gamma(nu) (sqrt(2nu) r/ell)^nu K_nu(sqrt(2nu) r/ell)
             S(p) = sigma^2 2^d pi^{d/2} Gamma(nu+d/2) (2nu)^nu / (Gamma(nu) ell^{2nu})
                    * (2nu/ell^2 + 4 pi^2 |p|^2)^{-(nu+d/2)}
             (Rasmussen & Williams 2006, eq. 4.14/4.15)
* Exponential C(r) = sigma^2 exp(-r/ell)   (the Matern case nu = 1/2)
* The family of Section 4, eq. (5) (written there for d = 2, here for any d):
             S(p) = (m^{kl} + (sum_i p_i^{2k})^l)^{-n},  k, l, n >= 1, m > 0;
             anisotropic for k >= 2.  With sigma, S is scaled by sigma^2.
* A tabulated S: values of S at the grid frequencies of the half-spectrum.

The adjoint needs d log S / d theta for theta = (sigma, ell, nu); those are
written out below from the formulas above.
"""
import numpy as np
from scipy import special

GAUSSIAN = 0
MATERN = 1
EXPONENTIAL = 2

KIND_NAMES = {"gaussian": GAUSSIAN, "matern": MATERN, "exponential": EXPONENTIAL}


def _nu_of(kind, nu):
    return 0.5 if kind == EXPONENTIAL else float(nu)


def spectral_density(kind, p2, d, sigma, ell, nu=0.5):
    """S at squared frequency |p|^2 = p2 (cycles), dimension d."""
    p2 = np.asarray(p2, dtype=np.float64)
    sigma, ell = float(sigma), float(ell)
    if kind == GAUSSIAN:
        return sigma ** 2 * (2 * np.pi * ell ** 2) ** (d / 2) * np.exp(-2 * np.pi ** 2 * ell ** 2 * p2)
    if kind in (MATERN, EXPONENTIAL):
        nu = _nu_of(kind, nu)
        logc = (d * np.log(2.0) + 0.5 * d * np.log(np.pi) + special.gammaln(nu + d / 2)
                + nu * np.log(2 * nu) - special.gammaln(nu) - 2 * nu * np.log(ell))
        u = 2 * nu / ell ** 2 + 4 * np.pi ** 2 * p2
        return sigma ** 2 * np.exp(logc) * u ** (-(nu + d / 2))
    raise ValueError(f"unknown covariance kind {kind}")


def dlog_spectral_density(kind, p2, d, sigma, ell, nu=0.5):
    """(d log S/d sigma, d log S/d ell, d log S/d nu) at |p|^2 = p2.

    A parameter that the family does not have (nu for the Gaussian and the
    exponential family) gets derivative 0.
    """
    p2 = np.asarray(p2, dtype=np.float64)
    sigma, ell = float(sigma), float(ell)
    ds = np.full_like(p2, 2.0 / sigma)
    if kind == GAUSSIAN:
        dl = d / ell - 4 * np.pi ** 2 * ell * p2
        return ds, dl, np.zeros_like(p2)
    if kind in (MATERN, EXPONENTIAL):
        nu = _nu_of(kind, nu)
        u = 2 * nu / ell ** 2 + 4 * np.pi ** 2 * p2
        a = nu + d / 2
        dl = -2 * nu / ell + a * 4 * nu / (ell ** 3 * u)
        if kind == EXPONENTIAL:
            return ds, dl, np.zeros_like(p2)
        dn = (special.digamma(a) - special.digamma(nu) + np.log(2 * nu) + 1.0
              - 2 * np.log(ell) - np.log(u) - a * (2.0 / ell ** 2) / u)
        return ds, dl, dn
    raise ValueError(f"unknown covariance kind {kind}")


def covariance(kind, r, sigma, ell, nu=0.5):
    """Closed-form C(r), r = |x| >= 0 (independent of d)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    sigma, ell = float(sigma), float(ell)
    if kind == GAUSSIAN:
        return sigma ** 2 * np.exp(-r ** 2 / (2 * ell ** 2))
    if kind == EXPONENTIAL:
        return sigma ** 2 * np.exp(-r / ell)
    if kind == MATERN:
        nu = float(nu)
        t = np.sqrt(2 * nu) * r / ell
        with np.errstate(invalid="ignore", divide="ignore"):
            c = sigma ** 2 * 2 ** (1 - nu) / special.gamma(nu) * t ** nu * special.kv(nu, t)
        return np.where(t == 0, sigma ** 2, c)
    raise ValueError(f"unknown covariance kind {kind}")


def wrapped_index(n):
    """kappa(k) for k = 0..n-1: k below n/2, k - n from n/2 on (numpy fftfreq * n)."""
    k = np.arange(n)
    return np.where(k < n // 2, k, k - n).astype(np.float64)


def freq2_grid(dims, lengths, half=True):
    """|p_k|^2 on the (half-)spectrum grid, p_k = kappa(k) / l per axis.

    half=True: the last axis runs over k_d = 0..N_d/2 (kappa(N_d/2) = -N_d/2).
    """
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    out = 0.0
    for i, (n, l) in enumerate(zip(dims, lengths)):
        kap = wrapped_index(n)
        if half and i == d - 1:
            kap = kap[: n // 2 + 1].copy()
            kap[n // 2] = -(n // 2)
        shape = [1] * d
        shape[i] = kap.size
        out = out + (kap.reshape(shape) / float(l)) ** 2
    return np.asarray(out, dtype=np.float64)


def filter_h(dims, lengths, kind, sigma, ell, nu=0.5, half=True):
    """h_k = sqrt(S(p_k) / |D|) on the (half-)spectrum grid, |D| = prod l_i."""
    d = len(dims)
    vol = float(np.prod(lengths))
    p2 = freq2_grid(dims, lengths, half=half)
    return np.sqrt(spectral_density(kind, p2, d, sigma, ell, nu) / vol)


def freq_components(dims, lengths, half=True):
    """Per-axis frequencies p_i = kappa(k_i) / l_i on the (half-)spectrum grid,
    as broadcastable arrays (one per axis)."""
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    comps = []
    for i, (n, l) in enumerate(zip(dims, lengths)):
        kap = wrapped_index(n)
        if half and i == d - 1:
            kap = kap[: n // 2 + 1].copy()
            kap[n // 2] = -(n // 2)
        shape = [1] * d
        shape[i] = kap.size
        comps.append(kap.reshape(shape) / float(l))
    return comps


def paper_density(m, k, l, n):
    """S of Section 4, eq. (5), as a function of the per-axis frequencies."""
    m, k, l, n = float(m), int(k), int(l), int(n)

    def S(comps):
        q = 0.0
        for p in comps:
            q = q + p ** (2 * k)
        return (m ** (k * l) + q ** l) ** (-n)
    return S


def density_on_grid(dims, lengths, density, half=True):
    """S(p_k) on the (half-)spectrum grid for a density given as a function of
    the per-axis frequencies."""
    comps = freq_components(dims, lengths, half=half)
    shape = tuple(int(n) for n in dims[:-1]) + ((int(dims[-1]) // 2 + 1) if half else int(dims[-1]),)
    return np.broadcast_to(np.asarray(density(comps), dtype=np.float64), shape).copy()


def filter_from_density(dims, lengths, S, sigma=1.0):
    """h_k = sigma sqrt(S_k / |D|) from S on the same grid (half or full)."""
    vol = float(np.prod(lengths))
    return float(sigma) * np.sqrt(np.asarray(S, dtype=np.float64) / vol)

