"""Float64 CPU oracle for FFT-based Gaussian random field sampling.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, independent
restatement of Lang & Potthoff, "Fast simulation of Gaussian random fields"
(Sections 2-3 and the appendix): the noise contract (Philox + Box-Muller),
the Hermitian data arrangement, the spectral filter, both sampling algorithms,
the adjoint, the recursive exact-count variant, and the cosine / sine
transform variant for reflecting boundaries.  Only the tests, the smoke check and the benchmark's CPU
baseline may import it; the GPU library never does, and it never imports the
GPU library.  Every function is pinned by a CPU test against something other
than itself (published known-answer vectors, naive DFTs, closed forms, exact
covariance identities, finite differences).
"""
from . import philox, noise, spectra, grf, adjoint, dft, reflect, recursive  # noqa: F401
from .spectra import GAUSSIAN, MATERN, EXPONENTIAL  # noqa: F401
