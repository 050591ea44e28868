"""Seeded synthetic workload descriptions shared by the tests and the
benchmark.  Only descriptions and random inputs live here -- none of the
sampler's arithmetic -- so that the float64 oracle and the GPU library can both
be driven from the same inputs without sharing code."""
import numpy as np

CONFIG4_SIDES = (64, 96, 128, 360, 512, 1000, 1024)
CONFIG4_NUS = (0.5, 1.5, 2.5)


def uneven_fields(n=4096, seed=0, sides=CONFIG4_SIDES, nus=CONFIG4_NUS, ell_range=(0.02, 0.2)):
    """n two-dimensional fields: N_1 and N_2 drawn independently and uniformly
    from `sides`, Matern nu uniformly from `nus`, length scale uniform in
    ell_range, sigma 1, unit torus, field f sampled with Philox key f.  The
    description is drawn from numpy.random.default_rng(seed)."""
    rng = np.random.default_rng(seed)
    n1 = rng.choice(sides, size=n)
    n2 = rng.choice(sides, size=n)
    nu = rng.choice(nus, size=n)
    ell = rng.uniform(ell_range[0], ell_range[1], size=n)
    return [dict(dims=(int(n1[f]), int(n2[f])), cov="matern", sigma=1.0, length_scale=float(ell[f]),
                 nu=float(nu[f]), seed=f, lengths=(1.0, 1.0)) for f in range(n)]


def loss_weights(shape, seed=1):
    """w ~ U[0, 1] for the quadratic loss L = sum w phi^2."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=shape)
