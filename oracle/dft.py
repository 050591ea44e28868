"""Naive O(P^2) discrete Fourier transforms from the definition (test
infrastructure): the pin for every fast transform the oracle uses.

F_sign[x]_k = sum_j x_j exp(sign * 2 pi i sum_i k_i j_i / N_i) over all j of the
d-dimensional grid, written as one dense P x P matrix.  Tiny grids only.
"""
import numpy as np


def dft_matrix(dims, sign):
    dims = tuple(int(n) for n in dims)
    idx = np.indices(dims).reshape(len(dims), -1).astype(np.float64)   # [d, P]
    phase = np.zeros((idx.shape[1], idx.shape[1]))
    for i, n in enumerate(dims):
        phase += np.outer(idx[i], idx[i]) / n
    return np.exp(sign * 2j * np.pi * phase)


def naive_dft(x, sign=-1):
    """sign=-1: forward; sign=+1: unnormalised inverse."""
    x = np.asarray(x)
    return (dft_matrix(x.shape, sign) @ x.reshape(-1)).reshape(x.shape)
