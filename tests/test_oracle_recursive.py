"""Pins of the recursive algorithm of Section 3 (oracle/recursive.py):
* its draw order equals the order derived by hand from the listing
  (tests/golden/alg3_draw_order.txt);
* it draws exactly P normals, sets every entry, and A is Hermitian;
* its law: the output is linear in the stream, and the covariance summed over
  the unit streams equals the exact covariance of the periodic algorithms
  (the circulant of the filter, computed by the periodic oracle)."""
import os

import numpy as np
import pytest

from oracle import grf, noise, recursive, spectra

HERE = os.path.dirname(__file__)


def _golden():
    cases, cur = [], None
    for line in open(os.path.join(HERE, "golden", "alg3_draw_order.txt")):
        line = line.split("#")[0].split()
        if not line:
            continue
        if line[0] == "grid":
            cur = (tuple(int(v) for v in line[1:]), [])
            cases.append(cur)
        else:
            i = line.index("re")
            cur[1].append((tuple(int(v) for v in line[1:i]), int(line[i + 1]), int(line[i + 3])))
    return cases


@pytest.mark.parametrize("case", _golden(), ids=lambda c: str(c[0]))
def test_draw_order_matches_hand_derivation(case):
    dims, entries = case
    P = int(np.prod(dims))
    stream = np.arange(1, P + 1, dtype=np.float64)        # draw j has value j + 1
    A, n = recursive.spectrum_from_stream(stream, dims, np.ones(dims))
    assert n == P
    s = 2.0 ** -0.5
    for k, re, im in entries:
        if im < 0:
            assert A[k] == re + 1
        else:
            assert A[k] == pytest.approx(s * (re + 1) + 1j * s * (im + 1), abs=1e-15)
            km = tuple((-a) % n for a, n in zip(k, dims))
            assert A[km] == np.conj(A[k])
    # the fixture lists every directly set entry
    direct = {k for k, _, _ in entries}
    mirrors = {tuple((-a) % n for a, n in zip(k, dims)) for k, _, im in entries if im >= 0}
    assert len(direct | mirrors) == P


@pytest.mark.parametrize("dims", [(6,), (16,), (4, 6), (8, 8), (2, 4, 6), (4, 4, 4)], ids=str)
def test_exact_count_and_hermitian(dims):
    P = int(np.prod(dims))
    z = np.random.default_rng(P).normal(size=P + 5)
    A, n = recursive.spectrum_from_stream(z, dims, np.ones(dims))
    assert n == P
    assert not np.isnan(A).any()
    neg = tuple(slice(None) for _ in dims)
    Am = A[neg]
    for ax in range(len(dims)):
        Am = np.roll(np.flip(Am, axis=ax), 1, axis=ax)
    np.testing.assert_array_equal(Am, np.conj(A))
    assert np.abs(np.fft.ifftn(A).imag).max() <= 1e-15 * np.abs(A).max()


@pytest.mark.parametrize("dims,lengths", [((8,), (1.0,)), ((4, 6), (1.0, 1.5)), ((4, 4, 4), (1.0, 1.0, 2.0))], ids=str)
def test_law_is_the_periodic_covariance(dims, lengths):
    P = int(np.prod(dims))
    cols = np.empty((P, P))
    for j in range(P):
        e = np.zeros(P)
        e[j] = 1.0
        cols[:, j] = recursive.alg3_from_stream(e, dims, lengths, spectra.MATERN, 1.3, 0.4, 1.5).ravel()
    cov = cols @ cols.T
    C = grf.discrete_covariance(dims, lengths, spectra.MATERN, 1.3, 0.4, 1.5)
    idx = np.indices(dims).reshape(len(dims), -1).T
    for a in range(0, P, max(1, P // 7)):
        diff = tuple(((idx[:, i] - idx[a, i]) % dims[i]) for i in range(len(dims)))
        np.testing.assert_allclose(cov[a], C[diff], atol=1e-12 * C.max())


def test_sample_reads_the_tag3_stream_in_row_major_order():
    dims = (4, 6)
    phi = recursive.sample(dims, (1.0, 1.0), spectra.GAUSSIAN, 1.0, 0.2, seed=5, batch=2)
    for b in range(2):
        z = noise.field_noise(dims, 5 + b, 3)
        np.testing.assert_array_equal(phi[b], recursive.alg3_from_stream(z.ravel(), dims, (1.0, 1.0),
                                                                          spectra.GAUSSIAN, 1.0, 0.2))


# ---------------------------------------------------------------------------
# adjoint, pinned by central finite differences of the sampler itself

@pytest.mark.parametrize("dims", [(8,), (4, 6), (4, 4, 4)], ids=str)
def test_adjoint_finite_differences(dims):
    lengths = tuple(1.0 + 0.5 * i for i in range(len(dims)))
    z = noise.field_noise(dims, 2, 3).ravel()
    w = np.random.default_rng(1).uniform(size=dims)
    th = np.array([1.1, 0.3, 1.5])
    phi = lambda t, zz: recursive.alg3_from_stream(zz, dims, lengths, spectra.MATERN, *t)
    loss = lambda t, zz: np.sum(w * phi(t, zz) ** 2)
    g = 2 * w * phi(th, z)
    got = recursive.grad_theta(z, g, lengths, spectra.MATERN, *th)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1e-6 * th[i]
        fd = (loss(th + e, z) - loss(th - e, z)) / (2 * e[i])
        assert got[i] == pytest.approx(fd, rel=1e-6)
    gz = recursive.grad_stream(g, lengths, spectra.MATERN, *th).ravel()
    dz = np.random.default_rng(2).normal(size=z.size)
    fd = (loss(th, z + 1e-6 * dz) - loss(th, z - 1e-6 * dz)) / 2e-6
    assert np.dot(gz, dz) == pytest.approx(fd, rel=1e-7)
