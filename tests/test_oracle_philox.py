"""Pins for the oracle's noise contract (CPU only)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import noise, philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            w, r = int(t[0]), int(t[1])
            v = [int(x, 16) for x in t[2:]]
            rows.append((w, r, v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("row", _kat(), ids=lambda r: f"w{r[0]}")
def test_known_answer_vectors(row):
    w, r, ctr, key, out = row
    assert philox.philox_scalar(ctr, key, width=w, rounds=r) == out


def test_width64_matches_numpy_philox():
    # numpy's Philox is the 4x64-10 instance; it advances the counter before
    # it produces a block, so its n-th block is the block of counter c + n + 1.
    for key, ctr0 in [((5, 7), 0), ((0xDEADBEEF, 123456789), 2 ** 63 - 5)]:
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array([ctr0, 0, 0, 0], dtype=np.uint64))
        raw = [int(x) for x in bg.random_raw(12)]
        for n in range(3):
            c = ctr0 + n + 1
            ctr = [c & (2 ** 64 - 1), c >> 64, 0, 0]
            assert philox.philox_scalar(ctr, key, width=64) == raw[4 * n:4 * n + 4]


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2 ** 32, size=(200, 4), dtype=np.uint64)
    for seed in [0, 1, 2 ** 40 + 17, 2 ** 64 - 1]:
        k0, k1 = philox.key_of(seed)
        v = philox.philox4x32(c[:, 0], c[:, 1], c[:, 2], c[:, 3], k0, k1)
        for i in range(0, 200, 13):
            assert [int(x[i]) for x in v] == philox.philox_scalar(c[i], (k0, k1), width=32)


def test_noise_layout_is_the_contract():
    dims = (3, 10)
    seed = 41
    for tag in (0, 1):
        z = noise.field_noise(dims, seed, tag)
        k0, k1 = philox.key_of(seed)
        for row in range(3):
            for s in range(10):
                x = philox.philox_scalar([s // 4, row, tag, 0], (k0, k1))
                u = [(xx + 0.5) * 2.0 ** -32 for xx in x]
                lane = s % 4
                a, b = (u[0], u[1]) if lane < 2 else (u[2], u[3])
                r = np.sqrt(-2 * np.log(a))
                want = r * (np.cos(2 * np.pi * b) if lane % 2 == 0 else np.sin(2 * np.pi * b))
                assert z[row, s] == pytest.approx(want, rel=1e-15, abs=1e-15)


def test_batch_uses_consecutive_seeds():
    a = noise.batch_noise((4, 8), 10, 3, 1)
    for b in range(3):
        np.testing.assert_array_equal(a[b], noise.field_noise((4, 8), 10 + b, 1))


def test_normals_are_standard_normal():
    z = noise.field_noise((256, 256), 7, 1).ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    # lag-1 correlation along the slot axis (pairs share a block)
    zz = z.reshape(256, 256)
    c = np.mean(zz[:, :-1] * zz[:, 1:])
    assert abs(c) < 5 / np.sqrt(zz[:, 1:].size)


def test_uniforms_open_interval():
    u = noise.uniforms(np.array([0, 2 ** 32 - 1], dtype=np.uint64))
    assert 0 < u[0] < u[1] < 1
