"""Pins for the Hermitian data arrangement (Section 2 rules a-e, Lemma 1,
eq. (3), Remark 2, the one-FFT and recursive algorithms of Section 3, and the
appendix construction of the half-set).  CPU only."""
import itertools
import os

import numpy as np
import pytest

from oracle import grf

HERE = os.path.dirname(os.path.abspath(__file__))
GRIDS = [(2,), (4,), (6,), (10,), (2, 2), (4, 4), (4, 6), (6, 4), (8, 8), (2, 4, 4), (4, 2, 6), (6, 4, 2)]


def neg(k, dims):
    return tuple((-a) % n for a, n in zip(k, dims))


def all_k(dims):
    return list(itertools.product(*[range(n) for n in dims]))


def is_valid_half_set(S, dims):
    """Exactly one of {k, -k} for every k; self-conjugate points included."""
    S = set(S)
    for k in all_k(dims):
        nk = neg(k, dims)
        if nk == k:
            if k not in S:
                return False
        elif (k in S) == (nk in S):
            return False
    return True


def full_xi_map(dims):
    """The linear map z -> full-spectrum xi as a P x P complex matrix."""
    P = int(np.prod(dims))
    M = np.zeros((P, P), dtype=complex)
    for i in range(P):
        z = np.zeros(P)
        z[i] = 1.0
        M[:, i] = grf.hermitian_extend(grf.hermitian_noise(z.reshape(dims)), dims).reshape(-1)
    return M


def test_fig1_self_conjugate_points_and_pair():
    dims = (4, 4)
    sc, pairs = set(), []
    with open(os.path.join(HERE, "golden", "fig1_grid4x4.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "selfconj":
                sc.add((int(t[1]), int(t[2])))
            else:
                pairs.append(((int(t[1]), int(t[2])), (int(t[3]), int(t[4]))))
    assert {k for k in all_k(dims) if neg(k, dims) == k} == sc
    rng = np.random.default_rng(0)
    full = grf.hermitian_extend(grf.hermitian_noise(rng.standard_normal(dims)), dims)
    for k in sc:
        assert full[k].imag == 0.0
    for a, b in pairs:
        assert neg(a, dims) == b
        assert full[a] == np.conj(full[b])


@pytest.mark.parametrize("dims", GRIDS)
def test_discrete_lemma1_law(dims):
    """E xi_k conj(xi_l) = delta_{k,l},  E xi_k xi_l = delta_{k,-l}  (the
    discrete form of the covariances of FW in Section 2 and Lemma 1), exactly,
    for z ~ N(0, I): the map z -> xi is M with M M^H = I and M M^T = J."""
    P = int(np.prod(dims))
    M = full_xi_map(dims)
    J = np.zeros((P, P))
    for i, k in enumerate(all_k(dims)):
        J[i, np.ravel_multi_index(neg(k, dims), dims)] = 1
    np.testing.assert_allclose(M @ M.conj().T, np.eye(P), atol=1e-15)
    np.testing.assert_allclose(M @ M.T, J, atol=1e-15)


@pytest.mark.parametrize("dims", GRIDS)
def test_hermitian_bitwise(dims):
    rng = np.random.default_rng(1)
    full = grf.hermitian_extend(grf.hermitian_noise(rng.standard_normal(dims)), dims)
    for k in all_k(dims):
        assert full[k] == np.conj(full[neg(k, dims)])


def our_independent_set(dims):
    """Entries of the half-spectrum that carry fresh normals in our rule."""
    m = dims[-1] // 2
    lead = dims[:-1]
    negrow = grf.neg_row_index(dims)
    S = []
    for r, kl in enumerate(itertools.product(*[range(n) for n in lead]) if lead else [()]):
        for kd in range(1, m):
            S.append(kl + (kd,))
        if r <= negrow[r]:
            S.append(kl + (0,))
            S.append(kl + (m,))
    return S


def paper_d2_half_set(dims):
    """The explicit d = 2 half-set of Section 2 (first axis halved)."""
    n1, n2 = dims
    m1, m2 = n1 // 2, n2 // 2
    S = [(a, b) for a in range(0, m1 + 1) for b in range(0, m2 + 1)]
    S += [(a, b) for a in range(1, m1) for b in range(m2 + 1, 2 * m2)]
    return S


def appendix_half_set(dims):
    """The appendix construction L = L_0 + L_1 + ... + L_d.  The second
    coordinate rule is read for i = 2..n (for i = 1 it would contradict the
    first rule)."""
    d = len(dims)
    M = [n // 2 for n in dims]
    S = [k for k in all_k(dims) if all(k[i] in (0, M[i]) for i in range(d))]
    for n in range(1, d + 1):
        for J in itertools.combinations(range(d), n):
            rest = [i for i in range(d) if i not in J]
            ranges = [None] * d
            ranges[J[0]] = list(range(1, M[J[0]]))
            for j in J[1:]:
                ranges[j] = [a for a in range(1, dims[j]) if a != M[j]]
            for i in rest:
                ranges[i] = [0, M[i]]
            S += list(itertools.product(*ranges))
    return S


def paper_recursive_draws(dims):
    """The recursive algorithm of Section 3 (create_random_field/set_array),
    with the IF/ELSE after the loop and the loop bound N_i - 1.  Returns the
    number of R() draws and the set of entries that received a value (directly
    or by conjugation)."""
    d = len(dims)
    M = [n // 2 for n in dims]
    draws = [0]
    setk = {}

    def assign(k, kind):
        assert k not in setk, f"entry {k} set twice"
        setk[k] = kind

    def set_array(j, tail):
        lead = [range(dims[i]) for i in range(j - 1)]
        for kk in itertools.product(*lead, range(1, M[j - 1])):
            k = tuple(kk) + tuple(tail)
            draws[0] += 2
            assign(k, "rep")
            assign(neg(k, dims), "mirror")
        if j == 1:
            for a in (0, M[0]):
                draws[0] += 1
                assign((a,) + tuple(tail), "real")
        else:
            set_array(j - 1, (0,) + tuple(tail))
            set_array(j - 1, (M[j - 1],) + tuple(tail))

    set_array(d, ())
    return draws[0], setk


@pytest.mark.parametrize("dims", GRIDS)
def test_half_sets_agree(dims):
    ours = our_independent_set(dims)
    assert is_valid_half_set(ours, dims)
    assert len(ours) == len(set(ours))
    app = appendix_half_set(dims)
    assert len(app) == len(set(app))
    assert is_valid_half_set(app, dims)
    assert len(app) == len(ours)
    if len(dims) == 2:
        pd2 = paper_d2_half_set(dims)
        assert is_valid_half_set(pd2, dims)
        assert len(pd2) == len(ours) == dims[0] * dims[1] // 2 + 2


@pytest.mark.parametrize("dims", GRIDS)
def test_recursive_algorithm_draws_exactly_P(dims):
    P = int(np.prod(dims))
    ndraw, setk = paper_recursive_draws(dims)
    assert ndraw == P
    assert set(setk) == set(all_k(dims))
    # our map also consumes exactly P normals: every slot of z is read
    M = full_xi_map(dims)
    assert np.all(np.abs(M).sum(axis=0) > 0)
    assert ndraw == M.shape[1]


def test_draw_count_of_simple_enumeration():
    """Remark 2 / the one-FFT algorithm's loop k_d = 0..N_d/2 draws
    2 N_1..N_{d-1} (N_d/2 + 1) - 2^d numbers: the surplus over P lives on the
    two boundary hyperplanes only."""
    for dims in [(8, 8), (4, 6, 10), (16,)]:
        lead = int(np.prod(dims[:-1])) if len(dims) > 1 else 1
        m = dims[-1] // 2
        selfc = 2 ** len(dims)
        simple = 2 * lead * (m + 1) - selfc
        P = int(np.prod(dims))
        assert simple - P == 2 * lead - selfc
