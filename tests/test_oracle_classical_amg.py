"""Pins of the oracle's classical-AMG definitions: linear interpolation and
the halved coarse Laplacian in 1-D, preserved constants on zero-row-sum
rows, hand-computed strength and weights with positive couplings."""
import numpy as np
import scipy.sparse as sp

from oracle import classical_amg as ca


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def test_1d_linear_interpolation_and_coarse_operator():
    n = 9
    A = lap1d(n)
    S = ca.strength(A, 0.25)
    assert S.nnz == 2 * (n - 1)  # every coupling is strong
    cf = np.arange(n) % 2 == 1   # coarse: 1, 3, 5, 7
    P = ca.direct_interpolation(A, S, cf).toarray()
    expect = np.zeros((n, 4))
    for c, i in enumerate([1, 3, 5, 7]):
        expect[i, c] = 1.0
        expect[i - 1, c] += 0.5
        expect[i + 1, c] += 0.5
    np.testing.assert_allclose(P, expect, rtol=0, atol=1e-15)
    Ac = ca.galerkin(A, P).toarray()
    np.testing.assert_allclose(Ac, 0.5 * lap1d(4).toarray(), rtol=0, atol=1e-15)


def test_constants_preserved_on_zero_row_sums():
    """Graph Laplacian (zero row sums, negative couplings): every fine row with
    a strong coarse neighbour interpolates constants exactly."""
    rng = np.random.default_rng(3)
    nx = ny = 7
    n = nx * ny
    A = sp.lil_matrix((n, n))
    for j in range(ny):
        for i in range(nx):
            p = i + nx * j
            for q in ([p + 1] if i + 1 < nx else []) + ([p + nx] if j + 1 < ny else []):
                w = rng.uniform(0.1, 3.0)
                A[p, q] = A[q, p] = -w
                A[p, p] += w
                A[q, q] += w
    A = A.tocsr()
    S = ca.strength(A, 0.25)
    cf = ((np.arange(n) % nx) + (np.arange(n) // nx)) % 2 == 0  # checkerboard
    P = ca.direct_interpolation(A, S, cf)
    rs = np.asarray(P.sum(axis=1)).ravel()
    nonempty = np.diff(P.indptr) > 0
    assert nonempty[~cf].sum() > 0.8 * (~cf).sum()
    np.testing.assert_allclose(rs[nonempty], 1.0, rtol=1e-14)
    ind, cov, lonely = ca.pmis_valid(S, cf)
    assert ind  # a checkerboard has no two coarse points adjacent on the 5-point graph


def test_strength_and_positive_couplings_by_hand():
    # row 0: a_01 = -2 (strong), a_02 = +0.5 (positive: never strong),
    # a_03 = -0.4 (weak: 0.4 < 0.25 * 2 is false -> 0.4 < 0.5, weak)
    A = sp.csr_matrix(np.array([[3.0, -2.0, 0.5, -0.4],
                                [-2.0, 4.0, -1.0, 0.0],
                                [0.5, -1.0, 2.0, -0.3],
                                [-0.4, 0.0, -0.3, 1.5]]))
    S = ca.strength(A, 0.25).toarray()
    assert S[0].tolist() == [False, True, False, False]
    assert S[2].tolist() == [False, True, False, True]  # max -a = 1.0, 0.3 >= 0.25
    cf = np.array([False, True, False, False])
    P = ca.direct_interpolation(A, S, cf).toarray()
    # alpha = (-2 - 0.4) / (-2); diag = 3 + 0.5; w = -alpha * (-2) / 3.5
    np.testing.assert_allclose(P[0, 0], 2.4 / 3.5, rtol=1e-15)
    np.testing.assert_allclose(P[1, 0], 1.0)
    # row 2: neighbours 1 (C, -1.0, strong), 3 (F, -0.3), 0 (+0.5)
    np.testing.assert_allclose(P[2, 0], ((1.0 + 0.3) / 1.0) * 1.0 / (2.0 + 0.5), rtol=1e-15)
    assert P[3, 0] == 0.0  # row 3 has no strong coarse neighbour (a_31 = 0)
    ind, cov, lonely = ca.pmis_valid(sp.csr_matrix(S), cf)
    # row 3 depends on 0 and 2 (both fine) and point 2 depends on it: a PMIS
    # splitting could not leave it fine without a coarse point to lean on
    assert ind and lonely == 1 and not cov
    assert ca.pmis_valid(sp.csr_matrix(S), np.array([False, True, False, True]))[:2] == (True, True)
    # 1 and 2 depend on each other: both coarse is never a PMIS result
    assert not ca.pmis_valid(sp.csr_matrix(S), np.array([False, True, True, False]))[0]
