"""Pins of the oracle's block-Jacobi ILU(0) against cases whose answer the
mathematics fixes: exact LU where ILU(0) creates no fill, Jacobi at block
size 1, the defining property (L U)_ij = a_ij on the pattern, and an
elimination with the loops in the other order (k outer) on tiny matrices."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ilu


def tridiag(n, seed):
    rng = np.random.default_rng(seed)
    off = -rng.uniform(0.5, 1.5, n - 1)
    d = np.abs(np.concatenate([[0], off])) + np.abs(np.concatenate([off, [0]])) + rng.uniform(0.1, 1.0, n)
    return sp.diags([off, d, off], [-1, 0, 1], format="csr")


def laplace5(nx, ny, seed):
    """5-point operator on an nx x ny grid with random positive couplings."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    A = sp.lil_matrix((n, n))
    for j in range(ny):
        for i in range(nx):
            p = i + nx * j
            for q in ([p + 1] if i + 1 < nx else []) + ([p + nx] if j + 1 < ny else []):
                w = rng.uniform(0.2, 2.0)
                A[p, q] = A[q, p] = -w
                A[p, p] += w
                A[q, q] += w
            A[p, p] += 0.05
    return A.tocsr()


def kij_ilu0(A, B):
    """ILU(0) with the elimination step k outermost, dense storage, updates
    restricted to the stored pattern of the diagonal blocks."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    M = np.zeros((n, n))
    P = np.zeros((n, n), bool)
    for i in range(n):
        for q in range(A.indptr[i], A.indptr[i + 1]):
            c = A.indices[q]
            if c // B == i // B:
                M[i, c] += A.data[q]
                P[i, c] = True
    for k in range(n):
        for i in range(k + 1, n):
            if P[i, k]:
                M[i, k] /= M[k, k]
                for j in range(k + 1, n):
                    if P[i, j] and P[k, j]:
                        M[i, j] -= M[i, k] * M[k, j]
    return np.tril(M, -1) + np.eye(n), np.triu(M)


def test_tridiagonal_is_exact_lu():
    A = tridiag(23, 1)
    r = np.random.default_rng(2).standard_normal(23)
    z = ilu.bj_ilu0_apply(ilu.bj_ilu0(A, 23), r)
    np.testing.assert_allclose(z, np.linalg.solve(A.toarray(), r), rtol=1e-12, atol=1e-12)


def test_blocks_drop_couplings():
    """Tridiagonal blocks of 4 (the last one ragged): M is the exact inverse of
    the block-diagonal part."""
    n, B = 18, 4
    A = tridiag(n, 3)
    D = A.toarray()
    for i in range(n):
        for j in range(n):
            if i // B != j // B:
                D[i, j] = 0.0
    r = np.random.default_rng(4).standard_normal(n)
    z = ilu.bj_ilu0_apply(ilu.bj_ilu0(A, B), r)
    np.testing.assert_allclose(z, np.linalg.solve(D, r), rtol=1e-12, atol=1e-12)


def test_block_size_one_is_jacobi():
    A = laplace5(5, 4, 5)
    r = np.random.default_rng(6).standard_normal(20)
    z = ilu.bj_ilu0_apply(ilu.bj_ilu0(A, 1), r)
    np.testing.assert_allclose(z, r / A.diagonal(), rtol=1e-14)


@pytest.mark.parametrize("B", [7, 11, 100])
def test_defining_property_and_kij_order(B):
    """(L U)_ij = a_ij at every stored position of the blocks, L and U inside
    the pattern, fill (L U - A) nonzero somewhere off the pattern, and the
    factors equal those of the k-outer elimination."""
    nx, ny = 6, 5
    A = laplace5(nx, ny, 7)
    n = nx * ny
    rows = ilu.bj_ilu0(A, B)
    L, U = ilu.to_dense(rows)
    Lk, Uk = kij_ilu0(A, B)
    np.testing.assert_allclose(L, Lk, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(U, Uk, rtol=1e-13, atol=1e-15)
    Ad = A.toarray()
    pat = (Ad != 0)
    blk = np.equal.outer(np.arange(n) // B, np.arange(n) // B)
    pat &= blk
    LU = L @ U
    np.testing.assert_allclose(LU[pat], Ad[pat], rtol=1e-12, atol=1e-13)
    off = (L - np.eye(n) != 0) | (U != 0)
    assert not (off & ~pat).any()
    if B >= 2 * nx:
        assert np.abs((LU - Ad)[blk & ~pat]).max() > 1e-3  # ILU(0) is not the exact LU here
    r = np.random.default_rng(8).standard_normal(n)
    z = ilu.bj_ilu0_apply(rows, r)
    np.testing.assert_allclose(LU @ z, r, rtol=1e-12, atol=1e-12)


def test_stored_zero_is_a_position():
    """An arrow matrix fills in completely under elimination; with the fill
    positions stored as explicit zeros, ILU(0) is the exact LU."""
    n = 6
    D = np.eye(n) * 4.0
    D[0, 1:] = D[1:, 0] = -0.5
    full = np.ones((n, n), bool)
    rows_i, cols_i = np.nonzero(full)
    A = sp.csr_matrix((D[rows_i, cols_i], (rows_i, cols_i)), shape=(n, n))
    assert A.nnz == n * n  # explicit zeros kept
    r = np.arange(1.0, n + 1)
    z = ilu.bj_ilu0_apply(ilu.bj_ilu0(A, n), r)
    np.testing.assert_allclose(z, np.linalg.solve(D, r), rtol=1e-13)
    # without the stored zeros the same matrix gives a different (inexact) M
    z0 = ilu.bj_ilu0_apply(ilu.bj_ilu0(sp.csr_matrix(D), n), r)
    assert np.abs(z0 - z).max() > 1e-3
