"""Block-Jacobi ILU(0) preconditioner — TEST INFRASTRUCTURE (oracle side).

Only ``tests/`` may import this module.  It shares no code with the GPU
library.

The paper's solver study (§5.3, the tables of iteration counts and times on
the 128^3 mesh) pairs GMRES and BiCGStab with a block Jacobi preconditioner
whose blocks are factored by incomplete LU without fill, ILU(0); there the
blocks are the rows owned by each MPI process.  Here the blocks are runs of
``block_rows`` consecutive unknowns of the system's own order (free nodes by
node index, then fracture faces), and the preconditioner is stated by its
definition:

* the block D_b = A[I_b, I_b], I_b = [b B, min(n, (b + 1) B)); couplings
  between blocks are dropped;
* ILU(0) of D_b: L unit lower triangular and U upper triangular, with the
  sparsity of the strictly lower and the upper part of D_b (every stored
  entry counts, also one whose value is zero), such that (L U)_ij = a_ij at
  every stored position (i, j) of D_b.  Gaussian elimination row by row in
  the natural order (the "IKJ" ordering of the loops, as in Saad's
  *Iterative Methods for Sparse Linear Systems*) that updates only stored
  positions produces exactly these factors;
* z = M^-1 r with M = blockdiag(L_b U_b): forward then backward substitution
  in each block.

Plain Python loops over dictionaries: meant for small systems.
"""
from __future__ import annotations

import numpy as np


def bj_ilu0(A, block_rows):
    """Factors of block-Jacobi ILU(0) of the CSR matrix A.

    Returns a list of rows; row i is a dict {column: value} over the stored
    positions of A in i's block: columns < i hold L (unit diagonal implied),
    the others U."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    n = A.shape[0]
    B = int(block_rows)
    if B < 1:
        raise ValueError("block_rows must be positive")
    rows = []
    for i in range(n):
        b0 = (i // B) * B
        lo, hi = A.indptr[i], A.indptr[i + 1]
        d = {}
        for c, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            if b0 <= c < b0 + B:
                d[int(c)] = d.get(int(c), 0.0) + float(v)
        if i not in d:
            raise ValueError(f"row {i} has no stored diagonal")
        rows.append(d)
    # row by row: subtract multiples of the already final rows k < i, in
    # increasing k, at the positions row i stores (no fill)
    for i in range(n):
        ri = rows[i]
        for k in sorted(c for c in ri if c < i):
            rk = rows[k]
            lik = ri[k] / rk[k]
            ri[k] = lik
            for j, ukj in rk.items():
                if j > k and j in ri:
                    ri[j] -= lik * ukj
    return rows


def bj_ilu0_apply(rows, r):
    """z = (L U)^-1 r block by block (the blocks are independent: L and U
    hold no entry across a block boundary)."""
    n = len(rows)
    r = np.asarray(r, float)
    y = np.zeros(n)
    for i in range(n):
        s = r[i]
        for c, v in rows[i].items():
            if c < i:
                s -= v * y[c]
        y[i] = s
    z = np.zeros(n)
    for i in range(n - 1, -1, -1):
        s = y[i]
        for c, v in rows[i].items():
            if c > i:
                s -= v * z[c]
        z[i] = s / rows[i][i]
    return z


def to_dense(rows):
    """(L, U) as dense arrays (L with its unit diagonal)."""
    n = len(rows)
    L = np.eye(n)
    U = np.zeros((n, n))
    for i, d in enumerate(rows):
        for c, v in d.items():
            if c < i:
                L[i, c] = v
            else:
                U[i, c] = v
    return L, U
