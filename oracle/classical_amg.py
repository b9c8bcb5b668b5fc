"""Classical (Ruge-Stueben type) AMG components — TEST INFRASTRUCTURE (oracle side).

Only ``tests/`` may import this module; it shares no code with the GPU library.

The paper's solver study (§5.3) runs BoomerAMG, a classical algebraic
multigrid, beside aggregation AMG and block Jacobi ILU(0).  The parts of a
classical hierarchy that a coarse/fine splitting determines uniquely are
stated here by their textbook definitions (Ruge and Stueben 1987; Stueben,
"A review of algebraic multigrid", 2001):

* strength: j strongly influences i when -a_ij >= theta * max_{k != i} (-a_ik)
  and -a_ij > 0 (positive couplings are never strong);
* direct interpolation for a fine point i with strong coarse neighbours C_i:
  e_i = sum_{j in C_i} w_ij e_j with
  w_ij = -alpha_i a_ij / a~_ii,
  alpha_i = (sum_{k != i} a_ik^-) / (sum_{j in C_i} a_ij^-),
  a~_ii = a_ii + sum_{k != i} a_ik^+   (x^- = min(x, 0), x^+ = max(x, 0));
  a fine point without strong coarse neighbours gets an empty row; a coarse
  point interpolates from itself with weight 1;
* the coarse operator is the Galerkin product P^T A P.

The splitting itself depends on the tie-breaking of the parallel independent
set and has many valid answers; ``pmis_valid`` states what every answer of
the PMIS rule (De Sterck, Yang and Heys 2006) satisfies.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def strength(A, theta):
    """Boolean CSR matrix S (same pattern as A, diagonal excluded): S_ij = 1
    when j strongly influences i."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rows, cols = [], []
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        neg = [-v for c, v in zip(A.indices[lo:hi], A.data[lo:hi]) if c != i]
        m = max(neg) if neg else 0.0
        for c, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            if c != i and -v > 0 and -v >= theta * m:
                rows.append(i)
                cols.append(int(c))
    return sp.csr_matrix((np.ones(len(rows), bool), (rows, cols)), shape=(n, n))


def direct_interpolation(A, S, is_coarse):
    """P (n x nc) of direct interpolation for the splitting is_coarse; coarse
    points are numbered in increasing fine index."""
    A = sp.csr_matrix(A)
    S = sp.csr_matrix(S)
    n = A.shape[0]
    is_coarse = np.asarray(is_coarse, bool)
    cidx = np.cumsum(is_coarse) - 1
    nc = int(is_coarse.sum())
    rows, cols, vals = [], [], []
    for i in range(n):
        if is_coarse[i]:
            rows.append(i)
            cols.append(int(cidx[i]))
            vals.append(1.0)
            continue
        lo, hi = A.indptr[i], A.indptr[i + 1]
        strong = set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist())
        aii = 0.0
        neg_all = pos_all = neg_c = 0.0
        ci = []
        for c, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            c = int(c)
            if c == i:
                aii += v
                continue
            neg_all += min(v, 0.0)
            pos_all += max(v, 0.0)
            if c in strong and is_coarse[c]:
                ci.append((c, v))
                neg_c += min(v, 0.0)
        if not ci:
            continue
        alpha = neg_all / neg_c
        diag = aii + pos_all
        for c, v in ci:
            rows.append(i)
            cols.append(int(cidx[c]))
            vals.append(-alpha * v / diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def galerkin(A, P):
    """P^T A P."""
    P = sp.csr_matrix(P)
    return sp.csr_matrix(P.T @ sp.csr_matrix(A) @ P)


def pmis_valid(S, is_coarse):
    """(independent, covered, lonely) of a splitting under the PMIS rule.

    PMIS picks, round after round, undecided points whose measure beats that
    of every undecided strong neighbour, then makes fine every undecided
    point that strongly depends on a new coarse point; points that influence
    no one start fine.  Every splitting it can produce therefore has:
    independent: no two coarse points depend strongly on each other (the
    first chosen would have made the other fine; two points chosen in one
    round are not neighbours); one-way dependence between coarse points
    chosen in different rounds is allowed;
    covered: every fine point that strongly influences some point depends
    strongly on a coarse point.
    lonely counts the fine points with strong dependencies but no coarse one
    among them (they receive an empty interpolation row)."""
    S = sp.csr_matrix(S).astype(bool)
    M = S.multiply(S.T).tocsr()  # mutual strong dependence
    lam = np.asarray(S.sum(axis=0)).ravel()  # points that depend on each point
    is_coarse = np.asarray(is_coarse, bool)
    independent = covered = True
    lonely = 0
    for i in range(S.shape[0]):
        mut = M.indices[M.indptr[i]:M.indptr[i + 1]]
        dep = S.indices[S.indptr[i]:S.indptr[i + 1]]
        if is_coarse[i] and is_coarse[mut[mut != i]].any():
            independent = False
        if not is_coarse[i]:
            has_c = bool(is_coarse[dep].any())
            if lam[i] > 0 and not has_c:
                covered = False
            if len(dep) and not has_c:
                lonely += 1
    return independent, covered, lonely
