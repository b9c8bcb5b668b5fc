"""Reference elimination of fracture-face groups, for tests only.

Takes the oracle's cell-eliminated system over (free nodes, fracture faces)
and eliminates groups of faces exactly with dense linear algebra, to give the
system the library assembles when it eliminates the faces.  A group is a
connected component of the face-face block's sparsity pattern (faces coupled
through a shared cell); it is eliminated when it has at most ``max_faces``
faces and its rows reach at most ``max_nodes`` free nodes, else its faces stay
unknowns.  Reduced unknown order: free nodes, then kept faces, ascending.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def face_groups(A, n_free):
    A = sp.csr_matrix(A)
    n = A.shape[0]
    Aff = A[n_free:, n_free:]
    pat = sp.csr_matrix((np.ones(Aff.nnz), Aff.indices, Aff.indptr), shape=Aff.shape)
    nc, lab = connected_components(pat, directed=False)
    groups = []
    for c in range(nc):
        faces = np.flatnonzero(lab == c)
        rows = A[n_free + faces, :n_free]
        nodes = np.unique(rows.indices)
        groups.append((faces, nodes))
    groups.sort(key=lambda g: g[0][0])
    return groups


def eliminate(A, b, n_free, max_faces=32, max_nodes=64):
    """Returns (S, bs, kept, eliminated): the reduced dense system over the
    kept unknowns and the index lists (in the full numbering)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    elim = []
    for faces, nodes in face_groups(A, n_free):
        if len(faces) <= max_faces and len(nodes) <= max_nodes:
            elim.extend((n_free + faces).tolist())
    elim = np.array(sorted(elim), dtype=np.int64)
    kept = np.setdiff1d(np.arange(n), elim)
    D = A.toarray()
    Akk = D[np.ix_(kept, kept)]
    if len(elim) == 0:
        return Akk, b[kept].copy(), kept, elim
    Ake = D[np.ix_(kept, elim)]
    Aee = D[np.ix_(elim, elim)]
    X = np.linalg.solve(Aee, np.column_stack([Ake.T, b[elim]]))
    S = Akk - Ake @ X[:, :-1]
    bs = b[kept] - Ake @ X[:, -1]
    return S, bs, kept, elim


def csr_to_dense(rp, col, val, n):
    return sp.csr_matrix((val, col, rp), shape=(n, n)).toarray()
