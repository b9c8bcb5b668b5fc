"""CPU pins of the test-side fracture-face elimination (tests/schur_ref.py).

The reduced system must have the same solution at the kept unknowns as the
full cell-eliminated system (a textbook identity of block elimination), and
the groups must have the shapes that the geometry fixes: one face per group
on a single plane, four faces around an intersection line, twelve at a
triple point (each meeting the free nodes of its cells).
"""
import numpy as np
import scipy.sparse.linalg as spla

import oracle
import schur_ref
import synth


def _full_solution(A, b):
    return spla.spsolve(A.tocsc(), b)


def test_single_plane_groups_are_single_faces():
    p = synth.config1()
    A, b = oracle.system(p)
    n_free = int((p.dirichlet == 0).sum())
    groups = schur_ref.face_groups(A, n_free)
    assert len(groups) == p.n_frac
    assert all(len(f) == 1 and len(nodes) == 12 for f, nodes in groups)


def test_intersection_group_shapes():
    n = 8
    p = synth.cartesian_problem(n, planes=[(0, 4, 0, n, 0, n), (1, 4, 0, n, 0, n), (2, 4, 0, n, 0, n)])
    A, b = oracle.system(p)
    n_free = int((p.dirichlet == 0).sum())
    groups = schur_ref.face_groups(A, n_free)
    sizes = sorted(len(f) for f, _ in groups)
    # the 8 cells around the triple point: 12 faces, 27 nodes
    big = [g for g in groups if len(g[0]) == 12]
    assert len(big) == 1 and len(big[0][1]) == 27
    # 4 cells around each cell edge of the 3 intersection lines, except at the
    # triple point: 18 nodes, 9 free where the line meets a Dirichlet plane
    four = [g for g in groups if len(g[0]) == 4]
    assert len(four) == 3 * (n - 2)
    m = sorted(len(nodes) for _, nodes in four)
    assert m == [9, 9] + [18] * (3 * (n - 2) - 2)
    assert sizes.count(1) == 3 * n * n - 4 * len(four) - 12


def test_reduced_solution_equals_full():
    p = synth.random_problem((7, 6, 5), 3, n_patches=8)
    A, b = oracle.system(p)
    n_free = int((p.dirichlet == 0).sum())
    S, bs, kept, elim = schur_ref.eliminate(A, b, n_free)
    assert len(elim) > 0
    x = _full_solution(A, b)
    xr = np.linalg.solve(S, bs)
    assert np.linalg.norm(xr - x[kept]) <= 1e-10 * np.linalg.norm(x)
    # symmetric positive definite, as a Schur complement of an SPD matrix
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    np.linalg.cholesky(S)


def test_group_limits_keep_long_chains():
    planes = [(0, x, 2, 3, 2, 3) for x in range(1, 20)]
    p = synth.planes_problem((20, 5, 5), planes)
    A, b = oracle.system(p)
    n_free = int((p.dirichlet == 0).sum())
    groups = schur_ref.face_groups(A, n_free)
    assert len(groups) == 1 and len(groups[0][0]) == 19
    S, bs, kept, elim = schur_ref.eliminate(A, b, n_free)
    assert len(elim) == 0                      # 80 free nodes > 64
    S2, bs2, kept2, elim2 = schur_ref.eliminate(A, b, n_free, max_nodes=200)
    assert len(elim2) == 19
