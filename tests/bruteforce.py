"""Brute-force Galerkin solution of the VAG Darcy problem on tiny meshes.

Independent of the oracle's cell-by-cell route: it assembles the *global* P1
stiffness on the whole tetrahedral sub-mesh T (§3.1) over every vertex (cell
centres, nodes, one centre per mesh face), adds the fracture P1 stiffness on
the fracture triangles, imposes the face-centre interpolation
v(x_sigma) = mean of the face's nodes for non-fracture faces as a linear
constraint, fixes the Dirichlet nodes and solves the dense Galerkin system
(equation varformVAG) with ``numpy.linalg.solve``.

Fluxes use the first form of equations VAGFluxMatrix / VAGFluxFracture,
F_{K,nu} = -int_K Lambda/mu grad(pi u) . grad(eta_nu), i.e. minus the row nu of
the cell-restricted reduced stiffness applied to u.
"""
from __future__ import annotations

import numpy as np

HEX_FACES = [[0, 4, 7, 3], [1, 2, 6, 5], [0, 1, 5, 4], [3, 7, 6, 2], [0, 3, 2, 1], [4, 5, 6, 7]]


def _tet_stiffness(V, L):
    J = (V[1:] - V[0]).T
    G = np.linalg.inv(J)
    g = np.vstack([-G.sum(0), G])
    vol = abs(np.linalg.det(J)) / 6.0
    return vol * g @ L @ g.T


def _tri_stiffness(V, kappa):
    # P1 on a triangle embedded in 3-D, via the local 2-D frame of its plane
    e1 = V[1] - V[0]
    e2 = V[2] - V[0]
    t1 = e1 / np.linalg.norm(e1)
    nrm = np.cross(e1, e2)
    t2 = np.cross(nrm / np.linalg.norm(nrm), t1)
    P2 = np.array([[0.0, 0.0], [e1 @ t1, e1 @ t2], [e2 @ t1, e2 @ t2]])
    J = (P2[1:] - P2[0]).T
    G = np.linalg.inv(J)
    g = np.vstack([-G.sum(0), G])
    area = abs(np.linalg.det(J)) / 2.0
    return kappa * area * g @ g.T


def solve(prob):
    xyz = prob.xyz
    hex8 = prob.hex8
    nn, nc, nf = len(xyz), len(hex8), len(prob.frac_nodes)
    # mesh faces, each once
    face_id = {}
    faces = []
    for K in range(nc):
        for lf in HEX_FACES:
            key = tuple(sorted(hex8[K, lf]))
            if key not in face_id:
                face_id[key] = len(faces)
                faces.append(hex8[K, lf])
    nF = len(faces)
    frac_of_face = {}
    for f in range(nf):
        frac_of_face[face_id[tuple(sorted(prob.frac_nodes[f]))]] = f
    # vertices: [cells | nodes | face centres]
    nv = nc + nn + nF
    S = np.zeros((nv, nv))
    cellS = []
    for K in range(nc):
        X = xyz[hex8[K]]
        xK = X.mean(0)
        p = prob.perm[K]
        L = np.array([[p[0], p[3], p[4]], [p[3], p[1], p[5]], [p[4], p[5], p[2]]]) / prob.mu
        SK = {}
        for lf in HEX_FACES:
            F = face_id[tuple(sorted(hex8[K, lf]))]
            xs = xyz[hex8[K, lf]].mean(0)
            for e in range(4):
                s1, s2 = hex8[K, lf[e]], hex8[K, lf[(e + 1) % 4]]
                V = np.array([xK, xs, xyz[s1], xyz[s2]])
                ids = [K, nc + nn + F, nc + s1, nc + s2]
                St = _tet_stiffness(V, L)
                for i in range(4):
                    for j in range(4):
                        S[ids[i], ids[j]] += St[i, j]
                        SK[(ids[i], ids[j])] = SK.get((ids[i], ids[j]), 0.0) + St[i, j]
        cellS.append(SK)
    fracS = []
    for f in range(nf):
        fn = prob.frac_nodes[f]
        F = face_id[tuple(sorted(fn))]
        xs = xyz[fn].mean(0)
        kappa = prob.frac_width[f] * prob.frac_perm[f] / prob.mu
        SF = {}
        for e in range(4):
            s1, s2 = fn[e], fn[(e + 1) % 4]
            ids = [nc + nn + F, nc + s1, nc + s2]
            St = _tri_stiffness(np.array([xs, xyz[s1], xyz[s2]]), kappa)
            for i in range(3):
                for j in range(3):
                    S[ids[i], ids[j]] += St[i, j]
                    SF[(ids[i], ids[j])] = SF.get((ids[i], ids[j]), 0.0) + St[i, j]
        fracS.append(SF)
    # reduced unknowns: [cells | nodes | fracture faces]
    nr = nc + nn + nf
    Pm = np.zeros((nv, nr))
    for i in range(nc + nn):
        Pm[i, i] = 1.0
    for F, fnodes in enumerate(faces):
        if F in frac_of_face:
            Pm[nc + nn + F, nc + nn + frac_of_face[F]] = 1.0
        else:
            for s in fnodes:
                Pm[nc + nn + F, nc + s] += 0.25
    A = Pm.T @ S @ Pm
    dir_idx = nc + np.nonzero(prob.dirichlet)[0]
    free = np.setdiff1d(np.arange(nr), dir_idx)
    u = np.zeros(nr)
    u[dir_idx] = prob.p_bar[prob.dirichlet.astype(bool)]
    rhs = -A[np.ix_(free, dir_idx)] @ u[dir_idx]
    u[free] = np.linalg.solve(A[np.ix_(free, free)], rhs)

    def restricted(Sdict):
        M = np.zeros((nv, nv))
        for (i, j), v in Sdict.items():
            M[i, j] = v
        return Pm.T @ M @ Pm

    F_cell = np.zeros((nc, 8))
    F_cell_frac = np.zeros((nf, 2))
    sides = np.zeros(nf, int)
    frac_cells = [[] for _ in range(nf)]
    for K in range(nc):
        AK = restricted(cellS[K])
        flux = -(AK @ u)
        for a in range(8):
            F_cell[K, a] = flux[nc + hex8[K, a]]
        for lf in HEX_FACES:
            F = face_id[tuple(sorted(hex8[K, lf]))]
            if F in frac_of_face:
                f = frac_of_face[F]
                frac_cells[f].append((K, flux[nc + nn + f]))
    for f in range(nf):
        for side, (K, val) in enumerate(sorted(frac_cells[f])):
            F_cell_frac[f, side] = val
        sides[f] = len(frac_cells[f])
    F_frac = np.zeros((nf, 4))
    for f in range(nf):
        AF = restricted(fracS[f])
        flux = -(AF @ u)
        for i, s in enumerate(prob.frac_nodes[f]):
            F_frac[f, i] = flux[nc + s]
    return dict(u_cell=u[:nc], u_node=u[nc:nc + nn], u_frac=u[nc + nn:], F_cell=F_cell,
                F_cell_frac=F_cell_frac, F_frac=F_frac, A_full=A, free=free)
