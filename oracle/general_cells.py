"""VAG on general cells (tetrahedra, prisms, hexahedra) — TEST INFRASTRUCTURE (oracle side).

Only ``tests/`` may import this module; it shares no code with the GPU library.

The scheme of §3.1 is stated for generalised polyhedral cells; the paper's
experiments use hexahedra (§5.1-§5.3), tetrahedra (§5.4) and prisms (§5.5).
This module computes the same discrete solution as ``vag_oracle.c`` for any
mix of these cells, in plain numpy (small meshes), following the same steps:

* cell centre x_K = mean of its nodes, face centre x_sigma = mean of the
  face's nodes (beta = 1 / |V_sigma|); the sub-tetrahedra (x_K, x_sigma, s_e,
  s_e+1) over the cyclic edges of every face (reading C1-C3);
* P1 stiffness of Lambda_K / mu on the sub-tetrahedra over {K, nodes, face
  centres}; the centres of non-fracture faces are replaced by beta-weighted
  node values, the fracture faces stay unknowns; a_{K,nu}^{nu'} is the block
  over {nodes, fracture faces} (eq VAGFluxMatrix);
* on a fracture face, P1 on the triangles (x_sigma, s_e, s_e+1) with
  d_f Lambda_f / mu (eq VAGFluxFracture);
* the cell unknowns eliminated (eq eqschur), a direct sparse solve for the
  nodes and fracture faces, the cell values by eq eqschurcell, the fluxes;
* porous volumes with alpha_{K,s} = 1 / (2 |V_K|) and alpha_{sigma,s} =
  1 / (2 |V_sigma|) (reading C7: 1/16 and 1/8 on hexahedra and quadrangles);
* the CFL bound and the explicit upwind steps of §3.2.2;
* Peaceman wells on fracture faces (§5.5): a well k perforating face sigma
  brings the inflow Q_k = WI_k (p_w,k - u_sigma) + q_k into sigma's
  conservation equation; in transport a producer (Q_k < 0) takes c_sigma |Q_k|
  out of sigma and counts in its outflow, an injector brings c_inj,k Q_k.

Cells are given as tuples of node indices in VTK order: 4 (tetrahedron:
base triangle, apex), 6 (prism: bottom triangle, top triangle above it) or
8 (hexahedron).  Fracture faces are triangles or quadrangles, nodes in cyclic
order.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# local faces of each cell type, cyclic and ordered so that the
# sub-tetrahedra (x_K, x_sigma, s_e, s_e+1) of a valid cell have positive volume
FACES = {
    8: [(0, 4, 7, 3), (1, 2, 6, 5), (0, 1, 5, 4), (3, 7, 6, 2), (0, 3, 2, 1), (4, 5, 6, 7)],
    6: [(0, 2, 1), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (0, 3, 5, 2)],
    4: [(0, 2, 1), (0, 1, 3), (1, 2, 3), (0, 3, 2)],
}


class Mesh:
    """A mesh of general cells with fracture faces and boundary data."""

    def __init__(self, xyz, cells, perm, poro, frac_faces=(), frac_width=(), frac_perm=(), frac_poro=(),
                 dirichlet=None, p_bar=None, c_bar=None, mu=1.0, wells=None):
        self.xyz = np.asarray(xyz, float)
        self.cells = [tuple(int(v) for v in c) for c in cells]
        self.perm = np.asarray(perm, float).reshape(-1, 6)
        self.poro = np.asarray(poro, float)
        self.frac = [tuple(int(v) for v in f) for f in frac_faces]
        self.frac_width = np.asarray(frac_width, float)
        self.frac_perm = np.asarray(frac_perm, float)
        self.frac_poro = np.asarray(frac_poro, float)
        nn = len(self.xyz)
        self.dirichlet = np.zeros(nn, np.uint8) if dirichlet is None else np.asarray(dirichlet, np.uint8)
        self.p_bar = np.zeros(nn) if p_bar is None else np.asarray(p_bar, float)
        self.c_bar = np.zeros(nn) if c_bar is None else np.asarray(c_bar, float)
        self.mu = float(mu)
        w = wells or {}
        self.well_face = np.asarray(w.get("face", []), np.int64)
        self.well_wi, self.well_pw, self.well_q, self.well_cinj = (
            np.asarray(w.get(k, []), float) for k in ("wi", "pw", "q", "cinj"))
        if len(set(self.well_face.tolist())) != len(self.well_face) or np.any(self.well_face < 0) or \
                np.any(self.well_face >= len(self.frac)):
            raise ValueError("a well must perforate a distinct fracture face")

    @classmethod
    def from_problem(cls, p):
        """The hexahedral problems of the synthetic generators."""
        return cls(p.xyz, p.hex8, p.perm, p.poro, np.asarray(p.frac_nodes).reshape(-1, 4), p.frac_width,
                   p.frac_perm, p.frac_poro, p.dirichlet, p.p_bar, p.c_bar, p.mu, getattr(p, "wells", None))


def _tensor(p6):
    xx, yy, zz, xy, xz, yz = p6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def tet_gradients(p0, p1, p2, p3):
    """Gradients of the barycentric coordinates (4 x 3) and signed volume."""
    J = np.column_stack([p1 - p0, p2 - p0, p3 - p0])
    det = np.linalg.det(J)
    G = np.linalg.inv(J)          # row i: gradient of lambda_{i+1}
    g = np.vstack([-G.sum(axis=0), G])
    return g, det / 6.0


def tri_gradients(p0, p1, p2):
    """In-plane gradients of the barycentric coordinates of a triangle in 3-D
    (3 x 3) and its area: grad lambda_i = n x (p_{i+2} - p_{i+1}) / |n|^2."""
    P = (p0, p1, p2)
    n = np.cross(p1 - p0, p2 - p0)
    nn = n @ n
    g = np.array([np.cross(n, P[(i + 2) % 3] - P[(i + 1) % 3]) / nn for i in range(3)])
    return g, 0.5 * np.sqrt(nn)


def _face_key(nodes):
    return tuple(sorted(nodes))


def topology(m):
    """cell_frac[K][f] = fracture index of local face f (-1 if none) and the
    cells of each fracture face (ascending, -1 for a missing second cell)."""
    fmap = {_face_key(f): i for i, f in enumerate(m.frac)}
    if len(fmap) != len(m.frac):
        raise ValueError("a fracture face is listed twice")
    cell_frac = []
    frac_cells = [[] for _ in m.frac]
    for K, c in enumerate(m.cells):
        row = []
        for lf in FACES[len(c)]:
            i = fmap.get(_face_key([c[v] for v in lf]), -1)
            row.append(i)
            if i >= 0:
                frac_cells[i].append(K)
        cell_frac.append(row)
    for i, cs in enumerate(frac_cells):
        if not cs:
            raise ValueError(f"fracture face {i} is not a face of the mesh")
    return cell_frac, [sorted(cs) + [-1] * (2 - len(cs)) for cs in frac_cells]


def cell_matrix(m, K, cell_frac_row=None):
    """a_{K,nu}^{nu'} over [cell nodes (VTK order), fracture faces of K (by
    local face)] and the cell volume; raises on a non-positive sub-tetrahedron."""
    c = m.cells[K]
    nv = len(c)
    faces = FACES[nv]
    X = m.xyz[list(c)]
    xK = X.mean(axis=0)
    L = _tensor(m.perm[K]) / m.mu
    nF = len(faces)
    S = np.zeros((1 + nv + nF, 1 + nv + nF))
    vol = 0.0
    for f, lf in enumerate(faces):
        xs = X[list(lf)].mean(axis=0)
        for e in range(len(lf)):
            s1, s2 = lf[e], lf[(e + 1) % len(lf)]
            g, v = tet_gradients(xK, xs, X[s1], X[s2])
            if not v > 0:
                raise ValueError(f"cell {K}: non-positive sub-tetrahedron")
            vol += v
            ids = [0, 1 + nv + f, 1 + s1, 1 + s2]
            S[np.ix_(ids, ids)] += v * (g @ L @ g.T)
    fr = [f for f in range(nF) if cell_frac_row is not None and cell_frac_row[f] >= 0]
    nr = 1 + nv + len(fr)
    Q = np.zeros((1 + nv + nF, nr))
    Q[0, 0] = 1.0
    for s in range(nv):
        Q[1 + s, 1 + s] = 1.0
    for f, lf in enumerate(faces):
        if f in fr:
            Q[1 + nv + f, 1 + nv + fr.index(f)] = 1.0
        else:
            for s in lf:
                Q[1 + nv + f, 1 + s] += 1.0 / len(lf)
    R = Q.T @ S @ Q
    return R[1:, 1:], vol


def frac_matrix(m, f):
    """(1 + k) x (1 + k) matrix over (sigma, its k nodes) and the face area."""
    nodes = m.frac[f]
    X = m.xyz[list(nodes)]
    xs = X.mean(axis=0)
    k = len(nodes)
    A = np.zeros((1 + k, 1 + k))
    area = 0.0
    kap = m.frac_width[f] * m.frac_perm[f] / m.mu
    for e in range(k):
        i1, i2 = e, (e + 1) % k
        g, a = tri_gradients(xs, X[i1], X[i2])
        ids = [0, 1 + i1, 1 + i2]
        A[np.ix_(ids, ids)] += kap * a * (g @ g.T)
        area += a
    return A, area


def _local_unknowns(m, K, cell_frac, node_unk, nfree):
    c = m.cells[K]
    unk = [node_unk[s] for s in c] + [nfree + i for i in cell_frac[K] if i >= 0]
    ids = list(c) + [-1] * sum(1 for i in cell_frac[K] if i >= 0)
    return unk, ids


def system(m):
    """The cell-eliminated system over (free nodes, fracture faces): A (CSR), b
    and the local data kept for recovery."""
    cell_frac, frac_cells = topology(m)
    nn, nf = len(m.xyz), len(m.frac)
    node_unk = np.full(nn, -1)
    free = np.where(m.dirichlet == 0)[0]
    node_unk[free] = np.arange(len(free))
    nfree = len(free)
    n = nfree + nf
    rows, cols, vals = [], [], []
    b = np.zeros(n)
    local = []
    for K in range(len(m.cells)):
        a, vol = cell_matrix(m, K, cell_frac[K])
        local.append((a, vol))
        r = a.sum(axis=1)
        AKK = r.sum()
        M = a - np.outer(r, r) / AKK
        unk, ids = _local_unknowns(m, K, cell_frac, node_unk, nfree)
        for i, ui in enumerate(unk):
            if ui < 0:
                continue
            for j, uj in enumerate(unk):
                if uj >= 0:
                    rows.append(ui)
                    cols.append(uj)
                    vals.append(M[i, j])
                else:
                    b[ui] -= M[i, j] * m.p_bar[ids[j]]
    fmat = []
    for f in range(nf):
        A5, area = frac_matrix(m, f)
        fmat.append((A5, area))
        unk = [nfree + f] + [node_unk[s] for s in m.frac[f]]
        ids = [-1] + list(m.frac[f])
        for i, ui in enumerate(unk):
            if ui < 0:
                continue
            for j, uj in enumerate(unk):
                if uj >= 0:
                    rows.append(ui)
                    cols.append(uj)
                    vals.append(A5[i, j])
                else:
                    b[ui] -= A5[i, j] * m.p_bar[ids[j]]
    for k, f in enumerate(m.well_face):  # Q_k = WI (p_w - u_sigma) + q enters sigma's row
        rows.append(nfree + f)
        cols.append(nfree + f)
        vals.append(m.well_wi[k])
        b[nfree + f] += m.well_wi[k] * m.well_pw[k] + m.well_q[k]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sum_duplicates()
    return A, b, dict(cell_frac=cell_frac, frac_cells=frac_cells, node_unk=node_unk, nfree=nfree,
                      local=local, fmat=fmat)


def solve_darcy(m):
    """Pressures (nodes, cells, fracture faces) and fluxes: F_cell[K] lists
    F_{K,s} per cell node then F_{K,sigma} per fracture face of K; F_frac[f]
    lists F_{sigma,s} per face node; well_rate[k] = Q_k."""
    A, b, d = system(m)
    x = spla.spsolve(A.tocsc(), b) if A.shape[0] else np.zeros(0)
    nn, nf = len(m.xyz), len(m.frac)
    u_node = m.p_bar.copy()
    free = d["node_unk"] >= 0
    u_node[free] = x[d["node_unk"][free]]
    u_frac = x[d["nfree"]:]
    u_cell = np.zeros(len(m.cells))
    F_cell = []
    for K, c in enumerate(m.cells):
        a, _ = d["local"][K]
        u = np.concatenate([u_node[list(c)], [u_frac[i] for i in d["cell_frac"][K] if i >= 0]])
        r = a.sum(axis=1)
        uK = r @ u / r.sum()
        u_cell[K] = uK
        F_cell.append(a @ (uK - u))
    F_frac = []
    for f in range(nf):
        A5, _ = d["fmat"][f]
        us = u_node[list(m.frac[f])]
        F_frac.append(A5[1:, 1:] @ (u_frac[f] - us))
    well_rate = m.well_wi * (m.well_pw - u_frac[m.well_face]) + m.well_q
    return dict(u_node=u_node, u_cell=u_cell, u_frac=u_frac, F_cell=F_cell, F_frac=F_frac, well_rate=well_rate,
                A=A, b=b, x=x,
                cell_frac=d["cell_frac"], frac_cells=d["frac_cells"], local=d["local"], fmat=d["fmat"])


def porous_volumes(m, sol, alpha_rule=0):
    """phi_K, phi_sigma, phi_s (0 at Dirichlet nodes), §3.2.1 with
    alpha_{K,s} = 1/(2|V_K|), alpha_{sigma,s} = 1/(2|V_sigma|).  alpha_rule 1:
    a node takes a share only from the adjacent cells (fracture faces at a
    fracture node) of largest permeability, a cell's permeability being the
    trace of its tensor over 3."""
    nn = len(m.xyz)
    frac_node = np.zeros(nn, bool)
    for f in m.frac:
        frac_node[list(f)] = True
    kcell = [(L[0] + L[1] + L[2]) / 3.0 for L in m.perm]
    pmax = np.full(nn, -1.0)
    for K, c in enumerate(m.cells):
        for s in c:
            if not frac_node[s]:
                pmax[s] = max(pmax[s], kcell[K])
    for f, nodes in enumerate(m.frac):
        for s in nodes:
            pmax[s] = max(pmax[s], m.frac_perm[f])
    phi_node = np.zeros(nn)
    phi_cell = np.zeros(len(m.cells))
    for K, c in enumerate(m.cells):
        pore = sol["local"][K][1] * m.poro[K]
        alpha = 1.0 / (2 * len(c))
        taken = 0.0
        for s in c:
            if m.dirichlet[s] or frac_node[s]:
                continue
            if alpha_rule == 1 and kcell[K] < pmax[s]:
                continue
            taken += alpha
            phi_node[s] += alpha * pore
        phi_cell[K] = (1.0 - taken) * pore
    phi_frac = np.zeros(len(m.frac))
    for f, nodes in enumerate(m.frac):
        pore = m.frac_width[f] * sol["fmat"][f][1] * m.frac_poro[f]
        alpha = 1.0 / (2 * len(nodes))
        taken = 0.0
        for s in nodes:
            if m.dirichlet[s]:
                continue
            if alpha_rule == 1 and m.frac_perm[f] < pmax[s]:
                continue
            taken += alpha
            phi_node[s] += alpha * pore
        phi_frac[f] = (1.0 - taken) * pore
    return dict(phi_cell=phi_cell, phi_frac=phi_frac, phi_node=phi_node)


def _edges(m, sol):
    """Every flux as (upstream-if-positive CV, downstream-if-positive CV, F):
    control volumes are cells [0, nc), faces [nc, nc + nf), nodes after."""
    nc, nf = len(m.cells), len(m.frac)
    out = []
    for K, c in enumerate(m.cells):
        F = sol["F_cell"][K]
        for i, s in enumerate(c):
            out.append((K, nc + nf + s, F[i]))
        j = len(c)
        for i in sol["cell_frac"][K]:
            if i >= 0:
                out.append((K, nc + i, F[j]))
                j += 1
    for f, nodes in enumerate(m.frac):
        for i, s in enumerate(nodes):
            out.append((nc + f, nc + nf + s, sol["F_frac"][f][i]))
    return out


def cfl_dt(m, sol, phi, cfl):
    """cfl x min over control volumes of porous volume / outgoing flux (the
    Dirichlet nodes excluded); a producing well's |Q_k| counts as outflow of
    its face."""
    nc, nf, nn = len(m.cells), len(m.frac), len(m.xyz)
    out = np.zeros(nc + nf + nn)
    for i, j, F in _edges(m, sol):
        if F > 0:
            out[i] += F
        else:
            out[j] -= F
    for f, Q in zip(m.well_face, _well_rates(m, sol)):
        out[nc + f] += max(-Q, 0.0)
    vol = np.concatenate([phi["phi_cell"], phi["phi_frac"], phi["phi_node"]])
    ok = out > 0
    ok[nc + nf:] &= m.dirichlet == 0
    return cfl * float(np.min(vol[ok] / out[ok]))


def _well_rates(m, sol):
    Q = sol.get("well_rate")
    if len(m.well_face) and Q is None:
        raise ValueError("the mesh has wells: the fluxes need their well_rate")
    return np.zeros(0) if Q is None else np.asarray(Q, float)


def transport(m, sol, phi, dt, n_steps):
    """Explicit upwind steps from c = 0 (Dirichlet nodes at c_bar); wells as
    sources c_inj Q^+ and sinks c_sigma Q^- of their faces."""
    nc, nf, nn = len(m.cells), len(m.frac), len(m.xyz)
    c = np.zeros(nc + nf + nn)
    dn = np.where(m.dirichlet == 1)[0]
    c[nc + nf + dn] = m.c_bar[dn]
    vol = np.concatenate([phi["phi_cell"], phi["phi_frac"], phi["phi_node"]])
    edges = _edges(m, sol)
    wrate = _well_rates(m, sol)
    for _ in range(n_steps):
        s = np.zeros_like(c)
        for i, j, F in edges:
            H = c[i] * max(F, 0.0) + c[j] * min(F, 0.0)
            s[i] += H
            s[j] -= H
        for k, f in enumerate(m.well_face):
            Q = wrate[k]
            s[nc + f] += c[nc + f] * max(-Q, 0.0) - m.well_cinj[k] * max(Q, 0.0)
        upd = np.ones(len(c), bool)
        upd[nc + nf + dn] = False
        c[upd] -= dt / vol[upd] * s[upd]
    return dict(c_cell=c[:nc], c_frac=c[nc:nc + nf], c_node=c[nc + nf:])
