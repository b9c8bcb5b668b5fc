"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these tests touches the GPU.  Each pin is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
operand, a wrong volume) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import bruteforce
import oracle
import synth
from oracle import analytic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
HEXF = [[0, 4, 7, 3], [1, 2, 6, 5], [0, 1, 5, 4], [3, 7, 6, 2], [0, 3, 2, 1], [4, 5, 6, 7]]


def one_cell(X, perm6, frac_faces=()):
    """A single hexahedron with given node coordinates, optional fracture faces."""
    hex8 = np.arange(8, dtype=np.int32)[None, :]
    fn = np.array([[HEXF[f][i] for i in range(4)] for f in frac_faces], np.int32).reshape(-1, 4)
    nf = len(fn)
    return synth.Problem(
        name="cell", dims=(1, 1, 1), xyz=np.asarray(X, float), hex8=hex8, frac_nodes=fn,
        frac_width=np.full(nf, 0.01), frac_perm=np.full(nf, 1e4), frac_poro=np.ones(nf),
        perm=np.asarray(perm6, float)[None, :], poro=np.ones(1), mu=1.0,
        dirichlet=np.ones(8, np.uint8), p_bar=np.zeros(8), c_bar=np.zeros(8))


CUBE = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)


# ---------------------------------------------------------------------------
# local matrices
# ---------------------------------------------------------------------------

def test_unit_cube_closed_form():
    """Axis-aligned cube of side h, isotropic lambda, no fracture face.

    On every sub-tetrahedron T_{K,sigma,e} the cell basis eta_K vanishes on the
    face plane and is 1 at x_K, a distance h/2 away, so |grad eta_K| = 2/h and
    A_KK = int lambda |grad eta_K|^2 = 4 lambda h.  By the cube's symmetry
    (and a hand computation on one sub-tetrahedron) the node block is
    diagonal: a_{K,s}^{s'} = (lambda h / 2) delta_{s s'} (VAG is two-point on a
    cube).  Hence the row sums r_s are lambda h / 2 and sum to A_KK.
    """
    h, lam = 0.37, 2.3
    a, vol = oracle.cell_matrix(one_cell(CUBE * h, [lam, lam, lam, 0, 0, 0]), 0)
    assert a.shape == (8, 8)
    np.testing.assert_allclose(a, lam * h / 2 * np.eye(8), atol=1e-14 * lam * h)
    assert a.sum() == pytest.approx(4 * lam * h, rel=1e-13)
    assert vol == pytest.approx(h ** 3, rel=1e-13)


def test_unit_cube_with_fracture_face():
    """Same cube with its x- face a fracture face.

    The 4 sub-tetrahedra on that face now see the face unknown instead of the
    interpolated centre: the face diagonal becomes 4 lambda h / 3, its coupling
    to each of its 4 nodes -lambda h / 6, the node block stays
    (lambda h / 2) I, so the row sums are lambda h / 3 on the face's nodes,
    lambda h / 2 on the others and 2 lambda h / 3 on the face: A_KK = 4 lambda h
    is unchanged (eta_K does not depend on which faces are fractures).
    """
    h, lam = 0.5, 1.7
    P = one_cell(CUBE * h, [lam, lam, lam, 0, 0, 0], frac_faces=(0,))
    a, _ = oracle.cell_matrix(P, 0, cell_frac6=[0, -1, -1, -1, -1, -1])
    assert a.shape == (9, 9)
    face_nodes = HEXF[0]
    expect = np.zeros((9, 9))
    expect[:8, :8] = lam * h / 2 * np.eye(8)
    expect[8, 8] = 4 * lam * h / 3
    for s in face_nodes:
        expect[8, s] = expect[s, 8] = -lam * h / 6
    np.testing.assert_allclose(a, expect, atol=1e-14)
    r = a.sum(1)
    np.testing.assert_allclose(r[face_nodes], lam * h / 3, rtol=1e-13)
    assert a.sum() == pytest.approx(4 * lam * h, rel=1e-13)


def test_square_fracture_face_closed_form():
    """A square fracture face of any side, kappa = d_f Lambda_f / mu.

    Each of its 4 triangles (x_sigma, s_e, s_e+1) is right-isoceles with the
    right angle at x_sigma; by the cotangent formula the node-node coupling of
    a triangle is -cot(90 deg)/2 = 0 and each node gets kappa/2 from each of
    its two triangles: a_sigma = kappa I, rho_s = kappa, R_sigma = 4 kappa.
    """
    h = 0.25
    P = one_cell(CUBE * h, [1, 1, 1, 0, 0, 0], frac_faces=(3,))
    P.frac_width[:] = 0.02
    P.frac_perm[:] = 300.0
    kappa = 0.02 * 300.0
    A5, area = oracle.frac_matrix(P, 0)
    np.testing.assert_allclose(A5[1:, 1:], kappa * np.eye(4), atol=1e-12)
    np.testing.assert_allclose(A5[0, 1:], -kappa, rtol=1e-13)
    assert A5[0, 0] == pytest.approx(4 * kappa, rel=1e-13)
    assert area == pytest.approx(h * h, rel=1e-13)


def _divergence_flux(X, lam, g, frac_faces):
    """-(Lambda g) . int_K grad eta_nu dx by the divergence theorem.

    int_K grad eta_nu = sum over boundary triangles (x_sigma, s_e, s_e+1) of the
    outward area vector times the mean of eta_nu over the triangle, and
    eta_nu is P1 there with value 1/4 at a non-fracture face centre of a face
    containing node nu, 1 at the centre of fracture face nu, delta at nodes.
    """
    xK = X.mean(0)
    m = 8 + len(frac_faces)
    integral = np.zeros((m, 3))
    for f, fn in enumerate(HEXF):
        xs = X[fn].mean(0)
        for e in range(4):
            s1, s2 = fn[e], fn[(e + 1) % 4]
            av = 0.5 * np.cross(X[s1] - xs, X[s2] - xs)
            if av @ (xs - xK) < 0:
                av = -av
            w = np.zeros(m)
            w[s1] += 1 / 3
            w[s2] += 1 / 3
            if f in frac_faces:
                w[8 + list(frac_faces).index(f)] += 1 / 3
            else:
                for s in fn:
                    w[s] += 0.25 / 3
            integral += w[:, None] * av[None, :]
    return -integral @ (lam @ g)


@pytest.mark.parametrize("seed", range(6))
def test_local_matrix_linear_consistency(seed):
    """For affine v, sum_nu' a_{nu nu'} (v_K - v_nu') equals -(Lambda g).int_K grad eta_nu.

    pi_T reproduces affine functions (the face centre is the mean of its nodes,
    so I_sigma is exact), hence F_{K,nu}(v) = -int_K Lambda g . grad eta_nu,
    evaluated here independently by the divergence theorem on the boundary
    triangles of a jittered cell with a full anisotropic tensor.
    """
    rng = np.random.default_rng(seed)
    X = CUBE + rng.uniform(-0.2, 0.2, size=(8, 3))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    lam = Q @ np.diag(np.exp(rng.standard_normal(3))) @ Q.T
    perm6 = [lam[0, 0], lam[1, 1], lam[2, 2], lam[0, 1], lam[0, 2], lam[1, 2]]
    frac = tuple(sorted(rng.choice(6, size=seed % 3, replace=False).tolist()))
    P = one_cell(X, perm6, frac_faces=frac)
    cf = [-1] * 6
    for i, f in enumerate(frac):
        cf[f] = i
    a, vol = oracle.cell_matrix(P, 0, cell_frac6=cf)
    np.testing.assert_allclose(a, a.T, rtol=1e-12, atol=1e-14)
    assert np.linalg.eigvalsh(0.5 * (a + a.T)).min() > 0
    g = rng.standard_normal(3)
    pos = np.vstack([X, np.array([X[HEXF[f]].mean(0) for f in frac]).reshape(-1, 3)])
    v = pos @ g
    vK = X.mean(0) @ g
    F = (a * (vK - v[None, :])).sum(1)
    np.testing.assert_allclose(F, _divergence_flux(X, lam, g, frac), rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------------------
# global system, solve, fluxes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,seed", [((3, 2, 2), 0), ((2, 3, 2), 1), ((3, 3, 2), 2), ((2, 2, 3), 3)])
def test_oracle_equals_bruteforce(dims, seed):
    """Cell-wise Schur route + PCG == dense global Galerkin solve on tiny meshes."""
    p = synth.random_problem(dims, seed, n_patches=3)
    bf = bruteforce.solve(p)
    o = oracle.solve_darcy(p, rtol=1e-15)
    scale = 1.0
    for k in ["u_node", "u_cell", "u_frac"]:
        np.testing.assert_allclose(o[k], bf[k], atol=1e-9 * scale)
    for k in ["F_cell", "F_cell_frac", "F_frac"]:
        np.testing.assert_allclose(o[k], bf[k], atol=1e-9 * np.abs(bf[k]).max())


@pytest.mark.parametrize("seed", range(3))
def test_linear_exactness_jittered_anisotropic(seed):
    """Affine boundary data on all boundary nodes, constant anisotropic tensor,
    jittered mesh, no fracture: the Galerkin solution is the affine function at
    nodes and cells (u_K = u(x_K))."""
    n = 5
    p = synth.random_problem((n, n, n), seed, n_patches=0)
    rng = np.random.default_rng(100 + seed)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    lam = Q @ np.diag(np.exp(rng.standard_normal(3))) @ Q.T
    p.perm[:] = [lam[0, 0], lam[1, 1], lam[2, 2], lam[0, 1], lam[0, 2], lam[1, 2]]
    bnd = ~synth.meshes.interior_mask(p.dims)
    g, c = rng.standard_normal(3), rng.standard_normal()
    p.dirichlet = bnd.astype(np.uint8)
    p.p_bar = p.xyz @ g + c
    o = oracle.solve_darcy(p, rtol=1e-14)
    np.testing.assert_allclose(o["u_node"], p.xyz @ g + c, atol=1e-11)
    xK = p.xyz[p.hex8].mean(1)
    np.testing.assert_allclose(o["u_cell"], xK @ g + c, atol=1e-11)


def test_linear_exactness_config1():
    """Config 1: u = 1 - x solves the problem (isotropic, walls parallel to the
    gradient, fracture normal to it): u_s = 1 - x_s, u_sigma = 0.5, F_sigma,s = 0."""
    p = synth.config1()
    o = oracle.solve_darcy(p, rtol=1e-14)
    np.testing.assert_allclose(o["u_node"], 1 - p.xyz[:, 0], atol=1e-12)
    np.testing.assert_allclose(o["u_frac"], 0.5, atol=1e-12)
    np.testing.assert_allclose(o["F_frac"], 0.0, atol=1e-12)
    np.testing.assert_allclose(o["u_cell"], 1 - p.xyz[p.hex8].mean(1)[:, 0], atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_schur_system_spd(seed):
    """Lax-Milgram gives an SPD form; the Schur complement of an SPD matrix on
    its diagonal block is SPD: Cholesky succeeds and the matrix is symmetric."""
    p = synth.random_problem((4, 3, 4), seed, n_patches=4)
    A, b = oracle.system(p)
    D = A.toarray()
    np.testing.assert_allclose(D, D.T, rtol=0, atol=1e-14 * np.abs(D).max())
    np.linalg.cholesky(0.5 * (D + D.T))
    assert np.linalg.eigvalsh(0.5 * (D + D.T)).min() > 0


def test_neumann_rows_sum_to_zero():
    """Constants are in the kernel of the full operator: every row whose
    unknown has no Dirichlet neighbour has zero row sum."""
    p = synth.random_problem((5, 4, 4), 7, n_patches=4)
    A, b = oracle.system(p)
    cf, fc, _ = oracle.topology(p)
    nfree = int((p.dirichlet == 0).sum())
    node_unk = -np.ones(p.n_nodes, int)
    node_unk[p.dirichlet == 0] = np.arange(nfree)
    touches = np.zeros(A.shape[0], bool)
    for K in range(p.n_cells):
        nodes = p.hex8[K]
        if p.dirichlet[nodes].any():
            unk = [node_unk[s] for s in nodes if node_unk[s] >= 0]
            unk += [nfree + f for f in cf[K] if f >= 0]
            touches[unk] = True
    rs = np.asarray(A.sum(1)).ravel()
    scale = np.abs(A).max()
    assert (~touches).sum() > 10
    np.testing.assert_allclose(rs[~touches], 0.0, atol=1e-13 * scale)
    np.testing.assert_allclose(b[~touches], 0.0, atol=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_conservation(seed):
    """Discrete conservation (§3.1): cells exactly, fracture faces and free nodes
    to the solver tolerance; the Dirichlet-node fluxes sum to zero."""
    p = synth.random_problem((5, 4, 4), seed, n_patches=4)
    o = oracle.solve_darcy(p, rtol=1e-14)
    cf, fc, _ = oracle.topology(p)
    Fs = np.abs(o["F_cell"]).max()
    cell_sum = o["F_cell"].sum(1)
    for f in range(p.n_frac):
        for side in range(2):
            if fc[f, side] >= 0:
                cell_sum[fc[f, side]] += o["F_cell_frac"][f, side]
    np.testing.assert_allclose(cell_sum, 0.0, atol=1e-12 * Fs)
    frac_res = o["F_frac"].sum(1) - o["F_cell_frac"].sum(1)
    node_res = np.zeros(p.n_nodes)
    np.add.at(node_res, p.hex8.ravel(), -o["F_cell"].ravel())
    np.add.at(node_res, p.frac_nodes.ravel(), -o["F_frac"].ravel())
    free = p.dirichlet == 0
    tol = 1e-8 * max(Fs, np.abs(o["F_frac"]).max())
    np.testing.assert_allclose(frac_res, 0.0, atol=tol)
    np.testing.assert_allclose(node_res[free], 0.0, atol=tol)
    assert abs(node_res[~free].sum()) < tol


# ---------------------------------------------------------------------------
# control volumes, CFL, transport
# ---------------------------------------------------------------------------

def test_porous_volume_partition():
    """The control volumes partition the pore space (§3.2.1): summed over all
    control volumes the porous volumes give int phi_m over Omega plus
    sum d_f |sigma| phi_f; the cells of a jittered unit cube fill volume 1."""
    p = synth.random_problem((5, 5, 4), 3, n_patches=5)
    p.poro[:] = np.random.default_rng(0).uniform(0.1, 0.4, p.n_cells)
    phi = oracle.porous_volumes(p)
    vols = np.array([oracle.cell_matrix(p, K)[1] for K in range(p.n_cells)])
    assert vols.sum() == pytest.approx(1.0, rel=1e-13)
    areas = np.array([oracle.frac_matrix(p, f)[1] for f in range(p.n_frac)])
    total = (vols * p.poro).sum() + (p.frac_width * areas * p.frac_poro).sum()
    got = phi["phi_cell"].sum() + phi["phi_frac"].sum() + phi["phi_node"].sum()
    assert got == pytest.approx(total, rel=1e-13)
    assert (phi["phi_node"][p.dirichlet == 1] == 0).all()
    assert (phi["phi_cell"] > 0).all() and (phi["phi_frac"] > 0).all()
    assert (phi["phi_node"][p.dirichlet == 0] > 0).all()


def test_cfl_uniform_flow_cube():
    """Cartesian n^3, no fracture, u = 1 - x: F_{K,s} = +-h^2/4 (two-point VAG,
    a = h/2, u_K - u_s = -+h/2).  An interior cell has porous volume
    (1 - 8/16) h^3 and outflow 4 h^2/4: dt = h/2; a free node has h^3/2 and
    outflow h^2: dt = h/2; cells touching a Dirichlet plane have 3h^3/4 and
    outflow h^2.  Hence min = h/2 exactly."""
    n = 6
    p = synth.cartesian_problem(n)
    o = oracle.solve_darcy(p, rtol=1e-14)
    h = 1.0 / n
    np.testing.assert_allclose(np.abs(o["F_cell"]), h * h / 4, rtol=1e-10)
    phi = oracle.porous_volumes(p)
    dt3 = oracle.cfl_bounds(p, o, phi)
    assert dt3[0] == pytest.approx(h / 2, rel=1e-10)
    assert dt3[2] == pytest.approx(h / 2, rel=1e-10)
    assert math.isinf(dt3[1])


def _config1_grid():
    """Config 1 (n = 10, fracture plane i = 5) with the grid indices of its
    nodes and cells, counted from the logical grid alone."""
    p = synth.config1()
    n = 10
    k, j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    node_ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], 1)
    assert (synth.node_index((n, n, n), *node_ijk.T) == np.arange(p.n_nodes)).all()
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cell_ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], 1)
    return p, n, node_ijk, cell_ijk


def test_config1_porous_volumes_closed_form():
    """Control volumes of config 1, one by one (§3.2.1, volume fractions of
    the single-rock-type reading: alpha_{K,s} = 1/16 for the free nodes of K
    that are not fracture nodes, alpha_{sigma,s} = 1/8 for the free nodes of
    sigma).  With h = 1/10, phi_m = phi_f = 1, d_f = 0.01:

    * a node on the fracture plane takes its porous volume from the fracture
      faces only, 1/8 of d_f h^2 from each of the m faces around it (4 inside
      the plane, 2 on a wall edge, 1 at a corner): m d_f h^2 / 8;
    * any other free node takes 1/16 of h^3 from each of its c cells (8, 4 on
      a wall, 2 on a wall edge): c h^3 / 16;
    * a fracture face keeps (1 - 4/8) of its volume: d_f h^2 / 2;
    * a cell keeps h^3 (1 - q/16) with q its free nodes off the fracture
      plane: 8 inside (h^3/2), 4 beside the fracture or a Dirichlet plane
      (3 h^3 / 4);
    * Dirichlet nodes hold none.
    Fracture nodes taking a matrix share, or another alpha_{sigma,s}, change
    these values."""
    p, n, nijk, cijk = _config1_grid()
    h, df = 1.0 / n, 0.01
    phi = oracle.porous_volumes(p)
    dirichlet = (nijk[:, 0] == 0) | (nijk[:, 0] == n)
    assert (dirichlet == (p.dirichlet == 1)).all()
    on_wall = lambda a: (a == 0) | (a == n)  # noqa: E731
    per_axis = lambda a: np.where(on_wall(a), 1, 2)  # noqa: E731
    m_faces = per_axis(nijk[:, 1]) * per_axis(nijk[:, 2])
    n_cells = m_faces * per_axis(nijk[:, 0])
    frac_node = nijk[:, 0] == n // 2
    expect_node = np.where(frac_node, m_faces * df * h * h / 8, n_cells * h ** 3 / 16)
    expect_node[dirichlet] = 0.0
    np.testing.assert_allclose(phi["phi_node"], expect_node, rtol=1e-12, atol=0)
    beside = (cijk[:, 0] == n // 2 - 1) | (cijk[:, 0] == n // 2) | (cijk[:, 0] == 0) | (cijk[:, 0] == n - 1)
    expect_cell = np.where(beside, 0.75, 0.5) * h ** 3
    np.testing.assert_allclose(phi["phi_cell"], expect_cell, rtol=1e-12, atol=0)
    np.testing.assert_allclose(phi["phi_frac"], df * h * h / 2, rtol=1e-12, atol=0)


def test_alpha_rule_ties_reduce_to_single_rock_type():
    """§3.2.1's largest-permeability rule on config 1, one matrix rock type
    and one fracture permeability: every cell (face) around a node ties for
    the largest permeability, so every one gives its share and the porous
    volumes are those of the single-rock-type reading, bit for bit."""
    p = synth.config1()
    a, b = oracle.porous_volumes(p, 0), oracle.porous_volumes(p, 1)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_alpha_rule_two_rock_types_closed_form():
    """§3.2.1's rule for nodes between rock types, control volume by control
    volume on config 1 (h = 1/10, d_f = 0.01) with the cells of x-index >= 7
    at permeability 10 I (the rest I) and the fracture faces above y = 1/2
    at 100 times the others' permeability:

    * a node of the rock interface i = 7 takes 1/16 of h^3 from the c_r cells
      on its high side only (4 inside, 2 on a wall, 1 on a wall edge);
    * a cell of index 6 gives nothing to its 4 nodes at i = 7 and keeps
      (1 - 4/16) h^3, a cell of index 7 gives to all 8: h^3/2;
    * a fracture node on the line j = 5 takes 1/8 of d_f h^2 from the faces
      above it only (2 inside the plane, 1 on a wall);
    * a fracture face just below the line gives nothing to its 2 nodes on
      it: (1 - 2/8) d_f h^2; the other faces keep d_f h^2 / 2;
    * every other control volume is as with one rock type.
    Taking the lowest-permeability cells, or the largest over the wrong
    neighbours, or comparing with > instead of >=, changes these values."""
    p, n, nijk, cijk = _config1_grid()
    h, df = 1.0 / n, 0.01
    hi_cell = cijk[:, 0] >= 7
    p.perm[hi_cell] = [10.0, 10.0, 10.0, 0.0, 0.0, 0.0]
    fy = p.xyz[np.asarray(p.frac_nodes).reshape(-1, 4)][:, :, 1].mean(1)
    hi_face = fy > 0.5
    p.frac_perm[hi_face] *= 100.0
    phi = oracle.porous_volumes(p, 1)
    base = oracle.porous_volumes(synth.config1(), 0)
    on_wall = lambda a: (a == 0) | (a == n)  # noqa: E731
    per_axis = lambda a: np.where(on_wall(a), 1, 2)  # noqa: E731
    expect_node = base["phi_node"].copy()
    iface = nijk[:, 0] == 7
    expect_node[iface] = per_axis(nijk[iface, 1]) * per_axis(nijk[iface, 2]) * h ** 3 / 16
    line = (nijk[:, 0] == n // 2) & (nijk[:, 1] == n // 2)
    expect_node[line] = per_axis(nijk[line, 2]) * df * h * h / 8
    np.testing.assert_allclose(phi["phi_node"], expect_node, rtol=1e-12, atol=0)
    expect_cell = base["phi_cell"].copy()
    expect_cell[cijk[:, 0] == 6] = 0.75 * h ** 3
    expect_cell[cijk[:, 0] == 7] = 0.5 * h ** 3
    np.testing.assert_allclose(phi["phi_cell"], expect_cell, rtol=1e-12, atol=0)
    below = (fy > 0.5 - h) & (fy < 0.5)
    expect_frac = np.where(below, 0.75, 0.5) * df * h * h
    np.testing.assert_allclose(phi["phi_frac"], expect_frac, rtol=1e-12, atol=0)
    # shares only move between control volumes: the total is unchanged
    total = sum(v.sum() for v in phi.values())
    assert total == pytest.approx(sum(v.sum() for v in base.values()), rel=1e-13)


def test_config1_cfl_closed_form():
    """eq eq_CFL on config 1, where u = 1 - x is the exact discrete solution.

    With the cube forms (node block (lambda h/2) I, fracture face diagonal
    4 lambda h/3 and coupling -lambda h/6 to its nodes, lambda = 1) and
    u_K - u_s = -+h/2 across a cell:
    * cells: an interior cell sends h^2/4 through each of its 4 downstream
      nodes; its volume h^3/2 gives dt_M = h/2.  The cells beside the plane
      (volume 3h^3/4, outflow h^2) give 3h/4.
    * fracture faces: F_{sigma,s} = 0, the upstream cell K sends
      F_{K,sigma} = (4/3 - 4/6) h (h/2) = h^2/3 into sigma, and the
      downstream cell L receives (-F_{L,sigma})^+ = h^2/3 from it: the only
      outflow of sigma.  dt_F = (d_f h^2/2) / (h^2/3) = 3 d_f / 2.
    * nodes: a fracture node sends (h/2 - h/6)(h/2) = h^2/6 into each of its
      4 downstream cells (2 h^2/3 in total) from d_f h^2/2: 3 d_f / 4; the
      others h^2 from h^3/2: h/2.
    Dropping the cell-to-face outflow term leaves sigma without outflow
    (dt_F infinite)."""
    p, n, _, _ = _config1_grid()
    h, df = 1.0 / n, 0.01
    o = oracle.solve_darcy(p, rtol=1e-14)
    phi = oracle.porous_volumes(p)
    dt3 = oracle.cfl_bounds(p, o, phi)
    assert dt3[0] == pytest.approx(h / 2, rel=1e-9)
    assert dt3[1] == pytest.approx(1.5 * df, rel=1e-9)
    assert dt3[2] == pytest.approx(0.75 * df, rel=1e-9)
    cf, fc, _ = oracle.topology(p)
    assert (fc >= 0).all()
    np.testing.assert_allclose(o["F_cell_frac"][:, 0], h * h / 3, rtol=1e-9)
    np.testing.assert_allclose(o["F_cell_frac"][:, 1], -h * h / 3, rtol=1e-9)


def _dirichlet_outflow(p, o, c):
    """sum over Dirichlet nodes s of sum_K H_{K,s} + sum_sigma H_{sigma,s}."""
    cf, fc, _ = oracle.topology(p)
    pos = lambda x: np.maximum(x, 0)  # noqa: E731
    neg = lambda x: np.minimum(x, 0)  # noqa: E731
    cK = c["c_cell"][:, None]
    cs = c["c_node"][p.hex8]
    H = cK * pos(o["F_cell"]) + cs * neg(o["F_cell"])
    d = p.dirichlet[p.hex8] == 1
    total = H[d].sum()
    Hf = c["c_frac"][:, None] * pos(o["F_frac"]) + c["c_node"][p.frac_nodes] * neg(o["F_frac"])
    total += Hf[p.dirichlet[p.frac_nodes] == 1].sum()
    return total


def test_mass_balance_and_max_principle():
    """Telescoping of the upwind fluxes: the pore mass changes only through
    the Dirichlet nodes, M^{n+1} - M^n = -dt * sum_{s Dirichlet} H_s (H_{K,s} is
    the flux from K into s); and under
    the CFL condition the scheme is monotone: 0 <= c <= 1."""
    p = synth.random_problem((6, 5, 5), 11, n_patches=4)
    o = oracle.solve_darcy(p, rtol=1e-14)
    phi = oracle.porous_volumes(p)
    dt = 0.9 * oracle.cfl_bounds(p, o, phi).min()
    c = dict(c_cell=np.zeros(p.n_cells), c_frac=np.zeros(p.n_frac), c_node=np.where(p.dirichlet == 1, p.c_bar, 0.0))
    mass = lambda c: (phi["phi_cell"] @ c["c_cell"] + phi["phi_frac"] @ c["c_frac"]  # noqa: E731
                      + phi["phi_node"] @ c["c_node"])
    for _ in range(20):
        m0 = mass(c)
        flow = _dirichlet_outflow(p, o, c)
        c = oracle.transport(p, o, phi, dt, 1, c0=c)
        scale = max(abs(m0), abs(dt * flow), 1e-300)
        assert abs(mass(c) - m0 + dt * flow) <= 1e-12 * scale
        for k in ("c_cell", "c_frac", "c_node"):
            assert c[k].min() >= -1e-9 and c[k].max() <= 1 + 1e-9


def test_steady_state_equals_direct_solve():
    """The fixed point of the explicit recursion solves sum_nu H_nu(c) = 0 for
    every control volume with c = c_bar at Dirichlet nodes, a sparse linear
    system solved here directly with scipy."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    p = synth.random_problem((5, 4, 4), 5, n_patches=3, ratios=(1e2,))
    o = oracle.solve_darcy(p, rtol=1e-14)
    phi = oracle.porous_volumes(p)
    dt = 0.9 * oracle.cfl_bounds(p, o, phi).min()
    cf, fc, _ = oracle.topology(p)
    nc, nf, nn = p.n_cells, p.n_frac, p.n_nodes
    N = nc + nf + nn
    rows, cols, vals = [], [], []
    rhs = np.zeros(N)

    def add_flux(i, j, F):
        # flux F from CV i to CV j: H = c_i F+ + c_j F-; eq_i += H, eq_j -= H
        for r, sgn in ((i, 1.0), (j, -1.0)):
            rows.extend([r, r])
            cols.extend([i, j])
            vals.extend([sgn * max(F, 0.0), sgn * min(F, 0.0)])

    for K in range(nc):
        for a in range(8):
            add_flux(K, nc + nf + p.hex8[K, a], o["F_cell"][K, a])
    for f in range(nf):
        for side in range(2):
            if fc[f, side] >= 0:
                add_flux(fc[f, side], nc + f, o["F_cell_frac"][f, side])
        for i in range(4):
            add_flux(nc + f, nc + nf + p.frac_nodes[f, i], o["F_frac"][f, i])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(N, N)).tolil()
    for s in np.nonzero(p.dirichlet)[0]:
        M.rows[nc + nf + s] = [nc + nf + s]
        M.data[nc + nf + s] = [1.0]
        rhs[nc + nf + s] = p.c_bar[s]
    c_direct = spla.spsolve(M.tocsr(), rhs)
    c = oracle.transport(p, o, phi, dt, 24000)
    np.testing.assert_allclose(c["c_cell"], c_direct[:nc], atol=1e-9)
    np.testing.assert_allclose(c["c_frac"], c_direct[nc:nc + nf], atol=1e-9)
    np.testing.assert_allclose(c["c_node"], c_direct[nc + nf:], atol=1e-9)


# ---------------------------------------------------------------------------
# the paper's analytical test cases
# ---------------------------------------------------------------------------

def test_paper_parameters_golden():
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    e2 = analytic.E2(g["e2"]["tan_theta1"], g["e2"]["tan_theta2"], g["e2"]["lambda_f1"], g["e2"]["lambda_f3"])
    (a, b), (c, d) = g["e2"]["x0_exact_fraction"]
    assert e2.x0 == pytest.approx(a / b, rel=1e-15)
    assert e2.y0 == pytest.approx(c / d, rel=1e-15)
    e1 = analytic.E1(g["e1"]["tan_theta"], g["e1"]["lambda_f"], g["e1"]["d_f"])
    # beta = sin(theta)/d_f with tan(theta) = 1/2 -> sin = 1/sqrt(5); k = 20 * 4/5
    assert e1.beta == pytest.approx(100 / math.sqrt(5), rel=1e-14)
    assert e1.k == pytest.approx(16.0, rel=1e-14)


def test_e1_closed_form_solves_fracture_equation():
    """c_f of §5.1 satisfies L c_f = beta c_m1 along the fracture characteristics:
    for x/k < t < x the matrix above is still 0, so (d/dt + k d/dx + beta) c_f = 0."""
    e1 = analytic.E1()
    x, t, eps = 0.7, 0.5, 1e-6
    c = lambda x, t: float(e1.cf(x, t))  # noqa: E731
    dt_ = (c(x, t + eps) - c(x, t - eps)) / (2 * eps)
    dx_ = (c(x + eps, t) - c(x - eps, t)) / (2 * eps)
    assert dt_ + e1.k * dx_ + e1.beta * c(x, t) == pytest.approx(0.0, abs=1e-6)
    assert c(0.3, 0.5) == 1.0 and c(9.0, 0.5) == 0.0


def test_e2_closed_form_vs_ode():
    """The stationary fracture concentrations of §5.2 solve the steady fracture
    ODEs of equation test_traceur4frac; integrate them numerically and compare
    (this pins the sign reading of the c_{f,3} exponent)."""
    from scipy.integrate import solve_ivp
    e2 = analytic.E2()
    # c_f2: k1 c' + b1 c = b1 c_f4(1/4 + x tan1),  c(x0) = c0
    s2 = solve_ivp(lambda x, c: [(e2.b1 * e2.cf4(0.25 + x * e2.tan1) - e2.b1 * c[0]) / e2.k1],
                   (e2.x0, 1.0), [e2.c0], rtol=1e-12, atol=1e-14, dense_output=True)
    for x in (0.7, 0.85, 1.0):
        assert float(e2.cf2(x)) == pytest.approx(s2.sol(x)[0], rel=1e-9)

    # c_f3: -k2 c' + b2 c = b2 c_m3(.., y),  c(y0) = c0, integrated downwards
    def cm3(y):
        return 0.0 if y < 0.25 else float(e2.cf1((y - 0.25) / e2.tan1))

    s3 = solve_ivp(lambda y, c: [(e2.b2 * c[0] - e2.b2 * cm3(y)) / e2.k2],
                   (e2.y0, 0.0), [e2.c0], rtol=1e-12, atol=1e-14, dense_output=True, max_step=1e-3)
    for y in (0.5, 0.3, 0.2, 0.0):
        assert float(e2.cf3(y)) == pytest.approx(s3.sol(y)[0], rel=1e-8)
    # c0 is the flux-weighted mix at the intersection
    assert e2.c0 == pytest.approx((e2.cf1(e2.x0) + e2.r * e2.cf4(e2.y0)) / (1 + e2.r), rel=1e-14)


def _quad_area(P):
    x, y = P[:, 0], P[:, 1]
    return 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def _errors_e1(n):
    p = synth.e1_problem(n)
    r = oracle.run(p)
    e1 = analytic.E1()
    xK = p.xyz[p.hex8].mean(1)
    w = np.array([_quad_area(p.xyz[h[:4]]) for h in p.hex8])
    em = analytic.rel_l1(w, r["c_cell"], e1.cm(xK[:, 0], xK[:, 1], 0.5))
    xs = p.xyz[p.frac_nodes].mean(1)
    wf = np.linalg.norm(p.xyz[p.frac_nodes[:, 1]] - p.xyz[p.frac_nodes[:, 0]], axis=1)
    ef = analytic.rel_l1(wf, r["c_frac"], e1.cf(xs[:, 0], 0.5))
    return em, ef


def _errors_e2(n):
    p = synth.e2_problem(n)
    r = oracle.run(p)
    e2 = analytic.E2()
    xK = p.xyz[p.hex8].mean(1)
    w = np.array([_quad_area(p.xyz[h[:4]]) for h in p.hex8])
    em = analytic.rel_l1(w, r["c_cell"], e2.cm(xK[:, 0], xK[:, 1]))
    xs = p.xyz[p.frac_nodes].mean(1)
    wf = np.linalg.norm(p.xyz[p.frac_nodes[:, 1]] - p.xyz[p.frac_nodes[:, 0]], axis=1)
    ef = analytic.rel_l1(wf, r["c_frac"], e2.cf_branch(p.meta["branch"], xs[:, 0], xs[:, 1]))
    return em, ef


def test_e1_convergence():
    """§5.1: the numerical solution converges to the analytical one under mesh
    refinement, faster in the fracture (rates themselves: parity unpinned)."""
    errs = [_errors_e1(n) for n in (16, 32, 64)]
    em = [e[0] for e in errs]
    ef = [e[1] for e in errs]
    assert em[0] > em[1] > em[2]
    assert ef[0] > ef[1] > ef[2]
    assert math.log2(em[1] / em[2]) > 0.3
    assert math.log2(ef[1] / ef[2]) > 0.6
    assert ef[2] < 0.1


def test_e2_convergence():
    """§5.2: convergence to the stationary analytical solution."""
    errs = [_errors_e2(n) for n in (16, 32, 64)]
    em = [e[0] for e in errs]
    ef = [e[1] for e in errs]
    assert em[0] > em[1] > em[2]
    assert ef[0] > ef[1] > ef[2]
    assert ef[2] < 0.05


# ---------------------------------------------------------------------------
# matrix-free residual (the full-size certificate of the GPU solves)
# ---------------------------------------------------------------------------

def _unknowns(p, res):
    """Stack free-node and face entries in the assembled system's order."""
    free = p.dirichlet == 0
    return np.concatenate([res[0][free], res[1]])


@pytest.mark.parametrize("seed,wells", [(0, False), (1, True), (2, False)])
def test_residual_equals_assembled_system(seed, wells):
    """orc_residual evaluates the conservation equations cell by cell; the
    assembled Schur system (triplets summed into CSR, Dirichlet columns moved
    to b) must give the same b and the same b - A x for any x."""
    p = synth.random_problem((5, 4, 6), seed, n_patches=4)
    if wells:
        synth.add_wells(p, seed, n_inj=1, n_prod=2)
    A, b = oracle.system(p)
    rng = np.random.default_rng(seed)
    free = p.dirichlet == 0
    u_node = np.where(free, rng.standard_normal(p.n_nodes), 123.0)  # Dirichlet entries are ignored
    u_frac = rng.standard_normal(p.n_frac)
    x = np.concatenate([u_node[free], u_frac])
    r = oracle.residual(p, u_node, u_frac)
    scale = np.abs(A).max() * (np.abs(x).max() + np.abs(p.p_bar).max())
    np.testing.assert_allclose(_unknowns(p, (r["b_node"], r["b_frac"])), b, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(_unknowns(p, (r["res_node"], r["res_frac"])), b - A @ x, rtol=0, atol=1e-13 * scale)
    assert (r["res_node"][~free] == 0).all() and (r["b_node"][~free] == 0).all()


def test_residual_vanishes_on_affine_solution():
    """Config 1: u = 1 - x at the nodes and 1/2 on the fracture is the exact
    discrete solution, so every conservation equation holds to rounding."""
    p = synth.config1()
    r = oracle.residual(p, 1 - p.xyz[:, 0], np.full(p.n_frac, 0.5))
    assert r["rel_residual"] < 1e-14
    assert np.linalg.norm(np.concatenate([r["b_node"], r["b_frac"]])) > 0.1
