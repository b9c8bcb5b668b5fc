"""Pins of the general-cell oracle (tetrahedra, prisms, hexahedra): on
hexahedra it reproduces the C oracle; on tetrahedral and prismatic meshes,
with or without a fracture plane, it reproduces affine pressures exactly
(the scheme is exact for affine solutions); mass balance of the transport.
Wells (§5.5) on general cells: on hexahedra they reproduce the C oracle's
wells, whose closed forms are pinned on their own; on tetrahedra and prisms
what the wells bring leaves through the Dirichlet nodes, a producer at its
face's own pressure changes nothing, and the transport balances mass."""
import numpy as np
import pytest

import oracle
import synth
from oracle import general_cells as gc
from synth import meshes as sm


def test_reference_cells_positive():
    """Every sub-tetrahedron of the reference tetrahedron, prism and cube is
    positively oriented with the local face tables, and the volumes add up."""
    ref = {4: [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]],
           6: [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [0, 1, 1]],
           8: [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]]}
    vol = {4: 1 / 6, 6: 1 / 2, 8: 1.0}
    for nv, X in ref.items():
        m = gc.Mesh(X, [tuple(range(nv))], [[1, 1, 1, 0, 0, 0]], [1.0])
        a, v = gc.cell_matrix(m, 0)
        assert v == pytest.approx(vol[nv], rel=1e-14)
        assert a.shape == (nv, nv)
        np.testing.assert_allclose(a, a.T, atol=1e-14)


def test_hexahedra_equal_the_c_oracle():
    p = synth.random_problem((5, 4, 4), 41, n_patches=3, n_steps=12)
    o = oracle.run(p, rtol=1e-14)
    m = gc.Mesh.from_problem(p)
    s = gc.solve_darcy(m)
    od = o["darcy"]
    np.testing.assert_allclose(s["u_node"], od["u_node"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(s["u_frac"], od["u_frac"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(s["u_cell"], od["u_cell"], rtol=0, atol=1e-10)
    scale = np.abs(od["F_cell"]).max()
    np.testing.assert_allclose(np.array([F[:8] for F in s["F_cell"]]), od["F_cell"], rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(np.array(s["F_frac"]), od["F_frac"], rtol=0, atol=1e-9 * scale)
    phi = gc.porous_volumes(m, s)
    for k in ("phi_cell", "phi_frac", "phi_node"):
        np.testing.assert_allclose(phi[k], o["phi"][k], rtol=1e-13, atol=1e-16)
    dt = gc.cfl_dt(m, s, phi, p.cfl)
    assert dt == pytest.approx(o["dt"], rel=1e-8)
    c = gc.transport(m, s, phi, o["dt"], p.n_steps)
    for k in ("c_cell", "c_frac", "c_node"):
        np.testing.assert_allclose(c[k], o[k], rtol=0, atol=1e-9)


def test_alpha_rule_hexahedra_equal_the_c_oracle():
    """The largest-permeability rule of §3.2.1 on hexahedra with lognormal
    tensors (every node between rock types) and fracture patches of several
    permeabilities: the numpy oracle's porous volumes equal the C oracle's,
    whose rule is pinned by closed forms."""
    p = synth.random_problem((6, 5, 4), 43, n_patches=4, n_steps=0)
    m = gc.Mesh.from_problem(p)
    s = gc.solve_darcy(m)
    a = oracle.porous_volumes(p, 1)
    phi = gc.porous_volumes(m, s, alpha_rule=1)
    for k in ("phi_cell", "phi_frac", "phi_node"):
        np.testing.assert_allclose(phi[k], a[k], rtol=1e-13, atol=1e-16)
    b = oracle.porous_volumes(p, 0)
    assert np.abs(a["phi_node"] - b["phi_node"]).max() > 1e-3 * np.abs(b["phi_node"]).max()


def test_wells_hexahedra_equal_the_c_oracle():
    """Two rate injectors and two pressure wells on hexahedra: pressures, well
    rates, time step and concentrations equal the C oracle's."""
    p = synth.add_wells(synth.random_problem((6, 5, 4), 45, n_patches=4, n_steps=15), 5, n_inj=2, n_prod=2)
    o = oracle.run(p, rtol=1e-14)
    m = gc.Mesh.from_problem(p)
    assert len(m.well_face) == 4
    s = gc.solve_darcy(m)
    od = o["darcy"]
    np.testing.assert_allclose(s["u_node"], od["u_node"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(s["u_frac"], od["u_frac"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(s["well_rate"], od["well_rate"], rtol=0, atol=1e-10)
    phi = gc.porous_volumes(m, s)
    dt = gc.cfl_dt(m, s, phi, p.cfl)
    assert dt == pytest.approx(o["dt"], rel=1e-8)
    c = gc.transport(m, s, phi, o["dt"], p.n_steps)
    for k in ("c_cell", "c_frac", "c_node"):
        np.testing.assert_allclose(c[k], o[k], rtol=0, atol=1e-9)
    assert c["c_frac"][p.wells["face"][0]] > 0.05


def _dirichlet_inflow(m, s):
    """Total flux from the domain into the Dirichlet nodes."""
    nc, nf = len(m.cells), len(m.frac)
    return sum(F for i, j, F in gc._edges(m, s) if j >= nc + nf and m.dirichlet[j - nc - nf])


def _with_wells(m, face, wi, pw, q, cinj):
    return gc.Mesh(m.xyz, m.cells, m.perm, m.poro, m.frac, m.frac_width, m.frac_perm, m.frac_poro, m.dirichlet,
                   m.p_bar, m.c_bar, m.mu, dict(face=face, wi=wi, pw=pw, q=q, cinj=cinj))


@pytest.mark.parametrize("kind", ["tet", "prism"])
def test_wells_conservation(kind):
    """At steady state the wells' total inflow leaves through the Dirichlet
    nodes, and without wells the Dirichlet fluxes balance to zero."""
    m0 = _general_mesh(kind, (4, 3, 3), 46, aniso=True, frac=True, dirichlet_all=False)
    s0 = gc.solve_darcy(m0)
    scale = max(np.abs(F).max() for F in s0["F_cell"])
    assert abs(_dirichlet_inflow(m0, s0)) <= 1e-10 * scale
    nf = len(m0.frac)
    m = _with_wells(m0, [0, nf // 2, nf - 1], [0.0, 0.3, 0.1], [0.0, 0.2, 0.9], [0.4, 0.0, 0.0], [1.0, 0.0, 0.0])
    s = gc.solve_darcy(m)
    Q = s["well_rate"]
    assert Q[0] == pytest.approx(0.4) and Q[1] < 0 and Q[2] > 0
    assert abs(Q.sum() - _dirichlet_inflow(m, s)) <= 1e-10 * scale


@pytest.mark.parametrize("kind", ["tet", "prism"])
def test_producer_at_the_face_pressure_changes_nothing(kind):
    m0 = _general_mesh(kind, (4, 3, 3), 47, aniso=True, frac=True, dirichlet_all=False)
    s0 = gc.solve_darcy(m0)
    f = int(np.argmax(np.abs(s0["u_frac"] - 0.5)))
    s1 = gc.solve_darcy(_with_wells(m0, [f], [50.0], [s0["u_frac"][f]], [0.0], [0.0]))
    assert abs(s1["well_rate"][0]) <= 1e-9
    np.testing.assert_allclose(s1["u_node"], s0["u_node"], rtol=0, atol=1e-10)
    # a lower well pressure draws fluid out and lowers the face pressure
    s2 = gc.solve_darcy(_with_wells(m0, [f], [50.0], [s0["u_frac"][f] - 0.2], [0.0], [0.0]))
    assert s2["well_rate"][0] < 0 and s2["u_frac"][f] < s0["u_frac"][f]


@pytest.mark.parametrize("kind", ["tet", "prism"])
def test_wells_transport_mass_balance(kind):
    """M^{n+1} - M^n = dt (c_inj Q^+ - c_sigma Q^- summed over the wells -
    flux into the Dirichlet nodes); c stays in [0, 1]."""
    m0 = _general_mesh(kind, (4, 3, 3), 48, aniso=True, frac=True, dirichlet_all=False)
    nf = len(m0.frac)
    m = _with_wells(m0, [1, nf - 2], [0.0, 0.2], [0.0, 0.1], [0.3, 0.0], [1.0, 0.0])
    s = gc.solve_darcy(m)
    Q = s["well_rate"]
    assert Q[0] > 0 and Q[1] < 0
    phi = gc.porous_volumes(m, s)
    dt = gc.cfl_dt(m, s, phi, 0.9)
    vol = np.concatenate([phi["phi_cell"], phi["phi_frac"], phi["phi_node"]])
    nc = len(m.cells)
    c = gc.transport(m, s, phi, dt, 0)
    for n in range(1, 12):
        cv = np.concatenate([c["c_cell"], c["c_frac"], c["c_node"]])
        out = 0.0
        for i, j, F in gc._edges(m, s):
            if j >= nc + nf and m.dirichlet[j - nc - nf]:
                out += cv[i] * max(F, 0.0) + cv[j] * min(F, 0.0)
        wells = Q[0] - cv[nc + m.well_face[1]] * (-Q[1])
        c2 = gc.transport(m, s, phi, dt, n)
        cv2 = np.concatenate([c2["c_cell"], c2["c_frac"], c2["c_node"]])
        assert abs(vol @ cv2 - vol @ cv - dt * (wells - out)) <= 1e-12 * max(1.0, abs(vol @ cv))
        assert cv2.min() >= -1e-12 and cv2.max() <= 1 + 1e-12
        c = c2
    assert c["c_frac"][m.well_face[0]] > 0.05


def _general_mesh(kind, dims, seed, aniso=True, frac=False, dirichlet_all=True):
    xyz, _ = sm.structured_hex(*dims)
    rng = np.random.default_rng(seed)
    h = 1.0 / np.array(dims)
    interior = np.all((xyz > 1e-12) & (xyz < 1 - 1e-12), axis=1)
    # jitter y and z only, so that the x planes (and the fracture plane) stay planar
    xyz[interior, 1:] += rng.uniform(-0.2, 0.2, (interior.sum(), 2)) * h[1:]
    cells = sm.simplex_cells(dims, kind)
    cells = sm.orient_tets(xyz, cells)
    nc = len(cells)
    if aniso:
        R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
        L = R @ np.diag([1.0, 3.0, 0.5]) @ R.T
        perm = np.tile([L[0, 0], L[1, 1], L[2, 2], L[0, 1], L[0, 2], L[1, 2]], (nc, 1))
    else:
        perm = np.tile([1.0, 1.0, 1.0, 0, 0, 0], (nc, 1))
    if dirichlet_all:
        d = (~interior).astype(np.uint8)
    else:
        d = ((xyz[:, 0] < 1e-12) | (xyz[:, 0] > 1 - 1e-12)).astype(np.uint8)
    ff = sm.plane_x_faces(dims, cells, dims[0] // 2) if frac else []
    nf = len(ff)
    return gc.Mesh(xyz, cells, perm, np.ones(nc), ff, np.full(nf, 0.01), np.full(nf, 1e3), np.ones(nf), d,
                   1.0 - xyz[:, 0] + 0.3 * xyz[:, 1] - 0.2 * xyz[:, 2] if dirichlet_all else 1.0 - xyz[:, 0],
                   (xyz[:, 0] < 1e-12).astype(float))


@pytest.mark.parametrize("kind", ["tet", "prism"])
def test_affine_pressure_exact(kind):
    """Affine Dirichlet data on every boundary node, a constant anisotropic
    tensor, jittered nodes: nodal and cell pressures are the affine function."""
    m = _general_mesh(kind, (4, 3, 3), 42)
    s = gc.solve_darcy(m)
    x = m.xyz
    f = lambda y: 1.0 - y[..., 0] + 0.3 * y[..., 1] - 0.2 * y[..., 2]  # noqa: E731
    np.testing.assert_allclose(s["u_node"], f(x), rtol=0, atol=1e-12)
    xK = np.array([x[list(c)].mean(axis=0) for c in m.cells])
    np.testing.assert_allclose(s["u_cell"], f(xK), rtol=0, atol=1e-12)
    for F in s["F_cell"]:
        assert abs(F.sum()) <= 1e-12 * max(1.0, np.abs(F).max())  # sum of the cell's fluxes vanishes


@pytest.mark.parametrize("kind", ["tet", "prism"])
def test_fracture_plane_normal_to_the_gradient(kind):
    """u = 1 - x with a fracture plane x = 1/2 (triangles or quadrangles),
    no-flow walls parallel to the gradient, isotropic matrix: exact, and no
    flow inside the fracture."""
    m = _general_mesh(kind, (4, 3, 3), 43, aniso=False, frac=True, dirichlet_all=False)
    assert len(m.frac) > 0 and all(len(f) == (3 if kind == "tet" else 4) for f in m.frac)
    s = gc.solve_darcy(m)
    np.testing.assert_allclose(s["u_node"], 1.0 - m.xyz[:, 0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(s["u_frac"], 0.5, rtol=0, atol=1e-12)
    assert np.abs(np.concatenate(s["F_frac"])).max() <= 1e-11


@pytest.mark.parametrize("kind", ["tet", "prism"])
def test_transport_mass_balance(kind):
    """M^{n+1} - M^n = -dt (flux into the Dirichlet nodes), c in [0, 1]."""
    m = _general_mesh(kind, (4, 3, 3), 44, aniso=True, frac=True, dirichlet_all=False)
    s = gc.solve_darcy(m)
    phi = gc.porous_volumes(m, s)
    dt = gc.cfl_dt(m, s, phi, 0.9)
    vol = np.concatenate([phi["phi_cell"], phi["phi_frac"], phi["phi_node"]])
    nc, nf = len(m.cells), len(m.frac)
    c = gc.transport(m, s, phi, dt, 0)
    for n in range(1, 12):
        cv = np.concatenate([c["c_cell"], c["c_frac"], c["c_node"]])
        out = 0.0
        for i, j, F in gc._edges(m, s):
            if j >= nc + nf and m.dirichlet[j - nc - nf]:
                out += cv[i] * max(F, 0.0) + cv[j] * min(F, 0.0)
        c2 = gc.transport(m, s, phi, dt, n)
        cv2 = np.concatenate([c2["c_cell"], c2["c_frac"], c2["c_node"]])
        assert abs(vol @ cv2 - vol @ cv + dt * out) <= 1e-12 * max(1.0, abs(vol @ cv))
        assert cv2.min() >= -1e-12 and cv2.max() <= 1 + 1e-12
        c = c2
