"""GPU parity of general cells (cells given by their faces): tetrahedra and
prisms (the cells of §5.4 and §5.5) and hexahedra, against the numpy oracle
of the scheme on general cells (oracle/general_cells.py), through the C-ABI.

- pressures (nodes, cells, fracture faces) relative L2 <= 1e-8 with the
  library solved to 1e-12 and the oracle solved directly;
- fluxes max-abs <= 1e-8 of the largest flux, compared per node (the
  library orders a cell's nodes by first appearance along its faces, the
  oracle by VTK order);
- porous volumes to 1e-13, the time step on identical fluxes to 1e-13;
- transport on the oracle's fluxes: concentrations max-abs <= 1e-12;
- affine pressures exact on a jittered anisotropic tetrahedral mesh;
- a hexahedral mesh given by its faces equals the hex8 path (system entry by
  entry with the fracture faces kept, pressures, fluxes, transport);
- Peaceman wells on the fracture faces of tetrahedral and prismatic meshes
  (§5.5): pressures, fluxes and well rates against the oracle, then the time
  step and transport on the oracle's fluxes and well rates.
Meshes are jittered, faces listed in random orientation and order per cell.
"""
import numpy as np
import pytest

import synth
from oracle import general_cells as gc

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_l2(a, b):
    a, b = np.asarray(a, float).ravel(), np.asarray(b, float).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_mesh(p):
    return gc.Mesh(p.xyz, p.cells, p.perm, p.poro, p.frac_faces(), p.frac_width, p.frac_perm, p.frac_poro,
                   p.dirichlet, p.p_bar, p.c_bar, p.mu, p.wells)


def flux_maps(p, sol):
    """Index maps between the library's flux layout and the oracle's lists."""
    cell_idx = []  # library flat index -> (cell, position in the oracle's F_cell[K])
    for K, c in enumerate(p.cells):
        for s in p.cell_node_order(K):
            cell_idx.append((K, list(c).index(s)))
    nv = [len(c) for c in p.cells]
    side_idx = []  # (face, side) -> (cell, position) or None
    for f, cs in enumerate(sol["frac_cells"]):
        for K in cs:
            if K < 0:
                side_idx.append(None)
                continue
            fr = [i for i in sol["cell_frac"][K] if i >= 0]
            side_idx.append((K, nv[K] + fr.index(f)))
    return cell_idx, side_idx


def oracle_fluxes_flat(p, sol):
    cell_idx, side_idx = flux_maps(p, sol)
    F_cell = np.array([sol["F_cell"][K][i] for K, i in cell_idx])
    F_cf = np.array([0.0 if t is None else sol["F_cell"][t[0]][t[1]] for t in side_idx]).reshape(-1, 2)
    F_frac = np.concatenate([np.asarray(v) for v in sol["F_frac"]]) if p.n_frac else np.zeros(0)
    return dict(F_cell=F_cell, F_cell_frac=F_cf, F_frac=F_frac)


def gpu(p, **opt):
    _torch()
    from paper_1602_03641_amd import vag
    opt.setdefault("rtol", 1e-12)
    opt.setdefault("max_iter", 20000)
    opt.setdefault("cfl", p.cfl)
    h = vag.Handle(p, **opt)
    info = h.solve_pressure()
    return h, info, vag


@pytest.mark.parametrize("kind,dims,seed", [("tet", (6, 5, 4), 1), ("prism", (7, 5, 4), 2), ("tet", (10, 9, 7), 3),
                                            ("prism", (11, 8, 6), 4), ("hex", (7, 6, 5), 5)])
@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_general_cells_parity(kind, dims, seed, precond):
    p = synth.general_problem(kind, dims, seed, frac_plane=dims[0] // 2, ratio=1e3)
    pc = {"jacobi": 0, "amg": 1}[precond]
    h, info, vag = gpu(p, precond=pc)
    print(f"{kind}{dims}: {p.n_cells} cells, {p.n_frac} fracture faces, {info['iterations']} iterations, "
          f"residual {info['rel_residual']:.2e}")
    assert info["status"] in (0, 1) and info["rel_residual"] <= 1e-11
    m = oracle_mesh(p)
    sol = gc.solve_darcy(m)
    g = vag.to_numpy(h.pressure())
    assert rel_l2(g["u_node"], sol["u_node"]) <= 1e-8
    assert rel_l2(g["u_cell"], sol["u_cell"]) <= 1e-8
    assert rel_l2(g["u_frac"], sol["u_frac"]) <= 1e-8
    of = oracle_fluxes_flat(p, sol)
    gf = vag.to_numpy(h.fluxes())
    scale = max(np.abs(of["F_cell"]).max(), np.abs(of["F_frac"]).max(initial=0.0))
    for k in ("F_cell", "F_cell_frac", "F_frac"):
        assert np.abs(gf[k] - of[k]).max(initial=0.0) <= 1e-8 * scale, k
    phi = gc.porous_volumes(m, sol)
    gphi = vag.to_numpy(h.porous_volumes())
    for k in ("phi_cell", "phi_frac", "phi_node"):
        np.testing.assert_allclose(gphi[k], phi[k], rtol=1e-13, atol=1e-18, err_msg=k)
    # transport on the oracle's fluxes
    h.set_fluxes(of)
    t = h.transport(n_steps=p.n_steps)
    dt = gc.cfl_dt(m, sol, phi, p.cfl)
    assert t["dt"] == pytest.approx(dt, rel=1e-13)
    oc = gc.transport(m, sol, phi, t["dt"], p.n_steps)
    gcn = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(gcn[k] - oc[k]).max(initial=0.0) <= 1e-12, k
    h.close()


@pytest.mark.parametrize("kind,dims,seed", [("tet", (8, 7, 6), 11), ("prism", (9, 7, 6), 12)])
def test_general_alpha_rule_parity(kind, dims, seed):
    """alpha_rule = 1 (§3.2.1, only the largest-permeability cells or fracture
    faces around a node give it a share) on lognormal tensors and fracture
    faces of two permeabilities: porous volumes to 1e-13 against the oracle's
    rule, then the time step and transport on the oracle's fluxes."""
    p = synth.general_problem(kind, dims, seed, frac_plane=dims[0] // 2, ratio=1e3)
    fy = np.array([p.xyz[list(p.face(f))][:, 1].mean() for f in p.frac_face_ids])
    p.frac_perm[fy > 0.5] *= 30.0
    h, info, vag = gpu(p, precond=1, alpha_rule=1)
    m = oracle_mesh(p)
    sol = gc.solve_darcy(m)
    phi = gc.porous_volumes(m, sol, alpha_rule=1)
    gphi = vag.to_numpy(h.porous_volumes())
    for k in ("phi_cell", "phi_frac", "phi_node"):
        np.testing.assert_allclose(gphi[k], phi[k], rtol=1e-13, atol=1e-18, err_msg=k)
    base = gc.porous_volumes(m, sol)
    assert np.abs(phi["phi_node"] - base["phi_node"]).max() > 1e-3 * np.abs(base["phi_node"]).max()
    h.set_fluxes(oracle_fluxes_flat(p, sol))
    t = h.transport(n_steps=p.n_steps)
    dt = gc.cfl_dt(m, sol, phi, p.cfl)
    assert t["dt"] == pytest.approx(dt, rel=1e-13)
    oc = gc.transport(m, sol, phi, t["dt"], p.n_steps)
    gcn = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(gcn[k] - oc[k]).max(initial=0.0) <= 1e-12, k
    h.close()


@pytest.mark.parametrize("kind", ["tet", "prism"])
def test_general_affine_exact(kind):
    """Affine Dirichlet data on every boundary node and a constant tensor:
    the scheme reproduces the affine function at nodes and cells."""
    p = synth.general_problem(kind, (6, 5, 5), 7, aniso_sigma=None, dirichlet="all")
    p.perm[:] = [2.0, 1.0, 0.5, 0.3, -0.2, 0.1]
    h, info, vag = gpu(p, rtol=1e-13, precond=1)
    g = vag.to_numpy(h.pressure())
    f = lambda y: 1.0 - y[..., 0] + 0.3 * y[..., 1] - 0.2 * y[..., 2]  # noqa: E731
    np.testing.assert_allclose(g["u_node"], f(p.xyz), rtol=0, atol=1e-10)
    xK = np.array([p.xyz[list(c)].mean(axis=0) for c in p.cells])
    np.testing.assert_allclose(g["u_cell"], f(xK), rtol=0, atol=1e-10)
    h.close()


def test_general_fracture_plane_no_flow_inside():
    """u = 1 - x with a fracture plane of triangles normal to the gradient:
    exact, u_sigma = 1/2 and no flow along the fracture."""
    p = synth.general_problem("tet", (6, 4, 4), 8, aniso_sigma=None, frac_plane=3, ratio=1e3, planar_x=True)
    h, info, vag = gpu(p, rtol=1e-13, precond=1)
    g = vag.to_numpy(h.pressure())
    np.testing.assert_allclose(g["u_node"], 1.0 - p.xyz[:, 0], rtol=0, atol=1e-10)
    np.testing.assert_allclose(g["u_frac"], 0.5, rtol=0, atol=1e-10)
    assert np.abs(vag.to_numpy(h.fluxes())["F_frac"]).max() <= 1e-9
    h.close()


def test_hex_faces_equal_hex8_path():
    """A hexahedral problem given by its faces (shuffled, random orientation)
    goes through the general path; it must agree with the hex8 path with the
    fracture faces kept: the assembled system entry by entry, pressures,
    fluxes per node, porous volumes and transport on identical fluxes."""
    _torch()
    from paper_1602_03641_amd import vag
    p = synth.random_problem((9, 7, 6), 21, n_patches=5, n_steps=30)
    q = synth.general_from_hex(p, seed=3)
    h8 = vag.Handle(p, rtol=1e-13, max_iter=20000, precond=1, eliminate_frac_faces=0)
    hg = vag.Handle(q, rtol=1e-13, max_iter=20000, precond=1)
    i8, ig = h8.solve_pressure(), hg.solve_pressure()
    assert i8["n_unknowns"] == ig["n_unknowns"] and i8["nnz"] == ig["nnz"]
    rp8, c8, v8, b8 = h8.system()
    rpg, cg, vg, bg = hg.system()
    np.testing.assert_array_equal(rp8, rpg)
    np.testing.assert_array_equal(c8, cg)
    np.testing.assert_allclose(vg, v8, rtol=1e-12, atol=1e-14 * np.abs(v8).max())
    np.testing.assert_allclose(bg, b8, rtol=1e-12, atol=1e-14 * np.abs(b8).max())
    a, b = vag.to_numpy(h8.pressure()), vag.to_numpy(hg.pressure())
    for k in ("u_node", "u_cell", "u_frac"):
        assert rel_l2(b[k], a[k]) <= 1e-9, k
    f8, fg = vag.to_numpy(h8.fluxes()), vag.to_numpy(hg.fluxes())
    idx = [(K, list(q.cells[K]).index(s)) for K in range(q.n_cells) for s in q.cell_node_order(K)]
    f8_flat = np.array([f8["F_cell"][K, i] for K, i in idx])
    scale = np.abs(f8["F_cell"]).max()
    assert np.abs(fg["F_cell"] - f8_flat).max() <= 1e-8 * scale
    assert np.abs(fg["F_cell_frac"] - f8["F_cell_frac"]).max() <= 1e-8 * scale
    # the face list may list a fracture face reversed: compare per node
    for f in range(q.n_frac):
        order = [list(p.frac_nodes[f]).index(s) for s in q.face(q.frac_face_ids[f])]
        np.testing.assert_allclose(fg["F_frac"][4 * f:4 * f + 4], f8["F_frac"][f][order], rtol=0,
                                   atol=1e-8 * scale)
    p8, pg = vag.to_numpy(h8.porous_volumes()), vag.to_numpy(hg.porous_volumes())
    for k in p8:
        np.testing.assert_allclose(pg[k], p8[k], rtol=1e-13, atol=1e-18, err_msg=k)
    # transport on the hex8 path's fluxes
    hg.set_fluxes(dict(F_cell=f8_flat, F_cell_frac=f8["F_cell_frac"],
                       F_frac=np.concatenate([f8["F_frac"][f][[list(p.frac_nodes[f]).index(s)
                                                                for s in q.face(q.frac_face_ids[f])]]
                                              for f in range(q.n_frac)])))
    t8, tg = h8.transport(n_steps=30), hg.transport(n_steps=30)
    assert tg["dt"] == pytest.approx(t8["dt"], rel=1e-13)
    c8, cg_ = vag.to_numpy(h8.concentration()), vag.to_numpy(hg.concentration())
    for k in c8:
        assert np.abs(cg_[k] - c8[k]).max() <= 1e-12, k
    h8.close()
    hg.close()


@pytest.mark.parametrize("kind,dims,seed", [("prism", (10, 8, 6), 21), ("tet", (8, 7, 6), 22)])
@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_general_wells_parity(kind, dims, seed, precond):
    """Two rate injectors and two pressure wells on a fracture plane of a
    jittered anisotropic mesh."""
    p = synth.add_wells(synth.general_problem(kind, dims, seed, frac_plane=dims[0] // 2, ratio=1e3, n_steps=40),
                        seed, n_inj=2, n_prod=2)
    h, info, vag = gpu(p, precond={"jacobi": 0, "amg": 1}[precond])
    print(f"{kind}{dims} wells: {p.n_cells} cells, {p.n_frac} fracture faces, {info['iterations']} iterations")
    assert info["status"] in (0, 1) and info["rel_residual"] <= 1e-11
    m = oracle_mesh(p)
    assert len(m.well_face) == 4
    sol = gc.solve_darcy(m)
    g = vag.to_numpy(h.pressure())
    for k in ("u_node", "u_cell", "u_frac"):
        assert rel_l2(g[k], sol[k]) <= 1e-8, k
    Q, Qo = h.well_rates(), sol["well_rate"]
    assert np.abs(Q - Qo).max() <= 1e-8 * np.abs(Qo).max()
    assert np.all(Qo[:2] > 0) and np.all(Qo[2:] < 0)  # the producers produce
    of = oracle_fluxes_flat(p, sol)
    gf = vag.to_numpy(h.fluxes())
    scale = max(np.abs(of["F_cell"]).max(), np.abs(of["F_frac"]).max(initial=0.0))
    for k in ("F_cell", "F_cell_frac", "F_frac"):
        assert np.abs(gf[k] - of[k]).max(initial=0.0) <= 1e-8 * scale, k
    phi = gc.porous_volumes(m, sol)
    t0 = h.transport(n_steps=0)
    assert t0["dt"] == pytest.approx(gc.cfl_dt(m, sol, phi, p.cfl), rel=1e-8)
    # transport on the oracle's fluxes and well rates
    h.set_fluxes(of)
    h.set_well_rates(Qo)
    np.testing.assert_array_equal(h.well_rates(), Qo)
    t = h.transport(n_steps=p.n_steps)
    assert t["dt"] == pytest.approx(gc.cfl_dt(m, sol, phi, p.cfl), rel=1e-13)
    oc = gc.transport(m, sol, phi, t["dt"], p.n_steps)
    gcn = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(gcn[k] - oc[k]).max(initial=0.0) <= 1e-12, k
    assert gcn["c_frac"][p.wells["face"][0]] > 0.05  # the injected tracer arrived
    h.close()


def test_general_noalloc_unsupported():
    h, info, vag = gpu(synth.general_problem("tet", (3, 3, 3), 9, frac_plane=1))
    with pytest.raises(vag.VagError) as e:
        h.transport_noalloc(n_steps=2)
    assert e.value.status == vag.VAG_ERR_UNSUPPORTED
    h.close()
