"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle.

Tolerances (FP64 path):
- pressures relative L2 <= 1e-8 with both sides solved to a relative residual
  of 1e-12..1e-13; fluxes max-abs <= 1e-6 of the largest flux;
- the assembled system entry by entry (same unknown order): 1e-12 relative,
  only the summation order differs;
- transport on identical fluxes (the oracle's, passed to the library with
  vag_set_fluxes): concentrations max-abs <= 1e-12;
- end to end, concentrations max-abs <= 1e-10 when the two pressure solutions
  agree to 1e-12; with high contrast the solver error (condition number times
  residual) can exceed that, and the bar grows in proportion:
  1e-10 * max(1, pressure agreement / 1e-12).
"""
import numpy as np
import pytest

import oracle
import synth

import schur_ref

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def reached(info, bound=1e-12):
    """Requests of rtol 1e-13 stop at the FP64 rounding floor of the true
    residual (reported as VAG_WARN_NOT_CONVERGED when it lies above 1e-13);
    parity needs the residual below `bound`."""
    return info["status"] in (0, 1) and info["rel_residual"] <= bound


def residual_floor(p, o):
    """eps || |A| |x| || / ||b|| for the oracle's system and solution: the size
    of the rounding error of one FP64 product A x relative to b, below which
    no FP64 solver's residual can be expected to fall (at permeability
    contrast 1e6 it reaches 1e-11)."""
    A, b = oracle.system(p)
    free = p.dirichlet == 0
    x = np.concatenate([o["darcy"]["u_node"][free], o["darcy"]["u_frac"]])
    return float(np.finfo(float).eps * np.linalg.norm(abs(A) @ np.abs(x)) / np.linalg.norm(b))


def rel_l2(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_run(p, n_steps=None, t_final=None, **opt):
    _torch()
    from paper_1602_03641_amd import vag
    opt.setdefault("cfl", p.cfl)
    h = vag.Handle(p, **opt)
    info = h.solve_pressure()
    out = dict(info=info, **vag.to_numpy(h.pressure()), **vag.to_numpy(h.fluxes()),
               **vag.to_numpy(h.porous_volumes()))
    n_steps = p.n_steps if n_steps is None else n_steps
    t_final = p.t_final if t_final is None else t_final
    if n_steps or t_final:
        out["tinfo"] = h.transport(n_steps=n_steps, t_final=t_final)
        out.update(vag.to_numpy(h.concentration()))
    out["handle"] = h
    return out


def flux_err(a, b, scale):
    """max |a - b| relative to the global flux scale (fluxes may vanish exactly)."""
    a = np.asarray(a, float)
    return float(np.abs(a - b).max() / scale) if a.size else 0.0


def compare(p, g, o, c_tol=1e-10, p_tol=1e-8, flux_tol=None):
    d = o["darcy"]
    flux_tol = 1e2 * p_tol if flux_tol is None else flux_tol
    p_err = rel_l2(g["u_node"], d["u_node"])
    c_tol = c_tol * max(1.0, p_err / 1e-12)
    assert p_err <= p_tol
    assert rel_l2(g["u_cell"], d["u_cell"]) <= p_tol
    # element by element as well: a rel-L2 bound alone lets one unknown of a
    # large vector be off by sqrt(n) times the bound
    pscale = np.abs(d["u_node"]).max()
    for k in ("u_node", "u_cell") + (("u_frac",) if p.n_frac else ()):
        assert np.abs(g[k] - d[k]).max() <= 10 * p_tol * pscale, k
    scale = max(np.abs(d["F_cell"]).max(), np.abs(d["F_frac"]).max() if p.n_frac else 0.0)
    assert flux_err(g["F_cell"], d["F_cell"], scale) <= flux_tol
    if p.n_frac:
        assert rel_l2(g["u_frac"], d["u_frac"]) <= p_tol
        assert flux_err(g["F_frac"], d["F_frac"], scale) <= flux_tol
        assert flux_err(g["F_cell_frac"], d["F_cell_frac"], scale) <= flux_tol
    for k in ("phi_cell", "phi_frac", "phi_node"):
        assert rel_l2(g[k], o["phi"][k]) <= 1e-13
    if "c_cell" in g:
        assert g["tinfo"]["n_steps"] == o["n_steps"]
        assert g["tinfo"]["dt"] == pytest.approx(o["dt"], rel=1e-9)
        for k in ("c_cell", "c_frac", "c_node"):
            if g[k].size:
                assert np.abs(g[k] - o[k]).max() <= c_tol, k


def test_config1_parity():
    p = synth.config1()
    g = gpu_run(p, rtol=1e-13, max_iter=5000)
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"])
    assert g["info"]["rel_residual"] <= 1e-12
    compare(p, g, o)
    # exact linear solution of config 1
    np.testing.assert_allclose(g["u_node"], 1 - p.xyz[:, 0], atol=1e-11)
    np.testing.assert_allclose(g["u_frac"], 0.5, atol=1e-11)


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_alpha_rule_parity(precond):
    """The largest-permeability rule of §3.2.1 (alpha_rule = 1) on a jittered
    mesh with lognormal tensors (every node between rock types) and fracture
    patches of contrasts 1e2..1e6: porous volumes to 1e-13 against the
    oracle's rule, then the time step and transport end to end; with the
    rule off, the library's volumes differ (the rule is really applied)."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((13, 11, 9), 23, n_patches=10, n_steps=40)
    pc = {"jacobi": vag.VAG_PC_JACOBI, "amg": vag.VAG_PC_AMG}[precond]
    g = gpu_run(p, rtol=1e-13, max_iter=20000, precond=pc, alpha_rule=1)
    o = oracle.run(p, rtol=1e-13, alpha_rule=1)
    for k in ("phi_cell", "phi_frac", "phi_node"):
        np.testing.assert_allclose(g[k], o["phi"][k], rtol=1e-13, atol=1e-18, err_msg=k)
    compare(p, g, o)
    base = oracle.porous_volumes(p, 0)
    assert np.abs(g["phi_node"] - base["phi_node"]).max() > 1e-3 * np.abs(base["phi_node"]).max()


def test_config1_system_entries():
    """With the fracture faces kept, the assembled cell-eliminated system equals
    the oracle's entry by entry (same pattern, same unknown order)."""
    p = synth.config1()
    g = gpu_run(p, n_steps=0, eliminate_frac_faces=0)
    rp, col, val, b = g["handle"].system()
    A, bo = oracle.system(p)
    np.testing.assert_array_equal(rp, A.indptr)
    np.testing.assert_array_equal(col, A.indices)
    scale = np.abs(A.data).max()
    assert np.abs(val - A.data).max() <= 1e-13 * scale
    assert np.abs(b - bo).max() <= 1e-13 * max(np.abs(bo).max(), 1e-300)


def check_eliminated_system(p, g):
    """The library's face-eliminated system equals the dense elimination of the
    oracle's system (tests/schur_ref.py)."""
    rp, col, val, b = g["handle"].system()
    A, bo = oracle.system(p)
    n_free = int((p.dirichlet == 0).sum())
    S, bs, kept, elim = schur_ref.eliminate(A, bo, n_free)
    n = len(kept)
    assert len(rp) == n + 1
    G = schur_ref.csr_to_dense(rp, col, val, n)
    scale = np.abs(S).max()
    assert np.abs(G - S).max() <= 1e-12 * scale
    assert np.abs(b - bs).max() <= 1e-12 * max(np.abs(bs).max(), 1e-300)
    return len(elim)


def test_config1_system_eliminated():
    """Every fracture face of config 1 is its own group and is eliminated."""
    p = synth.config1()
    g = gpu_run(p, n_steps=0)
    assert check_eliminated_system(p, g) == p.n_frac
    assert g["info"]["n_unknowns"] == int((p.dirichlet == 0).sum())


@pytest.mark.parametrize("dims,seed,patches", [((9, 7, 5), 1, 4), ((6, 11, 4), 2, 6), ((13, 5, 6), 3, 8),
                                               ((5, 5, 5), 4, 12)])
def test_random_parity(dims, seed, patches):
    """Jittered cells, full anisotropic tensors, random fracture patches with
    contrasts 1e2..1e6 (intersections, boundary fractures); several blocks of
    each kernel plus a ragged tail."""
    p = synth.random_problem(dims, seed, n_patches=patches, n_steps=30)
    g = gpu_run(p, rtol=1e-13, max_iter=20000)
    o = oracle.run(p, rtol=1e-13)
    check_eliminated_system(p, g)
    compare(p, g, o)


def test_random_parity_faces_kept():
    """The faces-kept route: system entry by entry and results."""
    p = synth.random_problem((9, 7, 5), 1, n_patches=6, n_steps=30)
    g = gpu_run(p, rtol=1e-13, max_iter=20000, eliminate_frac_faces=0)
    o = oracle.run(p, rtol=1e-13)
    rp, col, val, b = g["handle"].system()
    A, bo = oracle.system(p)
    np.testing.assert_array_equal(col, A.indices)
    assert np.abs(val - A.data).max() <= 1e-12 * np.abs(A.data).max()
    compare(p, g, o)


def stacked_problem():
    """A chain of 39 fracture faces through consecutive cells (too large a
    group: its faces stay unknowns), three intersecting planes (groups of 4
    along the intersection lines, a larger group at the triple point) and
    boundary fractures, on a jittered anisotropic 40x7x6 box."""
    planes = [(0, x, 2, 3, 2, 3) for x in range(1, 40)]
    planes += [(0, 20, 3, 7, 3, 6), (1, 5, 15, 25, 0, 6), (2, 4, 15, 25, 3, 7), (1, 0, 30, 36, 1, 5)]
    return synth.planes_problem((40, 7, 6), planes, ratio=1e4, jitter=0.2, aniso_sigma=1.0, seed=11,
                                name="stacked", rtol=1e-13, cfl=0.9, n_steps=30)


def test_stacked_groups_parity():
    p = stacked_problem()
    g = gpu_run(p, rtol=1e-13, max_iter=20000)
    o = oracle.run(p, rtol=1e-13)
    A, _ = oracle.system(p)
    n_free = int((p.dirichlet == 0).sum())
    sizes = sorted(len(f) for f, _ in schur_ref.face_groups(A, n_free))
    assert sizes[-1] == 39 and 4 in sizes and sizes[-2] > 4
    n_elim = check_eliminated_system(p, g)
    assert 0 < n_elim < p.n_frac
    compare(p, g, o)


def test_eliminated_equals_kept():
    """Both routes give the same discrete solution."""
    p = synth.random_problem((8, 6, 5), 5, n_patches=10, n_steps=20)
    a = gpu_run(p, rtol=1e-13, max_iter=20000)
    b = gpu_run(p, rtol=1e-13, max_iter=20000, eliminate_frac_faces=0)
    assert a["info"]["n_unknowns"] < b["info"]["n_unknowns"]
    for k in ("u_node", "u_cell", "u_frac"):
        assert rel_l2(a[k], b[k]) <= 1e-10, k
    scale = np.abs(b["F_cell"]).max()
    for k in ("F_cell", "F_frac", "F_cell_frac"):
        assert flux_err(a[k], b[k], scale) <= 1e-8, k


def test_e1_time_grid_parity():
    """§5.1 case: final time reached with a shortened last step."""
    p = synth.e1_problem(32)
    g = gpu_run(p, rtol=1e-13, max_iter=20000)
    o = oracle.run(p, rtol=1e-13)
    assert g["tinfo"]["last_dt"] == pytest.approx(o["last_dt"], rel=1e-8)
    compare(p, g, o)


def test_config2_full_size():
    """The benchmark workload (64^3, four clipped fractures, contrast 1e4)."""
    p = synth.config2()
    g = gpu_run(p, rtol=1e-13, max_iter=20000)
    o = oracle.run(p, rtol=1e-12)
    print(f"config2 Jacobi-CG: {g['info']['iterations']} iterations, residual {g['info']['rel_residual']:.2e}")
    assert reached(g["info"], 1e-11)  # 266k unknowns at contrast 1e4: the FP64 floor lies near 1e-12
    compare(p, g, o, p_tol=1e-8, c_tol=1e-10)


def test_determinism_bitwise():
    """Row-gathered assembly (one thread per row, fixed order) and fixed-shape
    reductions: two runs agree bit for bit."""
    p = synth.random_problem((8, 6, 7), 9, n_patches=5, n_steps=20)
    a = gpu_run(p, rtol=1e-13)
    b = gpu_run(p, rtol=1e-13)
    for k in ("u_node", "u_cell", "u_frac", "F_cell", "F_frac", "c_cell", "c_node", "c_frac"):
        np.testing.assert_array_equal(a[k], b[k])


def test_not_converged_warning():
    from paper_1602_03641_amd import vag
    _torch()
    h = vag.Handle(synth.config1(), rtol=1e-14, max_iter=2, check_every=1)
    info = h.solve_pressure()
    assert info["status"] == vag.VAG_WARN_NOT_CONVERGED
    assert info["iterations"] == 2


def test_inverted_cell_reported():
    from paper_1602_03641_amd import vag
    _torch()
    p = synth.cartesian_problem(3)
    p.hex8 = p.hex8[:, [4, 5, 6, 7, 0, 1, 2, 3]].copy()  # cell 0..: top and bottom swapped
    p.hex8[1:] = synth.cartesian_problem(3).hex8[1:]
    h = vag.Handle(p)
    with pytest.raises(vag.VagError) as e:
        h.solve_pressure()
    assert e.value.status == vag.VAG_ERR_MESH and "cell 0" in str(e.value)


@pytest.mark.parametrize("what", ["negative", "indefinite", "nan", "frac_perm", "frac_width"])
def test_invalid_coefficients_rejected(what):
    """A permeability tensor that is not symmetric positive definite (a
    negative diagonal, positive diagonals with a leading 2x2 minor below zero,
    a NaN), or a fracture face with zero permeability or negative width:
    vag_solve_pressure names the first offending cell or face."""
    from paper_1602_03641_amd import vag
    _torch()
    p = synth.random_problem((6, 5, 5), 36, n_patches=3, n_steps=0)
    p.perm = p.perm.copy()
    if what == "negative":
        p.perm[7, 1] = -1.0
    elif what == "indefinite":
        p.perm[7, :] = [1.0, 1.0, 1.0, 2.0, 0.0, 0.0]   # xx yy - xy^2 = -3
    elif what == "nan":
        p.perm[7, 5] = np.nan
    elif what == "frac_perm":
        p.frac_perm = p.frac_perm.copy()
        p.frac_perm[2] = 0.0
    else:
        p.frac_width = p.frac_width.copy()
        p.frac_width[2] = -0.01
    h = vag.Handle(p)
    with pytest.raises(vag.VagError) as e:
        h.solve_pressure()
    assert e.value.status == vag.VAG_ERR_ARG
    assert ("cell 7:" if what in ("negative", "indefinite", "nan") else "fracture face 2:") in str(e.value)
    h.close()


def test_free_node_of_no_cell_rejected():
    """A node that no cell names and no Dirichlet flag fixes has an empty
    conservation equation: vag_create reports it as a mesh error."""
    from paper_1602_03641_amd import vag
    _torch()
    p = synth.cartesian_problem(2)
    p.xyz = np.vstack([p.xyz, [[2.0, 2.0, 2.0]]])
    for k in ("dirichlet", "p_bar", "c_bar"):
        setattr(p, k, np.append(getattr(p, k), 0))
    with pytest.raises(vag.VagError) as e:
        vag.Handle(p)
    assert e.value.status == vag.VAG_ERR_MESH and "no cell" in str(e.value)


def test_transport_before_solve():
    from paper_1602_03641_amd import vag
    _torch()
    h = vag.Handle(synth.config1())
    with pytest.raises(vag.VagError) as e:
        h.transport(n_steps=1)
    assert e.value.status == vag.VAG_ERR_STATE


def test_tiny_meshes():
    """Degenerate sizes: one cell (every node Dirichlet), and two cells split
    by one fracture face whose nodes are all free except the x-walls."""
    p = synth.cartesian_problem(1, n_steps=3)
    g = gpu_run(p)
    o = oracle.run(p)
    compare(p, g, o)
    p = synth.cartesian_problem(2, planes=[(0, 1, 0, 2, 0, 2)], ratio=1e6, n_steps=5)
    g = gpu_run(p, rtol=1e-13)
    o = oracle.run(p, rtol=1e-13)
    compare(p, g, o)


def test_continue_and_restart_transport():
    """Transport in two calls equals one call; passing c0 restarts from it."""
    from paper_1602_03641_amd import vag
    _torch()
    p = synth.random_problem((6, 5, 4), 5, n_patches=3)
    h = vag.Handle(p, rtol=1e-12)
    h.solve_pressure()
    h.transport(n_steps=10)
    mid = vag.to_numpy(h.concentration())
    h.transport(n_steps=15)
    a = vag.to_numpy(h.concentration())
    h.transport(n_steps=15, c0=mid)
    b = vag.to_numpy(h.concentration())
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


# ---------------------------------------------------------------------------
# aggregation AMG preconditioner
# ---------------------------------------------------------------------------
def _amg():
    from paper_1602_03641_amd import vag
    return dict(precond=vag.VAG_PC_AMG)


def test_amg_config1_parity():
    p = synth.config1()
    g = gpu_run(p, rtol=1e-13, max_iter=2000, **_amg())
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"]) and g["info"]["amg_levels"] >= 2
    compare(p, g, o)


@pytest.mark.parametrize("dims,seed,patches", [((17, 13, 11), 1, 6), ((12, 20, 9), 2, 10), ((16, 16, 16), 3, 14)])
def test_amg_random_parity(dims, seed, patches):
    """Jittered, anisotropic, contrasts up to 1e6: AMG-CG reaches the oracle's solution."""
    p = synth.random_problem(dims, seed, n_patches=patches, n_steps=20)
    g = gpu_run(p, rtol=1e-13, max_iter=5000, **_amg())
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"], max(1e-12, residual_floor(p, o)))
    compare(p, g, o)


def test_amg_config2_full_size():
    """AMG-CG on the benchmark workload: oracle parity, far fewer iterations
    than Jacobi, small operator complexity, bitwise reproducible."""
    p = synth.config2()
    g = gpu_run(p, rtol=1e-13, max_iter=2000, **_amg())
    o = oracle.run(p, rtol=1e-12)
    info = g["info"]
    print("amg config2:", {k: info[k] for k in ("iterations", "amg_levels", "amg_operator_complexity",
                                                "ms_setup", "ms_solve")})
    assert reached(info, 1e-11)  # FP64 floor of the 266k-unknown system lies near 1e-12
    assert info["iterations"] < 200
    assert info["amg_operator_complexity"] < 2.0
    compare(p, g, o)
    g2 = gpu_run(p, rtol=1e-13, max_iter=2000, **_amg())
    np.testing.assert_array_equal(g["u_node"], g2["u_node"])
    np.testing.assert_array_equal(g["c_cell"], g2["c_cell"])


# ---------------------------------------------------------------------------
# mixed precision: FP32 AMG + FP32 inner CG under FP64 iterative refinement
# ---------------------------------------------------------------------------
def _mixed(ir=False, **kw):
    from paper_1602_03641_amd import vag
    return dict(precond=vag.VAG_PC_AMG, precision=vag.VAG_MIXED_IR if ir else vag.VAG_MIXED, **kw)


@pytest.mark.parametrize("name", ["config1", "random"])
@pytest.mark.parametrize("ir", [False, True])
def test_mixed_reaches_fp64_parity(name, ir):
    """FP32 hierarchy (and, with refinement, FP32 inner CG): the FP64 residual
    still reaches the tolerance and the solution meets the FP64 parity bar.
    On the 1e6-contrast mesh the attainable FP64 residual is about 1e-11
    (||A|| ||x|| eps / ||b||), so that case is solved to 1e-10."""
    p = synth.config1() if name == "config1" else synth.random_problem((14, 12, 10), 6, n_patches=8, n_steps=20)
    rtol = 1e-12 if name == "config1" else 1e-10
    g = gpu_run(p, rtol=rtol, inner_rtol=1e-3, max_iter=5000, **_mixed(ir))
    o = oracle.run(p, rtol=1e-13)
    info = g["info"]
    assert info["status"] == 0 and info["rel_residual"] <= rtol
    if ir:
        assert info["outer_iterations"] >= 2
    compare(p, g, o)


def test_mixed_same_iterations_as_fp64():
    """An FP32 V-cycle preconditions FP64 CG as well as the FP64 V-cycle."""
    p = synth.config2()
    a = gpu_run(p, rtol=1e-8, max_iter=2000, n_steps=0, **_amg())["info"]
    b = gpu_run(p, rtol=1e-8, max_iter=2000, n_steps=0, **_mixed())["info"]
    print("fp64 vs mixed iterations:", a["iterations"], b["iterations"])
    assert b["iterations"] <= a["iterations"] + 3


def test_mixed_config2_error_stated():
    """Benchmark tolerance (1e-8): the FP64 residual meets it and the error
    against the FP64 oracle is reported per result.  The pressures meet the
    1e-8 relative-L2 bar (measured: about 3e-10), and the concentrations the
    scaled bar of compare() (1e-10 times the pressure gap over 1e-12)."""
    p = synth.config2()
    g = gpu_run(p, rtol=1e-8, max_iter=2000, **_mixed())
    o = oracle.run(p, rtol=1e-12)
    info = g["info"]
    e_p = rel_l2(g["u_node"], o["darcy"]["u_node"])
    e_c = max(np.abs(g[k] - o[k]).max() for k in ("c_cell", "c_frac", "c_node"))
    print(f"mixed config2: inner={info['iterations']} outer={info['outer_iterations']} "
          f"res={info['rel_residual']:.2e} pressure relL2={e_p:.2e} conc maxabs={e_c:.2e}")
    assert info["status"] == 0 and info["rel_residual"] <= 1e-8
    assert e_p <= 1e-8
    assert e_c <= 1e-10 * max(1.0, e_p / 1e-12)


@pytest.mark.parametrize("kind", ["random_1e6", "config2"])
def test_transport_parity_identical_fluxes(kind):
    """Explicit upwind steps from the same fluxes: only rounding differs."""
    from paper_1602_03641_amd import vag
    _torch()
    p = (synth.random_problem((13, 11, 9), 21, n_patches=10, n_steps=60) if kind == "random_1e6"
         else synth.config2())
    od = oracle.solve_darcy(p, rtol=1e-10)
    phi = oracle.porous_volumes(p)
    dt = p.cfl * float(np.min(oracle.cfl_bounds(p, od, phi)))
    oc = oracle.transport(p, od, phi, dt, p.n_steps)
    h = vag.Handle(p, cfl=p.cfl)
    h.set_fluxes(od)
    gphi = vag.to_numpy(h.porous_volumes())
    for k in ("phi_cell", "phi_frac", "phi_node"):
        assert rel_l2(gphi[k], phi[k]) <= 1e-13
    t = h.transport(n_steps=p.n_steps)
    assert t["dt"] == pytest.approx(dt, rel=1e-12)
    gc = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(gc[k] - oc[k]).max() <= 1e-12, k


# ---------------------------------------------------------------------------
# GMRES(m) with CGS2 (right preconditioning)
# ---------------------------------------------------------------------------
def _gmres(**kw):
    from paper_1602_03641_amd import vag
    return dict(krylov=vag.VAG_GMRES, **kw)


@pytest.mark.parametrize("precond,precision", [("jacobi", "fp64"), ("amg", "fp64"), ("amg", "mixed")])
def test_gmres_parity(precond, precision):
    from paper_1602_03641_amd import vag
    p = synth.random_problem((10, 8, 7), 8, n_patches=6, n_steps=20)
    pc = vag.VAG_PC_JACOBI if precond == "jacobi" else vag.VAG_PC_AMG
    pr = vag.VAG_FP64 if precision == "fp64" else vag.VAG_MIXED
    g = gpu_run(p, rtol=1e-12, max_iter=20000, gmres_restart=100, precond=pc, precision=pr, **_gmres())
    o = oracle.run(p, rtol=1e-13)
    assert g["info"]["status"] == 0 and g["info"]["rel_residual"] <= 1e-12
    compare(p, g, o)


def test_gmres_short_restart():
    """GMRES(5): many restarts, same solution (a small coarsest level keeps
    the AMG preconditioner inexact on this small mesh)."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((9, 7, 6), 9, n_patches=4, n_steps=10)
    g = gpu_run(p, rtol=1e-12, max_iter=20000, gmres_restart=5, precond=vag.VAG_PC_AMG, amg_coarse_size=16,
                **_gmres())
    o = oracle.run(p, rtol=1e-13)
    assert g["info"]["status"] == 0 and g["info"]["iterations"] > 5
    compare(p, g, o)


def oracle_certificate(p, g):
    """||b - A x|| / ||b|| of the library's pressures in the oracle's own
    cell-eliminated system (free nodes, every fracture face), in FP64."""
    A, b = oracle.system(p)
    free = p.dirichlet == 0
    x = np.concatenate([g["u_node"][free], g["u_frac"]])
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))


def test_gmres_refinement_fp32_inner():
    """FP64 refinement around FP32 GMRES with the FP32 hierarchy (the mixed
    scheme of the 128^3 workload, to its tolerance 1e-8), on a scaled-down
    instance of its generator: the oracle's own system certifies the result."""
    from paper_1602_03641_amd import vag
    p = synth.config3(n=20, n_patches=10)
    g = gpu_run(p, n_steps=0, rtol=1e-8, inner_rtol=1e-2, max_iter=20000, gmres_restart=60,
                precond=vag.VAG_PC_AMG, precision=vag.VAG_MIXED_IR, **_gmres())
    info = g["info"]
    print(f"gmres ir: {info}")
    assert info["status"] == 0 and info["rel_residual"] <= 1e-8 and info["outer_iterations"] >= 2
    assert oracle_certificate(p, g) <= 1.5e-8


def test_gmres_matches_cg():
    from paper_1602_03641_amd import vag
    p = synth.random_problem((12, 9, 8), 10, n_patches=7, n_steps=0)
    a = gpu_run(p, rtol=1e-11, max_iter=20000, precond=vag.VAG_PC_AMG)
    b = gpu_run(p, rtol=1e-11, max_iter=20000, precond=vag.VAG_PC_AMG, **_gmres())
    assert a["info"]["status"] == 0 and b["info"]["status"] == 0
    # both solve the oracle's own system to the tolerance; at contrast 1e6 the
    # two iterates differ by up to condition number x residual
    assert oracle_certificate(p, a) <= 2e-11 and oracle_certificate(p, b) <= 2e-11
    assert rel_l2(a["u_node"], b["u_node"]) <= 1e-6


# ---------------------------------------------------------------------------
# BiCGStab (right preconditioning, device-resident scalars)
# ---------------------------------------------------------------------------
def _bicgstab(**kw):
    from paper_1602_03641_amd import vag
    return dict(krylov=vag.VAG_BICGSTAB, **kw)


@pytest.mark.parametrize("precond,precision", [("jacobi", "fp64"), ("amg", "fp64"), ("amg", "mixed")])
def test_bicgstab_parity(precond, precision):
    """Jittered anisotropic mesh, contrasts up to 1e6: the oracle's solution."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((10, 8, 7), 8, n_patches=6, n_steps=20)
    pc = vag.VAG_PC_JACOBI if precond == "jacobi" else vag.VAG_PC_AMG
    pr = vag.VAG_FP64 if precision == "fp64" else vag.VAG_MIXED
    g = gpu_run(p, rtol=1e-12, max_iter=20000, precond=pc, precision=pr, **_bicgstab())
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"], max(1e-12, residual_floor(p, o)))
    compare(p, g, o)


def test_bicgstab_config1_and_rejects_ir():
    from paper_1602_03641_amd import vag
    p = synth.config1()
    g = gpu_run(p, rtol=1e-13, max_iter=5000, precond=vag.VAG_PC_AMG, **_bicgstab())
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"])
    compare(p, g, o)
    with pytest.raises(vag.VagError) as e:
        vag.Handle(p, precision=vag.VAG_MIXED_IR, **_bicgstab())
    assert e.value.status == vag.VAG_ERR_UNSUPPORTED


def test_bicgstab_matches_cg():
    """Both Krylov methods solve the oracle's own system to the tolerance."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((12, 9, 8), 10, n_patches=7, n_steps=0)
    a = gpu_run(p, rtol=1e-11, max_iter=20000, precond=vag.VAG_PC_AMG)
    b = gpu_run(p, rtol=1e-11, max_iter=20000, precond=vag.VAG_PC_AMG, **_bicgstab())
    assert a["info"]["status"] == 0 and b["info"]["status"] == 0
    assert oracle_certificate(p, a) <= 2e-11 and oracle_certificate(p, b) <= 2e-11
    assert rel_l2(a["u_node"], b["u_node"]) <= 1e-6
    # two preconditioned products per BiCGStab iteration against one for CG
    print(f"iterations: CG {a['info']['iterations']}, BiCGStab {b['info']['iterations']}")


# ---------------------------------------------------------------------------
# Scaled-down instances of the 128^3 and 192^3 generators (jitter, full
# anisotropic tensors, many patches, contrasts up to 1e6): full parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gen,kw,rtol", [("config3", dict(n=24, n_patches=10), 1e-12),
                                         ("config5", dict(n=24, n_patches=25), 1e-10),
                                         ("config5", dict(n=32, n_patches=40), 1e-10)])
def test_scaled_workload_parity(gen, kw, rtol):
    """Pressures, fluxes and porous volumes end to end; concentrations on the
    oracle's own fluxes (at contrast 1e6 with small fracture control volumes
    the end-to-end concentration gap is the flux gap amplified by dt/phi over
    the steps, so the 1e-10 bar is checked where the fluxes are identical).
    With every fracture at contrast 1e6 the attainable FP64 residual is about
    1e-11 (||A|| ||x|| eps / ||b||), so those instances are solved to 1e-10, and
    a fracture flux is the face-node pressure gap times a transmissibility 1e4
    times the matrix one: the flux gap between two solutions at residual 1e-10
    reaches 1e-5 of the flux scale, while conservation holds to rounding."""
    from paper_1602_03641_amd import vag
    p = getattr(synth, gen)(**kw)
    p.n_steps = 20
    g = gpu_run(p, n_steps=0, rtol=rtol, max_iter=20000, precond=vag.VAG_PC_AMG, precision=vag.VAG_MIXED)
    o = oracle.run(p, rtol=1e-13, n_steps=0)
    assert g["info"]["status"] == 0 and g["info"]["rel_residual"] <= rtol
    assert oracle_certificate(p, g) <= 2 * rtol
    compare(p, g, o, flux_tol=1e-6 if rtol < 1e-11 else 1e-4)
    od, phi = o["darcy"], o["phi"]
    dt = p.cfl * float(np.min(oracle.cfl_bounds(p, od, phi)))
    oc = oracle.transport(p, od, phi, dt, p.n_steps)
    h = g["handle"]
    h.set_fluxes(od)
    h.transport(n_steps=p.n_steps)
    gc = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(gc[k] - oc[k]).max() <= 1e-10, k


@pytest.mark.parametrize("sweeps", [2, 3])
def test_amg_coarse_sweeps_parity(sweeps):
    """More smoothing on the coarse levels (symmetric, so CG still applies)."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((16, 12, 10), 12, n_patches=8, n_steps=10)
    g = gpu_run(p, rtol=1e-13, max_iter=2000, precond=vag.VAG_PC_AMG, amg_sweeps=sweeps, amg_coarse_size=40)
    base = gpu_run(p, rtol=1e-13, max_iter=2000, precond=vag.VAG_PC_AMG, amg_coarse_size=40)
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"], 1e-11) and g["info"]["amg_levels"] >= 3
    assert g["info"]["iterations"] <= base["info"]["iterations"]
    compare(p, g, o)



# ---------------------------------------------------------------------------
# K-cycles on the coarse levels (flexible outer CG)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kcycle", [1, 2, 4])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kcycle_parity(kcycle, precision):
    """Two flexible CG steps per visit on levels 1..kcycle (nested: level 2
    is visited four times per outer iteration at kcycle 2): the outer
    flexible CG still reaches the oracle's solution, in fewer iterations
    than with V-cycles alone."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((18, 14, 12), 13, n_patches=9, n_steps=20)
    pr = vag.VAG_FP64 if precision == "fp64" else vag.VAG_MIXED
    # distance-1 aggregates and a small coarsest level: five levels or more
    kw = dict(rtol=1e-12, max_iter=5000, precond=vag.VAG_PC_AMG, precision=pr, amg_coarse_size=20,
              amg_aggregate_hops=1)
    g = gpu_run(p, amg_kcycle=kcycle, **kw)
    v = gpu_run(p, n_steps=0, amg_kcycle=0, **kw)
    o = oracle.run(p, rtol=1e-13)
    info = g["info"]
    print(f"kcycle {kcycle} {precision}: {info['iterations']} iterations "
          f"(V-cycle {v['info']['iterations']}), levels {info['amg_levels']}")
    assert info["amg_levels"] >= min(kcycle, 3) + 2
    assert reached(info, max(1e-12, residual_floor(p, o)))
    assert info["iterations"] < v["info"]["iterations"]
    compare(p, g, o)


def test_kcycle_config2_fewer_iterations_bitwise():
    """Benchmark workload at its tolerance: the K-cycle cuts the outer
    iterations, and two handles give bitwise identical results."""
    from paper_1602_03641_amd import vag
    p = synth.config2()
    kw = dict(rtol=1e-8, max_iter=2000, precond=vag.VAG_PC_AMG, n_steps=0)
    v = gpu_run(p, amg_kcycle=0, **kw)["info"]
    a = gpu_run(p, amg_kcycle=2, **kw)
    b = gpu_run(p, amg_kcycle=2, **kw)
    print("config2 iterations: V-cycle", v["iterations"], "K-cycle", a["info"]["iterations"])
    assert a["info"]["status"] == 0 and a["info"]["rel_residual"] <= 1e-8
    assert a["info"]["iterations"] < v["iterations"]
    np.testing.assert_array_equal(a["u_node"], b["u_node"])
    np.testing.assert_array_equal(a["F_cell"], b["F_cell"])


def test_kcycle_ignored_where_not_flexible():
    """BiCGStab and the FP32 inner solves of refinement keep V-cycles: the
    option changes nothing there."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((12, 9, 8), 14, n_patches=5, n_steps=0)
    for kw in (dict(krylov=vag.VAG_BICGSTAB), dict(precision=vag.VAG_MIXED_IR, inner_rtol=1e-3),
               dict(precision=vag.VAG_MIXED_IR, inner_rtol=1e-2, krylov=vag.VAG_GMRES)):
        kw.update(rtol=1e-10, max_iter=5000, precond=vag.VAG_PC_AMG, amg_coarse_size=30)
        a = gpu_run(p, amg_kcycle=0, **kw)
        b = gpu_run(p, amg_kcycle=3, **kw)
        assert a["info"]["iterations"] == b["info"]["iterations"]
        np.testing.assert_array_equal(a["u_node"], b["u_node"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_kcycle_parity(precision):
    """Flexible GMRES keeps each preconditioned vector, so the nonlinear
    K-cycle preconditioner is allowed: it reaches the oracle's solution in
    fewer iterations than with V-cycles."""
    from paper_1602_03641_amd import vag
    # contrasts up to 1e4 keep rtol 1e-11 above the FP64 floor of the true
    # residual, which GMRES (unlike CG's warm restarts) would run into
    p = synth.random_problem((18, 14, 12), 13, n_patches=9, n_steps=20, ratios=(1e2, 1e4))
    pr = vag.VAG_FP64 if precision == "fp64" else vag.VAG_MIXED
    kw = dict(rtol=1e-11, max_iter=5000, precond=vag.VAG_PC_AMG, precision=pr, amg_coarse_size=20,
              amg_aggregate_hops=1, krylov=vag.VAG_GMRES)
    g = gpu_run(p, amg_kcycle=2, **kw)
    v = gpu_run(p, n_steps=0, amg_kcycle=0, **kw)
    o = oracle.run(p, rtol=1e-13)
    print(f"gmres {precision}: K-cycle {g['info']['iterations']}, V-cycle {v['info']['iterations']}")
    assert g["info"]["amg_levels"] >= 4
    assert g["info"]["status"] == 0 and v["info"]["status"] == 0
    assert g["info"]["iterations"] < v["info"]["iterations"]
    compare(p, g, o)


# ---------------------------------------------------------------------------
# block-Jacobi ILU(0) (with GMRES or BiCGStab), and the preconditioner entry
# ---------------------------------------------------------------------------
def _same_system_as_oracle(p, h):
    """The library's system with every fracture face kept has the oracle's
    unknown order and pattern; returns the oracle's (A, b)."""
    A, b = oracle.system(p)
    rp, col, val, _ = h.system()
    np.testing.assert_array_equal(rp, A.indptr)
    np.testing.assert_array_equal(col, A.indices)
    assert np.abs(val - A.data).max() <= 1e-12 * np.abs(A.data).max()
    return A, b


@pytest.mark.parametrize("B", [1, 64, 300, 8192])
def test_bjilu0_apply_matches_oracle(B):
    """z = M^-1 r element by element against the oracle's block-Jacobi
    ILU(0) of its own system (blocks of B unknowns, the last one ragged;
    B = 1 is Jacobi, 8192 one block)."""
    from paper_1602_03641_amd import vag
    from oracle import ilu
    p = synth.random_problem((11, 9, 8), 15, n_patches=6, n_steps=0, ratios=(1e2, 1e4))
    g = gpu_run(p, n_steps=0, rtol=1e-10, max_iter=5000, precond=vag.VAG_PC_BJILU0, krylov=vag.VAG_BICGSTAB,
                ilu_block_rows=B, eliminate_frac_faces=0)
    assert g["info"]["status"] == 0
    h = g["handle"]
    A, _ = _same_system_as_oracle(p, h)
    rows = ilu.bj_ilu0(A, B)
    rng = np.random.default_rng(16)
    for _ in range(2):
        r = rng.standard_normal(A.shape[0])
        z = h.apply_preconditioner(r)
        zr = ilu.bj_ilu0_apply(rows, r)
        assert np.abs(z - zr).max() <= 1e-11 * np.abs(zr).max()


@pytest.mark.parametrize("krylov", ["gmres", "bicgstab"])
def test_bjilu0_parity(krylov):
    """Jittered anisotropic mesh, contrasts up to 1e6, fracture faces
    eliminated: the oracle's solution."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((10, 8, 7), 8, n_patches=6, n_steps=20)
    kw = _gmres(gmres_restart=200) if krylov == "gmres" else _bicgstab()
    g = gpu_run(p, rtol=1e-12, max_iter=20000, precond=vag.VAG_PC_BJILU0, ilu_block_rows=128, **kw)
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"], max(1e-12, residual_floor(p, o)))
    compare(p, g, o)


def test_bjilu0_config1_and_config2():
    """Config 1 to the parity bar; config 2 at its tolerance, fewer
    iterations with larger blocks, bitwise reproducible."""
    from paper_1602_03641_amd import vag
    p = synth.config1()
    g = gpu_run(p, rtol=1e-13, max_iter=5000, precond=vag.VAG_PC_BJILU0, **_bicgstab())
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"])
    compare(p, g, o)
    p = synth.config2()
    kw = dict(n_steps=0, rtol=1e-8, max_iter=20000, precond=vag.VAG_PC_BJILU0, **_bicgstab())
    small = gpu_run(p, ilu_block_rows=256, **kw)["info"]
    a = gpu_run(p, ilu_block_rows=4096, **kw)
    b = gpu_run(p, ilu_block_rows=4096, **kw)
    print("config2 BiCGStab + BJ-ILU(0) iterations: blocks of 256:", small["iterations"], "of 4096:",
          a["info"]["iterations"], "ms solve", a["info"]["ms_solve"])
    assert a["info"]["status"] == 0 and a["info"]["rel_residual"] <= 1e-8
    assert a["info"]["iterations"] <= small["iterations"]
    np.testing.assert_array_equal(a["u_node"], b["u_node"])


def test_apply_preconditioner_jacobi_and_amg():
    """Jacobi: z = r / diag(A) of the oracle's system.  AMG with V-cycles:
    the cycle is a symmetric operator (r . M^-1 s = s . M^-1 r), which CG
    needs; with K-cycles it is not linear."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((9, 8, 7), 17, n_patches=5, n_steps=0)
    rng = np.random.default_rng(18)
    g = gpu_run(p, n_steps=0, rtol=1e-10, max_iter=5000, precond=vag.VAG_PC_JACOBI, eliminate_frac_faces=0)
    A, _ = _same_system_as_oracle(p, g["handle"])
    r = rng.standard_normal(A.shape[0])
    np.testing.assert_allclose(g["handle"].apply_preconditioner(r), r / A.diagonal(), rtol=1e-13)
    g = gpu_run(p, n_steps=0, rtol=1e-10, max_iter=5000, precond=vag.VAG_PC_AMG, amg_kcycle=0, amg_coarse_size=30)
    h = g["handle"]
    n = h.system()[3].size
    r, s = rng.standard_normal(n), rng.standard_normal(n)
    zr, zs = h.apply_preconditioner(r), h.apply_preconditioner(s)
    assert abs(r @ zs - s @ zr) <= 1e-12 * np.linalg.norm(r) * np.linalg.norm(zs)
    assert r @ zr > 0 and s @ zs > 0
    np.testing.assert_array_equal(h.apply_preconditioner(r), zr)


# ---------------------------------------------------------------------------
# classical AMG (PMIS, direct interpolation) and the exported hierarchy
# ---------------------------------------------------------------------------
def _csr(t, shape):
    import scipy.sparse as sp
    ptr, col, val = t
    return sp.csr_matrix((val, col, ptr), shape=shape)


def _levels(h):
    out = []
    for l in range(len(h.amg_levels())):
        d = h.amg_level(l)
        n = len(d["A"][0]) - 1
        d["Am"] = _csr(d["A"], (n, n))
        d["Pm"] = _csr(d["P"], (n, d["n_coarse"])) if d["P"] is not None else None
        out.append(d)
    return out


@pytest.mark.parametrize("kind", [0, 1])
def test_hierarchy_is_galerkin(kind):
    """Every coarse operator equals P^T A P of the level above, for the
    aggregation (kind 0) and the classical (kind 1) hierarchy; level 0 is the
    oracle's system (faces kept)."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((12, 10, 9), 19, n_patches=6, n_steps=0)
    g = gpu_run(p, n_steps=0, rtol=1e-10, max_iter=5000, precond=vag.VAG_PC_AMG, amg_kind=kind, amg_coarse_size=40,
                amg_kcycle=0, eliminate_frac_faces=0)
    lv = _levels(g["handle"])
    assert len(lv) >= 3
    A0, _ = oracle.system(p)
    assert abs(lv[0]["Am"] - A0).max() <= 1e-12 * abs(A0).max()
    for a, b in zip(lv[:-1], lv[1:]):
        G = (a["Pm"].T @ a["Am"] @ a["Pm"]).tocsr()
        assert abs(G - b["Am"]).max() <= 1e-12 * abs(G).max()
        if kind == 0:
            _check_aggregates(a["Am"], a["Pm"], theta=0.02)


def _check_aggregates(A, P, theta):
    """Validity of one aggregation level (many aggregations are correct, so
    the test checks the defining properties, not one particular answer): P
    is piecewise constant (exactly one entry, 1, per row), no aggregate is
    empty, and each aggregate is connected in the strength graph (i -> j
    when |a_ij| >= theta sqrt(|a_ii a_jj|), the rule the members join by)."""
    import scipy.sparse as sp
    from scipy.sparse import csgraph
    P = P.tocsr()
    assert np.array_equal(np.diff(P.indptr), np.ones(P.shape[0], np.int64))
    assert np.all(P.data == 1.0)
    agg = P.indices
    size = np.bincount(agg, minlength=P.shape[1])
    assert size.min() >= 1
    C = A.tocoo()
    d = A.diagonal()
    off = C.row != C.col
    r, c, v = C.row[off], C.col[off], C.data[off]
    keep = (np.abs(v) >= theta * np.sqrt(np.abs(d[r] * d[c]))) & (agg[r] == agg[c]) & (v != 0)
    S = sp.csr_matrix((np.ones(int(keep.sum())), (r[keep], c[keep])), shape=A.shape)
    ncomp, lab = csgraph.connected_components(S, directed=True, connection="weak")
    assert ncomp == P.shape[1], (ncomp, P.shape[1])
    # edges join members of one aggregate only, so each component lies in one
    # aggregate, and as many components as aggregates means each is one piece


def test_classical_interpolation_matches_oracle():
    """Level 0 of the classical hierarchy on the oracle's own system: the
    PMIS splitting is valid (no two coarse points depend strongly on each
    other, every fine point of positive measure depends strongly on a coarse
    one; it is one of many valid splittings), and for that splitting P
    equals the oracle's direct interpolation."""
    from paper_1602_03641_amd import vag
    from oracle import classical_amg as ca
    p = synth.random_problem((12, 10, 9), 20, n_patches=6, n_steps=0)
    g = gpu_run(p, n_steps=0, rtol=1e-10, max_iter=5000, precond=vag.VAG_PC_AMG, amg_kind=1,
                eliminate_frac_faces=0)
    d = g["handle"].amg_level(0)
    A, _ = oracle.system(p)
    S = ca.strength(A, 0.25)
    ci = d["coarse_index"]
    is_c = ci >= 0
    assert is_c.sum() == d["n_coarse"]
    independent, covered, lonely = ca.pmis_valid(S, is_c)
    assert independent and covered
    print(f"classical level 0: {A.shape[0]} rows, {is_c.sum()} coarse, {lonely} fine without a coarse neighbour")
    Po = ca.direct_interpolation(A, S, is_c).toarray()
    # oracle columns: coarse points by increasing index; the library's: ci
    order = np.argsort(np.where(is_c)[0])
    gcol_of_ocol = ci[np.where(is_c)[0][order]]
    Pg = _csr(d["P"], (A.shape[0], d["n_coarse"])).toarray()[:, gcol_of_ocol]
    np.testing.assert_allclose(Pg, Po, rtol=0, atol=1e-12 * np.abs(Po).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_classical_amg_parity(precision):
    """Classical AMG as the CG preconditioner (and in GMRES): the oracle's
    solution on a jittered anisotropic mesh with contrasts up to 1e6."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((14, 12, 10), 21, n_patches=8, n_steps=20)
    pr = vag.VAG_FP64 if precision == "fp64" else vag.VAG_MIXED
    g = gpu_run(p, rtol=1e-12, max_iter=5000, precond=vag.VAG_PC_AMG, amg_kind=1, precision=pr)
    o = oracle.run(p, rtol=1e-13)
    info = g["info"]
    print(f"classical {precision}: {info['iterations']} iterations, {info['amg_levels']} levels, "
          f"complexity {info['amg_operator_complexity']:.2f}")
    assert reached(info, max(1e-12, residual_floor(p, o)))
    compare(p, g, o)
    gm = gpu_run(p, rtol=1e-12, max_iter=5000, precond=vag.VAG_PC_AMG, amg_kind=1, precision=pr,
                 **_gmres(gmres_restart=100))
    assert reached(gm["info"], max(1e-12, residual_floor(p, o)))
    compare(p, gm, o)


def test_classical_amg_config2():
    """64^3 benchmark workload at its tolerance; bitwise reproducible."""
    from paper_1602_03641_amd import vag
    p = synth.config2()
    kw = dict(n_steps=0, rtol=1e-8, max_iter=2000, precond=vag.VAG_PC_AMG, amg_kind=1)
    a = gpu_run(p, **kw)
    b = gpu_run(p, **kw)
    info = a["info"]
    print("classical config2:", {k: info[k] for k in ("iterations", "amg_levels", "amg_operator_complexity",
                                                       "ms_setup", "ms_solve")})
    assert info["status"] == 0 and info["rel_residual"] <= 1e-8
    assert info["iterations"] < 200
    np.testing.assert_array_equal(a["u_node"], b["u_node"])


# ---------------------------------------------------------------------------
# Peaceman wells on fracture faces
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("eliminate", [1, 0])
@pytest.mark.parametrize("precond", ["amg", "jacobi"])
def test_wells_parity(eliminate, precond):
    """Two rate injectors and two pressure wells: pressures, fluxes, well
    rates and concentrations against the oracle (fracture faces eliminated
    or kept: a perforated face inside an eliminated group changes its block)."""
    from paper_1602_03641_amd import vag
    p = synth.add_wells(synth.random_problem((12, 10, 8), 33, n_patches=8, n_steps=30, ratios=(1e2, 1e4)), 3,
                        n_inj=2, n_prod=2)
    pc = vag.VAG_PC_AMG if precond == "amg" else vag.VAG_PC_JACOBI
    g = gpu_run(p, rtol=1e-13, max_iter=20000, precond=pc, eliminate_frac_faces=eliminate)
    o = oracle.run(p, rtol=1e-13)
    assert reached(g["info"], max(1e-12, residual_floor(p, o)))
    compare(p, g, o)
    Q, Qo = g["handle"].well_rates(), o["darcy"]["well_rate"]
    assert np.abs(Q - Qo).max() <= 1e-8 * np.abs(Qo).max()
    assert g["tinfo"]["dt"] == pytest.approx(o["dt"], rel=1e-9)


def test_wells_transport_identical_fluxes():
    """Transport with wells on the oracle's fluxes and well rates: only
    rounding differs."""
    from paper_1602_03641_amd import vag
    _torch()
    p = synth.add_wells(synth.random_problem((11, 9, 8), 34, n_patches=7, n_steps=80), 4, n_inj=2, n_prod=3)
    od = oracle.solve_darcy(p, rtol=1e-12)
    phi = oracle.porous_volumes(p)
    dt = p.cfl * float(np.min(oracle.cfl_bounds(p, od, phi)))
    oc = oracle.transport(p, od, phi, dt, p.n_steps)
    h = vag.Handle(p, cfl=p.cfl)
    h.set_fluxes(od)
    h.set_well_rates(od["well_rate"])
    np.testing.assert_array_equal(h.well_rates(), od["well_rate"])
    t = h.transport(n_steps=p.n_steps)
    assert t["dt"] == pytest.approx(dt, rel=1e-12)
    gc = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(gc[k] - oc[k]).max() <= 1e-12, k
    assert gc["c_frac"][p.wells["face"][0]] > 0.05  # the injected tracer arrived


def test_wells_rejected_and_removed():
    from paper_1602_03641_amd import vag
    _torch()
    p = synth.random_problem((6, 5, 5), 35, n_patches=3, n_steps=0)
    h = vag.Handle(p)
    one = np.ones(2)
    for face, wi in (([0, 0], one), ([0, p.n_frac], one), ([0, 1], -one), ([0, 1], np.array([1.0, np.nan]))):
        with pytest.raises(vag.VagError) as e:
            h.set_wells(face, wi, one, one, one)
        assert e.value.status == vag.VAG_ERR_ARG
    h.solve_pressure()
    u0 = vag.to_numpy(h.pressure())["u_node"]
    h.set_wells([1], [0.0], [0.0], [0.4], [1.0])
    h.solve_pressure()
    assert np.abs(vag.to_numpy(h.pressure())["u_node"] - u0).max() > 1e-3
    h.set_wells([], [], [], [], [])
    h.solve_pressure()
    np.testing.assert_array_equal(vag.to_numpy(h.pressure())["u_node"], u0)


def test_wide_planes_mix_column_widths():
    """181 x 181 x 2 cells: a node plane holds 33 124 nodes, so the slices of
    the middle plane span more than 65 536 columns and keep 32-bit columns
    while those of the outer planes take 16-bit offsets; both paths in one
    solve meet the parity bar."""
    from paper_1602_03641_amd import vag
    p = synth.random_problem((181, 181, 2), 36, n_patches=4, n_steps=10, ratios=(1e2,), jitter=0.1)
    g = gpu_run(p, rtol=1e-11, max_iter=20000, precond=vag.VAG_PC_AMG)
    o = oracle.run(p, rtol=1e-11)
    assert g["info"]["status"] == 0
    compare(p, g, o, p_tol=1e-8, c_tol=1e-9)


def test_switching_solvers_on_one_handle():
    """One handle through aggregation AMG, classical AMG, BiCGStab with
    block-Jacobi ILU(0), the FP32 hierarchy and back: every solve reaches the
    same solution, and the first configuration again gives it bitwise (no
    state of another solver leaks into a solve)."""
    from paper_1602_03641_amd import vag
    _torch()
    p = synth.random_problem((12, 10, 9), 37, n_patches=6, n_steps=10)
    h = vag.Handle(p, rtol=1e-12, max_iter=20000, precond=vag.VAG_PC_AMG)

    def solve():
        info = h.solve_pressure()
        h.transport(n_steps=p.n_steps)
        assert info["status"] in (0, 1) and info["rel_residual"] <= 1e-11
        return {**vag.to_numpy(h.pressure()), **vag.to_numpy(h.concentration())}

    ref = solve()
    steps = [dict(amg_kind=1), dict(precond=vag.VAG_PC_BJILU0, krylov=vag.VAG_BICGSTAB, amg_kind=0),
             dict(precond=vag.VAG_PC_AMG, krylov=vag.VAG_CG, precision=vag.VAG_MIXED),
             dict(krylov=vag.VAG_GMRES, precision=vag.VAG_FP64), dict(krylov=vag.VAG_CG)]
    for kw in steps:
        h.set_options(**kw)
        g = solve()
        assert rel_l2(g["u_node"], ref["u_node"]) <= 1e-9, kw
    for k in ("u_node", "u_frac", "c_cell", "c_node"):
        np.testing.assert_array_equal(g[k], ref[k])


# ---------------------------------------------------------------------------
# Checkpoint and resume of the transport
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["hex8", "tet"])
def test_transport_resume_bitwise(kind):
    """The explicit scheme's state is the concentration vector (the time step
    follows from the fluxes).  After a solve the state is 0; n steps, the
    concentrations saved to host memory, then m more steps (continuing on the
    handle, from the saved state on the same handle, and from it on a new
    handle of the same problem after its own solve) equal n + m uninterrupted
    steps, bitwise; a final-time run split at a step boundary agrees too."""
    _torch()
    from paper_1602_03641_amd import vag
    if kind == "hex8":
        p = synth.random_problem((9, 7, 6), 5, n_patches=4, n_steps=40)
    else:
        p = synth.general_problem("tet", (7, 6, 5), 5, frac_plane=3)
    opt = dict(rtol=1e-12, max_iter=20000, precond=vag.VAG_PC_AMG)
    keys = ("c_cell", "c_frac", "c_node")
    h = vag.Handle(p, **opt)
    h.solve_pressure()
    t_full = h.transport(n_steps=40)
    full = vag.to_numpy(h.concentration())
    h.solve_pressure()  # the state starts again from 0
    h.transport(n_steps=15)
    ck = vag.to_numpy(h.concentration())
    h.transport(n_steps=25)  # continues
    cont = vag.to_numpy(h.concentration())
    h.transport(n_steps=25, c0=ck)
    again = vag.to_numpy(h.concentration())
    h2 = vag.Handle(p, **opt)
    h2.solve_pressure()
    h2.transport(n_steps=25, c0=ck)
    fresh = vag.to_numpy(h2.concentration())
    assert np.abs(full["c_cell"] - ck["c_cell"]).max() > 1e-3  # the last 25 steps change the state
    for r in (cont, again, fresh):
        for k in keys:
            np.testing.assert_array_equal(r[k], full[k], err_msg=k)
    # final time 40 dt, and 15 dt followed by 25 dt
    dt = t_full["dt"]
    h.solve_pressure()
    h.transport(t_final=40 * dt)
    tf = vag.to_numpy(h.concentration())
    h.solve_pressure()
    h.transport(t_final=15 * dt)
    h.transport(t_final=25 * dt)
    tf2 = vag.to_numpy(h.concentration())
    for k in keys:
        np.testing.assert_allclose(tf2[k], tf[k], rtol=0, atol=1e-12, err_msg=k)
        np.testing.assert_allclose(tf[k], full[k], rtol=0, atol=1e-12, err_msg=k)
    h.close()
    h2.close()
