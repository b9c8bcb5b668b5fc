"""GPU checks at the full sizes of the 128^3 and 192^3 workloads, and of the
row loops that read large matrices with non-temporal loads.

At these sizes the oracle cannot converge a Jacobi-PCG solve of its own, so
it certifies the library's solution instead:
- the residual ||b - A x|| / ||b|| of the library's pressures, evaluated by
  the oracle cell by cell (its conservation equations, no assembled matrix),
  is within 1.5e-8 (the solves stop at 1e-8 on their own residual);
- every cell conserves its fluxes to rounding;
- the porous volumes equal the oracle's;
- the transport steps on the library's fluxes equal the oracle's to 1e-12.
The systems there exceed 128 MB, so these solves run the non-temporal row
loops; a forced run of those loops on the 64^3 workload must give results
bitwise equal to ordinary loads (only the cache policy differs).
"""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


@pytest.mark.parametrize("gen,solver", [("config3", "cg"), ("config3", "gmres_ir"), ("config5", "cg")])
def test_full_size_certificate(gen, solver):
    _torch()
    from paper_1602_03641_amd import vag
    _log(f"{gen} {solver}: generating")
    p = getattr(synth, gen)()
    opts = dict(rtol=1e-8, max_iter=5000, precond=vag.VAG_PC_AMG, cfl=p.cfl)
    if solver == "cg":
        opts.update(precision=vag.VAG_MIXED)
    else:  # the 128^3 workload's own solver: FP64 refinement around FP32 GMRES with the FP32 hierarchy
        opts.update(precision=vag.VAG_MIXED_IR, krylov=vag.VAG_GMRES, gmres_restart=100, inner_rtol=1e-2)
    _log(f"{gen}: {p.n_cells} cells, {p.n_frac} fracture faces; solving")
    h = vag.Handle(p, **opts)
    info = h.solve_pressure()
    _log(f"{gen}: status {info['status']}, {info['iterations']} iterations, residual {info['rel_residual']:.3e}")
    assert info["status"] == 0 and info["rel_residual"] <= 1e-8
    u = vag.to_numpy(h.pressure())
    r = oracle.residual(p, u["u_node"], u["u_frac"])
    _log(f"{gen}: oracle certificate {r['rel_residual']:.3e}")
    assert r["rel_residual"] <= 1.5e-8

    fl = vag.to_numpy(h.fluxes())
    cf, fc, _ = oracle.topology(p)
    cell_sum = fl["F_cell"].sum(1)
    for side in range(2):
        m = fc[:, side] >= 0
        np.add.at(cell_sum, fc[m, side], fl["F_cell_frac"][m, side])
    scale = np.abs(fl["F_cell"]).max()
    assert np.abs(cell_sum).max() <= 1e-12 * scale

    if solver == "gmres_ir":
        return
    _log(f"{gen}: porous volumes")
    phi = oracle.porous_volumes(p)
    gphi = vag.to_numpy(h.porous_volumes())
    for k in ("phi_cell", "phi_frac", "phi_node"):
        np.testing.assert_allclose(gphi[k], phi[k], rtol=1e-13, atol=0, err_msg=k)
    n = 10
    t = h.transport(n_steps=n)
    dt3 = oracle.cfl_bounds(p, fl, phi)
    assert t["dt"] == pytest.approx(p.cfl * dt3.min(), rel=1e-13)
    _log(f"{gen}: oracle transport, {n} steps")
    oc = oracle.transport(p, fl, phi, t["dt"], n)
    gc = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(gc[k] - oc[k]).max() <= 1e-12, k
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_forced_nontemporal_loads_bitwise(precision):
    """The 64^3 workload (90 MB system, ordinary loads by default) with the
    non-temporal row loops forced on, and with them forced off: the same
    arithmetic in the same order, so every output is bitwise the same."""
    _torch()
    from paper_1602_03641_amd import vag
    p = synth.config2()
    pr = vag.VAG_FP64 if precision == "fp64" else vag.VAG_MIXED
    out = {}
    for mode in (0, 1, 2):
        h = vag.Handle(p, rtol=1e-8, precond=vag.VAG_PC_AMG, precision=pr, stream_loads=mode)
        info = h.solve_pressure()
        h.transport(n_steps=p.n_steps)
        assert info["status"] == 0
        out[mode] = (info["iterations"], vag.to_numpy(h.pressure()), vag.to_numpy(h.concentration()))
        h.close()
    for mode in (1, 2):
        assert out[mode][0] == out[0][0]
        for d0, d1 in ((out[0][1], out[mode][1]), (out[0][2], out[mode][2])):
            for k in d0:
                assert np.array_equal(d0[k], d1[k]), (mode, k)

