"""GPU test of vag_transport_noalloc, the transport entry point that allocates
nothing (its scratch is the library's static device array).

Two calls in a row through the C-ABI, the second on a smaller problem (the
static array keeps the first call's contents), each checked against
vag_transport on the same handle: the same time step (bitwise: both run the
same CFL reduction) and concentrations within 1e-12 max-abs (only the order
of the additions inside a step differs; the FP64 path's bar is 1e-10), and
against the oracle's transport on the library's own fluxes and porous
volumes within 1e-10.
"""
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


def _host(d):
    return {k: v.detach().cpu().numpy() for k, v in d.items()}


def _check_case(p, n_steps, seed, t_final=0.0):
    torch = _torch()
    from paper_1602_03641_amd import vag
    print(f"noalloc case {p.name}: {p.n_cells} cells, {p.n_frac} faces, steps {n_steps}, t_final {t_final}",
          flush=True)
    h = vag.Handle(p, rtol=1e-12, max_iter=20000, cfl=p.cfl)
    h.solve_pressure()
    rng = np.random.default_rng(seed)
    c0 = dict(c_cell=rng.uniform(0, 1, p.n_cells), c_frac=rng.uniform(0, 1, p.n_frac),
              c_node=rng.uniform(0, 1, p.n_nodes))
    ref_info = h.transport(n_steps=n_steps, t_final=t_final, c0=c0)
    ref = vag.to_numpy(h.concentration())
    got_t, info = h.transport_noalloc(n_steps=n_steps, t_final=t_final, c0=c0)
    torch.cuda.synchronize()
    got = _host(got_t)
    assert info["dt"] == ref_info["dt"] and info["n_steps"] == ref_info["n_steps"]
    assert info["last_dt"] == ref_info["last_dt"]
    assert list(info["dt_bounds"]) == list(ref_info["dt_bounds"])
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(got[k] - ref[k]).max(initial=0.0) <= 1e-12, k
    # the handle's state is the result too
    state = vag.to_numpy(h.concentration())
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.array_equal(state[k], got[k]), k
    # the oracle on the library's own fluxes, porous volumes and time grid
    flux = vag.to_numpy(h.fluxes())
    if p.wells:
        flux["well_rate"] = h.well_rates()
    phi = vag.to_numpy(h.porous_volumes())
    c0o = dict(c0)
    c0o["c_node"] = np.where(p.dirichlet == 1, p.c_bar, c0["c_node"])
    last = info["last_dt"] if t_final > 0 else 0.0
    o = oracle.transport(p, flux, phi, info["dt"], info["n_steps"], last_dt=last, c0=c0o)
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(got[k] - o[k]).max(initial=0.0) <= 1e-10, k
    h.close()


def test_noalloc_equals_transport_twice_shrinking():
    big = synth.random_problem((16, 13, 11), 21, n_patches=6, n_steps=40)
    synth.add_wells(big, 3, n_inj=1, n_prod=1)
    small = synth.random_problem((5, 4, 6), 22, n_patches=2, n_steps=15)
    _check_case(big, big.n_steps, 1)
    _check_case(small, small.n_steps, 2)


def test_noalloc_final_time_and_no_sync():
    """t_final with a shortened last step; then a call without info queues
    its work only, and the handle's state is read afterwards."""
    torch = _torch()
    from paper_1602_03641_amd import vag
    p = synth.random_problem((7, 6, 5), 23, n_patches=3, n_steps=10)
    _check_case(p, 0, 3, t_final=0.37)
    h = vag.Handle(p, rtol=1e-12, max_iter=20000)
    h.solve_pressure()
    h.transport(n_steps=12)
    ref = vag.to_numpy(h.concentration())
    h.solve_pressure()  # back to a zero state
    got_t, info = h.transport_noalloc(n_steps=12, info=False)
    assert info is None
    torch.cuda.synchronize()
    got = _host(got_t)
    for k in ("c_cell", "c_frac", "c_node"):
        assert np.abs(got[k] - ref[k]).max(initial=0.0) <= 1e-12, k
    h.close()
