"""Pins of the oracle's Peaceman wells (§5.5): the closed-form well index
against the VAG scheme on the box it is derived from, global conservation
with sources and sinks, a producer at the face's own pressure changes
nothing, and the transport mass balance with wells."""
import math

import numpy as np
import pytest

import oracle
import synth


def box_problem(dx, dy, dz, lam):
    xyz = np.array([[0, 0, 0], [dx, 0, 0], [dx, dy, 0], [0, dy, 0],
                    [0, 0, dz], [dx, 0, dz], [dx, dy, dz], [0, dy, dz]], float)
    return synth.Problem(name="box", dims=(1, 1, 1), xyz=xyz, hex8=np.arange(8, dtype=np.int32)[None, :],
                         frac_nodes=np.zeros((0, 4), np.int32), frac_width=np.zeros(0), frac_perm=np.zeros(0),
                         frac_poro=np.zeros(0), perm=np.array([[lam, lam, lam, 0, 0, 0]], float),
                         poro=np.ones(1), mu=1.0, dirichlet=np.ones(8, np.uint8), p_bar=np.zeros(8),
                         c_bar=np.zeros(8))


@pytest.mark.parametrize("dx,df,dz", [(3.5, 1.0, 10.4), (2.0, 0.01, 2.0), (7.0, 1.0, 1.0)])
def test_peaceman_index_from_the_vag_box(dx, df, dz):
    """The well index is derived by imposing the radial well solution at the
    8 corners of the face expanded to a dx x df x dz box and the well's flow
    at its centre: all corners sit at the distance D = sqrt(dx^2 + df^2)/2 of
    the axis, so the VAG cell equation gives u_K - p_D = q dz / A_KK, and
    WI = q dz / (p_w - u_K) with p_D = p_w - q ln(D / rw) / (2 pi lam).  A_KK
    comes from the oracle's own cell matrix here; the closed form must agree."""
    lam, rw = 3.0, 0.1
    a, _ = oracle.cell_matrix(box_problem(dx, df, dz, lam), 0)
    AKK = a.sum()
    D = 0.5 * math.hypot(dx, df)
    wi_vag = 2 * math.pi * lam * dz / (math.log(D / rw) - 2 * math.pi * lam * dz / AKK)
    assert oracle.peaceman_wi(dx, dz, df, lam, rw) == pytest.approx(wi_vag, rel=1e-12)


def _dirichlet_flow(p, o):
    """Total flux from the domain into the Dirichlet nodes."""
    d = p.dirichlet[p.hex8] == 1
    total = o["F_cell"][d].sum()
    if p.n_frac:
        total += o["F_frac"][p.dirichlet[p.frac_nodes] == 1].sum()
    return total


def test_well_conservation():
    """At steady state what the wells put in leaves through the Dirichlet
    nodes: sum_k Q_k = flux into the Dirichlet nodes."""
    p = synth.add_wells(synth.random_problem((8, 7, 6), 30, n_patches=5, n_steps=0), 1, n_inj=2, n_prod=2)
    o = oracle.solve_darcy(p, rtol=1e-14)
    Q = o["well_rate"]
    assert np.all(Q[:2] == pytest.approx(0.5)) and np.all(Q[2:] != 0)
    scale = np.abs(o["F_cell"]).max()
    assert abs(Q.sum() - _dirichlet_flow(p, o)) <= 1e-9 * scale
    # without wells the Dirichlet flux balances to zero
    p.wells = None
    o0 = oracle.solve_darcy(p, rtol=1e-14)
    assert abs(_dirichlet_flow(p, o0)) <= 1e-9 * scale


def test_producer_at_the_face_pressure_changes_nothing():
    p = synth.random_problem((7, 6, 6), 31, n_patches=4, n_steps=0)
    o0 = oracle.solve_darcy(p, rtol=1e-14)
    f = int(np.argmax(np.abs(o0["u_frac"] - 0.5)))
    p.wells = dict(face=np.array([f], np.int32), wi=np.array([50.0]), pw=np.array([o0["u_frac"][f]]),
                   q=np.zeros(1), cinj=np.zeros(1))
    o1 = oracle.solve_darcy(p, rtol=1e-14)
    assert abs(o1["well_rate"][0]) <= 1e-9
    np.testing.assert_allclose(o1["u_node"], o0["u_node"], rtol=0, atol=1e-10)
    # a lower well pressure draws fluid out and lowers the face pressure
    p.wells["pw"] = np.array([o0["u_frac"][f] - 0.2])
    o2 = oracle.solve_darcy(p, rtol=1e-14)
    assert o2["well_rate"][0] < 0 and o2["u_frac"][f] < o0["u_frac"][f]


def test_well_transport_mass_balance():
    """M^{n+1} - M^n = dt (sum_inj c_inj Q - sum_prod c_sigma |Q| - Dirichlet
    outflow): the upwind fluxes telescope; concentrations stay in [0, 1]."""
    p = synth.add_wells(synth.random_problem((7, 6, 5), 32, n_patches=4, n_steps=0), 2)
    o = oracle.solve_darcy(p, rtol=1e-14)
    phi = oracle.porous_volumes(p)
    dt = 0.9 * oracle.cfl_bounds(p, o, phi).min()
    c = dict(c_cell=np.zeros(p.n_cells), c_frac=np.zeros(p.n_frac), c_node=np.where(p.dirichlet == 1, p.c_bar, 0.0))
    mass = lambda c: phi["phi_cell"] @ c["c_cell"] + phi["phi_frac"] @ c["c_frac"] + phi["phi_node"] @ c["c_node"]  # noqa: E731
    pos = lambda x: np.maximum(x, 0)  # noqa: E731
    neg = lambda x: np.minimum(x, 0)  # noqa: E731
    w, Q = p.wells, o["well_rate"]
    for _ in range(15):
        m0 = mass(c)
        H = c["c_cell"][:, None] * pos(o["F_cell"]) + c["c_node"][p.hex8] * neg(o["F_cell"])
        out = H[p.dirichlet[p.hex8] == 1].sum()
        Hf = c["c_frac"][:, None] * pos(o["F_frac"]) + c["c_node"][p.frac_nodes] * neg(o["F_frac"])
        out += Hf[p.dirichlet[p.frac_nodes] == 1].sum()
        wells = (w["cinj"] * pos(Q)).sum() - (c["c_frac"][w["face"]] * pos(-Q)).sum()
        c = oracle.transport(p, o, phi, dt, 1, c0=c)
        assert abs(mass(c) - m0 - dt * (wells - out)) <= 1e-12 * max(abs(m0), dt * abs(wells), 1e-300)
        for k in ("c_cell", "c_frac", "c_node"):
            assert c[k].min() >= -1e-9 and c[k].max() <= 1 + 1e-9
    assert c["c_frac"][w["face"][0]] > 0.1  # the injected tracer is there
