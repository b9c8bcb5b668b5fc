"""GPU tests of the serving loop (vag_server_*): every job's result is the same
alone and in the mix (bitwise: a job's rows get the same arithmetic in the same
order whatever else is on the device, its transport steps included, which run
batched with other jobs' steps), on hex8 meshes and on meshes given by their
faces, the batched steps equal a lone handle's, jobs
whose transports overlap share launches, admission by footprint keeps the
bytes in use within the budget, the footprint estimate bounds the real
footprint, cached handles are reused, cancel and out-of-memory rejection.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

OUT = ("u_node", "u_cell", "u_frac", "c_cell", "c_frac", "c_node")


def _vag():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_03641_amd import vag
    return vag


def _jobs(k=10):
    """Mixed sizes, contrasts and fracture counts; several exceed one block."""
    jobs = []
    for j in range(k):
        rng = np.random.default_rng([44, j])
        n = int(rng.integers(5, 19))
        dims = (n, int(rng.integers(4, 15)), int(rng.integers(4, 12)))
        p = synth.random_problem(dims, 100 + j, n_patches=int(rng.integers(1, 9)), n_steps=int(rng.integers(5, 40)))
        jobs.append(p)
    return jobs


def _opts(mode):
    from paper_1602_03641_amd import vag
    if mode == "fp64":
        return dict(precond=vag.VAG_PC_AMG, precision=vag.VAG_FP64, rtol=1e-10, max_iter=5000)
    if mode == "gmres_ir":  # FP64 refinement around flexible GMRES in FP32 (100 basis vectors)
        return dict(precond=vag.VAG_PC_AMG, precision=vag.VAG_MIXED_IR, krylov=vag.VAG_GMRES, gmres_restart=100,
                    inner_rtol=1e-2, rtol=1e-10, max_iter=5000)
    return dict(precond=vag.VAG_PC_AMG, precision=vag.VAG_MIXED, rtol=1e-10, max_iter=5000)


def _run(vag, jobs, mode, workers, together, budget=0):
    srv = vag.Server(hbm_budget=budget, n_workers=workers)
    try:
        res = []
        if together:
            ids = [srv.submit(p, n_steps=p.n_steps, **_opts(mode)) for p in jobs]
            res = [srv.wait(i) for i in ids]
        else:
            for p in jobs:
                res.append(srv.wait(srv.submit(p, n_steps=p.n_steps, **_opts(mode))))
        stats = srv.stats()
    finally:
        srv.close()
    return res, stats


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_alone_equals_mix_bitwise(mode):
    vag = _vag()
    jobs = _jobs(10)
    alone, _ = _run(vag, jobs, mode, workers=1, together=False)
    mix, stats = _run(vag, jobs, mode, workers=4, together=True)
    assert stats["finished"] == len(jobs) and stats["bytes_in_use"] == 0
    assert stats["job_steps"] == sum(p.n_steps for p in jobs) >= stats["step_launches"] > 0
    overlap = 0
    for a, m in zip(alone, mix):
        assert a["status"] == 0 and m["status"] == 0, (a["message"], m["message"])
        for k in OUT:
            np.testing.assert_array_equal(a[k], m[k], err_msg=k)
        assert a["solve"]["iterations"] == m["solve"]["iterations"]
    # the jobs of the mix did overlap in time
    iv = sorted((m["t_start"], m["t_end"]) for m in mix)
    overlap = sum(1 for i in range(1, len(iv)) if iv[i][0] < max(e for _, e in iv[:i]))
    assert overlap > 0
    print(f"{mode}: {overlap} of {len(mix)} jobs started while another was running")


def test_transport_steps_share_launches():
    """Eight jobs with long transports on eight workers: their steps run in
    shared launches (fewer launches than steps), and every result equals the
    job run alone, bitwise."""
    vag = _vag()
    jobs = [synth.random_problem((8, 7, 6), 200 + j, n_patches=3, n_steps=300) for j in range(8)]
    alone, st1 = _run(vag, jobs, "fp64", workers=1, together=False)
    assert st1["step_launches"] == st1["job_steps"] == 8 * 300  # one job at a time: one job per launch
    mix, st8 = _run(vag, jobs, "fp64", workers=8, together=True)
    assert st8["job_steps"] == 8 * 300
    print(f"{st8['job_steps']} steps in {st8['step_launches']} launches")
    assert st8["step_launches"] < st8["job_steps"]
    for a, m in zip(alone, mix):
        assert a["status"] == 0 and m["status"] == 0
        for k in OUT:
            np.testing.assert_array_equal(a[k], m[k], err_msg=k)


def test_served_final_time_matches_handle():
    """Jobs run to a final time (the last step a fraction of dt) in the mix:
    the batched steps, the partial last one included, equal a lone handle's
    transport to that time, bitwise."""
    vag = _vag()
    jobs = [synth.random_problem((7, 6, 5), 300 + j, n_patches=3, n_steps=0) for j in range(4)]
    srv = vag.Server(n_workers=4)
    try:
        ids = [srv.submit(p, t_final=0.037 * (j + 1), rtol=1e-12, max_iter=20000) for j, p in enumerate(jobs)]
        res = [srv.wait(i) for i in ids]
    finally:
        srv.close()
    for j, (p, r) in enumerate(zip(jobs, res)):
        assert r["status"] in (0, 1), r["message"]
        h = vag.Handle(p, rtol=1e-12, max_iter=20000)
        h.solve_pressure()
        t = h.transport(t_final=0.037 * (j + 1))
        assert t["last_dt"] < t["dt"] and r["transport"]["n_steps"] == t["n_steps"]
        d = vag.to_numpy(h.concentration())
        for k in ("c_cell", "c_frac", "c_node"):
            np.testing.assert_array_equal(r[k], d[k], err_msg=k)
        h.close()


def test_served_job_matches_handle_and_oracle():
    vag = _vag()
    p = synth.random_problem((9, 7, 6), 3, n_patches=5, n_steps=25)
    srv = vag.Server(n_workers=2)
    try:
        r = srv.wait(srv.submit(p, n_steps=p.n_steps, rtol=1e-13, max_iter=20000))
    finally:
        srv.close()
    assert r["status"] in (0, 1) and r["solve"]["rel_residual"] <= 1e-12  # 1: stopped at the rounding floor
    h = vag.Handle(p, rtol=1e-13, max_iter=20000)
    h.solve_pressure()
    h.transport(n_steps=p.n_steps)
    d = vag.to_numpy(h.pressure()) | vag.to_numpy(h.concentration())
    for k in OUT:
        np.testing.assert_array_equal(r[k], d[k], err_msg=k)
    o = oracle.run(p, rtol=1e-13)
    u = o["darcy"]["u_node"]
    assert np.linalg.norm(r["u_node"] - u) <= 1e-8 * np.linalg.norm(u)
    assert np.abs(r["c_cell"] - o["c_cell"]).max() <= 1e-10


def test_admission_respects_budget():
    vag = _vag()
    jobs = _jobs(8)
    est = [vag.estimate_footprint(p, **_opts("fp64")) for p in jobs]
    budget = int(2.2 * max(est))
    res, stats = _run(vag, jobs, "fp64", workers=4, together=True, budget=budget)
    assert all(r["status"] == 0 for r in res)
    assert stats["peak_bytes_in_use"] <= budget
    # at no time did the running jobs' estimates exceed the budget
    ev = sorted([(r["t_start"], 1, r["footprint_estimate"]) for r in res] +
                [(r["t_end"], 0, -r["footprint_estimate"]) for r in res])
    cur = 0
    for _, _, b in ev:
        cur += b
        assert cur <= budget


def test_footprint_estimate_bounds_actual():
    vag = _vag()
    for mode in ("fp64", "mixed"):
        for p in _jobs(6) + [synth.config4_job(3, n_range=(20, 28)), synth.config4_job(5, n_range=(40, 48))]:
            srv = vag.Server(n_workers=1)
            try:
                r = srv.wait(srv.submit(p, n_steps=3, **_opts(mode)))
            finally:
                srv.close()
            assert r["status"] == 0
            assert r["footprint_bytes"] <= r["footprint_estimate"], (p.name, mode, r["footprint_bytes"])
            if r["footprint_bytes"] > 20e6:  # tightness, once the fixed part no longer dominates
                assert r["footprint_estimate"] <= 3 * r["footprint_bytes"], (p.name, mode)


def _general_jobs():
    """Tetrahedra, prisms and hexahedra given by their faces, with fracture
    planes, mixed with hex8 jobs."""
    jobs = [synth.general_problem(kind, dims, 60 + k, frac_plane=dims[0] // 2, n_steps=12 + 5 * k)
            for k, (kind, dims) in enumerate([("tet", (7, 6, 5)), ("prism", (9, 7, 6)), ("hex", (8, 7, 6)),
                                              ("tet", (10, 8, 7)), ("prism", (6, 5, 4))])]
    return jobs + _jobs(3)


def test_general_jobs_alone_equal_mix_and_handle():
    """Jobs on meshes given by their faces run in the mix with hex8 jobs: each
    result equals the job run alone, bitwise, and a lone handle's."""
    vag = _vag()
    jobs = _general_jobs()
    alone, _ = _run(vag, jobs, "fp64", workers=1, together=False)
    mix, stats = _run(vag, jobs, "fp64", workers=4, together=True)
    assert stats["finished"] == len(jobs) and stats["bytes_in_use"] == 0
    assert stats["job_steps"] == sum(p.n_steps for p in jobs)
    for a, m in zip(alone, mix):
        assert a["status"] == 0 and m["status"] == 0, (a["message"], m["message"])
        for k in OUT:
            np.testing.assert_array_equal(a[k], m[k], err_msg=k)
    for p, r in zip(jobs[:2], mix[:2]):
        h = vag.Handle(p, **_opts("fp64"))
        h.solve_pressure()
        h.transport(n_steps=p.n_steps)
        d = vag.to_numpy(h.pressure()) | vag.to_numpy(h.concentration())
        h.close()
        for k in OUT:
            np.testing.assert_array_equal(r[k], d[k], err_msg=k)


def test_general_footprint_estimate_bounds_actual():
    """The mesh-based estimate bounds the footprint of jobs on tetrahedra,
    prisms and hexahedra given by their faces (CG in FP64 and with the FP32
    hierarchy, refinement around FP32 GMRES), within 3x once the mesh is
    large."""
    vag = _vag()
    for kind, dims in [("tet", (6, 5, 4)), ("prism", (9, 8, 6)), ("hex", (10, 9, 8)), ("tet", (28, 26, 24)),
                       ("prism", (36, 32, 30)), ("hex", (44, 40, 36))]:
        p = synth.general_problem(kind, dims, 7, frac_plane=dims[0] // 2)
        for mode in ("fp64", "mixed", "gmres_ir"):
            srv = vag.Server(n_workers=1)
            try:
                r = srv.wait(srv.submit(p, n_steps=3, **_opts(mode)))
            finally:
                srv.close()
            assert r["status"] == 0, r["message"]
            assert r["footprint_bytes"] <= r["footprint_estimate"], (kind, dims, mode, r["footprint_bytes"])
            print(f"{kind}{dims} {mode}: {r['footprint_bytes'] / 1e6:.1f} MB, estimate "
                  f"{r['footprint_estimate'] / 1e6:.1f} MB")
            if r["footprint_bytes"] > 20e6:
                assert r["footprint_estimate"] <= 3 * r["footprint_bytes"], (kind, dims, mode)


def test_oom_rejected_at_submit():
    vag = _vag()
    p = _jobs(1)[0]
    srv = vag.Server(hbm_budget=1 << 20, n_workers=1)
    try:
        with pytest.raises(vag.VagError) as e:
            srv.submit(p, n_steps=2)
        assert e.value.status == vag.VAG_ERR_OOM
    finally:
        srv.close()


def test_cancel_queued_job():
    vag = _vag()
    jobs = _jobs(4)
    srv = vag.Server(n_workers=1)
    try:
        ids = [srv.submit(p, n_steps=p.n_steps) for p in jobs]
        st = srv.cancel(ids[-1])
        res = [srv.wait(i) for i in ids]
    finally:
        srv.close()
    if st == vag.VAG_OK:
        assert res[-1]["status"] == vag.VAG_ERR_CANCELLED and res[-1]["worker"] == -1
    else:  # it had already started
        assert st == vag.VAG_ERR_STATE and res[-1]["status"] == 0
    assert all(r["status"] == 0 for r in res[:-1])


def test_cached_handle_reused_with_new_data():
    vag = _vag()
    p = synth.random_problem((8, 6, 5), 21, n_patches=4, n_steps=10)
    q = synth.random_problem((8, 6, 5), 21, n_patches=4, n_steps=10)
    q.perm = q.perm * 3.0
    q.p_bar = q.p_bar * 2.0
    srv = vag.Server(n_workers=2)
    try:
        r1 = srv.wait(srv.submit(p, n_steps=10, mesh_key=77, **_opts("fp64")))
        r2 = srv.wait(srv.submit(q, n_steps=10, mesh_key=77, **_opts("fp64")))
        st = srv.stats()
    finally:
        srv.close()
    assert r1["reused"] == 0 and r2["reused"] == 1
    assert st["cached_handles"] == 1
    fresh, _ = _run(vag, [q], "fp64", workers=1, together=False)
    for k in OUT:
        np.testing.assert_array_equal(r2[k], fresh[0][k], err_msg=k)
    assert not np.array_equal(r1["u_node"], r2["u_node"])


def test_pool_reuse_and_trim():
    """Handles created and destroyed in turn reuse the library's cached device
    blocks; trimming returns the unused blocks and later handles still work."""
    vag = _vag()
    p = synth.random_problem((7, 6, 5), 9, n_patches=3, n_steps=5)
    ref = None
    for k in range(3):
        h = vag.Handle(p, rtol=1e-12, max_iter=5000)
        h.solve_pressure()
        h.transport(n_steps=5)
        d = vag.to_numpy(h.pressure()) | vag.to_numpy(h.concentration())
        h.close()
        if k == 1:
            vag.trim_memory()
        if ref is None:
            ref = d
        for key in OUT:
            np.testing.assert_array_equal(d[key], ref[key], err_msg=key)


def test_jsonl_records(tmp_path):
    """vag.set_log: one JSON record per solve, transport call and served job,
    with the phases, iterations, residual and the job's times."""
    import json
    vag = _vag()
    path = str(tmp_path / "log.jsonl")
    vag.set_log(path)
    try:
        p = _jobs(1)[0]
        h = vag.Handle(p, **_opts("fp64"))
        h.solve_pressure()
        h.transport(n_steps=3)
        h.close()
        srv = vag.Server(n_workers=1)
        try:
            jid = srv.submit(p, n_steps=3, **_opts("fp64"))
            r = srv.wait(jid)
        finally:
            srv.close()
    finally:
        vag.set_log(None)
    recs = [json.loads(line) for line in open(path)]
    assert [x["kind"] for x in recs] == ["solve", "transport", "job"]
    s, t, j = recs
    assert s["n_cells"] == p.n_cells and s["iterations"] > 0 and s["rel_residual"] <= 1e-10
    assert all(s[k] >= 0 for k in ("ms_assembly", "ms_setup", "ms_solve", "ms_fluxes"))
    assert t["n_steps"] == 3 and len(t["dt_bounds"]) == 3
    assert j["job_id"] == jid and j["status"] == r["status"] == 0
    assert j["t_submit"] <= j["t_start"] <= j["t_end"] and j["solve"]["iterations"] == s["iterations"]
    assert j["transport"]["n_steps"] == 3


def test_general_job_errors():
    """A mesh given by its faces with decreasing offsets is rejected at
    submit; a job whose fracture face index is out of range fails in its own
    result (the library's message), and the jobs around it finish as if alone."""
    import copy
    vag = _vag()
    good = _general_jobs()[:2]
    bad_ptr = copy.copy(good[0])
    bad_ptr.cell_face_ptr = good[0].cell_face_ptr.copy()
    bad_ptr.cell_face_ptr[3] = bad_ptr.cell_face_ptr[2] - 1
    bad_fid = copy.copy(good[1])
    bad_fid.frac_face_ids = good[1].frac_face_ids.copy()
    bad_fid.frac_face_ids[0] = len(good[1].face_node_ptr) + 5
    alone, _ = _run(vag, good, "fp64", workers=1, together=False)
    srv = vag.Server(n_workers=2)
    try:
        with pytest.raises(vag.VagError) as e:
            srv.submit(bad_ptr, n_steps=3)
        assert e.value.status == vag.VAG_ERR_ARG
        ids = [srv.submit(good[0], n_steps=good[0].n_steps, **_opts("fp64")),
               srv.submit(bad_fid, n_steps=3, **_opts("fp64")),
               srv.submit(good[1], n_steps=good[1].n_steps, **_opts("fp64"))]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    finally:
        srv.close()
    assert res[1]["status"] == vag.VAG_ERR_ARG and "out of range" in res[1]["message"]
    for a, m in zip(alone, (res[0], res[2])):
        assert m["status"] == 0
        for k in OUT:
            np.testing.assert_array_equal(a[k], m[k], err_msg=k)
    assert st["bytes_in_use"] == 0


def test_general_cached_handle_reused():
    """A job on a mesh given by its faces keeps its handle under a mesh key; a
    second job on that mesh with new rock and boundary data reuses it and
    equals the same job run on a fresh handle, bitwise."""
    import copy
    vag = _vag()
    p = synth.general_problem("prism", (8, 7, 6), 41, frac_plane=4, n_steps=15)
    q = copy.copy(p)
    q.perm = p.perm * 2.5
    q.frac_perm = p.frac_perm * 0.5
    q.p_bar = p.p_bar * 1.5
    srv = vag.Server(n_workers=2)
    try:
        r1 = srv.wait(srv.submit(p, n_steps=15, mesh_key=91, **_opts("fp64")))
        r2 = srv.wait(srv.submit(q, n_steps=15, mesh_key=91, **_opts("fp64")))
        st = srv.stats()
    finally:
        srv.close()
    assert r1["status"] == 0 and r2["status"] == 0, (r1["message"], r2["message"])
    assert r1["reused"] == 0 and r2["reused"] == 1 and st["cached_handles"] == 1
    fresh, _ = _run(vag, [q], "fp64", workers=1, together=False)
    for k in OUT:
        np.testing.assert_array_equal(r2[k], fresh[0][k], err_msg=k)
    assert not np.array_equal(r1["u_node"], r2["u_node"])
