"""Python binding of libvag (argument marshalling only).

The functions ``vag_*`` mirror the C-ABI of ``include/vag.h`` one to one.
``Handle`` is a convenience owner of a ``vag_handle*`` that keeps inputs and
outputs in torch tensors on the GPU (torch provides device memory and the
stream; every step of the computation runs in the library's HIP kernels).

The library must be built (``paper_1602_03641_amd.build.build()``); loading
fails loudly otherwise — there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvag.so")
_log_path = os.environ.get("VAG_LOG_JSONL") or None

VAG_OK, VAG_WARN_NOT_CONVERGED = 0, 1
VAG_ERR_ARG, VAG_ERR_MESH, VAG_ERR_UNSUPPORTED, VAG_ERR_OOM, VAG_ERR_HIP, VAG_ERR_STATE = -1, -2, -3, -4, -5, -6
VAG_ERR_TIMEOUT, VAG_ERR_CANCELLED = -7, -8
VAG_MEM_HOST, VAG_MEM_DEVICE = 0, 1
VAG_FP64, VAG_MIXED, VAG_MIXED_IR = 0, 1, 2
VAG_CG, VAG_GMRES, VAG_BICGSTAB = 0, 1, 2
VAG_PC_JACOBI, VAG_PC_AMG, VAG_PC_BJILU0 = 0, 1, 2
VAG_KERNEL_SPMV, VAG_KERNEL_TRANSPORT_STEP, VAG_KERNEL_LOCAL, VAG_KERNEL_PRECOND = 0, 1, 2, 3

STATUS_NAMES = {0: "VAG_OK", 1: "VAG_WARN_NOT_CONVERGED", -1: "VAG_ERR_ARG", -2: "VAG_ERR_MESH",
                -3: "VAG_ERR_UNSUPPORTED", -4: "VAG_ERR_OOM", -5: "VAG_ERR_HIP", -6: "VAG_ERR_STATE",
                -7: "VAG_ERR_TIMEOUT", -8: "VAG_ERR_CANCELLED"}

vp = C.c_void_p


class vag_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_cells", C.c_int64), ("node_xyz", vp), ("hex8", vp),
                ("n_faces", C.c_int64), ("cell_face_ptr", vp), ("cell_faces", vp), ("face_node_ptr", vp),
                ("face_nodes", vp)]


class vag_fractures(C.Structure):
    _fields_ = [("n_frac", C.c_int64), ("face_nodes", vp), ("width", vp), ("perm", vp), ("porosity", vp),
                ("face_ids", vp)]


class vag_rock(C.Structure):
    _fields_ = [("perm", vp), ("porosity", vp), ("mu", C.c_double)]


class vag_bc(C.Structure):
    _fields_ = [("node_dirichlet", vp), ("p_bar", vp), ("c_bar", vp)]


class vag_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("krylov", C.c_int), ("precond", C.c_int), ("rtol", C.c_double),
                ("inner_rtol", C.c_double), ("max_iter", C.c_int), ("gmres_restart", C.c_int),
                ("check_every", C.c_int), ("cfl", C.c_double), ("amg_coarse_size", C.c_int),
                ("amg_max_levels", C.c_int), ("amg_theta", C.c_double), ("amg_sweeps", C.c_int),
                ("eliminate_frac_faces", C.c_int), ("amg_aggregate_hops", C.c_int), ("amg_kcycle", C.c_int),
                ("ilu_block_rows", C.c_int), ("amg_kind", C.c_int),
                ("amg_strong_theta", C.c_double), ("stream_loads", C.c_int),
                ("alpha_rule", C.c_int)]


class vag_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer_iterations", C.c_int), ("rel_residual", C.c_double),
                ("n_unknowns", C.c_int64), ("nnz", C.c_int64), ("amg_levels", C.c_int),
                ("amg_operator_complexity", C.c_double), ("ms_assembly", C.c_double),
                ("ms_setup", C.c_double), ("ms_solve", C.c_double), ("ms_fluxes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vag_transport_info(C.Structure):
    _fields_ = [("n_steps", C.c_int64), ("dt", C.c_double), ("last_dt", C.c_double),
                ("dt_bounds", C.c_double * 3), ("ms_setup", C.c_double), ("ms_steps", C.c_double),
                ("n_rows", C.c_int64), ("t_nnz", C.c_int64), ("t_stored", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["dt_bounds"] = list(self.dt_bounds)
        return d


class vag_job(C.Structure):
    _fields_ = [("mesh", C.POINTER(vag_mesh)), ("frac", C.POINTER(vag_fractures)), ("rock", C.POINTER(vag_rock)),
                ("bc", C.POINTER(vag_bc)), ("opt", C.POINTER(vag_options)), ("n_steps", C.c_int64),
                ("t_final", C.c_double), ("mesh_key", C.c_uint64),
                ("u_node", vp), ("u_cell", vp), ("u_frac", vp), ("c_cell", vp), ("c_frac", vp), ("c_node", vp)]


class vag_job_result(C.Structure):
    _fields_ = [("status", C.c_int), ("message", C.c_char * 200), ("solve", vag_solve_info),
                ("transport", vag_transport_info), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_end", C.c_double), ("worker", C.c_int), ("reused", C.c_int),
                ("footprint_estimate", C.c_size_t), ("footprint_bytes", C.c_size_t),
                ("ms_create", C.c_double), ("ms_run", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["message"] = self.message.decode(errors="replace")
        d["solve"] = self.solve.as_dict()
        d["transport"] = self.transport.as_dict()
        return d


class vag_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("queued", C.c_int64), ("running", C.c_int64), ("finished", C.c_int64),
                ("budget", C.c_size_t), ("bytes_in_use", C.c_size_t), ("peak_bytes_in_use", C.c_size_t),
                ("cached_bytes", C.c_size_t), ("cached_handles", C.c_int), ("step_launches", C.c_int64),
                ("job_steps", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (argtypes, restype)
_SIGS = {
    "vag_version": ([], C.c_char_p),
    "vag_default_options": ([C.POINTER(vag_options)], C.c_int),
    "vag_create": ([C.POINTER(vag_mesh), C.POINTER(vag_fractures), C.POINTER(vag_rock), C.POINTER(vag_bc),
                    C.POINTER(vag_options), C.c_int, vp, C.POINTER(vp)], C.c_int),
    "vag_update": ([vp, C.POINTER(vag_rock), C.POINTER(vag_fractures), vp, vp, C.c_int], C.c_int),
    "vag_set_stream": ([vp, vp], C.c_int),
    "vag_trim_memory": ([], C.c_int),
    "vag_set_options": ([vp, C.POINTER(vag_options)], C.c_int),
    "vag_solve_pressure": ([vp, C.POINTER(vag_solve_info)], C.c_int),
    "vag_transport": ([vp, C.c_int64, C.c_double, vp, vp, vp, C.c_int, C.POINTER(vag_transport_info)], C.c_int),
    "vag_transport_noalloc": ([vp, C.c_int64, C.c_double, vp, vp, vp, vp, vp, vp,
                               C.POINTER(vag_transport_info)], C.c_int),
    "vag_set_fluxes": ([vp, vp, vp, vp, C.c_int], C.c_int),
    "vag_get_pressure": ([vp, vp, vp, vp, C.c_int], C.c_int),
    "vag_get_fluxes": ([vp, vp, vp, vp, C.c_int], C.c_int),
    "vag_flux_layout": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "vag_get_porous_volumes": ([vp, vp, vp, vp, C.c_int], C.c_int),
    "vag_get_concentration": ([vp, vp, vp, vp, C.c_int], C.c_int),
    "vag_system_size": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "vag_get_system": ([vp, vp, vp, vp, vp, C.c_int], C.c_int),
    "vag_benchmark_kernel": ([vp, C.c_int, C.c_int, C.POINTER(C.c_double)], C.c_int),
    "vag_apply_preconditioner": ([vp, vp, vp, C.c_int], C.c_int),
    "vag_set_wells": ([vp, C.c_int64, vp, vp, vp, vp, vp, C.c_int], C.c_int),
    "vag_get_well_rates": ([vp, vp, C.c_int], C.c_int),
    "vag_set_well_rates": ([vp, vp, C.c_int], C.c_int),
    "vag_peaceman_wi": ([C.c_double] * 5, C.c_double),
    "vag_amg_level_csr": ([vp, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
    "vag_amg_levels": ([vp, C.POINTER(C.c_int), vp, vp, vp, C.c_int], C.c_int),
    "vag_footprint_bytes": ([vp], C.c_size_t),
    "vag_last_error": ([vp], C.c_char_p),
    "vag_destroy": ([vp], None),
    "vag_estimate_footprint": ([C.c_int64, C.c_int64, C.c_int64, C.POINTER(vag_options)], C.c_size_t),
    "vag_estimate_footprint_mesh": ([C.POINTER(vag_mesh), C.c_int64, C.POINTER(vag_options)], C.c_size_t),
    "vag_server_create": ([C.c_size_t, C.c_int, C.POINTER(vp)], C.c_int),
    "vag_server_submit": ([vp, C.POINTER(vag_job), C.POINTER(C.c_uint64)], C.c_int),
    "vag_server_wait": ([vp, C.c_uint64, C.c_double, C.POINTER(vag_job_result)], C.c_int),
    "vag_server_cancel": ([vp, C.c_uint64], C.c_int),
    "vag_server_get_stats": ([vp, C.POINTER(vag_server_stats)], C.c_int),
    "vag_server_clock": ([vp], C.c_double),
    "vag_server_destroy": ([vp], None),
}

_lib = None


def load():
    """Loads libvag.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1602_03641_amd.build.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def __getattr__(name):  # vag_* functions resolve to the C symbols
    if name.startswith("vag_") and name in _SIGS:
        return getattr(load(), name)
    raise AttributeError(name)


def set_log(path):
    """Appends one JSON record per line to `path` for every pressure solve,
    transport call and served job (None turns the log off).  The environment
    variable VAG_LOG_JSONL sets the path when the module is imported."""
    global _log_path
    _log_path = path


def _log(kind, rec):
    if not _log_path:
        return
    line = json.dumps({"kind": kind, "unix_time": time.time(), **rec},
                      default=lambda o: list(o) if hasattr(o, "__len__") else str(o))
    with open(_log_path, "a") as f:
        f.write(line + "\n")


class VagError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def default_options(**kw) -> vag_options:
    o = vag_options()
    load().vag_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


class Handle:
    """Owns a vag_handle built from a problem description (numpy arrays).

    Inputs are moved to the GPU as torch tensors and passed as device memory;
    the handle is bound to torch's current HIP stream.
    """

    def __init__(self, prob, options=None, device="cuda", **opt_kw):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        lib = load()
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.device)  # noqa: E731
        # general cells (cell -> faces, face -> nodes) when the problem gives faces
        self.general = getattr(prob, "face_node_ptr", None) is not None
        self.nn, self.nc = int(prob.xyz.shape[0]), int(prob.n_cells)
        self.nf = int(len(prob.frac_face_ids) if self.general else prob.frac_nodes.shape[0])
        self._in = dict(
            xyz=t(prob.xyz, torch.float64),
            frac_width=t(prob.frac_width, torch.float64), frac_perm=t(prob.frac_perm, torch.float64),
            frac_poro=t(prob.frac_poro, torch.float64), perm=t(prob.perm, torch.float64),
            poro=t(prob.poro, torch.float64), dirichlet=t(prob.dirichlet, torch.uint8),
            p_bar=t(prob.p_bar, torch.float64), c_bar=t(prob.c_bar, torch.float64))
        i = self._in
        if self.general:
            i.update(cfp=t(prob.cell_face_ptr, torch.int64), cf=t(prob.cell_faces, torch.int32),
                     fnp=t(prob.face_node_ptr, torch.int64), fn=t(prob.face_nodes, torch.int32),
                     fid=t(prob.frac_face_ids, torch.int32))
            self.mesh = vag_mesh(self.nn, self.nc, _dptr(i["xyz"]), None, int(len(prob.face_node_ptr) - 1),
                                 _dptr(i["cfp"]), _dptr(i["cf"]), _dptr(i["fnp"]), _dptr(i["fn"]))
            self.frac = vag_fractures(self.nf, None, _dptr(i["frac_width"]), _dptr(i["frac_perm"]),
                                      _dptr(i["frac_poro"]), _dptr(i["fid"]))
        else:
            i.update(hex8=t(prob.hex8, torch.int32),
                     frac_nodes=t(np.asarray(prob.frac_nodes).reshape(-1, 4), torch.int32))
            self.mesh = vag_mesh(self.nn, self.nc, _dptr(i["xyz"]), _dptr(i["hex8"]))
            self.frac = vag_fractures(self.nf, _dptr(i["frac_nodes"]), _dptr(i["frac_width"]),
                                      _dptr(i["frac_perm"]), _dptr(i["frac_poro"]))
        self.rock = vag_rock(_dptr(i["perm"]), _dptr(i["poro"]), float(prob.mu))
        self.bc = vag_bc(_dptr(i["dirichlet"]), _dptr(i["p_bar"]), _dptr(i["c_bar"]))
        self.options = options if options is not None else default_options(**opt_kw)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = C.c_void_p()
        st = lib.vag_create(C.byref(self.mesh), C.byref(self.frac), C.byref(self.rock), C.byref(self.bc),
                            C.byref(self.options), VAG_MEM_DEVICE, C.c_void_p(stream), C.byref(h))
        if st != VAG_OK:
            raise VagError(st, lib.vag_last_error(None).decode())
        self.h = h
        ncf, nff = C.c_int64(), C.c_int64()
        lib.vag_flux_layout(h, C.byref(ncf), C.byref(nff))
        self.n_cell_flux, self.n_frac_flux = ncf.value, nff.value
        self.nw = 0
        w = getattr(prob, "wells", None)
        if w:
            self.set_wells(w["face"], w["wi"], w["pw"], w["q"], w["cinj"])

    def _check(self, st):
        if st < 0:
            raise VagError(st, load().vag_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            load().vag_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.options, k, v)
        self._check(load().vag_set_options(self.h, C.byref(self.options)))

    def _sizes(self):
        o = self.options
        return dict(n_cells=self.nc, n_nodes=self.nn, n_frac=self.nf, general=self.general,
                    options=dict(precision=o.precision, krylov=o.krylov, precond=o.precond, rtol=o.rtol))

    def solve_pressure(self):
        info = vag_solve_info()
        st = self._check(load().vag_solve_pressure(self.h, C.byref(info)))
        d = info.as_dict()
        d["status"] = st
        _log("solve", {**self._sizes(), **d})
        return d

    def transport(self, n_steps=0, t_final=0.0, c0=None):
        info = vag_transport_info()
        args = (None, None, None)
        if c0 is not None:
            tt = [self.torch.as_tensor(np.ascontiguousarray(c0[k]), dtype=self.torch.float64, device=self.device)
                  for k in ("c_cell", "c_frac", "c_node")]
            self._c0 = tt
            args = tuple(_dptr(x) for x in tt)
        self._check(load().vag_transport(self.h, int(n_steps), float(t_final), *args, VAG_MEM_DEVICE,
                                         C.byref(info)))
        d = info.as_dict()
        d["dt_bounds"] = list(d["dt_bounds"])
        _log("transport", {**self._sizes(), **d})
        return d

    def transport_noalloc(self, n_steps=0, t_final=0.0, c0=None, info=True):
        """vag_transport_noalloc: the steps gathered from the fluxes, with the
        library's static scratch; returns (concentrations as device tensors,
        info dict or None)."""
        args = (None, None, None)
        if c0 is not None:
            tt = [self.torch.as_tensor(np.ascontiguousarray(c0[k]) if not hasattr(c0[k], "data_ptr") else c0[k],
                                       dtype=self.torch.float64, device=self.device)
                  for k in ("c_cell", "c_frac", "c_node")]
            self._c0 = tt
            args = tuple(_dptr(x) for x in tt)
        out = [self.torch.empty(n, dtype=self.torch.float64, device=self.device) for n in (self.nc, self.nf, self.nn)]
        ti = vag_transport_info() if info else None
        self._check(load().vag_transport_noalloc(self.h, int(n_steps), float(t_final), *args,
                                                 *[_dptr(o) for o in out], C.byref(ti) if info else None))
        return dict(c_cell=out[0], c_frac=out[1], c_node=out[2]), (ti.as_dict() if info else None)

    def set_fluxes(self, flux):
        tt = [self.torch.as_tensor(np.ascontiguousarray(flux[k]), dtype=self.torch.float64, device=self.device)
              for k in ("F_cell", "F_cell_frac", "F_frac")]
        self._check(load().vag_set_fluxes(self.h, *[_dptr(x) for x in tt], VAG_MEM_DEVICE))

    def _get3(self, fn, shapes):
        outs = [self.torch.empty(s, dtype=self.torch.float64, device=self.device) for s in shapes]
        self._check(fn(self.h, *[_dptr(o) for o in outs], VAG_MEM_DEVICE))
        return outs

    def pressure(self):
        u_node, u_cell, u_frac = self._get3(load().vag_get_pressure, [(self.nn,), (self.nc,), (self.nf,)])
        return dict(u_node=u_node, u_cell=u_cell, u_frac=u_frac)

    def fluxes(self):
        """F_cell [n_cells, 8] and F_frac [n_frac, 4] on hexahedra; on general
        cells both flat (cell after cell, face after face: vag_flux_layout)."""
        if self.general:
            shapes = [(self.n_cell_flux,), (self.nf, 2), (self.n_frac_flux,)]
        else:
            shapes = [(self.nc, 8), (self.nf, 2), (self.nf, 4)]
        a, b, c = self._get3(load().vag_get_fluxes, shapes)
        return dict(F_cell=a, F_cell_frac=b, F_frac=c)

    def porous_volumes(self):
        a, b, c = self._get3(load().vag_get_porous_volumes, [(self.nc,), (self.nf,), (self.nn,)])
        return dict(phi_cell=a, phi_frac=b, phi_node=c)

    def concentration(self):
        a, b, c = self._get3(load().vag_get_concentration, [(self.nc,), (self.nf,), (self.nn,)])
        return dict(c_cell=a, c_frac=b, c_node=c)

    def system(self):
        n = C.c_int64()
        nnz = C.c_int64()
        self._check(load().vag_system_size(self.h, C.byref(n), C.byref(nnz)))
        rp = np.zeros(n.value + 1, np.int64)
        col = np.zeros(nnz.value, np.int64)
        val = np.zeros(nnz.value)
        b = np.zeros(n.value)
        p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._check(load().vag_get_system(self.h, p(rp), p(col), p(val), p(b), VAG_MEM_HOST))
        return rp, col, val, b

    def set_wells(self, face, wi, pw, q, cinj):
        """Peaceman wells on fracture faces (host arrays)."""
        face = np.ascontiguousarray(face, np.int32)
        arr = [np.ascontiguousarray(a, np.float64) for a in (wi, pw, q, cinj)]
        p = lambda a: a.ctypes.data_as(C.c_void_p) if a.size else None  # noqa: E731
        self._check(load().vag_set_wells(self.h, len(face), p(face), *(p(a) for a in arr), VAG_MEM_HOST))
        self.nw = len(face)

    def well_rates(self):
        Q = np.zeros(self.nw)
        self._check(load().vag_get_well_rates(self.h, Q.ctypes.data_as(C.c_void_p) if self.nw else None,
                                              VAG_MEM_HOST))
        return Q

    def set_well_rates(self, Q):
        Q = np.ascontiguousarray(Q, np.float64)
        self._check(load().vag_set_well_rates(self.h, Q.ctypes.data_as(C.c_void_p) if Q.size else None,
                                              VAG_MEM_HOST))

    def apply_preconditioner(self, r):
        """z = M^-1 r (host arrays, the unknown order of system())."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._check(load().vag_apply_preconditioner(self.h, p(r), p(z), VAG_MEM_HOST))
        return z

    def amg_level(self, level):
        """Level `level` of the hierarchy: dict with A (CSR arrays), P (CSR
        arrays, None on the coarsest level), n_coarse and coarse_index."""
        sz = np.zeros(4, np.int64)
        p = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None  # noqa: E731
        lib = load()
        self._check(lib.vag_amg_level_csr(self.h, int(level), p(sz), None, None, None, None, None, None, None))
        n, annz, nc, pnnz = (int(v) for v in sz)
        ap, ac, av = np.zeros(n + 1, np.int64), np.zeros(annz, np.int64), np.zeros(annz)
        pp, pc, pv = np.zeros(n + 1, np.int64), np.zeros(pnnz, np.int64), np.zeros(pnnz)
        ci = np.zeros(n, np.int32)
        self._check(lib.vag_amg_level_csr(self.h, int(level), p(sz), p(ap), p(ac), p(av), p(pp), p(pc), p(pv), p(ci)))
        return dict(A=(ap, ac, av), P=(pp, pc, pv) if nc else None, n_coarse=nc, coarse_index=ci)

    def benchmark_kernel(self, kernel, reps=50):
        ms = C.c_double()
        self._check(load().vag_benchmark_kernel(self.h, int(kernel), int(reps), C.byref(ms)))
        return ms.value

    def amg_levels(self):
        """[(rows, nonzeros, stored entries)] per level of the last solve's hierarchy."""
        nl = C.c_int()
        rows, nnz, stored = (np.zeros(32, np.int64) for _ in range(3))
        p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._check(load().vag_amg_levels(self.h, C.byref(nl), p(rows), p(nnz), p(stored), 32))
        return [(int(rows[i]), int(nnz[i]), int(stored[i])) for i in range(nl.value)]

    def footprint_bytes(self):
        return int(load().vag_footprint_bytes(self.h))


def trim_memory():
    """Return the library's cached (unused) device blocks to the system."""
    st = load().vag_trim_memory()
    if st != VAG_OK:
        raise VagError(st, "vag_trim_memory failed")


def to_numpy(d):
    return {k: v.detach().cpu().numpy() if hasattr(v, "detach") else v for k, v in d.items()}


def _host_mesh(prob):
    """The mesh and fracture structs of a problem in either form, over host
    copies of its arrays (returned too: they must outlive the structs)."""
    c = np.ascontiguousarray
    p = lambda a: a.ctypes.data_as(C.c_void_p) if a.size else None  # noqa: E731
    keep = dict(xyz=c(prob.xyz, np.float64), fw=c(prob.frac_width, np.float64), fk=c(prob.frac_perm, np.float64),
                fp=c(prob.frac_poro, np.float64))
    nn = int(prob.xyz.shape[0])
    if getattr(prob, "face_node_ptr", None) is not None:
        keep.update(cfp=c(prob.cell_face_ptr, np.int64), cf=c(prob.cell_faces, np.int32),
                    fnp=c(prob.face_node_ptr, np.int64), fn=c(prob.face_nodes, np.int32),
                    fid=c(prob.frac_face_ids, np.int32))
        nc, nf = int(prob.n_cells), len(keep["fid"])
        mesh = vag_mesh(nn, nc, p(keep["xyz"]), None, len(keep["fnp"]) - 1, p(keep["cfp"]), p(keep["cf"]),
                        p(keep["fnp"]), p(keep["fn"]))
        frac = vag_fractures(nf, None, p(keep["fw"]), p(keep["fk"]), p(keep["fp"]), p(keep["fid"]))
    else:
        keep.update(hex8=c(prob.hex8, np.int32), fnodes=c(np.asarray(prob.frac_nodes, np.int32).reshape(-1, 4)))
        nc, nf = int(prob.hex8.shape[0]), int(keep["fnodes"].shape[0])
        mesh = vag_mesh(nn, nc, p(keep["xyz"]), p(keep["hex8"]))
        frac = vag_fractures(nf, p(keep["fnodes"]), p(keep["fw"]), p(keep["fk"]), p(keep["fp"]))
    return keep, mesh, frac


def estimate_footprint(prob, **opt_kw):
    """vag_estimate_footprint_mesh of the problem's mesh (either form)."""
    o = default_options(**opt_kw)
    keep, mesh, frac = _host_mesh(prob)
    return int(load().vag_estimate_footprint_mesh(C.byref(mesh), int(frac.n_frac), C.byref(o)))


class Server:
    """Owns a vag_server.  Jobs are problem descriptions (numpy arrays, host
    memory); results come back as numpy arrays with the job's timing."""

    OUTPUTS = ("u_node", "u_cell", "u_frac", "c_cell", "c_frac", "c_node")

    def __init__(self, hbm_budget=0, n_workers=4):
        lib = load()
        s = C.c_void_p()
        st = lib.vag_server_create(C.c_size_t(int(hbm_budget)), int(n_workers), C.byref(s))
        if st != VAG_OK:
            raise VagError(st, "vag_server_create failed")
        self.s = s
        self._jobs = {}

    def submit(self, prob, n_steps=0, t_final=0.0, mesh_key=0, outputs=OUTPUTS, **opt_kw):
        """Queues one job (a hex8 problem or one given by its faces); returns
        its id.  The server copies the inputs."""
        keep, mesh, frac = _host_mesh(prob)
        nn, nc, nf = int(mesh.n_nodes), int(mesh.n_cells), int(frac.n_frac)
        keep.update(perm=np.ascontiguousarray(prob.perm, np.float64), poro=np.ascontiguousarray(prob.poro, np.float64),
                    dir=np.ascontiguousarray(prob.dirichlet, np.uint8), pb=np.ascontiguousarray(prob.p_bar, np.float64),
                    cb=np.ascontiguousarray(prob.c_bar, np.float64))
        p = lambda a: a.ctypes.data_as(C.c_void_p) if a.size else None  # noqa: E731
        rock = vag_rock(p(keep["perm"]), p(keep["poro"]), float(prob.mu))
        bc = vag_bc(p(keep["dir"]), p(keep["pb"]), p(keep["cb"]))
        opt = default_options(**opt_kw)
        sizes = dict(u_node=nn, u_cell=nc, u_frac=nf, c_cell=nc, c_frac=nf, c_node=nn)
        outs = {k: np.empty(sizes[k]) for k in outputs}
        job = vag_job(C.pointer(mesh), C.pointer(frac), C.pointer(rock), C.pointer(bc), C.pointer(opt),
                      int(n_steps), float(t_final), int(mesh_key),
                      *[p(outs[k]) if k in outs else None for k in self.OUTPUTS])
        jid = C.c_uint64()
        st = load().vag_server_submit(self.s, C.byref(job), C.byref(jid))
        if st != VAG_OK:
            raise VagError(st, "vag_server_submit failed")
        self._jobs[jid.value] = outs  # output buffers stay alive until wait()
        return jid.value

    def wait(self, job_id, timeout=-1.0):
        """Result dict (status, timing, solve/transport info, output arrays),
        or None on timeout."""
        res = vag_job_result()
        st = load().vag_server_wait(self.s, C.c_uint64(job_id), float(timeout), C.byref(res))
        if st == VAG_ERR_TIMEOUT:
            return None
        if st != VAG_OK:
            raise VagError(st, f"vag_server_wait({job_id})")
        d = res.as_dict()
        d["transport"]["dt_bounds"] = list(d["transport"]["dt_bounds"])
        _log("job", {"job_id": job_id, **d})
        d.update(self._jobs.pop(job_id))
        return d

    def cancel(self, job_id):
        return load().vag_server_cancel(self.s, C.c_uint64(job_id))

    def stats(self):
        st = vag_server_stats()
        load().vag_server_get_stats(self.s, C.byref(st))
        return st.as_dict()

    def clock(self):
        return load().vag_server_clock(self.s)

    def close(self):
        if getattr(self, "s", None):
            load().vag_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def peaceman_wi(dx, dz, d_f, lambda_f, r_w):
    """Peaceman well index of a fracture face (the library's closed form)."""
    return float(load().vag_peaceman_wi(dx, dz, d_f, lambda_f, r_w))
