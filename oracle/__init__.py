"""CPU oracle of the VAG Darcy + upwind transport path — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``vag_oracle.c`` (plain FP64
C, compiled here with gcc) through ctypes and shares no code with the GPU
library in ``paper_1602_03641_amd``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vag_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP on the cell and mat-vec loops)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int64), ("n_cells", C.c_int64), ("n_frac", C.c_int64),
        ("xyz", C.c_void_p), ("hex8", C.c_void_p), ("frac_nodes", C.c_void_p),
        ("frac_width", C.c_void_p), ("frac_perm", C.c_void_p), ("frac_poro", C.c_void_p),
        ("perm", C.c_void_p), ("poro", C.c_void_p), ("mu", C.c_double),
        ("dirichlet", C.c_void_p), ("p_bar", C.c_void_p), ("c_bar", C.c_void_p),
        ("n_wells", C.c_int64), ("well_face", C.c_void_p), ("well_wi", C.c_void_p), ("well_pw", C.c_void_p),
        ("well_q", C.c_void_p), ("well_cinj", C.c_void_p),
    ]


def _lib_handle():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB_PATH)
        P = C.POINTER(_Problem)
        vp = C.c_void_p
        lib.orc_topology.argtypes = [P, vp, vp, vp]
        lib.orc_topology.restype = C.c_int
        lib.orc_cell_matrix.argtypes = [P, C.c_int64, vp, vp, C.POINTER(C.c_int), vp]
        lib.orc_cell_matrix.restype = C.c_double
        lib.orc_frac_matrix.argtypes = [P, C.c_int64, vp]
        lib.orc_frac_matrix.restype = C.c_double
        lib.orc_system_size.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.orc_system_size.restype = C.c_int64
        lib.orc_system_csr.argtypes = [P, vp, vp, vp, vp]
        lib.orc_system_csr.restype = C.c_int
        lib.orc_solve_darcy.argtypes = [P, C.c_double, C.c_int, vp, vp, vp, vp, vp, vp,
                                        C.POINTER(C.c_int), C.POINTER(C.c_double)]
        lib.orc_solve_darcy.restype = C.c_int
        lib.orc_residual.argtypes = [P, vp, vp, vp, vp, vp, vp]
        lib.orc_residual.restype = C.c_int
        lib.orc_porous_volumes.argtypes = [P, C.c_int, vp, vp, vp]
        lib.orc_porous_volumes.restype = C.c_int
        lib.orc_well_rates.argtypes = [P, vp, vp]
        lib.orc_well_rates.restype = C.c_int
        lib.orc_cfl.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_cfl.restype = C.c_int
        lib.orc_transport.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, C.c_double, C.c_int64, C.c_double,
                                      vp, vp, vp]
        lib.orc_transport.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


class OracleProblem:
    """Holds contiguous copies of a ``synth.Problem`` and the C struct view."""

    def __init__(self, prob):
        self.prob = prob
        self.xyz = np.ascontiguousarray(prob.xyz, np.float64)
        self.hex8 = np.ascontiguousarray(prob.hex8, np.int32)
        self.frac_nodes = np.ascontiguousarray(prob.frac_nodes, np.int32).reshape(-1, 4)
        self.frac_width = np.ascontiguousarray(prob.frac_width, np.float64)
        self.frac_perm = np.ascontiguousarray(prob.frac_perm, np.float64)
        self.frac_poro = np.ascontiguousarray(prob.frac_poro, np.float64)
        self.perm = np.ascontiguousarray(prob.perm, np.float64)
        self.poro = np.ascontiguousarray(prob.poro, np.float64)
        self.dirichlet = np.ascontiguousarray(prob.dirichlet, np.uint8)
        self.p_bar = np.ascontiguousarray(prob.p_bar, np.float64)
        self.c_bar = np.ascontiguousarray(prob.c_bar, np.float64)
        self.nn, self.nc, self.nf = len(self.xyz), len(self.hex8), len(self.frac_nodes)
        w = getattr(prob, "wells", None) or {}
        self.well_face = np.ascontiguousarray(w.get("face", []), np.int32)
        self.nw = len(self.well_face)
        self.well_wi, self.well_pw, self.well_q, self.well_cinj = (
            np.ascontiguousarray(w.get(k, np.zeros(self.nw)), np.float64) for k in ("wi", "pw", "q", "cinj"))
        self.s = _Problem(self.nn, self.nc, self.nf, _ptr(self.xyz), _ptr(self.hex8),
                          _ptr(self.frac_nodes), _ptr(self.frac_width), _ptr(self.frac_perm),
                          _ptr(self.frac_poro), _ptr(self.perm), _ptr(self.poro), float(prob.mu),
                          _ptr(self.dirichlet), _ptr(self.p_bar), _ptr(self.c_bar), self.nw,
                          _ptr(self.well_face), _ptr(self.well_wi), _ptr(self.well_pw), _ptr(self.well_q),
                          _ptr(self.well_cinj))

    @property
    def ref(self):
        return C.byref(self.s)


def _as(prob):
    return prob if isinstance(prob, OracleProblem) else OracleProblem(prob)


def topology(prob):
    op = _as(prob)
    cf = np.empty((op.nc, 6), np.int32)
    fc = np.empty((max(op.nf, 1), 2), np.int32)
    fl = np.empty((max(op.nf, 1), 2), np.int32)
    st = _lib_handle().orc_topology(op.ref, _ptr(cf), _ptr(fc), _ptr(fl))
    if st:
        raise ValueError(f"oracle topology error {st}")
    return cf, fc[: op.nf], fl[: op.nf]


def cell_matrix(prob, K, cell_frac6=None, with_full=False):
    """Local VAG matrix a_{K,nu}^{nu'} (m x m), cell volume, optional 15x15 stiffness."""
    op = _as(prob)
    cf = np.full(6, -1, np.int32) if cell_frac6 is None else np.ascontiguousarray(cell_frac6, np.int32)
    a = np.zeros(14 * 14)
    full = np.zeros(15 * 15) if with_full else None
    m = C.c_int(0)
    vol = _lib_handle().orc_cell_matrix(op.ref, int(K), _ptr(cf), _ptr(a), C.byref(m), _ptr(full))
    out = a[: m.value * m.value].reshape(m.value, m.value)
    if with_full:
        return out, vol, full.reshape(15, 15)
    return out, vol


def frac_matrix(prob, f):
    op = _as(prob)
    A5 = np.zeros(25)
    area = _lib_handle().orc_frac_matrix(op.ref, int(f), _ptr(A5))
    return A5.reshape(5, 5), area


def system(prob):
    """Schur-complement system over (free nodes, fracture faces): (CSR arrays, b)."""
    import scipy.sparse as sp
    op = _as(prob)
    n = C.c_int64(0)
    nnz = C.c_int64(0)
    lib = _lib_handle()
    st = lib.orc_system_size(op.ref, C.byref(n), C.byref(nnz))
    if st:
        raise ValueError(f"oracle system error {st}")
    rp = np.zeros(n.value + 1, np.int64)
    col = np.zeros(max(nnz.value, 1), np.int64)
    val = np.zeros(max(nnz.value, 1))
    b = np.zeros(max(n.value, 1))
    lib.orc_system_csr(op.ref, _ptr(rp), _ptr(col), _ptr(val), _ptr(b))
    A = sp.csr_matrix((val[: nnz.value], col[: nnz.value], rp), shape=(n.value, n.value))
    return A, b[: n.value]


def solve_darcy(prob, rtol=1e-12, max_iter=200000):
    op = _as(prob)
    out = dict(
        u_node=np.zeros(op.nn), u_cell=np.zeros(op.nc), u_frac=np.zeros(op.nf),
        F_cell=np.zeros((op.nc, 8)), F_cell_frac=np.zeros((op.nf, 2)), F_frac=np.zeros((op.nf, 4)))
    it = C.c_int(0)
    rr = C.c_double(0)
    st = _lib_handle().orc_solve_darcy(
        op.ref, float(rtol), int(max_iter), _ptr(out["u_node"]), _ptr(out["u_cell"]),
        _ptr(out["u_frac"]), _ptr(out["F_cell"]), _ptr(out["F_cell_frac"]), _ptr(out["F_frac"]),
        C.byref(it), C.byref(rr))
    if st:
        raise ValueError(f"oracle darcy error {st}")
    out["iters"] = it.value
    out["relres"] = rr.value
    out["well_rate"] = np.zeros(op.nw)
    if op.nw:
        _lib_handle().orc_well_rates(op.ref, _ptr(out["u_frac"]), _ptr(out["well_rate"]))
    return out


def residual(prob, u_node, u_frac):
    """Rows of b - A x of the system at the given pressures (the conservation
    equations of the free nodes and fracture faces, evaluated cell by cell
    without assembling A) and b itself: dict of res_node, res_frac, b_node,
    b_frac (0 at Dirichlet nodes) and the relative residual ||b - A x|| / ||b||."""
    op = _as(prob)
    u_node = np.ascontiguousarray(u_node, np.float64)
    u_frac = np.ascontiguousarray(u_frac, np.float64)
    out = dict(res_node=np.zeros(op.nn), res_frac=np.zeros(op.nf), b_node=np.zeros(op.nn), b_frac=np.zeros(op.nf))
    st = _lib_handle().orc_residual(op.ref, _ptr(u_node), _ptr(u_frac), _ptr(out["res_node"]), _ptr(out["res_frac"]),
                                    _ptr(out["b_node"]), _ptr(out["b_frac"]))
    if st:
        raise ValueError(f"oracle residual error {st}")
    r2 = float(out["res_node"] @ out["res_node"] + out["res_frac"] @ out["res_frac"])
    b2 = float(out["b_node"] @ out["b_node"] + out["b_frac"] @ out["b_frac"])
    out["rel_residual"] = math.sqrt(r2 / b2) if b2 > 0 else math.sqrt(r2)
    return out


def porous_volumes(prob, alpha_rule=0):
    """Porous volumes of §3.2.1; alpha_rule 1: only the largest-permeability
    cells (fracture faces) around a node give it a share."""
    op = _as(prob)
    out = dict(phi_cell=np.zeros(op.nc), phi_frac=np.zeros(op.nf), phi_node=np.zeros(op.nn))
    st = _lib_handle().orc_porous_volumes(op.ref, int(alpha_rule), _ptr(out["phi_cell"]), _ptr(out["phi_frac"]),
                                          _ptr(out["phi_node"]))
    if st:
        raise ValueError(f"oracle porous volume error {st}")
    return out


def _rates(op, flux):
    """Well rates of a flux dict (solve_darcy's, or given); None without wells."""
    if not op.nw:
        return None
    q = flux.get("well_rate")
    if q is None:
        raise ValueError("the problem has wells: the fluxes need their well_rate")
    return np.ascontiguousarray(q, np.float64)


def peaceman_wi(dx, dz, df, lam_f, rw):
    """Well index of a fracture face perforated by a vertical well (§5.5,
    Peaceman's method on the face expanded to a dx x df x dz box):
    WI = 2 pi dz lam_f / ln(r0 / rw), r0 = D exp(-2 pi dz / C),
    C = 4/3 (dx dz / df + dx df / dz + dz df / dx), D = sqrt(dx^2 + df^2) / 2."""
    C = 4.0 / 3.0 * (dx * dz / df + dx * df / dz + dz * df / dx)
    D = 0.5 * math.sqrt(dx * dx + df * df)
    r0 = D * math.exp(-2.0 * math.pi * dz / C)
    return 2.0 * math.pi * dz * lam_f / math.log(r0 / rw)


def cfl_bounds(prob, flux, phi):
    op = _as(prob)
    dt3 = np.zeros(3)
    st = _lib_handle().orc_cfl(op.ref, _ptr(flux["F_cell"]), _ptr(flux["F_cell_frac"]),
                               _ptr(flux["F_frac"]), _ptr(_rates(op, flux)), _ptr(phi["phi_cell"]),
                               _ptr(phi["phi_frac"]),
                               _ptr(phi["phi_node"]), _ptr(dt3))
    if st:
        raise ValueError(f"oracle cfl error {st}")
    return dt3


def transport(prob, flux, phi, dt, n_steps, last_dt=0.0, c0=None):
    op = _as(prob)
    c_cell = np.zeros(op.nc) if c0 is None else np.array(c0["c_cell"], np.float64)
    c_frac = np.zeros(op.nf) if c0 is None else np.array(c0["c_frac"], np.float64)
    c_node = np.zeros(op.nn) if c0 is None else np.array(c0["c_node"], np.float64)
    st = _lib_handle().orc_transport(
        op.ref, _ptr(flux["F_cell"]), _ptr(flux["F_cell_frac"]), _ptr(flux["F_frac"]),
        _ptr(_rates(op, flux)), _ptr(phi["phi_cell"]), _ptr(phi["phi_frac"]), _ptr(phi["phi_node"]), float(dt),
        int(n_steps), float(last_dt), _ptr(c_cell), _ptr(c_frac), _ptr(c_node))
    if st:
        raise ValueError(f"oracle transport error {st}")
    return dict(c_cell=c_cell, c_frac=c_frac, c_node=c_node)


def time_grid(dt, t_final):
    """§4.3 step 2: N = ceil(T/dt) steps of dt, the last one T - (N-1) dt."""
    N = max(1, math.ceil(t_final / dt))
    return N, t_final - (N - 1) * dt


def run(prob, rtol=None, max_iter=200000, n_steps=None, cfl=None, t_final=None, alpha_rule=0):
    """Darcy solve, porous volumes, CFL time step, then the transport steps."""
    op = _as(prob)
    p = op.prob
    rtol = p.rtol if rtol is None else rtol
    cfl = p.cfl if cfl is None else cfl
    t_final = p.t_final if t_final is None else t_final
    n_steps = p.n_steps if n_steps is None else n_steps
    darcy = solve_darcy(op, rtol, max_iter)
    phi = porous_volumes(op, alpha_rule)
    dt3 = cfl_bounds(op, darcy, phi)
    dt = cfl * float(np.min(dt3))
    last = 0.0
    if t_final and t_final > 0:
        n_steps, last = time_grid(dt, t_final)
    c = transport(op, darcy, phi, dt, n_steps, last)
    return dict(darcy=darcy, phi=phi, dt3=dt3, dt=dt, n_steps=n_steps, last_dt=last, **c)
