"""Seeded generators for hexahedral meshes with fracture faces.

Conventions shared by every consumer (they describe the *input format*, not
any computation of the scheme):

* Logical grid of ``nx * ny * nz`` hexahedra.  Node ``(i, j, k)`` has index
  ``i + (nx+1) * (j + (ny+1) * k)``; cell ``(i, j, k)`` has index
  ``i + nx * (j + ny * k)``.
* ``hex8[c]`` lists the cell's 8 nodes in VTK order: the bottom quad
  ``(i,j,k) (i+1,j,k) (i+1,j+1,k) (i,j+1,k)`` then the same four at ``k+1``.
* A fracture is a set of mesh faces (the paper's conforming assumption, §3.1);
  each fracture face is given by its 4 node indices in cyclic order.
* Permeability tensors are packed ``[xx, yy, zz, xy, xz, yz]``.
* Dirichlet nodes carry ``p_bar`` (pressure) and ``c_bar`` (injected
  concentration); every other node gets a conservation equation.

Random draws use ``numpy.random.default_rng(seed)`` in a fixed, documented order
so the same problem is rebuilt bit for bit on every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    dims: tuple
    xyz: np.ndarray          # [n_nodes, 3] float64
    hex8: np.ndarray         # [n_cells, 8] int32
    frac_nodes: np.ndarray   # [n_frac, 4] int32
    frac_width: np.ndarray   # [n_frac] float64   d_f
    frac_perm: np.ndarray    # [n_frac] float64   Lambda_f (isotropic in plane)
    frac_poro: np.ndarray    # [n_frac] float64   phi_f
    perm: np.ndarray         # [n_cells, 6] float64
    poro: np.ndarray         # [n_cells] float64  phi_m
    mu: float
    dirichlet: np.ndarray    # [n_nodes] uint8
    p_bar: np.ndarray        # [n_nodes] float64
    c_bar: np.ndarray        # [n_nodes] float64
    rtol: float = 1e-10
    cfl: float = 0.9
    n_steps: int = 50
    t_final: float = 0.0     # > 0: integrate to this time, last step shortened
    meta: dict = field(default_factory=dict)
    # wells on fracture faces: dict of arrays face, wi, pw, q, cinj (None: no wells)
    wells: dict = None

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.hex8.shape[0])

    @property
    def n_frac(self) -> int:
        return int(self.frac_nodes.shape[0])


# ----------------------------------------------------------------------------
# grid topology
# ----------------------------------------------------------------------------

def node_index(dims, i, j, k):
    nx, ny, _ = dims
    return i + (nx + 1) * (j + (ny + 1) * k)


def structured_hex(nx: int, ny: int, nz: int):
    """Unit-box coordinates and VTK-ordered connectivity of a logical grid."""
    i = np.arange(nx + 1, dtype=np.float64) / nx
    j = np.arange(ny + 1, dtype=np.float64) / ny
    k = np.arange(nz + 1, dtype=np.float64) / nz
    zz, yy, xx = np.meshgrid(k, j, i, indexing="ij")
    xyz = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    dims = (nx, ny, nz)
    n = lambda a, b, c: node_index(dims, a, b, c)  # noqa: E731
    hex8 = np.stack([
        n(ci, cj, ck), n(ci + 1, cj, ck), n(ci + 1, cj + 1, ck), n(ci, cj + 1, ck),
        n(ci, cj, ck + 1), n(ci + 1, cj, ck + 1), n(ci + 1, cj + 1, ck + 1), n(ci, cj + 1, ck + 1),
    ], axis=1).astype(np.int32)
    return xyz, hex8


def plane_faces(dims, axis: int, plane: int, a_lo: int, a_hi: int, b_lo: int, b_hi: int):
    """Grid faces on node plane ``plane`` normal to ``axis``.

    The two in-plane axes ``a < b`` are the remaining ones in increasing order;
    face indices run over ``[a_lo, a_hi) x [b_lo, b_hi)``.  Returns ``[m, 4]``
    node indices in cyclic order.
    """
    a_ax, b_ax = [d for d in range(3) if d != axis]
    A, B = np.meshgrid(np.arange(a_lo, a_hi), np.arange(b_lo, b_hi), indexing="ij")
    A = A.ravel()
    B = B.ravel()

    def idx(da, db):
        c = [None, None, None]
        c[axis] = np.full_like(A, plane)
        c[a_ax] = A + da
        c[b_ax] = B + db
        return node_index(dims, c[0], c[1], c[2])

    f = np.stack([idx(0, 0), idx(1, 0), idx(1, 1), idx(0, 1)], axis=1)
    return f.astype(np.int32)


def merge_patches(patches):
    """Union of (faces, value) patches; a face listed twice keeps the max value."""
    if not patches:
        return np.zeros((0, 4), np.int32), np.zeros(0)
    faces = np.concatenate([p[0] for p in patches])
    vals = np.concatenate([np.full(len(p[0]), float(p[1])) for p in patches])
    key = np.sort(faces, axis=1)
    order = np.lexsort((-vals, key[:, 3], key[:, 2], key[:, 1], key[:, 0]))
    key = key[order]
    keep = np.ones(len(order), bool)
    keep[1:] = np.any(key[1:] != key[:-1], axis=1)
    sel = np.sort(order[keep])
    return faces[sel].astype(np.int32), vals[sel]


def interior_mask(dims):
    nx, ny, nz = dims
    zz, yy, xx = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return ((xx > 0) & (xx < nx) & (yy > 0) & (yy < ny) & (zz > 0) & (zz < nz)).ravel()


def grid_i(dims):
    nx, ny, nz = dims
    return np.tile(np.arange(nx + 1), (ny + 1) * (nz + 1))


def jitter_nodes(xyz, dims, amp, rng):
    """Move every node off the domain boundary by U[-amp*h, amp*h] per axis."""
    m = interior_mask(dims)
    h = np.array([1.0 / dims[0], 1.0 / dims[1], 1.0 / dims[2]])
    d = rng.uniform(-1.0, 1.0, size=(int(m.sum()), 3)) * (amp * h)
    out = xyz.copy()
    out[m] += d
    return out


def lognormal_tensors(n_cells, sigma, rng):
    """Lambda = R diag(exp(z)) R^T with z ~ N(0, sigma^2), R Haar-distributed."""
    z = rng.standard_normal((n_cells, 3)) * sigma
    g = rng.standard_normal((n_cells, 3, 3))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    q = q * s[:, None, :]
    lam = np.einsum("nij,nj,nkj->nik", q, np.exp(z), q)
    return np.stack([lam[:, 0, 0], lam[:, 1, 1], lam[:, 2, 2],
                     lam[:, 0, 1], lam[:, 0, 2], lam[:, 1, 2]], axis=1)


def isotropic(n_cells, value=1.0):
    p = np.zeros((n_cells, 6))
    p[:, :3] = value
    return p


def random_patches(dims, n_patches, rng, ratios=(1e2, 1e4, 1e6), fixed_ratio=None):
    """Axis-aligned rectangular patches of grid faces.

    Per patch, in this draw order: axis ~ U{0,1,2}; plane ~ U{1..n-1};
    side lengths ~ U{ceil(n/16)..ceil(n/4)} per in-plane axis; corner ~ U over
    valid positions; ratio ~ U(ratios) unless ``fixed_ratio`` is given.
    """
    patches = []
    for _ in range(n_patches):
        axis = int(rng.integers(0, 3))
        n_ax = dims[axis]
        plane = int(rng.integers(1, n_ax))
        a_ax, b_ax = [d for d in range(3) if d != axis]
        lens = []
        for ax in (a_ax, b_ax):
            n = dims[ax]
            lo, hi = math.ceil(n / 16), math.ceil(n / 4)
            lens.append(int(rng.integers(lo, hi + 1)))
        corner = [int(rng.integers(0, dims[ax] - L + 1)) for ax, L in zip((a_ax, b_ax), lens)]
        ratio = fixed_ratio if fixed_ratio is not None else float(ratios[int(rng.integers(0, len(ratios)))])
        f = plane_faces(dims, axis, plane, corner[0], corner[0] + lens[0], corner[1], corner[1] + lens[1])
        patches.append((f, ratio))
    return patches


def x_dirichlet(dims, n_nodes, xyz):
    """Dirichlet pressure 1 / concentration 1 at x=0, pressure 0 / concentration 0 at x=1."""
    gi = grid_i(dims)
    dirichlet = ((gi == 0) | (gi == dims[0])).astype(np.uint8)
    p_bar = np.where(gi == 0, 1.0, 0.0)
    c_bar = np.where(gi == 0, 1.0, 0.0)
    return dirichlet, p_bar, c_bar


def _assemble(name, dims, xyz, hex8, faces, ratios, perm, df=0.01, lam_m=1.0, **kw):
    nf = len(faces)
    return Problem(
        name=name, dims=dims, xyz=np.ascontiguousarray(xyz, np.float64),
        hex8=np.ascontiguousarray(hex8, np.int32),
        frac_nodes=np.ascontiguousarray(faces, np.int32).reshape(nf, 4),
        frac_width=np.full(nf, df), frac_perm=np.asarray(ratios, np.float64) * lam_m,
        frac_poro=np.ones(nf), perm=np.ascontiguousarray(perm, np.float64),
        poro=np.ones(len(hex8)), mu=1.0, **kw)


def planes_problem(dims, planes=(), ratio=1e4, df=0.01, jitter=0.0, aniso_sigma=None,
                   seed=0, name=None, **kw):
    """Box of dims cells; ``planes`` = [(axis, plane, a_lo, a_hi, b_lo, b_hi), ...]."""
    dims = tuple(int(d) for d in dims)
    xyz, hex8 = structured_hex(*dims)
    nc = dims[0] * dims[1] * dims[2]
    rng = np.random.default_rng(seed)
    if jitter > 0:
        xyz = jitter_nodes(xyz, dims, jitter, rng)
    perm = lognormal_tensors(nc, aniso_sigma, rng) if aniso_sigma else isotropic(nc)
    patches = [(plane_faces(dims, *p), ratio) for p in planes]
    faces, ratios = merge_patches(patches)
    d, pb, cb = x_dirichlet(dims, len(xyz), xyz)
    return _assemble(name or f"box{dims}", dims, xyz, hex8, faces, ratios, perm, df=df,
                     dirichlet=d, p_bar=pb, c_bar=cb, **kw)


def cartesian_problem(n, planes=(), ratio=1e4, df=0.01, jitter=0.0, aniso_sigma=None,
                      seed=0, name=None, **kw):
    """Cube of n^3 cells; ``planes`` = [(axis, plane, a_lo, a_hi, b_lo, b_hi), ...]."""
    return planes_problem((n, n, n), planes, ratio=ratio, df=df, jitter=jitter, aniso_sigma=aniso_sigma,
                          seed=seed, name=name or f"cart{n}", **kw)


def random_problem(dims, seed, jitter=0.2, aniso_sigma=1.0, n_patches=3,
                   ratios=(1e2, 1e4, 1e6), name=None, **kw):
    """Small random instance: jitter, lognormal tensors, random face patches."""
    xyz, hex8 = structured_hex(*dims)
    rng = np.random.default_rng(seed)
    if jitter > 0:
        xyz = jitter_nodes(xyz, dims, jitter, rng)
    nc = len(hex8)
    perm = lognormal_tensors(nc, aniso_sigma, rng) if aniso_sigma else isotropic(nc)
    faces, r = merge_patches(random_patches(dims, n_patches, rng, ratios))
    d, pb, cb = x_dirichlet(dims, len(xyz), xyz)
    return _assemble(name or f"rand{dims}-{seed}", dims, xyz, hex8, faces, r, perm,
                     dirichlet=d, p_bar=pb, c_bar=cb, **kw)


# ----------------------------------------------------------------------------
# The five benchmark workloads
# ----------------------------------------------------------------------------

def config1():
    """10^3 unit cube, one fracture = all faces of plane x=0.5, d_f*Lambda_f = 100."""
    n = 10
    return cartesian_problem(n, planes=[(0, 5, 0, n, 0, n)], ratio=1e4, name="config1",
                             rtol=1e-10, cfl=0.9, n_steps=50)


def config2(n=64, seed=2):
    """n^3 cube, four clipped fractures on planes x=n/2, y=n/2, z=n/4, z=3n/4."""
    rng = np.random.default_rng(seed)
    planes = []
    lo_hi = lambda: (int(rng.integers(0, n * 12 // 64 + 1)), int(rng.integers(n * 52 // 64, n + 1)))  # noqa: E731
    for axis, plane in ((0, n // 2), (1, n // 2), (2, n // 4), (2, 3 * n // 4)):
        a_lo, a_hi = lo_hi()
        b_lo, b_hi = lo_hi()
        planes.append((axis, plane, a_lo, a_hi, b_lo, b_hi))
    return cartesian_problem(n, planes=planes, ratio=1e4, name=f"config2-n{n}",
                             rtol=1e-8, cfl=0.9, n_steps=200)


def config3(n=128, seed=3, n_patches=40):
    """Jittered n^3 mesh, lognormal anisotropic tensors, random face patches."""
    dims = (n, n, n)
    xyz, hex8 = structured_hex(*dims)
    rng = np.random.default_rng(seed)
    xyz = jitter_nodes(xyz, dims, 0.2, rng)
    perm = lognormal_tensors(n ** 3, 1.0, rng)
    faces, r = merge_patches(random_patches(dims, n_patches, rng))
    d, pb, cb = x_dirichlet(dims, len(xyz), xyz)
    return _assemble(f"config3-n{n}", dims, xyz, hex8, faces, r, perm,
                     dirichlet=d, p_bar=pb, c_bar=cb, rtol=1e-8, cfl=0.9, n_steps=200)


def config4_job(j, n_range=(16, 96)):
    """Serving job j: jittered n^3, isotropic matrix, 1-20 patches, one ratio per job."""
    rng = np.random.default_rng([4, j])
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    dims = (n, n, n)
    xyz, hex8 = structured_hex(*dims)
    xyz = jitter_nodes(xyz, dims, 0.2, rng)
    n_p = int(rng.integers(1, 21))
    ratio = float((1e2, 1e4, 1e6)[int(rng.integers(0, 3))])
    faces, r = merge_patches(random_patches(dims, n_p, rng, fixed_ratio=ratio))
    d, pb, cb = x_dirichlet(dims, len(xyz), xyz)
    return _assemble(f"config4-job{j}-n{n}", dims, xyz, hex8, faces, r, isotropic(n ** 3),
                     dirichlet=d, p_bar=pb, c_bar=cb, rtol=1e-8, cfl=0.9, n_steps=100)


def config5(n=192, seed=5, n_patches=200):
    """Largest instance: jittered n^3, lognormal tensors, patches at ratio 1e6."""
    dims = (n, n, n)
    xyz, hex8 = structured_hex(*dims)
    rng = np.random.default_rng(seed)
    xyz = jitter_nodes(xyz, dims, 0.2, rng)
    perm = lognormal_tensors(n ** 3, 1.0, rng)
    faces, r = merge_patches(random_patches(dims, n_patches, rng, fixed_ratio=1e6))
    d, pb, cb = x_dirichlet(dims, len(xyz), xyz)
    return _assemble(f"config5-n{n}", dims, xyz, hex8, faces, r, perm,
                     dirichlet=d, p_bar=pb, c_bar=cb, rtol=1e-8, cfl=0.9, n_steps=1000)


CONFIGS = {1: config1, 2: config2, 3: config3, 5: config5}


# ----------------------------------------------------------------------------
# The paper's two analytical test cases (§5.1, §5.2), extruded to one layer
# ----------------------------------------------------------------------------

def _extruded(n, xy):
    """n x n x 1 grid whose (i, j) node sits at xy[j, i]; layer thickness 1/n."""
    dims = (n, n, 1)
    xyz, hex8 = structured_hex(*dims)
    for k in range(2):
        sl = slice(k * (n + 1) ** 2, (k + 1) * (n + 1) ** 2)
        xyz[sl, 0] = xy[..., 0].ravel()
        xyz[sl, 1] = xy[..., 1].ravel()
        xyz[sl, 2] = k / n
    return dims, xyz, hex8


def e1_problem(n, tan_theta=0.5, lam_f=20.0, df=0.01, t_final=0.5):
    """§5.1: one fracture from (0,1/4) to (1,1/4+tan(theta)); u = 1 - x."""
    assert n % 2 == 0
    h = n // 2
    x = np.arange(n + 1) / n
    yf = 0.25 + x * tan_theta
    xy = np.zeros((n + 1, n + 1, 2))
    for j in range(n + 1):
        xy[j, :, 0] = x
        if j <= h:
            xy[j, :, 1] = (j / h) * yf
        else:
            xy[j, :, 1] = yf + ((j - h) / h) * (1.0 - yf)
    dims, xyz, hex8 = _extruded(n, xy)
    faces = plane_faces(dims, 1, h, 0, n, 0, 1)
    gi = grid_i(dims)
    dirichlet = ((gi == 0) | (gi == n)).astype(np.uint8)
    p_bar = 1.0 - xyz[:, 0]
    c_bar = np.where(gi == 0, 1.0, 0.0)
    nf = len(faces)
    return Problem(name=f"e1-n{n}", dims=dims, xyz=xyz, hex8=hex8, frac_nodes=faces,
                   frac_width=np.full(nf, df), frac_perm=np.full(nf, lam_f), frac_poro=np.ones(nf),
                   perm=isotropic(len(hex8)), poro=np.ones(len(hex8)), mu=1.0,
                   dirichlet=dirichlet, p_bar=p_bar, c_bar=c_bar, rtol=1e-13, cfl=1.0,
                   n_steps=0, t_final=t_final,
                   meta=dict(tan_theta=tan_theta, lam_f=lam_f, df=df, row=h))


def e2_problem(n, tan1=5 / 8, tan2=1 / 4, lam_f1=200.0, lam_f3=400.0, df=0.01, t_final=3.0):
    """§5.2: four fractures meeting at x0; mesh = 4 bilinear blocks conforming to both lines."""
    assert n % 2 == 0
    h = n // 2
    x0 = (3 - tan2) / (4 * (1 + tan1 * tan2))
    y0 = (1 + 3 * tan1) / (4 * (1 + tan1 * tan2))
    P = {
        "A": (0.0, 0.0), "B": (1.0, 0.0), "C": (1.0, 1.0), "D": (0.0, 1.0),
        "x1": (0.0, 0.25), "x2": (1.0, 0.25 + tan1), "x3": (0.75, 0.0), "x4": (0.75 - tan2, 1.0),
        "x0": (x0, y0),
    }
    P = {k: np.array(v) for k, v in P.items()}
    xy = np.zeros((n + 1, n + 1, 2))
    blocks = [  # (i range, j range, corners p00 p10 p11 p01)
        ((0, h), (0, h), ("A", "x3", "x0", "x1")),
        ((h, n), (0, h), ("x3", "B", "x2", "x0")),
        ((0, h), (h, n), ("x1", "x0", "x4", "D")),
        ((h, n), (h, n), ("x0", "x2", "C", "x4")),
    ]
    for (i0, i1), (j0, j1), (c00, c10, c11, c01) in blocks:
        for j in range(j0, j1 + 1):
            v = (j - j0) / (j1 - j0)
            for i in range(i0, i1 + 1):
                u = (i - i0) / (i1 - i0)
                xy[j, i] = ((1 - u) * (1 - v) * P[c00] + u * (1 - v) * P[c10]
                            + u * v * P[c11] + (1 - u) * v * P[c01])
    dims, xyz, hex8 = _extruded(n, xy)
    f1 = plane_faces(dims, 1, h, 0, h, 0, 1)      # Gamma_1: x1 -> x0
    f2 = plane_faces(dims, 1, h, h, n, 0, 1)      # Gamma_2: x0 -> x2
    f3 = plane_faces(dims, 0, h, 0, h, 0, 1)      # Gamma_3: x3 -> x0
    f4 = plane_faces(dims, 0, h, h, n, 0, 1)      # Gamma_4: x0 -> x4
    faces = np.concatenate([f1, f2, f3, f4])
    perm_f = np.concatenate([np.full(len(f1) + len(f2), lam_f1), np.full(len(f3) + len(f4), lam_f3)])
    branch = np.concatenate([np.full(len(f), b) for b, f in enumerate((f1, f2, f3, f4), start=1)])
    gi = grid_i(dims)
    gj = np.tile(np.repeat(np.arange(n + 1), n + 1), 2)
    tip3 = (gi == h) & (gj == 0)
    tip4 = (gi == h) & (gj == n)
    dirichlet = ((gi == 0) | (gi == n) | tip3 | tip4).astype(np.uint8)
    p_bar = 1.0 - xyz[:, 0]
    tip1 = (gi == 0) & (gj == h)
    c_bar = np.where(tip1 | tip4, 1.0, 0.0)
    nf = len(faces)
    return Problem(name=f"e2-n{n}", dims=dims, xyz=xyz, hex8=hex8, frac_nodes=faces,
                   frac_width=np.full(nf, df), frac_perm=perm_f, frac_poro=np.ones(nf),
                   perm=isotropic(len(hex8)), poro=np.ones(len(hex8)), mu=1.0,
                   dirichlet=dirichlet, p_bar=p_bar, c_bar=c_bar, rtol=1e-13, cfl=1.0,
                   n_steps=0, t_final=t_final,
                   meta=dict(tan1=tan1, tan2=tan2, lam_f1=lam_f1, lam_f3=lam_f3, df=df,
                             x0=x0, y0=y0, branch=branch))


def add_wells(prob, seed, n_inj=1, n_prod=2, q=0.5, pw=0.3, wi_range=(0.05, 0.2)):
    """Perforates distinct random fracture faces of prob (in place, returns it):
    n_inj rate injectors (wi 0, inflow q, injected concentration 1) and n_prod
    pressure-controlled wells at pressure pw with a well index drawn
    uniformly in wi_range (they produce where the face pressure exceeds pw)."""
    rng = np.random.default_rng([17, seed])
    n = n_inj + n_prod
    if prob.n_frac < n:
        raise ValueError("not enough fracture faces for the wells")
    face = rng.choice(prob.n_frac, size=n, replace=False).astype(np.int32)
    wi = np.zeros(n)
    wi[n_inj:] = rng.uniform(*wi_range, size=n_prod)
    prob.wells = dict(face=face, wi=wi, pw=np.where(np.arange(n) < n_inj, 0.0, pw),
                      q=np.where(np.arange(n) < n_inj, q, 0.0), cinj=np.where(np.arange(n) < n_inj, 1.0, 0.0))
    return prob


def simplex_cells(dims, kind):
    """Cells of a structured (nx, ny, nz) grid split into tetrahedra (kind
    "tet": 6 per hexahedron around its 0-6 diagonal, conforming) or prisms
    (kind "prism": 2 per hexahedron, split along the 0-2 diagonal of the
    bottom square), as node tuples in VTK order with positive orientation."""
    nx, ny, nz = dims
    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                h = [node_index(dims, i, j, k), node_index(dims, i + 1, j, k), node_index(dims, i + 1, j + 1, k),
                     node_index(dims, i, j + 1, k), node_index(dims, i, j, k + 1), node_index(dims, i + 1, j, k + 1),
                     node_index(dims, i + 1, j + 1, k + 1), node_index(dims, i, j + 1, k + 1)]
                if kind == "prism":
                    cells.append((h[0], h[1], h[2], h[4], h[5], h[6]))
                    cells.append((h[0], h[2], h[3], h[4], h[6], h[7]))
                else:
                    for a, b in ((1, 2), (2, 3), (3, 7), (7, 4), (4, 5), (5, 1)):
                        cells.append((h[0], h[a], h[b], h[6]))
    return cells


def orient_tets(xyz, cells):
    """Tetrahedra reordered (two nodes swapped) where needed so that the
    volume det[p1 - p0, p2 - p0, p3 - p0] / 6 is positive."""
    out = []
    for c in cells:
        if len(c) == 4:
            p = xyz[list(c)]
            if np.linalg.det(np.array([p[1] - p[0], p[2] - p[0], p[3] - p[0]])) < 0:
                c = (c[0], c[2], c[1], c[3])
        out.append(tuple(c))
    return out


def plane_x_faces(dims, cells, i0):
    """The cell faces lying on the grid plane x = i0 (triangles for
    tetrahedra, quadrangles for prisms), each once, nodes in cyclic order."""
    on = lambda s: s % (dims[0] + 1) == i0  # noqa: E731
    seen, faces = set(), []
    for c in cells:
        pts = [s for s in c if on(s)]
        want = 3 if len(c) == 4 else 4
        if len(pts) != want:
            continue
        key = tuple(sorted(pts))
        if key in seen:
            continue
        seen.add(key)
        if want == 4:  # cyclic order of the quadrangle: sort by (z, then y) around its centre
            js = [(s // (dims[0] + 1)) % (dims[1] + 1) for s in pts]
            ks = [s // ((dims[0] + 1) * (dims[1] + 1)) for s in pts]
            cj, ck = np.mean(js), np.mean(ks)
            pts = [p for _, p in sorted(zip([np.arctan2(k - ck, j - cj) for j, k in zip(js, ks)], pts))]
        faces.append(tuple(pts))
    return faces


# ----------------------------------------------------------------------------
# General cells given by their faces (the mesh form of §3.1)
# ----------------------------------------------------------------------------

# local faces of VTK cells, each cyclic and outward for a positively
# oriented cell (hexahedron, prism (wedge), tetrahedron)
CELL_FACES = {
    8: [(0, 4, 7, 3), (1, 2, 6, 5), (0, 1, 5, 4), (3, 7, 6, 2), (0, 3, 2, 1), (4, 5, 6, 7)],
    6: [(0, 2, 1), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (0, 3, 5, 2)],
    4: [(0, 2, 1), (0, 1, 3), (1, 2, 3), (0, 3, 2)],
}


@dataclass
class GeneralProblem:
    """A mesh of general cells: cell -> faces (CSR), face -> nodes (CSR, cyclic).
    ``cells`` keeps each cell's nodes in VTK order (for checkers that work
    with node tuples); ``frac_face_ids`` index the face list."""
    name: str
    xyz: np.ndarray
    cells: list
    cell_face_ptr: np.ndarray   # [n_cells + 1] int64
    cell_faces: np.ndarray      # int32 face ids
    face_node_ptr: np.ndarray   # [n_faces + 1] int64
    face_nodes: np.ndarray      # int32, cyclic per face
    frac_face_ids: np.ndarray   # [n_frac] int32
    frac_width: np.ndarray
    frac_perm: np.ndarray
    frac_poro: np.ndarray
    perm: np.ndarray            # [n_cells, 6]
    poro: np.ndarray
    mu: float
    dirichlet: np.ndarray
    p_bar: np.ndarray
    c_bar: np.ndarray
    rtol: float = 1e-10
    cfl: float = 0.9
    n_steps: int = 20
    t_final: float = 0.0
    wells: dict = None

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_cells(self) -> int:
        return len(self.cells)

    @property
    def n_frac(self) -> int:
        return int(len(self.frac_face_ids))

    def face(self, f):
        return tuple(int(v) for v in self.face_nodes[self.face_node_ptr[f]:self.face_node_ptr[f + 1]])

    def frac_faces(self):
        """The fracture faces as node tuples (the face list's cyclic order)."""
        return [self.face(f) for f in self.frac_face_ids]

    def cell_node_order(self, K):
        """The cell's nodes in the order they first appear along its faces."""
        out = []
        for q in range(self.cell_face_ptr[K], self.cell_face_ptr[K + 1]):
            for s in self.face(self.cell_faces[q]):
                if s not in out:
                    out.append(s)
        return out


def grid_cells(dims, kind):
    """Cells of a structured (nx, ny, nz) grid as an array of VTK node tuples:
    hexahedra, prisms (2 per hexahedron, split along the 0-2 diagonal of its
    bottom square) or tetrahedra (6 per hexahedron around its 0-6 diagonal),
    in the order of ``simplex_cells``."""
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    n = lambda a, b, c: node_index(dims, a, b, c)  # noqa: E731
    h = np.stack([n(i, j, k), n(i + 1, j, k), n(i + 1, j + 1, k), n(i, j + 1, k), n(i, j, k + 1),
                  n(i + 1, j, k + 1), n(i + 1, j + 1, k + 1), n(i, j + 1, k + 1)], axis=1).astype(np.int32)
    if kind == "hex":
        return h
    if kind == "prism":
        return np.stack([h[:, [0, 1, 2, 4, 5, 6]], h[:, [0, 2, 3, 4, 6, 7]]], axis=1).reshape(-1, 6)
    pairs = ((1, 2), (2, 3), (3, 7), (7, 4), (4, 5), (5, 1))
    return np.stack([h[:, [0, a, b, 6]] for a, b in pairs], axis=1).reshape(-1, 4)


def orient_tet_array(xyz, cells):
    """Tetrahedra with nodes 1 and 2 swapped where det[p1-p0, p2-p0, p3-p0] < 0."""
    cells = np.array(cells)
    if cells.shape[1] != 4:
        return cells
    p = xyz[cells]
    det = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
    neg = det < 0
    cells[neg, 1], cells[neg, 2] = cells[neg, 2].copy(), cells[neg, 1].copy()
    return cells


def faces_of_cells(cells, rng=None, shuffle=False, flip=False):
    """Face list of a conforming mesh of VTK cells (an array, one cell type):
    each distinct face once, with the node order of its first cell (reversed
    at random with ``flip``), and each cell's faces in local-face order (or
    shuffled per cell).  Returns cell_face_ptr, cell_faces, face_node_ptr,
    face_nodes and, per face, its node key (sorted nodes, -1 padded)."""
    cells = np.asarray(cells, np.int64)
    nc, nv = cells.shape
    table = CELL_FACES[nv]
    face_id = np.zeros((nc, len(table)), np.int64)
    ptr_parts, node_parts, key_parts, nfaces = [], [], [], 0
    for k in (3, 4):
        lfs = [lf for lf in range(len(table)) if len(table[lf]) == k]
        if not lfs:
            continue
        F = np.stack([cells[:, list(table[lf])] for lf in lfs], axis=1).reshape(-1, k)  # cell-major
        key = np.sort(F, axis=1)
        _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
        inv = inv.ravel()
        order = np.argsort(first, kind="stable")  # faces numbered by first appearance
        rank = np.empty_like(order)
        rank[order] = np.arange(len(order))
        nodes = F[first[order]]
        if flip and rng is not None:
            rev = rng.random(len(nodes)) < 0.5
            nodes[rev] = nodes[rev, ::-1]
        face_id[:, lfs] = (nfaces + rank[inv]).reshape(nc, len(lfs))
        node_parts.append(nodes.ravel())
        ptr_parts.append(np.full(len(nodes), k))
        kp = np.full((len(nodes), 4), -1, np.int64)
        kp[:, :k] = np.sort(nodes, axis=1)
        key_parts.append(kp)
        nfaces += len(nodes)
    if shuffle and rng is not None:
        perm = np.argsort(rng.random(face_id.shape), axis=1)
        face_id = np.take_along_axis(face_id, perm, axis=1)
    fptr = np.concatenate([[0], np.cumsum(np.concatenate(ptr_parts))]).astype(np.int64)
    cptr = (np.arange(nc + 1) * len(table)).astype(np.int64)
    return (cptr, face_id.ravel().astype(np.int32), fptr, np.concatenate(node_parts).astype(np.int32),
            np.concatenate(key_parts))


def _square_keys(dims, keys):
    """Grid square of each face lying on an axis plane (-1 if none): faces
    are given by their sorted node keys (-1 padded)."""
    nx, ny, nz = dims
    valid = keys >= 0
    s = np.where(valid, keys, keys[:, :1])
    g = np.stack([s % (nx + 1), (s // (nx + 1)) % (ny + 1), s // ((nx + 1) * (ny + 1))], axis=-1)  # [f, 4, 3]
    N = max(dims) + 1
    out = np.full(len(keys), -1, np.int64)
    for axis in range(3):
        a, b = [d for d in range(3) if d != axis]
        on = np.all(g[:, :, axis] == g[:, :1, axis], axis=1)
        code = ((axis * N + g[:, 0, axis]) * N + g[:, :, a].min(axis=1)) * N + g[:, :, b].min(axis=1)
        out = np.where(on & (out < 0), code, out)
    return out


def general_workload(kind, dims, seed, n_patches=40, ratios=(1e2, 1e4, 1e6), jitter=0.2, aniso_sigma=1.0,
                     df=0.01, n_steps=200, shuffle=False, flip=False, name=None):
    """Unit-box workload of tetrahedra, prisms or hexahedra (a jittered grid
    split into cells), lognormal anisotropic tensors, ``n_patches`` random
    axis-aligned fracture patches (the 128^3 workload's rule) whose cell faces
    (triangles or quadrangles lying in a patch's grid squares) are fracture
    faces, Dirichlet p = 1 - x, c = 1 at x = 0 and 0 at x = 1."""
    rng = np.random.default_rng([41, seed])
    xyz, _ = structured_hex(*dims)
    xyz = jitter_nodes(xyz, dims, jitter, rng)
    cells = orient_tet_array(xyz, grid_cells(dims, kind))
    nc = len(cells)
    perm = lognormal_tensors(nc, aniso_sigma, rng) if aniso_sigma else isotropic(nc)
    quads, ratio = merge_patches(random_patches(dims, n_patches, rng, ratios))
    cfp, cf, fnp, fn, keys = faces_of_cells(cells, rng, shuffle=shuffle, flip=flip)
    fkey = _square_keys(dims, keys)
    qkey = _square_keys(dims, np.sort(quads.astype(np.int64), axis=1)) if len(quads) else np.zeros(0, np.int64)
    order = np.argsort(qkey)
    pos = np.searchsorted(qkey[order], fkey)
    pos = np.minimum(pos, max(len(qkey) - 1, 0))
    hit = (fkey >= 0) & (len(qkey) > 0) & (qkey[order][pos] == fkey) if len(qkey) else np.zeros(len(fkey), bool)
    fids = np.nonzero(hit)[0].astype(np.int32)
    fr = ratio[order][pos[fids]] if len(fids) else np.zeros(0)
    d, pb, cb = x_dirichlet(dims, len(xyz), xyz)
    nf = len(fids)
    return GeneralProblem(
        name=name or f"{kind}{tuple(dims)}-{seed}", xyz=xyz, cells=cells, cell_face_ptr=cfp, cell_faces=cf,
        face_node_ptr=fnp, face_nodes=fn, frac_face_ids=fids, frac_width=np.full(nf, df), frac_perm=fr * 1.0,
        frac_poro=np.ones(nf), perm=perm, poro=np.ones(nc), mu=1.0, dirichlet=d, p_bar=pb, c_bar=cb, rtol=1e-8,
        cfl=0.9, n_steps=n_steps)


def general_problem(kind, dims, seed, jitter=0.2, aniso_sigma=1.0, frac_plane=None, ratio=1e3, df=0.01,
                    shuffle=True, flip=True, dirichlet="x", n_steps=20, planar_x=False, name=None):
    """Unit-box mesh of tetrahedra ("tet"), prisms ("prism") or hexahedra
    ("hex") on a (nx, ny, nz) grid: interior nodes jittered by U[-jitter h,
    jitter h] (only in y and z with ``planar_x``, so that x planes stay
    planar), lognormal anisotropic tensors (sigma aniso_sigma; None =
    isotropic 1), an optional fracture plane x = frac_plane (grid index) of
    the cells' faces with Lambda_f = ratio, d_f = df, Dirichlet data p = 1 - x
    and c = 1 at x = 0, 0 at x = 1 (``dirichlet="x"``) or p = 1 - x + 0.3 y -
    0.2 z on every boundary node ("all").  Faces are listed in random
    orientation and each cell's faces in random order (``flip``, ``shuffle``)."""
    rng = np.random.default_rng([31, seed])
    xyz, _ = structured_hex(*dims)
    h = 1.0 / np.array(dims, float)
    interior = np.all((xyz > 1e-12) & (xyz < 1 - 1e-12), axis=1)
    axes = slice(1, 3) if planar_x else slice(0, 3)
    width = 2 if planar_x else 3
    xyz[interior, axes] += rng.uniform(-jitter, jitter, (int(interior.sum()), width)) * h[axes]
    cells = orient_tet_array(xyz, grid_cells(dims, kind))
    nc = len(cells)
    perm = lognormal_tensors(nc, aniso_sigma, rng) if aniso_sigma else isotropic(nc)
    cfp, cf, fnp, fn, keys = faces_of_cells(cells, rng, shuffle=shuffle, flip=flip)
    if frac_plane is not None:
        on = lambda s: (s < 0) | (s % (dims[0] + 1) == frac_plane)  # noqa: E731
        fids = np.nonzero(np.all(on(keys), axis=1))[0].astype(np.int32)
    else:
        fids = np.zeros(0, np.int32)
    nf = len(fids)
    if dirichlet == "all":
        d = (~interior).astype(np.uint8)
        pb = 1.0 - xyz[:, 0] + 0.3 * xyz[:, 1] - 0.2 * xyz[:, 2]
    else:
        d = ((xyz[:, 0] < 1e-12) | (xyz[:, 0] > 1 - 1e-12)).astype(np.uint8)
        pb = 1.0 - xyz[:, 0]
    cb = (xyz[:, 0] < 1e-12).astype(float)
    return GeneralProblem(
        name=name or f"{kind}{tuple(dims)}-{seed}", xyz=xyz, cells=cells, cell_face_ptr=cfp, cell_faces=cf,
        face_node_ptr=fnp, face_nodes=fn, frac_face_ids=fids, frac_width=np.full(nf, df),
        frac_perm=np.full(nf, float(ratio)), frac_poro=np.ones(nf), perm=perm, poro=np.ones(nc), mu=1.0,
        dirichlet=d, p_bar=pb, c_bar=cb, n_steps=n_steps)


def general_from_hex(prob, seed=0, shuffle=True, flip=True):
    """The same hexahedral problem in the general (faces) form."""
    rng = np.random.default_rng([37, seed])
    cells = np.asarray(prob.hex8, np.int32)
    cfp, cf, fnp, fn, keys = faces_of_cells(cells, rng, shuffle=shuffle, flip=flip)
    look = {tuple(k): f for f, k in enumerate(keys.tolist())}
    fids = np.array([look[tuple(sorted(int(v) for v in f))] for f in np.asarray(prob.frac_nodes).reshape(-1, 4)],
                    np.int32)
    return GeneralProblem(
        name=prob.name + "-faces", xyz=prob.xyz, cells=cells, cell_face_ptr=cfp, cell_faces=cf, face_node_ptr=fnp,
        face_nodes=fn, frac_face_ids=fids, frac_width=prob.frac_width, frac_perm=prob.frac_perm,
        frac_poro=prob.frac_poro, perm=prob.perm, poro=prob.poro, mu=prob.mu, dirichlet=prob.dirichlet,
        p_bar=prob.p_bar, c_bar=prob.c_bar, rtol=prob.rtol, cfl=prob.cfl, n_steps=prob.n_steps)
