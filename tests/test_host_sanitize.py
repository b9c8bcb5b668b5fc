"""Host code under the address and undefined-behaviour sanitizers (CPU only).

The library's symbolic phases (hexahedra, with and without fracture-face
group elimination; general cells) and the C oracle (a whole run: system,
solve, residual, both volume rules, CFL, transport, wells) are built with
-fsanitize=address,undefined for the host, and run on small meshes with
fractures, intersections and wells, plus inputs the symbolic phase must
reject.  The host chunk pool the symbolic phases run on is driven by several
submitting threads at once, nested calls and a throwing chunk under the thread
sanitizer and under the address one.  A sanitizer report, a leak or a wrong
result code fails the test.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_1602_03641_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")


def _build(tmp, name, cmd):
    exe = os.path.join(tmp, name)
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"sanitizer build unavailable here: {r.stderr[-400:]}")
    return exe


@pytest.fixture(scope="module")
def tools(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("san"))
    if not shutil.which("gcc") or not os.path.exists(HIPCC):
        pytest.skip("no compiler")
    # the library's host code: every sanitizer flag goes to the host pass only
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    sym = _build(tmp, "symbolic_check",
                 [HIPCC, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", *host_san,
                  "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, os.path.join(HERE, "symbolic_check.cpp"),
                  os.path.join(CSRC, "symbolic.cpp"), os.path.join(CSRC, "symbolic_general.cpp"), "-lpthread"])
    orc = _build(tmp, "oracle_check",
                 ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", *SAN,
                  "-I" + os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_check.c"),
                  os.path.join(ROOT, "oracle", "vag_oracle.c"), "-lm"])
    return tmp, sym, orc


@pytest.mark.parametrize("san", [["-fsanitize=thread"], SAN])
def test_chunk_pool(tmp_path, san):
    if not shutil.which("g++"):
        pytest.skip("no compiler")
    exe = _build(str(tmp_path), "pool_check", ["g++", "-O1", "-g", "-std=c++17", *san, "-I" + CSRC,
                                               os.path.join(HERE, "pool_check.cpp"), "-lpthread"])
    env = dict(ENV, TSAN_OPTIONS="halt_on_error=1:exitcode=88")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out and "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert r.returncode == 0 and "pool ok" in r.stdout, (r.returncode, out[-2000:])


def _run(exe, path):
    r = subprocess.run([exe, path], capture_output=True, text=True, env=ENV, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out[-3000:]
    assert r.returncode == 0, (r.returncode, out[-2000:])
    return r.stdout


def _i64(*v):
    return np.array(v, np.int64).tobytes()


def _hex_file(path, p, expect_error=0):
    with open(path, "wb") as f:
        f.write(_i64(0, expect_error, p.n_nodes, p.n_cells, len(p.frac_nodes)))
        f.write(np.ascontiguousarray(p.hex8, np.int32).tobytes())
        f.write(np.ascontiguousarray(np.asarray(p.frac_nodes).reshape(-1, 4), np.int32).tobytes())
        f.write(np.ascontiguousarray(p.dirichlet, np.uint8).tobytes())


def _general_file(path, q, expect_error=0):
    with open(path, "wb") as f:
        f.write(_i64(1, expect_error, q.n_nodes, q.n_cells, len(q.face_node_ptr) - 1))
        f.write(np.ascontiguousarray(q.cell_face_ptr, np.int64).tobytes())
        f.write(np.ascontiguousarray(q.cell_faces, np.int32).tobytes())
        f.write(np.ascontiguousarray(q.face_node_ptr, np.int64).tobytes())
        f.write(np.ascontiguousarray(q.face_nodes, np.int32).tobytes())
        f.write(_i64(len(q.frac_face_ids)))
        f.write(np.ascontiguousarray(q.frac_face_ids, np.int32).tobytes())
        f.write(np.ascontiguousarray(q.dirichlet, np.uint8).tobytes())


def _oracle_file(path, p, n_steps):
    w = getattr(p, "wells", None) or {}
    nw = len(w.get("face", []))
    with open(path, "wb") as f:
        f.write(_i64(p.n_nodes, p.n_cells, len(p.frac_nodes), nw, n_steps))
        f.write(np.array([p.mu, 1e-12], np.float64).tobytes())
        for a, dt in ((p.xyz, np.float64), (p.hex8, np.int32), (np.asarray(p.frac_nodes).reshape(-1, 4), np.int32),
                      (p.frac_width, np.float64), (p.frac_perm, np.float64), (p.frac_poro, np.float64),
                      (p.perm, np.float64), (p.poro, np.float64), (p.dirichlet, np.uint8), (p.p_bar, np.float64),
                      (p.c_bar, np.float64)):
            f.write(np.ascontiguousarray(a, dt).tobytes())
        f.write(np.ascontiguousarray(w.get("face", []), np.int32).tobytes())
        for k in ("wi", "pw", "q", "cinj"):
            f.write(np.ascontiguousarray(w.get(k, np.zeros(nw)), np.float64).tobytes())


def test_symbolic_phases_clean(tools, tmp_path):
    tmp, sym, _ = tools
    cases = [synth.config1(), synth.random_problem((9, 7, 6), 21, n_patches=8, n_steps=0),
             synth.config2(n=12)]
    for k, p in enumerate(cases):
        path = str(tmp_path / f"hex{k}.bin")
        _hex_file(path, p)
        out = _run(sym, path)
        assert "check 0" in out, out
    for k, (kind, dims) in enumerate([("tet", (6, 5, 4)), ("prism", (7, 5, 4)), ("hex", (5, 4, 4))]):
        q = synth.general_problem(kind, dims, 30 + k, frac_plane=dims[0] // 2, ratio=1e3)
        path = str(tmp_path / f"gen{k}.bin")
        _general_file(path, q)
        out = _run(sym, path)
        assert "check 0" in out, out


def test_symbolic_rejections_clean(tools, tmp_path):
    """Invalid inputs end in an error, with nothing leaked or read out of bounds."""
    tmp, sym, _ = tools
    p = synth.cartesian_problem(3, planes=[(0, 1, 0, 3, 0, 3)])
    bad = [p.hex8.copy(), None, None]
    bad[0][0, 0] = p.n_nodes + 5                                # node index out of range
    fn = np.asarray(p.frac_nodes).reshape(-1, 4).copy()
    bad[1] = np.concatenate([fn, fn[:1, ::-1]])                 # a fracture face listed twice
    bad[2] = fn.copy()
    bad[2][0] = [0, 1, 2, 3]                                    # not a face of the mesh
    for k, variant in enumerate(bad):
        q = synth.cartesian_problem(3, planes=[(0, 1, 0, 3, 0, 3)])
        if k == 0:
            q.hex8 = variant
        else:
            q.frac_nodes = variant
        path = str(tmp_path / f"bad{k}.bin")
        _hex_file(path, q, expect_error=1)
        _run(sym, path)
    g = synth.general_problem("tet", (3, 3, 3), 5, frac_plane=1)
    g.cell_faces = np.asarray(g.cell_faces).copy()
    g.cell_faces[0] = len(g.face_node_ptr) + 7                   # face index out of range
    path = str(tmp_path / "badgen.bin")
    _general_file(path, g, expect_error=1)
    _run(sym, path)


@pytest.mark.parametrize("case", ["config1", "random", "wells"])
def test_oracle_run_clean(tools, tmp_path, case):
    tmp, _, orc = tools
    if case == "config1":
        p = synth.config1()
    else:
        p = synth.random_problem((7, 6, 5), 17, n_patches=6, n_steps=0)
        if case == "wells":
            p = synth.add_wells(p, 3)
    path = str(tmp_path / f"orc_{case}.bin")
    _oracle_file(path, p, 15)
    out = _run(orc, path)
    assert "oracle:" in out
