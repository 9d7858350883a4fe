"""The C oracle and the library's host graph steps built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code only), run
on small inputs: no sanitizer report, and the oracle's results equal those
of its ordinary build. The mesh generator is NumPy only (no native code)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import meshgen as mg
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1",
       "OMP_NUM_THREADS": "4"}

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="no gcc")


def _run(cmd, **kw):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert p.returncode == 0, p.stdout[-4000:]
    assert "runtime error" not in p.stdout and "AddressSanitizer" not in p.stdout, p.stdout[-4000:]
    return p.stdout


def test_host_graph_steps_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_graph_check")
    _run(["g++", "-std=c++17", *SAN, os.path.join(ROOT, "tests", "native", "host_graph_check.cpp"), "-o", exe])
    _run([exe], env=ENV)


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c99", *SAN, "-fopenmp", "-ffp-contract=off", os.path.join(ROOT, "oracle", "fea_oracle.c"),
          os.path.join(ROOT, "tests", "native", "oracle_check.c"), "-lm", "-o", exe])
    m = mg.heterogeneous(6, seed=81, brick=2, jitter=0.15)
    m.u = mg.smooth_field(m, 3, seed=82) * 0.5
    d = tmp_path / "mesh"
    d.mkdir()
    arrays = {"sizes.i64": np.array([m.n_nodes, m.n_elems, m.conn.size], np.int64), "types.u8": m.types,
              "conn_ptr.i64": m.conn_ptr, "conn.i32": m.conn, "x.f64": m.x, "y.f64": m.y, "z.f64": m.z,
              "young.f64": m.young, "nu.f64": m.nu, "nh.u8": m.nh_flag, "u.f64": m.u,
              "source.f64": np.ascontiguousarray(m.source[:, :3])}
    for k, v in arrays.items():
        np.ascontiguousarray(v).tofile(str(d / k))
    _run([exe, str(d)], env=ENV)

    def rd(name, dt):
        return np.fromfile(str(d / name), dtype=dt)

    g = oracle.mesh_graph(m)
    assert np.array_equal(rd("row_ptr.i64", np.int64), g.row_ptr)
    assert np.array_equal(rd("e2nnz.i32", np.int32), g.e2nnz)
    assert np.array_equal(rd("inv.i32", np.int32), g.inv)
    c, _ = oracle.colour_greedy(m.n_nodes, m.conn_ptr, m.conn)
    assert np.array_equal(rd("colour.i16", np.int16), c)
    mp = mg.Mesh(**{**m.__dict__, "source": np.ascontiguousarray(m.source[:, 2:3])})
    for tag, mesh, model, nh in (("p", mp, oracle.POISSON, False), ("l", m, oracle.ELASTIC, False),
                                 ("n", m, oracle.ELASTIC, True)):
        v, r = oracle.assemble(mesh, g, model=model, use_nh=nh)
        assert np.array_equal(rd(f"{tag}_vals.f64", np.float64), v), tag
        assert np.array_equal(rd(f"{tag}_rhs.f64", np.float64), r), tag
    v, _ = oracle.assemble(m, g, model=oracle.ELASTIC, use_nh=True)
    for tag in ("omp_atomic", "omp_colour"):
        assert np.abs(rd(f"{tag}_vals.f64", np.float64) - v).max() <= 1e-13 * np.abs(v).max()
    assert np.array_equal(rd("residual.f64", np.float64), oracle.residual(m, use_nh=True))
    _, sub = oracle.subscale(m, m.u, model=oracle.ELASTIC)
    assert np.array_equal(rd("subscale.f64", np.float64), sub.reshape(-1))
