"""CPU oracle for finite-element assembly -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library (paper_1805_03949_amd) never imports it;
the two share no code apart from the seeded input generator (meshgen).

Contents:
  fea_oracle.c   plain FP64 C: shape functions, Gauss rules, element
                 matrices (Poisson, linear elasticity, neo-Hookean tangent),
                 sparsity pattern / element-to-nonzero map / inverse map,
                 greedy colouring, Algorithm 1 assembly with |term| sums,
                 the Newton residual and the element-wise subgrid scale
  dense.py       a second, independent formulation (dense Voigt B^T D B) for
                 tiny meshes, used to cross-check fea_oracle.c
  mlp.py         FP64 NumPy forward/backward/Adam for the cost model
  sched.py       load-balance metric and list-scheduling simulation
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fea_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a library built elsewhere from a modified copy of fea_oracle.c, loaded
# instead of liboracle.so (the test that plants mistakes in the oracle)
_OVERRIDE = os.environ.get("FEA_ORACLE_LIB")

POISSON, ELASTIC = 0, 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O3, OpenMP for the parallel timing
    variants, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _OVERRIDE:
            L = ctypes.CDLL(_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.or_shape.argtypes = [ctypes.c_int, P, P, P]
        L.or_rule.argtypes = [ctypes.c_int, P, P]
        L.or_element.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_double,
                                 ctypes.c_double, P, P, P, P, P, P]
        L.or_element_fint.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_double, P, P]
        L.or_graph_rows.argtypes = [i64, i64, P, P, P, P, P]
        L.or_graph_rows.restype = i64
        L.or_graph_fill.argtypes = [i64, i64, P, P, P, P, P, P, P, P]
        L.or_colour_greedy.argtypes = [i64, i64, P, P, P]
        L.or_assemble.argtypes = [i64, i64, P, P, P, P, P, P, ctypes.c_int, P, P, P, P, P,
                                  P, P, P, P, P, P, P]
        L.or_assemble.restype = i64
        L.or_assemble_omp.argtypes = [ctypes.c_int, i64, i64, P, P, P, P, P, P, ctypes.c_int, P, P, P, P, P,
                                      P, P, P, P, P, ctypes.c_int, P, P]
        L.or_assemble_omp.restype = i64
        L.or_threads.restype = ctypes.c_int
        L.or_residual.argtypes = [i64, i64, P, P, P, P, P, P, P, P, P, P, P, P]
        L.or_residual.restype = i64
        L.or_shape2.argtypes = [ctypes.c_int, P, P]
        L.or_element_subscale.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_double, ctypes.c_double,
                                          P, P, P]
        L.or_subscale.argtypes = [i64, P, P, P, P, P, P, ctypes.c_int, P, P, P, P, P, P]
        L.or_subscale.restype = i64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


NODES = (4, 5, 6, 8)


def shape(etype, xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    N = np.zeros(8)
    dN = np.zeros((8, 3))
    nn = lib().or_shape(etype, _p(xi), _p(N), _p(dN))
    return N[:nn].copy(), dN[:nn].copy()


def rule(etype):
    pts = np.zeros((8, 3))
    w = np.zeros(8)
    nq = lib().or_rule(etype, _p(pts), _p(w))
    return pts[:nq].copy(), w[:nq].copy()


def element(etype, X, model=ELASTIC, young=1.0, nu=0.3, f=None, u=None, nh=False,
            with_terms=False):
    """Element matrix Ke[(nn*B),(nn*B)] (dof = a*B + i) and vector fe[nn*B]."""
    nn = NODES[etype]
    B = 1 if model == POISSON else 3
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(nn, 3)
    U = np.zeros((nn, 3)) if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(nn, 3)
    if f is None:
        f = np.ones(1) if B == 1 else np.array([0.0, 0.0, -1.0])
    f = np.ascontiguousarray(f, dtype=np.float64)
    Ke = np.zeros(nn * nn * B * B)
    fe = np.zeros(nn * B)
    Tk = np.zeros_like(Ke)
    Tf = np.zeros_like(fe)
    rc = lib().or_element(etype, model, int(bool(nh)), _p(X), young, nu, _p(U), _p(f), _p(Ke),
                          _p(fe), _p(Tk), _p(Tf))
    if rc != 0:
        raise ValueError(f"element rejected (code {rc}): detJ <= 0")
    # block order (a, b, i, j) -> dense (a*B+i, b*B+j)
    K = Ke.reshape(nn, nn, B, B).transpose(0, 2, 1, 3).reshape(nn * B, nn * B)
    if with_terms:
        T = Tk.reshape(nn, nn, B, B).transpose(0, 2, 1, 3).reshape(nn * B, nn * B)
        return K, fe, T, Tf
    return K, fe


def element_fint(etype, X, young, nu, u):
    nn = NODES[etype]
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(nn, 3)
    U = np.ascontiguousarray(u, dtype=np.float64).reshape(nn, 3)
    out = np.zeros(nn * 3)
    rc = lib().or_element_fint(etype, _p(X), young, nu, _p(U), _p(out))
    if rc != 0:
        raise ValueError("element rejected")
    return out


class Graph:
    """Block sparsity pattern + element-to-nonzero map + inverse map."""

    def __init__(self, row_ptr, col, map_ptr, e2nnz, inv_ptr, inv):
        self.row_ptr, self.col, self.map_ptr = row_ptr, col, map_ptr
        self.e2nnz, self.inv_ptr, self.inv = e2nnz, inv_ptr, inv

    @property
    def nnz(self):
        return int(self.col.shape[0])


class MeshError(ValueError):
    def __init__(self, elem):
        super().__init__(f"invalid element {elem}")
        self.elem = elem


def graph(n_nodes, types, conn_ptr, conn):
    types = np.ascontiguousarray(types, dtype=np.uint8)
    conn_ptr = np.ascontiguousarray(conn_ptr, dtype=np.int64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E = types.shape[0]
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    map_ptr = np.zeros(E + 1, dtype=np.int64)
    rc = lib().or_graph_rows(n_nodes, E, _p(types), _p(conn_ptr), _p(conn), _p(row_ptr),
                             _p(map_ptr))
    if rc != 0:
        raise MeshError(-rc - 1)
    nnz = int(row_ptr[-1])
    ml = int(map_ptr[-1])
    col = np.zeros(nnz, dtype=np.int32)
    e2nnz = np.zeros(ml, dtype=np.int32)
    inv_ptr = np.zeros(nnz + 1, dtype=np.int64)
    inv = np.zeros(ml, dtype=np.int32)
    rc = lib().or_graph_fill(n_nodes, E, _p(conn_ptr), _p(conn), _p(row_ptr), _p(map_ptr),
                             _p(col), _p(e2nnz), _p(inv_ptr), _p(inv))
    if rc != 0:
        raise RuntimeError(f"or_graph_fill failed ({rc})")
    return Graph(row_ptr, col, map_ptr, e2nnz, inv_ptr, inv)


def mesh_graph(mesh):
    return graph(mesh.n_nodes, mesh.types, mesh.conn_ptr, mesh.conn)


def colour_greedy(n_nodes, conn_ptr, conn):
    E = conn_ptr.shape[0] - 1
    colour = np.zeros(E, dtype=np.int16)
    nc = lib().or_colour_greedy(n_nodes, E, _p(np.ascontiguousarray(conn_ptr, dtype=np.int64)),
                                _p(np.ascontiguousarray(conn, dtype=np.int32)), _p(colour))
    return colour, nc


def assemble(mesh, g, model=ELASTIC, with_terms=False, use_nh=True):
    """Algorithm 1 assembly of the whole mesh. Returns (vals, rhs[, tvals, trhs])."""
    B = 1 if model == POISSON else 3
    nnz = g.nnz
    vals = np.zeros(nnz * B * B)
    rhs = np.zeros(mesh.n_nodes * B)
    tv = np.zeros_like(vals) if with_terms else None
    tr = np.zeros_like(rhs) if with_terms else None
    if mesh.source.shape[1] < B:
        raise ValueError("elasticity needs a 3-component source per element")
    src = np.ascontiguousarray(mesh.source[:, :B], dtype=np.float64)
    nh = np.ascontiguousarray(mesh.nh_flag, dtype=np.uint8) if use_nh else None
    rc = lib().or_assemble(mesh.n_nodes, mesh.n_elems, _p(mesh.types), _p(mesh.conn_ptr),
                           _p(mesh.conn), _p(mesh.x), _p(mesh.y), _p(mesh.z), model,
                           _p(mesh.young), _p(mesh.nu), _p(nh), _p(mesh.u), _p(src),
                           _p(g.row_ptr), _p(g.map_ptr), _p(g.e2nnz), _p(vals), _p(rhs),
                           _p(tv), _p(tr))
    if rc != 0:
        raise MeshError(-rc - 1)
    if with_terms:
        return vals, rhs, tv, tr
    return vals, rhs


def threads():
    """OpenMP threads the parallel variants use (OMP_NUM_THREADS, else all cores)."""
    return int(lib().or_threads())


def colour_buckets(colour, n_colours):
    """Element ids grouped by colour (ascending within a colour) and the
    bucket offsets cptr[n_colours + 1]."""
    celems = np.argsort(colour, kind="stable").astype(np.int32)
    cptr = np.zeros(n_colours + 1, dtype=np.int64)
    cptr[1:] = np.cumsum(np.bincount(colour.astype(np.int64), minlength=n_colours))
    return cptr, celems


def assemble_parallel(mesh, g, variant, model=ELASTIC, use_nh=True, buckets=None):
    """Algorithm 1 with the element loop on OpenMP threads (timing variants):
    variant "atomic" (Algorithm 4) or "colour" (Algorithm 5; buckets from
    colour_buckets, computed here when not given). Returns (vals, rhs),
    equal to assemble()'s up to rounding."""
    B = 1 if model == POISSON else 3
    vals = np.zeros(g.nnz * B * B)
    rhs = np.zeros(mesh.n_nodes * B)
    src = np.ascontiguousarray(mesh.source[:, :B], dtype=np.float64)
    nh = np.ascontiguousarray(mesh.nh_flag, dtype=np.uint8) if use_nh else None
    if variant == "colour":
        if buckets is None:
            colour, nc = colour_greedy(mesh.n_nodes, mesh.conn_ptr, mesh.conn)
            buckets = colour_buckets(colour, nc)
        cptr, celems = buckets
        v = 2
    elif variant == "atomic":
        cptr, celems, v = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int32), 1
    else:
        raise ValueError(variant)
    rc = lib().or_assemble_omp(v, mesh.n_nodes, mesh.n_elems, _p(mesh.types), _p(mesh.conn_ptr), _p(mesh.conn),
                               _p(mesh.x), _p(mesh.y), _p(mesh.z), model, _p(mesh.young), _p(mesh.nu), _p(nh),
                               _p(mesh.u), _p(src), _p(g.row_ptr), _p(g.map_ptr), _p(g.e2nnz), _p(cptr),
                               _p(celems), int(cptr.shape[0] - 1), _p(vals), _p(rhs))
    if rc != 0:
        raise MeshError(-rc - 1)
    return vals, rhs


def residual(mesh, use_nh=True):
    """Newton residual b = f_ext - f_int(mesh.u) of the elastic solid
    (neo-Hookean internal force where nh_flag is set and use_nh, linear
    K^e u^e elsewhere), node-major rhs[3 * n_nodes]."""
    if mesh.source.shape[1] < 3:
        raise ValueError("elasticity needs a 3-component source per element")
    src = np.ascontiguousarray(mesh.source[:, :3], dtype=np.float64)
    nh = np.ascontiguousarray(mesh.nh_flag, dtype=np.uint8) if use_nh else None
    u = np.ascontiguousarray(mesh.u, dtype=np.float64)
    rhs = np.zeros(mesh.n_nodes * 3)
    rc = lib().or_residual(mesh.n_nodes, mesh.n_elems, _p(mesh.types), _p(mesh.conn_ptr), _p(mesh.conn),
                           _p(mesh.x), _p(mesh.y), _p(mesh.z), _p(mesh.young), _p(mesh.nu), _p(nh), _p(u),
                           _p(src), _p(rhs))
    if rc != 0:
        raise MeshError(-rc - 1)
    return rhs


def shape2(etype, xi):
    """Second reference derivatives D2[a, j, l] = d2 N_a / dxi_j dxi_l."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    D2 = np.zeros((8, 3, 3))
    nn = lib().or_shape2(etype, _p(xi), _p(D2))
    return D2[:nn].copy()


def element_subscale(etype, X, u, model=ELASTIC, young=1.0, nu=0.3, f=None):
    """Subgrid scale of one element at its Gauss points, shape (nq, B):
    tau_e (f + L(u_h)(x_q)), L the Laplacian (Poisson) or div sigma
    (linear elasticity), tau_e = V_e^(2/3) / (4 k), k = 1 or mu."""
    nn = NODES[etype]
    B = 1 if model == POISSON else 3
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(nn, 3)
    U = np.ascontiguousarray(u, dtype=np.float64).reshape(nn * B)
    if f is None:
        f = np.ones(1) if B == 1 else np.array([0.0, 0.0, -1.0])
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(8 * B)
    rc = lib().or_element_subscale(etype, model, _p(X), young, nu, _p(U), _p(f), _p(out))
    if rc != 0:
        raise ValueError(f"element rejected (code {rc}): detJ <= 0")
    nq = rule(etype)[0].shape[0]
    return out[:nq * B].reshape(nq, B).copy()


def subscale(mesh, u, model=ELASTIC):
    """Subgrid scale of every element (element loop, nothing assembled).
    u: nodal field, B values per node (node-major). Returns (gp_ptr, out)
    with element e's Gauss points at rows gp_ptr[e] .. gp_ptr[e+1] of
    out[n_points, B]."""
    B = 1 if model == POISSON else 3
    if mesh.source.shape[1] < B:
        raise ValueError("elasticity needs a 3-component source per element")
    src = np.ascontiguousarray(mesh.source[:, :B], dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    if u.shape[0] != mesh.n_nodes * B:
        raise ValueError("u must hold B values per node")
    gp_ptr = np.zeros(mesh.n_elems + 1, dtype=np.int64)
    n_pts = int(sum(rule(t)[0].shape[0] * int(np.count_nonzero(mesh.types == t)) for t in range(4)))
    out = np.zeros(n_pts * B)
    rc = lib().or_subscale(mesh.n_elems, _p(mesh.types), _p(mesh.conn_ptr), _p(mesh.conn), _p(mesh.x),
                           _p(mesh.y), _p(mesh.z), model, _p(mesh.young), _p(mesh.nu), _p(u), _p(src),
                           _p(gp_ptr), _p(out))
    if rc != 0:
        raise MeshError(-rc - 1)
    return gp_ptr, out.reshape(n_pts, B)


def to_dense(g, vals, B, n_nodes):
    """Dense matrix (dof = node*B + i) from block CSR values (tiny meshes only)."""
    A = np.zeros((n_nodes * B, n_nodes * B))
    V = vals.reshape(-1, B, B)
    for r in range(n_nodes):
        for k in range(g.row_ptr[r], g.row_ptr[r + 1]):
            c = g.col[k]
            A[r * B:(r + 1) * B, c * B:(c + 1) * B] = V[k]
    return A
