"""Python binding of libfea.so, the gfx950 finite-element assembly library.

Argument marshalling only: every step of the graph build and the assembly
runs in the library's HIP kernels. PyTorch (ROCm) supplies device memory and
the stream. The C ABI is declared in include/fea.h.

If libfea.so has not been built, importing this package raises ImportError:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfea.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                      f"g.build()'` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

FEA_OK, FEA_EINVAL, FEA_EMESH, FEA_ENOMEM, FEA_EHIP, FEA_ERANGE = 0, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
ROWOWNER, ATOMIC, COLOUR, ROWGATHER, ROWSYM, TILECOLOUR = 0, 1, 2, 3, 4, 5
F64, F32 = 0, 1
POISSON, ELASTIC = 0, 1
VARIANTS = {"rowowner": ROWOWNER, "atomic": ATOMIC, "colour": COLOUR, "rowgather": ROWGATHER, "rowsym": ROWSYM,
            "tilecolour": TILECOLOUR}

_P = ctypes.c_void_p
_I64 = ctypes.c_int64


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("variant", ctypes.c_int),
                ("out_dtype", ctypes.c_int), ("timing", ctypes.c_int)]


class Material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("young", _P), ("nu", _P), ("nh_flag", _P), ("u", _P),
                ("residual", ctypes.c_int)]


_lib.fea_graph_build.argtypes = [_I64, _I64, _P, _P, _P, _P, ctypes.POINTER(_P)]
_lib.fea_graph_build.restype = ctypes.c_int
_lib.fea_graph_save.argtypes = [_P, ctypes.c_char_p]
_lib.fea_graph_load.argtypes = [ctypes.c_char_p, _I64, _I64, _P, _P, _P, _P, ctypes.POINTER(_P)]
_lib.fea_graph_sizes.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                 ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int)]
_lib.fea_graph_sym_sizes.argtypes = [_P] + [ctypes.POINTER(_I64)] * 4
_lib.fea_graph_export.argtypes = [_P] * 9 + [ctypes.POINTER(_I64), _P]
_lib.fea_graph_tile_colouring.argtypes = [_P, ctypes.POINTER(ctypes.c_int), _P, _P, _P, _P]
_lib.fea_graph_destroy.argtypes = [_P]
_lib.fea_graph_destroy.restype = None
_lib.fea_assemble.argtypes = [_P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(Material), _P,
                              ctypes.POINTER(Options), _P, _P, _P, _P]
_lib.fea_assemble_noalloc.argtypes = _lib.fea_assemble.argtypes
_lib.fea_last_timing.argtypes = [_P, ctypes.POINTER(ctypes.c_float)]
_lib.fea_graph_gauss_points.argtypes = [_P, ctypes.POINTER(_I64), _P, _P]
_lib.fea_subscale.argtypes = [_P, _P, _P, _P, ctypes.POINTER(Material), _P, _P, _P, _P, _P]
_lib.fea_batch_gauss_points.argtypes = [_P, _P, _P]
_lib.fea_batch_subscale.argtypes = [_P, _P, _P, _P]
_lib.fea_last_class_timing.argtypes = [_P, ctypes.POINTER(ctypes.c_float)]
_lib.fea_last_error.restype = ctypes.c_char_p
_lib.fea_version.restype = ctypes.c_char_p


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_nodes", _I64), ("n_elems", _I64), ("types", _P), ("conn_ptr", _P), ("conn", _P),
                ("x", _P), ("y", _P), ("z", _P), ("young", _P), ("nu", _P), ("nh_flag", _P),
                ("u", _P), ("source", _P)]


_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(_I64)
_lib.fea_batch_build.argtypes = [ctypes.c_int, ctypes.POINTER(MeshDesc), ctypes.c_int, _I32P, _P,
                                 ctypes.POINTER(_P)]
_lib.fea_batch_sizes.argtypes = [_P, _I64P, _I64P, _I64P, _I64P]
_lib.fea_batch_offsets.argtypes = [_P, _I64P, _I64P]
_lib.fea_batch_items.argtypes = [_P, _I32P]
_lib.fea_batch_set_tiles.argtypes = [_P, _I32P]
_lib.fea_batch_set_order.argtypes = [_P, _I32P]
_lib.fea_batch_get_order.argtypes = [_P, _I32P]
_lib.fea_batch_assemble.argtypes = [_P, ctypes.POINTER(Options), _P, _P, _P, _P]
_lib.fea_batch_capture.argtypes = [_P, ctypes.POINTER(Options), _P, _P, _P, _P]
_lib.fea_batch_replay.argtypes = [_P, ctypes.c_int, _P]
_lib.fea_batch_cycles.argtypes = [_P, _P, _P, _P, _P]
_lib.fea_batch_last_ms.argtypes = [_P, ctypes.POINTER(ctypes.c_float)]
_lib.fea_batch_workers.argtypes = [_P, ctypes.POINTER(ctypes.c_int)]
_lib.fea_batch_destroy.argtypes = [_P]
_lib.fea_batch_destroy.restype = None
_lib.fea_batch_autotune.argtypes = [_P, ctypes.POINTER(Options), ctypes.c_int, ctypes.c_char_p, _P, _I32P]
_lib.fea_tile_table_load.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, _I32P]
_lib.fea_batch_order.argtypes = [_P, ctypes.c_int, _P, _P]
_lib.fea_batch_partition.argtypes = [_P, ctypes.c_int, _P, _P]
_lib.fea_batch_features.argtypes = [_P, ctypes.c_int, _P, _P]
_lib.fea_cost_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(_P)]
_lib.fea_cost_destroy.argtypes = [_P]
_lib.fea_cost_destroy.restype = None
_F32P = ctypes.POINTER(ctypes.c_float)
_lib.fea_cost_get_params.argtypes = [_P, _F32P]
_lib.fea_cost_set_params.argtypes = [_P, _F32P]
_lib.fea_cost_set_norm.argtypes = [_P, _F32P, _F32P]
_lib.fea_cost_fit_norm.argtypes = [_P, _P, _I64, _P]
_lib.fea_cost_predict.argtypes = [_P, _P, _I64, _P, _P]
_lib.fea_cost_grad.argtypes = [_P, _P, _P, _I64, _P, _P, _P]
_lib.fea_cost_train.argtypes = [_P, _P, _P, _I64, ctypes.c_int, ctypes.c_float, _P, _P]
_lib.fea_cost_log_cycles.argtypes = [_P, _I64, _P, _P]
_lib.fea_cost_save.argtypes = [_P, ctypes.c_char_p]
_lib.fea_cost_load.argtypes = [_P, ctypes.c_char_p]

TYPE_SORTED, LEARNED, GP_WEIGHT, LEARNED_CLASSES = 0, 1, 2, 3
N_FEATURES, N_PARAMS = 12, 5057

# every exported symbol declared in include/fea.h
EXPORTS = ("fea_graph_build", "fea_graph_save", "fea_graph_load", "fea_graph_sizes", "fea_graph_sym_sizes",
           "fea_graph_export", "fea_graph_destroy",
           "fea_graph_tile_colouring",
           "fea_assemble", "fea_assemble_noalloc", "fea_last_timing", "fea_graph_gauss_points", "fea_subscale",
           "fea_batch_gauss_points", "fea_batch_subscale", "fea_last_class_timing", "fea_last_error", "fea_version",
           "fea_batch_build", "fea_batch_sizes", "fea_batch_offsets", "fea_batch_items",
           "fea_batch_set_tiles", "fea_batch_set_order", "fea_batch_get_order", "fea_batch_assemble", "fea_batch_capture",
           "fea_batch_replay", "fea_batch_cycles", "fea_batch_last_ms", "fea_batch_workers",
           "fea_batch_destroy", "fea_batch_autotune", "fea_tile_table_load", "fea_batch_order",
           "fea_batch_partition",
           "fea_batch_features", "fea_cost_create", "fea_cost_destroy", "fea_cost_get_params",
           "fea_cost_set_params", "fea_cost_set_norm", "fea_cost_fit_norm", "fea_cost_predict",
           "fea_cost_grad", "fea_cost_train", "fea_cost_log_cycles", "fea_cost_save", "fea_cost_load")


class FeaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fea error {code}: {msg}")
        self.code = code
        self.msg = msg


# Library objects released while a HIP graph is being captured on this
# thread's current stream: freeing device memory then (a garbage-collected
# Graph, Batch or CostModel) would invalidate the capture, so their
# destruction waits for the next release outside a capture.
_deferred = []


def _capturing():
    try:
        return torch.cuda.is_available() and torch.cuda.is_current_stream_capturing()
    except Exception:
        return False


def _release(destroy_fn, handle):
    if _capturing():
        _deferred.append((destroy_fn, handle))
        return
    while _deferred:
        fn, h = _deferred.pop()
        fn(h)
    destroy_fn(handle)


def _check(rc):
    if rc != FEA_OK:
        raise FeaError(rc, _lib.fea_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def version():
    return _lib.fea_version().decode()


def _dev(t, dtype):
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
    return t


class Graph:
    """Sparsity graph built on the GPU from device connectivity tensors, or
    read from a graph cache file written by save() (cache=path)."""

    def __init__(self, n_nodes, types, conn_ptr, conn, stream=None, cache=None):
        _dev(types, torch.uint8)
        _dev(conn_ptr, torch.int64)
        _dev(conn, torch.int32)
        h = _P()
        if cache is None:
            _check(_lib.fea_graph_build(int(n_nodes), int(types.numel()), _ptr(types), _ptr(conn_ptr),
                                        _ptr(conn), _stream(stream), ctypes.byref(h)))
        else:
            _check(_lib.fea_graph_load(str(cache).encode(), int(n_nodes), int(types.numel()), _ptr(types),
                                       _ptr(conn_ptr), _ptr(conn), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.device = types.device
        n, e, nnz, ml = _I64(), _I64(), _I64(), _I64()
        nc = ctypes.c_int()
        _check(_lib.fea_graph_sizes(h, ctypes.byref(n), ctypes.byref(e), ctypes.byref(nnz),
                                    ctypes.byref(ml), ctypes.byref(nc)))
        self.n_nodes, self.n_elems, self.nnz, self.map_len = n.value, e.value, nnz.value, ml.value
        self.n_colours = nc.value

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph destroyed")
        return self._h

    def save(self, path):
        """Writes the graph cache file (fea_graph_save)."""
        _check(_lib.fea_graph_save(self.handle, str(path).encode()))

    def export(self, stream=None):
        d = self.device
        out = dict(
            row_ptr=torch.empty(self.n_nodes + 1, dtype=torch.int64, device=d),
            col=torch.empty(self.nnz, dtype=torch.int32, device=d),
            map_ptr=torch.empty(self.n_elems + 1, dtype=torch.int64, device=d),
            e2nnz=torch.empty(self.map_len, dtype=torch.int32, device=d),
            inv_ptr=torch.empty(self.nnz + 1, dtype=torch.int64, device=d),
            inv=torch.empty(self.map_len, dtype=torch.int32, device=d),
            colour=torch.empty(self.n_elems, dtype=torch.int16, device=d),
            type_perm=torch.empty(self.n_elems, dtype=torch.int32, device=d),
        )
        seg = (_I64 * 5)()
        _check(_lib.fea_graph_export(self.handle, _ptr(out["row_ptr"]), _ptr(out["col"]),
                                     _ptr(out["map_ptr"]), _ptr(out["e2nnz"]), _ptr(out["inv_ptr"]),
                                     _ptr(out["inv"]), _ptr(out["colour"]), _ptr(out["type_perm"]),
                                     seg, _stream(stream)))
        out["type_seg"] = list(seg)
        return out

    def sym_sizes(self):
        """Sizes of the upper-triangle layout (after the first ROWSYM
        assembly): tiles, entries, tile_blocks, upper_blocks."""
        v = [_I64() for _ in range(4)]
        _check(_lib.fea_graph_sym_sizes(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(("tiles", "entries", "tile_blocks", "upper_blocks"), (x.value for x in v)))

    def tile_colouring(self, stream=None):
        """(n_colours, bucket_ptr[4 * (C + 1)], tiles (device int32), nneig)
        of the tile-coloured form (after its first assembly)."""
        nc = ctypes.c_int()
        _check(_lib.fea_graph_tile_colouring(self.handle, ctypes.byref(nc), None, None, None, _stream(stream)))
        import numpy as np
        sz = self.sym_sizes()
        bp = np.zeros(4 * (nc.value + 1), dtype=np.int64)
        nneig = np.zeros(max(sz["tiles"], 1), dtype=np.int32)
        tiles = torch.empty(max(sz["tiles"], 1), dtype=torch.int32, device=self.device)
        _check(_lib.fea_graph_tile_colouring(self.handle, ctypes.byref(nc), bp.ctypes.data_as(_P),
                                             _ptr(tiles), nneig.ctypes.data_as(_P), _stream(stream)))
        return nc.value, bp, tiles[:sz["tiles"]], nneig[:sz["tiles"]]

    def gauss_points(self, stream=None):
        """(n_points, gp_ptr): total Gauss points and the device offsets of
        each element's points, in element order."""
        n = _I64()
        gp_ptr = torch.empty(self.n_elems + 1, dtype=torch.int64, device=self.device)
        _check(_lib.fea_graph_gauss_points(self.handle, ctypes.byref(n), _ptr(gp_ptr), _stream(stream)))
        return n.value, gp_ptr

    def last_timing(self):
        """(element ms, second-phase ms, total ms) of the last timed assemble."""
        ms = (ctypes.c_float * 3)()
        _check(_lib.fea_last_timing(self.handle, ms))
        return tuple(float(v) for v in ms)

    def last_class_timing(self):
        """Per-class kernel ms (tet4, pyr5, pen6, hex8, interface rows) of the
        last timed row-gather assemble."""
        ms = (ctypes.c_float * 5)()
        _check(_lib.fea_last_class_timing(self.handle, ms))
        return tuple(float(v) for v in ms)

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _release(_lib.fea_graph_destroy, h)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def assemble(graph, x, y, z, types, conn_ptr, conn, source, model=ELASTIC, young=None, nu=None,
             nh_flag=None, u=None, precision=FP64, variant=ROWOWNER, out_dtype=F64, vals=None,
             rhs=None, status=None, stream=None, timing=False, residual=False, noalloc=False):
    """Assembles (vals, rhs, status) on the GPU; all tensors on the graph's device.
    residual: rhs is the Newton residual f_ext - f_int(u) (elasticity, FP64).
    noalloc: call fea_assemble_noalloc (row-owner, library workspaces in its
    static scratch; the caller's tensors are still allocated here when not
    given)."""
    B = 1 if model == POISSON else 3
    odt = torch.float64 if out_dtype == F64 else torch.float32
    d = graph.device
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    if vals is None:
        vals = torch.empty(graph.nnz * B * B, dtype=odt, device=d)
    if rhs is None:
        rhs = torch.empty(graph.n_nodes * B, dtype=odt, device=d)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=d)
    for t in (x, y, z, source):
        _dev(t, torch.float64)
    for t in (young, nu, u):
        if t is not None:
            _dev(t, torch.float64)
    if nh_flag is not None:
        _dev(nh_flag, torch.uint8)
    _dev(vals, odt)
    _dev(rhs, odt)
    mat = Material(model, _ptr(young), _ptr(nu), _ptr(nh_flag), _ptr(u), int(bool(residual)))
    opt = Options(precision, variant, out_dtype, int(bool(timing)))
    fn = _lib.fea_assemble_noalloc if noalloc else _lib.fea_assemble
    _check(fn(graph.handle, _ptr(x), _ptr(y), _ptr(z), _ptr(types), _ptr(conn_ptr), _ptr(conn), ctypes.byref(mat),
              _ptr(source), ctypes.byref(opt), _stream(stream), _ptr(vals), _ptr(rhs), _ptr(status)))
    return vals, rhs, status


def subscale(graph, x, y, z, u, source, model=ELASTIC, young=None, nu=None, out=None, status=None,
             stream=None):
    """Element-wise subgrid scale tau_e (f_e + L(u_h)) at every Gauss point,
    FP64, out[n_points, B] with element e's points at rows gp_ptr[e] ..
    gp_ptr[e+1] (Graph.gauss_points). u: nodal field, B values per node."""
    B = 1 if model == POISSON else 3
    d = graph.device
    if u.numel() != graph.n_nodes * B or source.numel() != graph.n_elems * B:
        raise ValueError(f"u needs {B} values per node and source {B} per element")
    n_pts, _ = graph.gauss_points(stream) if out is None else (None, None)
    if out is None:
        out = torch.empty((n_pts, B), dtype=torch.float64, device=d)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=d)
    for t in (x, y, z, u, source, out):
        _dev(t, torch.float64)
    for t in (young, nu):
        if t is not None:
            _dev(t, torch.float64)
    mat = Material(model, _ptr(young), _ptr(nu), None, None, 0)
    _check(_lib.fea_subscale(graph.handle, _ptr(x), _ptr(y), _ptr(z), ctypes.byref(mat), _ptr(u), _ptr(source),
                             _stream(stream), _ptr(out), _ptr(status)))
    return out, status


class DeviceMesh:
    """Device copies of a mesh's arrays (connectivity, coordinates, material)."""

    FIELDS = ("x", "y", "z", "types", "conn_ptr", "conn", "young", "nu", "nh_flag", "u")

    def __init__(self, mesh, device="cuda", dofs=3):
        dev = torch.device(device)
        self.n_nodes = mesh.n_nodes
        self.n_elems = mesh.n_elems
        for f in self.FIELDS:
            setattr(self, f, torch.from_numpy(getattr(mesh, f)).to(dev).contiguous())
        src = mesh.source[:, :dofs]
        self.source = torch.from_numpy(src.copy()).to(dev).contiguous()

    def graph(self, stream=None, cache=None):
        return Graph(self.n_nodes, self.types, self.conn_ptr, self.conn, stream=stream, cache=cache)

    def assemble(self, graph, model=ELASTIC, use_nh=False, residual=False, **kw):
        src = self.source
        if model == POISSON:
            src = src[:, :1].contiguous()
        return assemble(graph, self.x, self.y, self.z, self.types, self.conn_ptr, self.conn,
                        src, model=model, young=self.young,
                        nu=self.nu if model == ELASTIC else None,
                        nh_flag=self.nh_flag if (use_nh and model == ELASTIC) else None,
                        u=self.u if ((use_nh or residual) and model == ELASTIC) else None,
                        residual=residual, **kw)


    def subscale(self, graph, u, model=ELASTIC, **kw):
        """Subgrid scale of every element for the nodal field u (B values per
        node, a device FP64 tensor)."""
        src = self.source
        if model == POISSON:
            src = src[:, :1].contiguous()
        return subscale(graph, self.x, self.y, self.z, u, src, model=model, young=self.young,
                        nu=self.nu if model == ELASTIC else None, **kw)


def _np_i32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


class Batch:
    """Many meshes assembled by one persistent launch fed from a device queue."""

    def __init__(self, meshes, model=ELASTIC, tile=None, use_nh=False, stream=None):
        import numpy as np
        self.meshes = list(meshes)
        self.model = model
        self.device = self.meshes[0].x.device if self.meshes else torch.device("cuda")
        self._keep = []
        descs = (MeshDesc * max(1, len(self.meshes)))()
        for i, dm in enumerate(self.meshes):
            src = dm.source if model == ELASTIC else dm.source[:, :1].contiguous()
            self._keep.append(src)
            nh = dm.nh_flag if (use_nh and model == ELASTIC) else None
            descs[i] = MeshDesc(dm.n_nodes, dm.n_elems, _ptr(dm.types), _ptr(dm.conn_ptr), _ptr(dm.conn),
                                _ptr(dm.x), _ptr(dm.y), _ptr(dm.z), _ptr(dm.young),
                                _ptr(dm.nu) if model == ELASTIC else None, _ptr(nh),
                                _ptr(dm.u) if model == ELASTIC else None, _ptr(src))
        h = _P()
        tp = None
        if tile is not None:
            self._tile, tp = _np_i32(tile)
        _check(_lib.fea_batch_build(len(self.meshes), descs, model, tp, _stream(stream), ctypes.byref(h)))
        self._h = h
        self._refresh()

    def _refresh(self):
        import numpy as np
        v, r, ni, ne = _I64(), _I64(), _I64(), _I64()
        _check(_lib.fea_batch_sizes(self._h, ctypes.byref(v), ctypes.byref(r), ctypes.byref(ni),
                                    ctypes.byref(ne)))
        self.vals_len, self.rhs_len, self.n_items, self.n_elems = v.value, r.value, ni.value, ne.value
        n = len(self.meshes)
        vo = (_I64 * (n + 1))()
        ro = (_I64 * (n + 1))()
        _check(_lib.fea_batch_offsets(self._h, vo, ro))
        self.vals_off = np.array(list(vo), dtype=np.int64)
        self.rhs_off = np.array(list(ro), dtype=np.int64)
        items = np.zeros(max(1, self.n_items) * 4, dtype=np.int32)
        _check(_lib.fea_batch_items(self._h, items.ctypes.data_as(_I32P)))
        self.items = items[: self.n_items * 4].reshape(-1, 4)

    def set_tiles(self, tile):
        self._tile, tp = _np_i32(tile)
        _check(_lib.fea_batch_set_tiles(self._h, tp))
        self._refresh()

    def set_order(self, order):
        arr, p = _np_i32(order)
        _check(_lib.fea_batch_set_order(self._h, p))

    def get_order(self):
        import numpy as np
        out = np.zeros(max(1, self.n_items), dtype=np.int32)
        _check(_lib.fea_batch_get_order(self._h, out.ctypes.data_as(_I32P)))
        return out[: self.n_items]

    def outputs(self, out_dtype=F64):
        odt = torch.float64 if out_dtype == F64 else torch.float32
        return (torch.empty(self.vals_len, dtype=odt, device=self.device),
                torch.empty(self.rhs_len, dtype=odt, device=self.device),
                torch.empty(max(1, len(self.meshes)), dtype=torch.int32, device=self.device))

    def assemble(self, precision=FP64, out_dtype=F64, vals=None, rhs=None, status=None, stream=None,
                 timing=False, variant=ROWOWNER):
        if vals is None:
            vals, rhs, status = self.outputs(out_dtype)
        opt = Options(precision, variant, out_dtype, int(bool(timing)))
        _check(_lib.fea_batch_assemble(self._h, ctypes.byref(opt), _stream(stream), _ptr(vals), _ptr(rhs),
                                       _ptr(status)))
        return vals, rhs, status

    def capture(self, vals, rhs, status, precision=FP64, out_dtype=F64, stream=None, variant=ROWOWNER):
        opt = Options(precision, variant, out_dtype, 0)
        _check(_lib.fea_batch_capture(self._h, ctypes.byref(opt), _stream(stream), _ptr(vals), _ptr(rhs),
                                      _ptr(status)))

    def replay(self, n=1, stream=None):
        _check(_lib.fea_batch_replay(self._h, int(n), _stream(stream)))

    def cycles(self, stream=None):
        c = torch.empty(self.n_items, dtype=torch.int64, device=self.device)
        w = torch.empty(self.n_items, dtype=torch.int32, device=self.device)
        u = torch.empty(self.n_items, dtype=torch.int32, device=self.device)
        _check(_lib.fea_batch_cycles(self._h, _ptr(c), _ptr(w), _ptr(u), _stream(stream)))
        return c, w, u

    def last_ms(self):
        ms = ctypes.c_float()
        _check(_lib.fea_batch_last_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)

    def autotune(self, precision=FP64, out_dtype=F64, reps=5, table_path=None, stream=None, variant=ROWOWNER):
        import numpy as np
        if isinstance(variant, str):
            variant = VARIANTS[variant]
        opt = Options(precision, variant, out_dtype, 0)
        tile = np.zeros(4, dtype=np.int32)
        path = table_path.encode() if table_path else None
        _check(_lib.fea_batch_autotune(self._h, ctypes.byref(opt), int(reps), path, _stream(stream),
                                       tile.ctypes.data_as(_I32P)))
        self._refresh()
        return tile

    def order(self, schedule, pred=None, stream=None):
        _check(_lib.fea_batch_order(self._h, int(schedule), _ptr(pred), _stream(stream)))

    def partition(self, weights, pred=None, stream=None):
        _check(_lib.fea_batch_partition(self._h, int(weights), _ptr(pred), _stream(stream)))

    def features(self, fp64_geometry=True, stream=None):
        f = torch.empty((self.n_items, N_FEATURES), dtype=torch.float32, device=self.device)
        _check(_lib.fea_batch_features(self._h, int(bool(fp64_geometry)), _ptr(f), _stream(stream)))
        return f

    def workers(self):
        w = ctypes.c_int()
        _check(_lib.fea_batch_workers(self._h, ctypes.byref(w)))
        return int(w.value)

    def tile_colouring(self, stream=None):
        """(n_colours, bucket_ptr[4 * (C + 1)], tiles (device int32), nneig)
        of the tile-coloured form (after its first assembly)."""
        nc = ctypes.c_int()
        _check(_lib.fea_graph_tile_colouring(self.handle, ctypes.byref(nc), None, None, None, _stream(stream)))
        import numpy as np
        sz = self.sym_sizes()
        bp = np.zeros(4 * (nc.value + 1), dtype=np.int64)
        nneig = np.zeros(max(sz["tiles"], 1), dtype=np.int32)
        tiles = torch.empty(max(sz["tiles"], 1), dtype=torch.int32, device=self.device)
        _check(_lib.fea_graph_tile_colouring(self.handle, ctypes.byref(nc), bp.ctypes.data_as(_P),
                                             _ptr(tiles), nneig.ctypes.data_as(_P), _stream(stream)))
        return nc.value, bp, tiles[:sz["tiles"]], nneig[:sz["tiles"]]

    def gauss_points(self, stream=None):
        """Offsets (n_meshes + 1) of every mesh's Gauss points in the
        concatenated subgrid-scale output."""
        import numpy as np
        off = np.zeros(len(self.meshes) + 1, dtype=np.int64)
        _check(_lib.fea_batch_gauss_points(self._h, off.ctypes.data_as(_P), _stream(stream)))
        return off

    def subscale(self, out=None, status=None, stream=None):
        """Batched subgrid scale (linear elasticity, each mesh's u as the
        field): out[n_points, 3] in mesh order, status[n_meshes]."""
        n = int(self.gauss_points(stream)[-1])
        if out is None:
            out = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if status is None:
            status = torch.empty(len(self.meshes), dtype=torch.int32, device=self.device)
        if out.numel() != 3 * n or status.numel() != len(self.meshes):
            raise ValueError(f"out needs {3 * n} values and status {len(self.meshes)}")
        _dev(out, torch.float64)
        _check(_lib.fea_batch_subscale(self._h, _stream(stream), _ptr(out), _ptr(status)))
        return out, status

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _release(_lib.fea_batch_destroy, h)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tile_table_load(path, model, precision):
    import numpy as np
    tile = np.zeros(4, dtype=np.int32)
    _check(_lib.fea_tile_table_load(path.encode(), int(model), int(precision), tile.ctypes.data_as(_I32P)))
    return tile


class CostModel:
    """12 -> 64 -> 64 -> 1 ReLU perceptron predicting log(cycles) of a work item."""

    def __init__(self, seed=0, device="cuda"):
        h = _P()
        _check(_lib.fea_cost_create(int(seed), ctypes.byref(h)))
        self._h = h
        self.device = torch.device(device)

    def params(self):
        import numpy as np
        p = np.zeros(N_PARAMS, dtype=np.float32)
        _check(_lib.fea_cost_get_params(self._h, p.ctypes.data_as(_F32P)))
        return p

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(_lib.fea_cost_set_params(self._h, p.ctypes.data_as(_F32P)))

    def set_norm(self, mean, scale):
        import numpy as np
        m = np.ascontiguousarray(mean, dtype=np.float32)
        sc = np.ascontiguousarray(scale, dtype=np.float32)
        _check(_lib.fea_cost_set_norm(self._h, m.ctypes.data_as(_F32P), sc.ctypes.data_as(_F32P)))

    def fit_norm(self, feats, stream=None):
        _dev(feats, torch.float32)
        _check(_lib.fea_cost_fit_norm(self._h, _ptr(feats), feats.shape[0], _stream(stream)))

    def predict(self, feats, stream=None):
        _dev(feats, torch.float32)
        out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        _check(_lib.fea_cost_predict(self._h, _ptr(feats), feats.shape[0], _ptr(out), _stream(stream)))
        return out

    def grad(self, feats, target, stream=None):
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        _check(_lib.fea_cost_grad(self._h, _ptr(feats), _ptr(target), feats.shape[0], _ptr(g), _ptr(loss),
                                  _stream(stream)))
        return g, loss

    def train(self, feats, target, steps=500, lr=1e-3, stream=None):
        hist = torch.empty(max(1, steps), dtype=torch.float32, device=feats.device)
        _check(_lib.fea_cost_train(self._h, _ptr(feats), _ptr(target), feats.shape[0], int(steps),
                                   float(lr), _ptr(hist), _stream(stream)))
        return hist[:steps]

    @staticmethod
    def log_cycles(cycles, stream=None):
        out = torch.empty(cycles.shape[0], dtype=torch.float32, device=cycles.device)
        _check(_lib.fea_cost_log_cycles(_ptr(cycles), cycles.shape[0], _ptr(out), _stream(stream)))
        return out

    def save(self, path):
        _check(_lib.fea_cost_save(self._h, path.encode()))

    def load(self, path):
        _check(_lib.fea_cost_load(self._h, path.encode()))

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _release(_lib.fea_cost_destroy, h)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
