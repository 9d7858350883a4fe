"""The allocation-free entry point (fea_assemble_noalloc) against
fea_assemble's row-owner assembly and the oracle, through the C ABI: two
calls in a row on one GPU, the second on a smaller mesh, then the size and
option checks."""
import ctypes

import numpy as np
import pytest

import meshgen as mg
import oracle
from tests.helpers import fp64_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1805_03949_amd as fea  # noqa: E402


def _meshes():
    big = mg.hybrid_bands(8, seed=61, jitter=0.2)
    ct = np.random.default_rng(62).integers(0, 4, 4 ** 3).astype(np.uint8)
    small = mg.cube_mesh(4, ct, jitter=0.25, seed=63)
    return big, small


@pytest.mark.parametrize("precision,out_dtype", [(fea.FP64, fea.F64), (fea.MIXED, fea.F32)])
def test_noalloc_equals_rowowner_twice_second_smaller(precision, out_dtype):
    for m in _meshes():
        print(f"[noalloc] E={m.n_elems} N={m.n_nodes} precision={precision}", flush=True)
        dm = fea.DeviceMesh(m, device="cuda:0")
        g = dm.graph()
        ref = dm.assemble(g, variant=fea.ROWOWNER, precision=precision, out_dtype=out_dtype)
        got = dm.assemble(g, variant=fea.ROWOWNER, precision=precision, out_dtype=out_dtype, noalloc=True)
        torch.cuda.synchronize()
        assert int(got[2].item()) == -1
        # same kernels, same summation order: bitwise equal
        assert got[0].cpu().numpy().tobytes() == ref[0].cpu().numpy().tobytes()
        assert got[1].cpu().numpy().tobytes() == ref[1].cpu().numpy().tobytes()
        if precision == fea.FP64:
            og = oracle.mesh_graph(m)
            ov, orhs = oracle.assemble(m, og, model=oracle.ELASTIC)
            ev, er = fp64_errors(got[0].cpu().numpy(), ov, og.row_ptr, 3, got[1].cpu().numpy(), orhs)
            assert ev <= 1e-12 and er <= 1e-12, (ev, er)
        g.destroy()


def test_noalloc_null_status_and_poisson():
    m = mg.poisson_hex(6, jitter=0.2, seed=64)
    dm = fea.DeviceMesh(m, device="cuda:0")
    g = dm.graph()
    src = dm.source[:, :1].contiguous()
    ref = dm.assemble(g, model=fea.POISSON, variant=fea.ROWOWNER)
    vals = torch.empty_like(ref[0])
    rhs = torch.empty_like(ref[1])
    mat = fea.Material(fea.POISSON, fea._ptr(dm.young), None, None, None, 0)
    opt = fea.Options(fea.FP64, fea.ROWOWNER, fea.F64, 0)
    p = fea._ptr
    rc = fea._lib.fea_assemble_noalloc(g.handle, p(dm.x), p(dm.y), p(dm.z), p(dm.types), p(dm.conn_ptr),
                                       p(dm.conn), ctypes.byref(mat), p(src), ctypes.byref(opt),
                                       fea._stream(None), p(vals), p(rhs), None)
    assert rc == fea.FEA_OK, fea._lib.fea_last_error()
    torch.cuda.synchronize()
    assert vals.cpu().numpy().tobytes() == ref[0].cpu().numpy().tobytes()
    assert rhs.cpu().numpy().tobytes() == ref[1].cpu().numpy().tobytes()
    g.destroy()


def test_noalloc_rejects_large_meshes_and_other_options():
    # 36^3 cells: a row-owner FP64 workspace of about 330 MB, over the 256 MiB scratch
    m = mg.hybrid_bands(36, seed=65)
    dm = fea.DeviceMesh(m, device="cuda:0")
    g = dm.graph()
    assert (g.map_len * 9 + int(m.conn_ptr[-1]) * 3) * 8 > 256 << 20
    with pytest.raises(fea.FeaError) as ei:
        dm.assemble(g, variant=fea.ROWOWNER, noalloc=True)
    assert ei.value.code == fea.FEA_ERANGE
    for kw in ({"variant": fea.ROWSYM}, {"timing": True}):
        with pytest.raises(fea.FeaError) as ei:
            dm.assemble(g, noalloc=True, **{"variant": fea.ROWOWNER, **kw})
        assert ei.value.code == fea.FEA_EINVAL
    g.destroy()
