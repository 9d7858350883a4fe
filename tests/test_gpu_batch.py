"""GPU tests of the batched persistent assembly (work queue, tiles, graph
replay, cycle records) against the one-mesh path and the CPU oracle."""
import numpy as np
import pytest

import meshgen as mg
import oracle
from tests.helpers import fp32_bound_L, fp64_errors, row_scale, within_fp32_bound

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1805_03949_amd as fea  # noqa: E402


def small_batch_meshes(seed=40):
    rng = np.random.default_rng(seed)
    meshes = []
    for m in range(6):
        n = int(rng.integers(2, 7))
        frac = rng.dirichlet(np.ones(4))
        ct = rng.choice(4, size=n ** 3, p=frac).astype(np.uint8)
        mesh = mg.cube_mesh(n, ct, jitter=0.25, seed=seed + m)
        mesh.source[:, 0] = 0.3
        meshes.append(mesh)
    # one mesh with a neo-Hookean region
    meshes.append(mg.heterogeneous(8, seed=seed + 10, brick=2, jitter=0.1))
    meshes[-1].source[:, 0] = 0.3
    return meshes


_state = {}


def state():
    if not _state:
        meshes = small_batch_meshes()
        dms = [fea.DeviceMesh(m) for m in meshes]
        _state.update(meshes=meshes, dms=dms, graphs=[dm.graph() for dm in dms])
    return _state


def per_mesh(vals, rhs, b, m):
    return (vals[b.vals_off[m]:b.vals_off[m + 1]].cpu().numpy(),
            rhs[b.rhs_off[m]:b.rhs_off[m + 1]].cpu().numpy())


@pytest.mark.parametrize("precision", [fea.FP64, fea.MIXED])
@pytest.mark.parametrize("model", [fea.POISSON, fea.ELASTIC])
def test_batch_matches_single_mesh_path(model, precision):
    """Same element code and summation order as the one-mesh path; the two
    kernels are compiled separately, so FMA contraction may differ in the
    last bits: compared at 1e-13 of the row scale (FP64) or 1e-6 (mixed)."""
    st = state()
    use_nh = model == fea.ELASTIC
    b = fea.Batch(st["dms"], model=model, use_nh=use_nh)
    out = fea.F64 if precision == fea.FP64 else fea.F32
    vals, rhs, status = b.assemble(precision=precision, out_dtype=out)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == -1)
    for m, (dm, g) in enumerate(zip(st["dms"], st["graphs"])):
        v1, r1, s1 = dm.assemble(g, model=model, use_nh=use_nh, variant=fea.ROWOWNER,
                                 precision=precision, out_dtype=out)
        torch.cuda.synchronize()
        vb, rb = per_mesh(vals, rhs, b, m)
        B = 1 if model == fea.POISSON else 3
        ev, er = fp64_errors(vb.astype(np.float64), v1.cpu().numpy().astype(np.float64),
                             g.export()["row_ptr"].cpu().numpy(), B, rb.astype(np.float64),
                             r1.cpu().numpy().astype(np.float64))
        tol = 1e-13 if precision == fea.FP64 else 1e-6
        assert ev <= tol and er <= tol, (m, ev, er)


def test_batch_against_oracle():
    st = state()
    b = fea.Batch(st["dms"], model=fea.ELASTIC, use_nh=True)
    vals, rhs, _ = b.assemble()
    vmix, rmix, _ = b.assemble(precision=fea.MIXED, out_dtype=fea.F32)
    torch.cuda.synchronize()
    for m, mesh in enumerate(st["meshes"]):
        og = oracle.mesh_graph(mesh)
        ov, orr, tv, tr = oracle.assemble(mesh, og, with_terms=True)
        vb, rb = per_mesh(vals, rhs, b, m)
        ev, er = fp64_errors(vb, ov, og.row_ptr, 3, rb, orr)
        assert ev <= 1e-12 and er <= 1e-12, (m, ev, er)
        vm, rm = per_mesh(vmix, rmix, b, m)
        L = fp32_bound_L(mesh.types)
        assert within_fp32_bound(vm, ov, tv, L, 1e-12 * row_scale(ov, og.row_ptr, 3)) <= 1.0
        assert within_fp32_bound(rm, orr, tr, L, 1e-12 * np.abs(orr).max()) <= 1.0


def test_queue_order_and_tiles_do_not_change_results():
    st = state()
    b = fea.Batch(st["dms"], model=fea.ELASTIC, use_nh=True)
    v0, r0, _ = b.assemble()
    ref = (v0.cpu().numpy().tobytes(), r0.cpu().numpy().tobytes())
    rng = np.random.default_rng(7)
    for trial in range(3):
        b.set_order(rng.permutation(b.n_items))
        v, r, _ = b.assemble()
        assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref
    sym_epb = (25, 17, 12, 7)
    for tile in ([16, 10, 7, 4], [1, 3, 5, 7], [256, 160, 112, 64]):
        b.set_tiles(tile)
        counts = b.items[:, 3]
        fam = b.items[:, 1]
        for t in range(4):
            sel = fam == t
            if sel.any():
                # items are whole upper-triangle tiles (the last one of a
                # family may be partial) and start on tile boundaries
                assert counts[sel].max() <= -(-tile[t] // sym_epb[t]) * sym_epb[t]
                assert np.all(b.items[sel, 2] % sym_epb[t] == 0)
        v, r, _ = b.assemble()
        assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref
    with pytest.raises(fea.FeaError):
        b.set_order(np.zeros(b.n_items, dtype=np.int32))


def test_graph_replay_matches_eager():
    st = state()
    b = fea.Batch(st["dms"], model=fea.ELASTIC, use_nh=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        vals, rhs, status = b.outputs(fea.F32)
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs, status=status)
        s.synchronize()
        ref = (vals.cpu().numpy().tobytes(), rhs.cpu().numpy().tobytes())
        b.capture(vals, rhs, status, precision=fea.MIXED, out_dtype=fea.F32)
        for rep in range(4):
            vals.fill_(float("nan"))
            rhs.fill_(float("nan"))
            status.fill_(123)
            b.replay(1)
            s.synchronize()
            assert (vals.cpu().numpy().tobytes(), rhs.cpu().numpy().tobytes()) == ref, rep
            assert np.all(status.cpu().numpy() == -1)
        b.replay(3)
        s.synchronize()
        assert (vals.cpu().numpy().tobytes(), rhs.cpu().numpy().tobytes()) == ref


def test_cycle_records():
    st = state()
    b = fea.Batch(st["dms"], model=fea.ELASTIC, use_nh=True)
    b.assemble(timing=True)
    ms = b.last_ms()
    c, w, u = b.cycles()
    torch.cuda.synchronize()
    c, w, u = c.cpu().numpy(), w.cpu().numpy(), u.cpu().numpy()
    assert ms > 0
    assert np.all(c > 0)
    assert np.all((w >= 0) & (w < b.workers()))
    assert np.all(u >= 0)


def test_batch_status_per_mesh():
    meshes = small_batch_meshes(seed=50)[:3]
    bad_mesh, e = 1, 3
    m = meshes[bad_mesh]
    c = m.conn.copy()
    p = m.conn_ptr[e]
    c[p + 1], c[p + 2] = c[p + 2], c[p + 1]
    m.conn = c
    dms = [fea.DeviceMesh(x) for x in meshes]
    b = fea.Batch(dms, model=fea.ELASTIC)
    _, _, status = b.assemble()
    torch.cuda.synchronize()
    s = status.cpu().numpy()
    assert s[bad_mesh] == e and s[0] == -1 and s[2] == -1


@pytest.mark.parametrize("mesh_ids", [(0, 17, 63)])
def test_full_size_batched_workload_sampled_meshes(mesh_ids):
    """The 64-mesh batched workload at its real sizes in one persistent
    launch; three of its meshes (about 0.3M elements) are compared with the
    oracle in FP64 and mixed precision."""
    meshes = mg.batched(64)
    dms = [fea.DeviceMesh(m) for m in meshes]
    b = fea.Batch(dms, model=fea.ELASTIC)
    print(f"[case] batched64: {b.n_elems} elements, {b.n_items} items", flush=True)
    vals, rhs, status = b.assemble(precision=fea.MIXED, out_dtype=fea.F32)
    v64, r64, _ = b.assemble()
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == -1)
    for m in mesh_ids:
        og = oracle.mesh_graph(meshes[m])
        ov, orr, tv, tr = oracle.assemble(meshes[m], og, with_terms=True)
        vb, rb = per_mesh(v64, r64, b, m)
        ev, er = fp64_errors(vb, ov, og.row_ptr, 3, rb, orr)
        assert ev <= 1e-12 and er <= 1e-12, (m, ev, er)
        vm, rm = per_mesh(vals, rhs, b, m)
        L = fp32_bound_L(meshes[m].types)
        assert within_fp32_bound(vm, ov, tv, L, 1e-12 * row_scale(ov, og.row_ptr, 3)) <= 1.0


@pytest.mark.parametrize("precision", [fea.FP64, fea.MIXED])
@pytest.mark.parametrize("model", [fea.POISSON, fea.ELASTIC])
def test_batch_rowgather_equals_single_mesh_rowgather(model, precision):
    """The batched row-gather runs the one-mesh row-gather tiles of every
    mesh in one launch per class: each mesh's values equal its own
    row-gather assembly bitwise."""
    st = state()
    use_nh = model == fea.ELASTIC
    b = fea.Batch(st["dms"], model=model, use_nh=use_nh)
    out = fea.F64 if precision == fea.FP64 else fea.F32
    vals, rhs, status = b.assemble(precision=precision, out_dtype=out, variant=fea.ROWGATHER)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == -1)
    for m, (dm, g) in enumerate(zip(st["dms"], st["graphs"])):
        v1, r1, _ = dm.assemble(g, model=model, use_nh=use_nh, variant=fea.ROWGATHER,
                                precision=precision, out_dtype=out)
        torch.cuda.synchronize()
        vb, rb = per_mesh(vals, rhs, b, m)
        assert vb.tobytes() == v1.cpu().numpy().tobytes(), m
        assert rb.tobytes() == r1.cpu().numpy().tobytes(), m


def test_batch_rowgather_against_oracle_and_replay():
    st = state()
    b = fea.Batch(st["dms"], model=fea.ELASTIC, use_nh=True)
    vals, rhs, _ = b.assemble(variant=fea.ROWGATHER)
    torch.cuda.synchronize()
    for m, mesh in enumerate(st["meshes"]):
        og = oracle.mesh_graph(mesh)
        ov, orr, tv, tr = oracle.assemble(mesh, og, with_terms=True)
        vb, rb = per_mesh(vals, rhs, b, m)
        ev, er = fp64_errors(vb, ov, og.row_ptr, 3, rb, orr)
        assert ev <= 1e-12 and er <= 1e-12, (m, ev, er)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        v2, r2, st2 = b.outputs(fea.F32)
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=v2, rhs=r2, status=st2, variant=fea.ROWGATHER)
        s.synchronize()
        ref = (v2.cpu().numpy().tobytes(), r2.cpu().numpy().tobytes())
        for m, mesh in enumerate(st["meshes"]):
            og = oracle.mesh_graph(mesh)
            ov, orr, tv, tr = oracle.assemble(mesh, og, with_terms=True)
            vm, rm = per_mesh(v2, r2, b, m)
            L = fp32_bound_L(mesh.types)
            assert within_fp32_bound(vm, ov, tv, L, 1e-12 * row_scale(ov, og.row_ptr, 3)) <= 1.0
            assert within_fp32_bound(rm, orr, tr, L, 1e-12 * np.abs(orr).max()) <= 1.0
        b.capture(v2, r2, st2, precision=fea.MIXED, out_dtype=fea.F32, variant=fea.ROWGATHER)
        for rep in range(3):
            v2.fill_(float("nan"))
            r2.fill_(float("nan"))
            st2.fill_(123)
            b.replay(1)
            s.synchronize()
            assert (v2.cpu().numpy().tobytes(), r2.cpu().numpy().tobytes()) == ref, rep
            assert np.all(st2.cpu().numpy() == -1)


@pytest.mark.parametrize("precision", [fea.FP64, fea.MIXED])
@pytest.mark.parametrize("model", [fea.POISSON, fea.ELASTIC])
def test_batch_rowsym_matches_single_mesh_rowsym(model, precision):
    """The batched upper-triangle form runs the one-mesh tiles (items start
    on tile boundaries) with the same summation order; the persistent and
    one-mesh kernels are compiled separately, so FMA contraction may differ
    in the last bits: compared at 1e-13 of the row scale (FP64) or 1e-6
    (mixed)."""
    st = state()
    use_nh = model == fea.ELASTIC
    b = fea.Batch(st["dms"], model=model, use_nh=use_nh)
    out = fea.F64 if precision == fea.FP64 else fea.F32
    vals, rhs, status = b.assemble(precision=precision, out_dtype=out, variant=fea.ROWSYM)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == -1)
    B = 1 if model == fea.POISSON else 3
    for m, (dm, g) in enumerate(zip(st["dms"], st["graphs"])):
        v1, r1, _ = dm.assemble(g, model=model, use_nh=use_nh, variant=fea.ROWSYM,
                                precision=precision, out_dtype=out)
        torch.cuda.synchronize()
        vb, rb = per_mesh(vals, rhs, b, m)
        ev, er = fp64_errors(vb.astype(np.float64), v1.cpu().numpy().astype(np.float64),
                             g.export()["row_ptr"].cpu().numpy(), B, rb.astype(np.float64),
                             r1.cpu().numpy().astype(np.float64))
        tol = 1e-13 if precision == fea.FP64 else 1e-6
        assert ev <= tol and er <= tol, (m, ev, er)


def test_batch_rowsym_against_oracle_order_tiles_and_replay():
    st = state()
    b = fea.Batch(st["dms"], model=fea.ELASTIC, use_nh=True)
    vals, rhs, _ = b.assemble(variant=fea.ROWSYM)
    torch.cuda.synchronize()
    ref64 = (vals.cpu().numpy().tobytes(), rhs.cpu().numpy().tobytes())
    for m, mesh in enumerate(st["meshes"]):
        og = oracle.mesh_graph(mesh)
        ov, orr, tv, tr = oracle.assemble(mesh, og, with_terms=True)
        vb, rb = per_mesh(vals, rhs, b, m)
        ev, er = fp64_errors(vb, ov, og.row_ptr, 3, rb, orr)
        assert ev <= 1e-12 and er <= 1e-12, (m, ev, er)
    # queue order, static partitions and item sizes do not change the result
    rng = np.random.default_rng(11)
    b.set_order(rng.permutation(b.n_items))
    v, r, _ = b.assemble(variant=fea.ROWSYM)
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref64
    b.set_tiles([50, 17, 36, 28])
    v, r, _ = b.assemble(variant=fea.ROWSYM)
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref64
    b.order(fea.GP_WEIGHT)
    b.partition(fea.GP_WEIGHT)
    v, r, _ = b.assemble(variant=fea.ROWSYM)
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref64
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        v2, r2, st2 = b.outputs(fea.F32)
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=v2, rhs=r2, status=st2, variant=fea.ROWSYM)
        s.synchronize()
        ref = (v2.cpu().numpy().tobytes(), r2.cpu().numpy().tobytes())
        for m, mesh in enumerate(st["meshes"]):
            og = oracle.mesh_graph(mesh)
            ov, orr, tv, tr = oracle.assemble(mesh, og, with_terms=True)
            vm, rm = per_mesh(v2, r2, b, m)
            L = fp32_bound_L(mesh.types)
            assert within_fp32_bound(vm, ov, tv, L, 1e-12 * row_scale(ov, og.row_ptr, 3)) <= 1.0
            assert within_fp32_bound(rm, orr, tr, L, 1e-12 * np.abs(orr).max()) <= 1.0
        b.capture(v2, r2, st2, precision=fea.MIXED, out_dtype=fea.F32, variant=fea.ROWSYM)
        for rep in range(3):
            v2.fill_(float("nan"))
            r2.fill_(float("nan"))
            st2.fill_(123)
            b.replay(1)
            s.synchronize()
            assert (v2.cpu().numpy().tobytes(), r2.cpu().numpy().tobytes()) == ref, rep
            assert np.all(st2.cpu().numpy() == -1)


def test_batch_rowgather_status_per_mesh():
    meshes = [mg.cube_mesh(3, np.full(27, mg.TET4, dtype=np.uint8)) for _ in range(3)]
    e = 29
    c = meshes[1].conn.copy()
    c[meshes[1].conn_ptr[e] + 1], c[meshes[1].conn_ptr[e] + 2] = c[meshes[1].conn_ptr[e] + 2], c[meshes[1].conn_ptr[e] + 1]
    meshes[1].conn = c
    b = fea.Batch([fea.DeviceMesh(m) for m in meshes], model=fea.ELASTIC)
    _, _, status = b.assemble(variant=fea.ROWGATHER)
    torch.cuda.synchronize()
    assert list(status.cpu().numpy()) == [-1, e, -1]
    with pytest.raises(fea.FeaError):
        b.assemble(variant=fea.COLOUR)
