"""Benchmark: finite-element assembly on one MI355X.

A step is one fea_assemble call over the whole workload (element quadrature
for every element plus the race-free scatter into the 3x3 block matrix and
the right-hand side), with the mesh, graph and outputs resident in HBM.
The graph build is timed once and reported separately.

Workload (default, the largest single-GPU configuration): linear elasticity
on a 256^3-cell hybrid mesh, z-bands of 102 / 77 / 51 / 26 cell layers
(hex8 / tet4 / pen6 / pyr5), E = 1, nu per element U[0.2, 0.35], body force
(0, 0, -1); 53,870,592 elements, 18,678,529 nodes, FP64 upper-triangle
form. Companion workloads (extra keys): the 96^3-cell hybrid mesh with every
scatter form, the subgrid scale, the batched and heterogeneous-cost
workloads and the persistent form of the large mesh.

Prints one JSON line. Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload hybrid256|hybrid96]
                  [--variant rowsym] [--precision fp64|mixed] [--no-cpu] [--no-variants]
                  [--no-small] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector
METRIC = "elements assembled/s + scatter HBM GB/s (% peak); learned+mixed vs plain FP64"


def reduce_bytes(g, B, s_c, s_v):
    """Algorithmic bytes of one launch of the row-owner block-value kernel:
    every slot contribution read once (the workspace is sorted by
    destination, so no map is read), each block's segment bound read once
    (int64), every block value written once."""
    return g.map_len * B * B * s_c + (g.nnz + 1) * 8 + g.nnz * B * B * s_v


def sym_tile_blocks(mesh, np):
    """(entries, tile-blocks) of the upper-triangle layout, from its
    definition: per family the type-sorted elements in tiles of
    256 // (n(n+1)/2); per element one entry per local pair a <= b (two where
    its nodes coincide); tile-blocks = distinct (tile, upper block) pairs."""
    order = np.argsort(mesh.types, kind="stable")
    ent, keys, tile0, N = 0, [], 0, int(mesh.n_nodes)
    for t in range(4):
        idx = order[mesh.types[order] == t]
        if idx.size == 0:
            continue
        n = NODES[t]
        epb = 256 // (n * (n + 1) // 2)
        c = mesh.conn[mesh.conn_ptr[idx][:, None] + np.arange(n)[None, :]].astype(np.int64)
        a, b = np.triu_indices(n)
        na, nb = c[:, a], c[:, b]
        tile = tile0 + (np.arange(idx.size, dtype=np.int64) // epb)[:, None]
        ent += na.size + int(((na == nb) & (a != b)[None, :]).sum())
        keys.append(((tile * N + np.minimum(na, nb)) * N + np.maximum(na, nb)).ravel())
        tile0 += (idx.size + epb - 1) // epb
    return ent, int(np.unique(np.concatenate(keys)).size) if keys else 0


def sym_reduce_bytes(ulen, nup, nnz, B, s_c, s_v):
    """Algorithmic bytes of one launch of the upper-triangle block-value
    kernel: every tile sum (ulen tile-blocks) read once, per upper block its
    segment bound (int64), its block index and its lower partner (int32),
    every block value (upper and transposed lower) written once, and with
    3x3 blocks the right-hand side of every row that has a diagonal block
    (2 nup - nnz rows), which those blocks' tile sums carry."""
    rows = 2 * nup - nnz if B == 3 else 0
    return ulen * B * B * s_c + (nup + 1) * 8 + nup * 8 + nnz * B * B * s_v + rows * B * s_v


def element_bytes(g, B, s_c, s_v, conn_len, n_nodes, n_elems, variant, sym=None):
    """Algorithmic bytes of the element phase: node coordinates once, the
    connectivity and per-element data once, and its outputs once (the slot
    contributions for row-owner; for the upper-triangle form the tile sums
    plus its tile entries (2 bytes), tile-block ends and slots (6 bytes) and
    tile ranges (16 bytes), and with 1x1 blocks the per-element
    right-hand-side contributions (3x3 blocks carry them in the tile sums);
    for row-gather the final values, plus the pair-ordered node lists, lane
    bytes and segment bounds it reads)."""
    inputs = n_nodes * 24 + conn_len * 4 + n_elems * (8 + 4 + 8 + 16 + 8 * B)
    if variant == "rowowner":
        return inputs + g.map_len * B * B * s_c + conn_len * B * s_c
    if variant == "rowsym":
        return (inputs + sym["tile_blocks"] * (B * B * s_c + 6) + sym["entries"] * 2 + sym["tiles"] * 16
                + (conn_len * B * s_c if B == 1 else 0))
    if variant == "rowgather":
        maps = g.map_len * (4 + 1) + conn_len * 5 + (g.nnz + 1) * 8 + (n_nodes + 1) * 8
        return inputs + maps + g.nnz * B * B * s_v + n_nodes * B * s_v
    return inputs + g.map_len * 4 + g.nnz * B * B * 8 * 2 + n_nodes * B * 8 * 2


GATHER_FAMILIES = ("tet4", "pyr5", "pen6", "hex8", "interface")
NODES = (4, 5, 6, 8)
GAUSS = (1, 8, 6, 8)


def gather_pair_flops(t, B=3):
    """FP64 (or mixed) floating-point operations the row-gather kernel
    executes for one (row, element) pair of family t, recomputation
    included: per Gauss point the Jacobian (18 n), its determinant (14) and
    inverse (37), the row node's weighted gradient (19) and the pair's
    right-hand-side term (7); per element node b and Gauss point the
    gradient of b (15) and the 3x3 outer-product update (18), then the
    block from S (33); per element node one 9-value addition into the
    block sums."""
    n, q = NODES[t], GAUSS[t]
    return q * (18 * n + 70 + 7) + n * (q * 33 + 33) + n * B * B


# Algorithmic flops per element of the element matrix, exploiting the
# sparsity of B (the per-element figures of the measurement plan): tet4,
# pyr5, pen6, hex8.
ELEMENT_FLOPS = (1.5e3, 16.9e3, 17.1e3, 37.2e3)


def gather_class_flops(mesh, np):
    """Per row-tile class kernel (pure tet4, pyr5, pen6, hex8 rows, interface
    rows) for one assembly: (algorithmic flops, executed flops). A (row,
    element) pair computes 1/n of its element's matrix, so a kernel's
    algorithmic flops are its pairs' share of the per-element figure;
    executed flops count the kernel's own operations, the geometry it
    recomputes per pair included."""
    et = mesh.types[np.repeat(np.arange(mesh.n_elems), np.diff(mesh.conn_ptr))]
    mask = np.zeros(mesh.n_nodes, dtype=np.int64)
    np.bitwise_or.at(mask, mesh.conn, (1 << et.astype(np.int64)))
    single = (mask & (mask - 1)) == 0
    cls = np.where(single, np.log2(np.maximum(mask, 1)).astype(np.int64), 4)
    pair_cls = cls[mesh.conn]
    alg = np.array([ELEMENT_FLOPS[t] / NODES[t] for t in range(4)], dtype=np.float64)[et]
    exe = np.array([gather_pair_flops(t) for t in range(4)], dtype=np.float64)[et]
    return ([float(alg[pair_cls == c].sum()) for c in range(5)],
            [float(exe[pair_cls == c].sum()) for c in range(5)])


def traffic_from_profile(kernel_key, source):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    names this kernel and matches the current source file of the kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    import hashlib
    src = open(os.path.join(ROOT, "paper_1805_03949_amd", "csrc", source), "rb").read()
    digest = hashlib.sha256(src).hexdigest()[:16]
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get(f"source_sha256_16[{source}]") != digest:
        return None
    v = rec.get(f"{kernel_key}_bytes")
    return float(v) if v else None


SUB_NN = (4, 5, 6, 8)   # nodes per family (tet4, pyr5, pen6, hex8)
SUB_NQ = (1, 8, 6, 8)   # Gauss points per family


def subscale_flops_per_point(t, B):
    """Algorithmic flops of the subgrid scale at one Gauss point of family t
    (FMA = 2). tet4: per node J (9 FMA). The others, per field (the three
    coordinates and the B field components): the lane's polynomial
    coefficient of it from the node values (hex8 and the pyramid: eight
    signed additions and a scaling by 1/8; pen6: at most five operations)
    and its first and mixed second reference derivatives at the point
    (hex8, pyramid: 9 FMA; pen6: 4 FMA). Then J^-1 with its determinant and
    w detJ (43), the second-derivative transform and the operator (282 for
    elasticity, 56 for Poisson; tet4: none), the volume sum (1) and tau r
    (B)."""
    if t == 0:
        return SUB_NN[0] * 18 + 43 + 1 + B
    per_field = 27 if t in (1, 3) else 13
    post = 282 if B == 3 else 56
    return (3 + B) * per_field + 43 + post + 1 + B


def subscale_work(mesh, B, np):
    """(algorithmic bytes, algorithmic flops) of one subgrid-scale call:
    per element its id (4 B), node ids (4 B each), material (young and nu,
    16 B, elasticity only), source (8B), Gauss-point offset (8) and outputs
    (8B per Gauss point); per node its coordinates and field (24 + 8B),
    read once."""
    cnt = np.bincount(mesh.types, minlength=4)
    byts, flops = mesh.n_nodes * (24 + 8 * B), 0
    for t in range(4):
        per_elem = 4 + 4 * SUB_NN[t] + (16 if B == 3 else 0) + 8 * B + 8 + 8 * B * SUB_NQ[t]
        byts += int(cnt[t]) * per_elem
        flops += int(cnt[t]) * SUB_NQ[t] * subscale_flops_per_point(t, B)
    return byts, flops


def subscale_workload(fea, mg, torch, np, mesh, dm, g, reps=20, name="hybrid96"):
    """The element-wise subgrid scale of linear elasticity on the headline
    mesh at a smooth displacement field: four family launches, nothing
    assembled."""
    u = torch.from_numpy(mg.smooth_field(mesh, 3, seed=11)).to(dm.x.device)
    out, st = dm.subscale(g, u)
    for _ in range(3):
        dm.subscale(g, u, out=out, status=st)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dm.subscale(g, u, out=out, status=st)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    byts, flops = subscale_work(mesh, 3, np)
    gbs = byts / (ms * 1e-3) / 1e9
    tfs = flops / (ms * 1e-3) / 1e12
    n_pts = int(out.shape[0])
    alu = flops / (PEAK_FP64_TFLOPS * 1e12) >= byts / (PEAK_HBM_GBS * 1e9)
    roof = ({"bound": "alu", "achieved": round(tfs, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
             "frac": round(tfs / PEAK_FP64_TFLOPS, 4)} if alu else
            {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": round(gbs / PEAK_HBM_GBS, 4)})
    roof.update({"kernel": "k_subscale<family, elasticity> (4 launches)",
                 "traffic": traffic_from_profile("k_subscale,elastic", "subscale.hip"),
                 "algorithmic_bytes": int(byts), "algorithmic_flops": int(flops),
                 "hbm_GBps": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                 "fp64_TFLOPs": round(tfs, 2), "fp64_frac": round(tfs / PEAK_FP64_TFLOPS, 4)})
    res = {"workload": f"{name} elasticity, smooth displacement field, FP64", "ms": round(ms, 4),
           "elements_per_s": round(mesh.n_elems / (ms * 1e-3), 1),
           "gauss_points_per_s": round(n_pts / (ms * 1e-3), 1), "gauss_points": n_pts,
           "roofline": roof, "status_ok": int(st.item()) == -1}
    return res, u


def _median_ms(fn, reps):
    import numpy as np
    vals = [fn() for _ in range(reps)]
    return float(np.median(vals))


def batched_workload(fea, mg, torch):
    """64 independent meshes (8^3..48^3 cells, random family mix, jitter
    0.25 h) in one persistent launch of the upper-triangle form, mixed
    precision, tiles autotuned, replayed 100 times from a HIP graph; then
    the same batch in the row-owner and row-gather forms, also replayed
    from graphs."""
    import tempfile
    meshes = mg.batched(64)
    for k, m in enumerate(meshes):
        # displacement field of the subgrid-scale timing (the linear
        # assembly does not read it)
        m.u = mg.smooth_field(m, 3, seed=100 + k)
    dms = [fea.DeviceMesh(m) for m in meshes]
    b = fea.Batch(dms, model=fea.ELASTIC)
    n_items_default = b.n_items
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        vals, rhs, status = b.outputs(fea.F32)
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs, status=status, timing=True,
                   variant=fea.ROWSYM)
        side.synchronize()
        default_ms = _median_ms(lambda: (b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs,
                                                    status=status, timing=True, variant=fea.ROWSYM),
                                         b.last_ms())[1], 5)
        # the tuner's search starts from the smallest items (one
        # upper-triangle tile each), timed first, so that what it finds is
        # measured against where it started as well as against the defaults
        start = [25, 17, 12, 7]
        b.set_tiles(start)
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs, status=status, timing=True,
                   variant=fea.ROWSYM)
        start_ms = _median_ms(lambda: (b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs,
                                                  status=status, timing=True, variant=fea.ROWSYM),
                                       b.last_ms())[1], 5)
        with tempfile.TemporaryDirectory() as d:
            tile = b.autotune(precision=fea.MIXED, out_dtype=fea.F32, reps=3, table_path=f"{d}/tiles.txt",
                              variant=fea.ROWSYM)
        tuned_ms = _median_ms(lambda: (b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs,
                                                  status=status, timing=True, variant=fea.ROWSYM),
                                       b.last_ms())[1], 5)
        b.capture(vals, rhs, status, precision=fea.MIXED, out_dtype=fea.F32, variant=fea.ROWSYM)
        b.replay(3)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(side)
        b.replay(100)
        e1.record(side)
        side.synchronize()
        ms = e0.elapsed_time(e1) / 100
        ok = bool((status.cpu() == -1).all())
        # the same batch in the row-owner form (same items) and the
        # row-gather form (one launch per tile class)
        gather = {}
        b.capture(vals, rhs, status, precision=fea.MIXED, out_dtype=fea.F32, variant=fea.ROWOWNER)
        b.replay(3)
        e0.record(side)
        b.replay(100)
        e1.record(side)
        side.synchronize()
        oms = e0.elapsed_time(e1) / 100
        gather["rowowner_mixed"] = {"ms_per_replay": round(oms, 4),
                                    "elements_per_s": round(b.n_elems / (oms * 1e-3), 1),
                                    "status_ok": bool((status.cpu() == -1).all())}
        for pname, p, o in (("fp64", fea.FP64, fea.F64), ("mixed", fea.MIXED, fea.F32)):
            gv, gr, gs = b.outputs(o)
            b.assemble(precision=p, out_dtype=o, vals=gv, rhs=gr, status=gs, variant=fea.ROWGATHER)
            b.capture(gv, gr, gs, precision=p, out_dtype=o, variant=fea.ROWGATHER)
            b.replay(3)
            e0.record(side)
            b.replay(100)
            e1.record(side)
            side.synchronize()
            gms = e0.elapsed_time(e1) / 100
            gather[f"rowgather_{pname}"] = {"ms_per_replay": round(gms, 4),
                                            "elements_per_s": round(b.n_elems / (gms * 1e-3), 1),
                                            "status_ok": bool((gs.cpu() == -1).all())}
            del gv, gr, gs
        # the subgrid scale of every mesh (nothing scattered): the batch's
        # per-family queues feeding persistent workgroups, against one
        # call (four family launches) per mesh
        del vals, rhs
        sub_out, sub_st = b.subscale(stream=side)
        for _ in range(2):
            b.subscale(out=sub_out, status=sub_st, stream=side)
        e0.record(side)
        for _ in range(10):
            b.subscale(out=sub_out, status=sub_st, stream=side)
        e1.record(side)
        side.synchronize()
        q_ms = e0.elapsed_time(e1) / 10
        off = b.gauss_points(stream=side)
        graphs = [dm.graph(stream=side) for dm in dms]
        one = [dm.subscale(g, dm.u, stream=side) for dm, g in zip(dms, graphs)]
        for _ in range(2):
            for (o, st), dm, g in zip(one, dms, graphs):
                dm.subscale(g, dm.u, out=o, status=st, stream=side)
        e0.record(side)
        for _ in range(10):
            for (o, st), dm, g in zip(one, dms, graphs):
                dm.subscale(g, dm.u, out=o, status=st, stream=side)
        e1.record(side)
        side.synchronize()
        m_ms = e0.elapsed_time(e1) / 10
        same = all(torch.equal(sub_out[int(off[k]):int(off[k + 1])], o) for k, (o, _) in enumerate(one))
        gather["subscale"] = {"gauss_points": int(off[-1]), "queue_ms": round(q_ms, 4),
                              "one_call_per_mesh_ms": round(m_ms, 4),
                              "speedup_queue_vs_per_mesh": round(m_ms / q_ms, 3),
                              "gauss_points_per_s": round(int(off[-1]) / (q_ms * 1e-3), 1),
                              "bitwise_equal": bool(same),
                              "status_ok": bool((sub_st.cpu() == -1).all())
                              and all(int(st.item()) == -1 for _, st in one)}
        del one, graphs, sub_out
    return {"workload": "batched64-elasticity (64 meshes, 8^3..48^3 cells, jitter 0.25h)",
            "elements": int(b.n_elems), "items": int(b.n_items), "items_default_tiles": int(n_items_default),
            "precision": "mixed", "variant": "rowsym", "tiles": [int(t) for t in tile],
            "persistent_kernel_ms_default_tiles": round(default_ms, 4),
            "autotune_start_tiles": start, "persistent_kernel_ms_start_tiles": round(start_ms, 4),
            "persistent_kernel_ms_tuned_tiles": round(tuned_ms, 4),
            "speedup_tuned_vs_start": round(start_ms / tuned_ms, 4),
            "ms_per_replay": round(ms, 4), "elements_per_s": round(b.n_elems / (ms * 1e-3), 1),
            "replays": 100, "workers": b.workers(), "status_ok": ok, **gather}


def copy_bandwidth(torch):
    """Device-to-device copy of 2 GiB (read + write), GB/s: the practical
    streaming ceiling next to the 8 TB/s nominal peak."""
    a = torch.empty(1 << 28, dtype=torch.float64, device="cuda:0")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    return round(2 * a.numel() * 8 / (ms * 1e-3) / 1e9, 1)


def large_workload(fea, mg, torch, np, cells=256, mesh=None):
    """53.9M-element hybrid mesh (40/30/20/10 hex/tet/pen/pyr layers) through
    the persistent path in the upper-triangle form (plain FP64 against mixed
    precision with the learned schedule; row-owner FP64 for reference), then
    one-mesh assemblies in the row-gather form and the subgrid scale."""
    if mesh is None:
        mesh = mg.hybrid_split(cells, seed=5)
    dm = fea.DeviceMesh(mesh)
    b = fea.Batch([dm], model=fea.ELASTIC)
    out = {"workload": f"hybrid{cells}-elasticity (40/30/20/10 hex/tet/pen/pyr layers)",
           "elements": int(mesh.n_elems), "nodes": int(mesh.n_nodes), "nnz_blocks": int(b.vals_len // 9),
           "items": int(b.n_items)}

    def run(precision, reps=5, variant=fea.ROWSYM):
        outd = fea.F64 if precision == fea.FP64 else fea.F32
        vals, rhs, st = b.outputs(outd)
        b.assemble(precision=precision, out_dtype=outd, vals=vals, rhs=rhs, status=st, variant=variant)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tot = []
        for _ in range(reps):
            e0.record()
            b.assemble(precision=precision, out_dtype=outd, vals=vals, rhs=rhs, status=st, variant=variant)
            e1.record()
            torch.cuda.synchronize()
            tot.append(e0.elapsed_time(e1))
        ok = bool((st.cpu() == -1).all())
        del vals, rhs
        return {"total_ms": round(float(np.median(tot)), 3),
                "elements_per_s": round(mesh.n_elems / (float(np.median(tot)) * 1e-3), 1), "status_ok": ok}

    out["fp64_type_sorted_rowowner"] = run(fea.FP64, variant=fea.ROWOWNER)
    out["fp64_type_sorted"] = run(fea.FP64)
    out["mixed_type_sorted"] = run(fea.MIXED)
    c, _, _ = b.cycles()
    target = fea.CostModel.log_cycles(c)
    feats = b.features(fp64_geometry=False)
    cm = fea.CostModel(seed=7)
    cm.fit_norm(feats)
    cm.train(feats, target, steps=600, lr=3e-3)
    pred = cm.predict(feats)
    b.partition(fea.LEARNED, pred)
    out["mixed_static_learned"] = run(fea.MIXED)
    b.order(fea.LEARNED, pred)
    out["mixed_queue_learned_lpt"] = run(fea.MIXED)
    # the learned schedule: predicted cost classes, type-sorted within a class
    b.order(fea.LEARNED_CLASSES, pred)
    out["mixed_queue_learned_classes"] = run(fea.MIXED)
    lc = out["mixed_queue_learned_classes"]["total_ms"]
    out["speedup_learned_mixed_vs_fp64"] = round(out["fp64_type_sorted"]["total_ms"] / lc, 4)
    out["speedup_learned_vs_type_sorted_queue_mixed"] = round(out["mixed_type_sorted"]["total_ms"] / lc, 4)
    # the same ratio with the exact longest-predicted-first queue
    out["speedup_learned_lpt_mixed_vs_fp64"] = round(
        out["fp64_type_sorted"]["total_ms"] / out["mixed_queue_learned_lpt"]["total_ms"], 4)
    b.destroy()
    torch.cuda.empty_cache()

    # the same mesh through the fused row-gather form (no workspace) and the
    # upper-triangle row-owner form
    g = dm.graph()
    for vname in ("rowgather",):
        for pname, p, o in (("fp64", fea.FP64, fea.F64), ("mixed", fea.MIXED, fea.F32)):
            var = fea.VARIANTS[vname]
            vals, rhs, st = dm.assemble(g, variant=var, precision=p, out_dtype=o)
            tot = []
            for _ in range(5):
                dm.assemble(g, variant=var, precision=p, out_dtype=o, vals=vals, rhs=rhs, status=st, timing=True)
                tot.append(g.last_timing()[2])
            ok = int(st.item()) == -1
            out[f"{vname}_{pname}"] = {"total_ms": round(float(np.median(tot)), 3),
                                       "elements_per_s": round(mesh.n_elems / (float(np.median(tot)) * 1e-3), 1),
                                       "status_ok": ok}
            del vals, rhs, st
    # the element-wise subgrid scale of the whole mesh at a smooth field
    u = torch.from_numpy(mg.smooth_field(mesh, 3, seed=12)).to(dm.x.device)
    so, ss = dm.subscale(g, u)
    dm.subscale(g, u, out=so, status=ss)
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dm.subscale(g, u, out=so, status=ss)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    sms = float(np.median(ts))
    out["subscale_fp64"] = {"ms": round(sms, 3), "gauss_points": int(so.shape[0]),
                            "gauss_points_per_s": round(int(so.shape[0]) / (sms * 1e-3), 1),
                            "elements_per_s": round(mesh.n_elems / (sms * 1e-3), 1),
                            "status_ok": int(ss.item()) == -1}
    del so, ss, u
    g.destroy()
    return out


def _batch_runner(fea, torch, np, b):
    def run(precision, reps=9, variant=fea.ROWSYM):
        outd = fea.F64 if precision == fea.FP64 else fea.F32
        vals, rhs, st = b.outputs(outd)
        b.assemble(precision=precision, out_dtype=outd, vals=vals, rhs=rhs, status=st, variant=variant)
        kern, tot = [], []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(reps):
            e0.record()
            b.assemble(precision=precision, out_dtype=outd, vals=vals, rhs=rhs, status=st, timing=True,
                       variant=variant)
            e1.record()
            torch.cuda.synchronize()
            kern.append(b.last_ms())
            tot.append(e0.elapsed_time(e1))
        c, w, _ = b.cycles()
        c = c.cpu().numpy().astype(np.float64)
        w = w.cpu().numpy()
        # load balance of the four per-family launches together: busy time
        # over the time their workers were held (each launch lasts as long
        # as its busiest worker)
        fam = b.items[:, 1]
        busy_sum, held = 0.0, 0.0
        for t in range(4):
            sel = fam == t
            if not sel.any():
                continue
            busy = np.bincount(w[sel], weights=c[sel])
            busy = busy[busy > 0]
            busy_sum += busy.sum()
            held += busy.size * busy.max()
        return {"kernel_ms": round(float(np.median(kern)), 4), "total_ms": round(float(np.median(tot)), 4),
                "load_balance": round(float(busy_sum / held), 4)}, vals, st
    return run


def _measured_log_cycles(fea, torch, b, runs=5):
    """Per-item log-cycles averaged over `runs` type-sorted mixed runs (one
    run is noisy: concurrent workgroups share caches and memory channels)."""
    vals, rhs, st = b.outputs(fea.F32)
    logs = []
    for _ in range(runs):
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs, status=st, variant=fea.ROWSYM)
        c, _, _ = b.cycles()
        logs.append(fea.CostModel.log_cycles(c))
    return torch.stack(logs).mean(dim=0).contiguous()


def static_split_cuts(np, wts, parts):
    """Cut points of a static split of items (in their order) into `parts`
    contiguous parts of about equal total weight: part k ends at the first
    item whose weight midpoint lies past (k+1)/parts of the total, so every
    part is within one item's weight of an even share."""
    wts = np.asarray(wts, dtype=np.float64)
    cs = np.cumsum(wts)
    return np.searchsorted(cs - 0.5 * wts, cs[-1] * np.arange(1, parts) / parts)


def heterogeneous_workload(fea, mg, torch, np, cells=128):
    """Hybrid split meshes (40/30/20/10 hex/tet/pen/pyr layers) where 30% of
    8^3-cell bricks use the neo-Hookean tangent. The cost model is trained
    on the cycles recorded on one mesh (seed 4) and judged on another
    (seed 6: other bricks, other displacement field) that it never saw:
    prediction quality against measured cycles, the load balance of a
    static 8-way split of the whole mesh (the sharding over 8 GPUs, judged
    by measured cycles), and the queue orders and static partitions of the
    persistent kernels, against the type-sorted order and the Gauss-point
    weights of the paper's Section 4.1."""
    mesh = mg.heterogeneous(cells, seed=4)
    dm = fea.DeviceMesh(mesh)
    b = fea.Batch([dm], model=fea.ELASTIC, use_nh=True)
    run = _batch_runner(fea, torch, np, b)
    out = {"workload": f"hetero{cells}-elasticity (30% neo-Hookean bricks, 40/30/20/10 hex/tet/pen/pyr)",
           "train_mesh_seed": 4, "heldout_mesh_seed": 6,
           "elements": int(mesh.n_elems), "items": int(b.n_items), "workers": 0,
           "variant": "rowsym (persistent kernel)"}
    out["fp64_type_sorted_rowowner"], _, _ = run(fea.FP64, variant=fea.ROWOWNER)
    fp64_ts, v64, st64 = run(fea.FP64)
    out["fp64_type_sorted"] = fp64_ts
    mix_ts, vmx, stm = run(fea.MIXED)
    out["mixed_type_sorted"] = mix_ts
    target = _measured_log_cycles(fea, torch, b)
    feats = b.features(fp64_geometry=False)
    cm = fea.CostModel(seed=7)
    cm.fit_norm(feats)
    t0 = time.perf_counter()
    hist = cm.train(feats, target, steps=600, lr=3e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    pred = cm.predict(feats)

    def r2(x, y):
        x = x - x.mean()
        y = y - y.mean()
        return float((x @ y) ** 2 / ((x @ x) * (y @ y)))

    def split_lb(cyc, wts, parts=8):
        # cut the type-sorted items by weight, then rate the split by the
        # measured cycles of its parts
        cut = static_split_cuts(np, wts, parts)
        sums = np.array([c.sum() for c in np.split(cyc, cut)])
        return round(float(sums.mean() / sums.max()), 4)

    def executed_split(msh, bb, wts, parts=8, reps=5):
        # the cut of split_lb, each part then assembled as a mesh of its own
        # (upper-triangle form, FP64, neo-Hookean tangent where flagged) and
        # timed alone on the GPU: what each of 8 GPUs would run, so the
        # makespan is the slowest part's time
        perm = np.argsort(msh.types, kind="stable")
        seg = np.concatenate([[0], np.cumsum(np.bincount(msh.types, minlength=4))])
        cut = static_split_cuts(np, wts, parts)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms, ne = [], []
        for sel in np.split(np.arange(bb.items.shape[0]), cut):
            el = [perm[seg[f] + z: seg[f] + z + c] for _, f, z, c in bb.items[sel]]
            el = np.concatenate(el) if el else np.zeros(0, np.int64)
            ne.append(int(el.size))
            if el.size == 0:
                ms.append(0.0)
                continue
            sdm = fea.DeviceMesh(mg.submesh(msh, el))
            sg = sdm.graph()
            kw = dict(use_nh=True, variant=fea.ROWSYM, precision=fea.FP64, out_dtype=fea.F64)
            v, r, st = sdm.assemble(sg, **kw)
            ts = []
            for _ in range(reps + 2):
                e0.record()
                sdm.assemble(sg, vals=v, rhs=r, status=st, **kw)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            assert int(st.item()) == -1
            ms.append(float(np.median(ts[2:])))
            del v, r, st
            sg.destroy()
            del sdm
        torch.cuda.empty_cache()
        ms = np.array(ms)
        return {"part_elements": ne, "part_ms": [round(float(x), 3) for x in ms],
                "makespan_ms": round(float(ms.max()), 3), "balance": round(float(ms.mean() / ms.max()), 4)}

    def judge(bb, tgt, prd):
        t = tgt.cpu().numpy().astype(np.float64)
        p = prd.cpu().numpy().astype(np.float64)
        gp = np.log(bb.items[:, 3] * np.array([1, 8, 6, 8])[bb.items[:, 1]])
        cyc = np.exp(t)
        return {"r2_learned_vs_measured": round(r2(p, t), 4),
                "r2_gauss_point_weight_vs_measured": round(r2(gp, t), 4),
                "static_split_8_load_balance": {"elements": split_lb(cyc, bb.items[:, 3].astype(np.float64)),
                                                "gauss_points": split_lb(cyc, np.exp(gp)),
                                                "learned": split_lb(cyc, np.exp(p)),
                                                "measured_cycles": split_lb(cyc, cyc)}}

    out["cost_model"] = {"train_steps": 600, "train_s": round(train_s, 3),
                         "loss_first": round(float(hist[0].item()), 5), "loss_last": round(float(hist[-1].item()), 5),
                         "in_sample": judge(b, target, pred)}
    del vmx, stm
    # the held-out mesh: the trained model predicts, measured cycles judge
    hmesh = mg.heterogeneous(cells, seed=6)
    hdm = fea.DeviceMesh(hmesh)
    hb = fea.Batch([hdm], model=fea.ELASTIC, use_nh=True)
    hrun = _batch_runner(fea, torch, np, hb)
    hfeats = hb.features(fp64_geometry=False)
    hpred = cm.predict(hfeats)
    htarget = _measured_log_cycles(fea, torch, hb)
    out["cost_model"]["held_out"] = judge(hb, htarget, hpred)
    # the 8-part static split executed: each part assembled alone
    w_el = hb.items[:, 3].astype(np.float64)
    ex = {"form": "each part a mesh of its own, upper-triangle FP64, timed alone (median of 5)"}
    for key, w in (("elements", w_el), ("gauss_points", w_el * np.array([1, 8, 6, 8])[hb.items[:, 1]]),
                   ("learned", np.exp(hpred.cpu().numpy().astype(np.float64))),
                   ("measured_cycles", np.exp(htarget.cpu().numpy().astype(np.float64)))):
        ex[key] = executed_split(hmesh, hb, w)
    for key in ("elements", "gauss_points"):
        ex[f"makespan_gain_learned_vs_{key}"] = round(ex[key]["makespan_ms"] / ex["learned"]["makespan_ms"], 4)
    out["cost_model"]["held_out"]["executed_split_8"] = ex
    ho = {"elements": int(hmesh.n_elems), "items": int(hb.n_items)}
    ho["fp64_type_sorted"], hv64, hst64 = hrun(fea.FP64)
    ho["mixed_type_sorted"], _, _ = hrun(fea.MIXED)
    hb.order(fea.GP_WEIGHT)
    ho["mixed_queue_gp_weight_lpt"], _, _ = hrun(fea.MIXED)
    hb.order(fea.LEARNED, hpred)
    ho["mixed_queue_learned_lpt"], _, _ = hrun(fea.MIXED)
    hb.order(fea.LEARNED_CLASSES, hpred)
    ho["mixed_queue_learned_classes"], _, _ = hrun(fea.MIXED)
    hb.partition(fea.TYPE_SORTED)
    ho["mixed_static_by_elements"], _, _ = hrun(fea.MIXED)
    hb.partition(fea.GP_WEIGHT)
    ho["mixed_static_by_gauss_points"], _, _ = hrun(fea.MIXED)
    hb.partition(fea.LEARNED, hpred)
    ho["mixed_static_learned"], hvl, hstl = hrun(fea.MIXED)
    hb.order(fea.TYPE_SORTED)
    # the learned schedule: predicted cost classes, type-sorted within a class
    lc = ho["mixed_queue_learned_classes"]["total_ms"]
    ho["speedup_learned_mixed_vs_fp64_type_sorted"] = round(ho["fp64_type_sorted"]["total_ms"] / lc, 4)
    ho["speedup_learned_vs_type_sorted_queue_mixed"] = round(ho["mixed_type_sorted"]["total_ms"] / lc, 4)
    ho["speedup_learned_lpt_vs_type_sorted_queue_mixed"] = round(
        ho["mixed_type_sorted"]["total_ms"] / ho["mixed_queue_learned_lpt"]["total_ms"], 4)
    ho["speedup_learned_lpt_mixed_vs_fp64_type_sorted"] = round(
        ho["fp64_type_sorted"]["total_ms"] / ho["mixed_queue_learned_lpt"]["total_ms"], 4)
    ho["speedup_learned_static_vs_gauss_point_static"] = round(
        ho["mixed_static_by_gauss_points"]["total_ms"] / ho["mixed_static_learned"]["total_ms"], 4)
    # the most any queue order can gain on this GPU: the dynamic queue's
    # measured load balance already bounds the idle share of the launches
    ho["max_gain_any_order"] = round(1.0 / ho["mixed_type_sorted"]["load_balance"], 4)
    ho["mixed_vs_fp64_rel_frobenius"] = float(((hvl.double() - hv64).norm() / hv64.norm()).item())
    ho["status_ok"] = bool((hst64.cpu() == -1).all()) and bool((hstl.cpu() == -1).all())
    out["held_out"] = ho
    out["workers"] = hb.workers()
    del hv64, hvl
    hb.destroy()
    del hb, hdm
    torch.cuda.empty_cache()
    out["status_ok"] = bool((st64.cpu() == -1).all())
    del v64
    # the training mesh (neo-Hookean bricks included) in the row-gather and
    # upper-triangle row-owner forms, one mesh per call
    g = dm.graph()
    for vname in ("rowgather", "rowsym"):
        var = fea.VARIANTS[vname]
        for pname, p, o in (("fp64", fea.FP64, fea.F64), ("mixed", fea.MIXED, fea.F32)):
            gv, gr, gs = dm.assemble(g, variant=var, use_nh=True, precision=p, out_dtype=o)
            tot = []
            for _ in range(5):
                dm.assemble(g, variant=var, use_nh=True, precision=p, out_dtype=o, vals=gv, rhs=gr,
                            status=gs, timing=True)
                tot.append(g.last_timing()[2])
            out[f"{vname}_{pname}"] = {"total_ms": round(float(np.median(tot)), 4),
                                       "status_ok": int(gs.item()) == -1}
            del gv, gr, gs
    # one Newton step's assembly: the tangent A and the residual
    # b = f_ext - f_int(u) together (upper-triangle form, FP64)
    gv, gr, gs = dm.assemble(g, variant=fea.ROWSYM, use_nh=True, residual=True)
    tot = []
    for _ in range(5):
        dm.assemble(g, variant=fea.ROWSYM, use_nh=True, residual=True, vals=gv, rhs=gr, status=gs, timing=True)
        tot.append(g.last_timing()[2])
    out["rowsym_fp64_newton_residual"] = {"total_ms": round(float(np.median(tot)), 4),
                                          "status_ok": int(gs.item()) == -1}
    del gv, gr, gs
    g.destroy()
    b.destroy()
    return out


def workload_mesh(mg, name):
    """The seeded synthetic meshes: hybrid256 (256^3 cells, 40/30/20/10
    hex8/tet4/pen6/pyr5 layers, seed 5) and hybrid96 (96^3 cells, four equal
    bands hex8/pen6/tet4/pyr5, seed 2)."""
    if name == "hybrid256":
        return mg.hybrid_split(256, seed=5)
    if name == "hybrid96":
        return mg.hybrid_bands(96, seed=2)
    raise ValueError(name)


WORKLOAD_DESC = {
    "hybrid256": "hybrid256-elasticity (256^3 cells, 40/30/20/10 hex8/tet4/pen6/pyr5 z-bands, 3x3 BSR)",
    "hybrid96": "hybrid96-elasticity (96^3 cells, hex8/pen6/tet4/pyr5 z-bands, 3x3 BSR)",
}
PRECISIONS = {"fp64": (0, 0), "mixed": (1, 1)}  # (fea precision, fea out dtype)


def timed_steps(torch, step, steps, warmup):
    """ms per step over `steps` calls after `warmup`, bracketed by
    synchronisations (torch events on the current stream, where the library
    enqueues)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def phase_medians(np, g, step, reps):
    """Median (element phase, block-value kernel, whole call) in ms from the
    HIP events the library records on its stream."""
    ph = []
    for _ in range(reps):
        step(True)
        ph.append(g.last_timing())
    return [float(x) for x in np.median(np.array(ph), axis=0)]


def sym_roofline(g, sym, B, s_c, s_v, k_ms, copy_gbps, key):
    kb = sym_reduce_bytes(sym["tile_blocks"], sym["upper_blocks"], g.nnz, B, s_c, s_v)
    achieved = kb / (k_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "kernel": "k_segsum_sym<9>" + ("" if s_c == 8 else ",mixed"),
           "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_from_profile(key, "segsum.h"),
           "algorithmic_bytes": int(kb), "kernel_ms": round(k_ms, 4)}
    if copy_gbps:
        out.update({"copy_GBps": copy_gbps, "frac_of_copy": round(achieved / copy_gbps, 4)})
    return out


def one_mesh_workload(fea, torch, np, mesh, name, args, variant_names, copy_gbps):
    """One fea_assemble per step over the whole mesh: the headline form
    (args.variant, args.precision) timed over args.steps, its phases, and
    the other forms of variant_names in both precisions (five timed calls
    each). Returns (result dict, device mesh, graph)."""
    B = 3
    dm = fea.DeviceMesh(mesh, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = dm.graph()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3
    prec, outd = PRECISIONS[args.precision]
    var = fea.VARIANTS[args.variant]
    s_c, s_v = (8, 8) if prec == fea.FP64 else (4, 4)
    conn_len = int(mesh.conn_ptr[-1])
    # the first call builds the layout of its form (upper-triangle tiles)
    t0 = time.perf_counter()
    vals, rhs, st = dm.assemble(g, variant=var, precision=prec, out_dtype=outd)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3

    def step(timing=False):
        dm.assemble(g, variant=var, precision=prec, out_dtype=outd, vals=vals, rhs=rhs, status=st, timing=timing)

    ms = timed_steps(torch, step, args.steps, args.warmup)
    assert int(st.item()) == -1, "an element was rejected"
    print(f"[bench] {name}: {args.steps} steps, {ms:.3f} ms/step", file=sys.stderr, flush=True)
    ph = phase_medians(np, g, step, max(5, min(args.steps, 20)))
    dm.assemble(g, variant=fea.ROWSYM)  # builds the upper-triangle layout if the headline form did not
    sym = g.sym_sizes()
    eb = element_bytes(g, B, s_c, s_v, conn_len, mesh.n_nodes, mesh.n_elems, args.variant, sym)
    out = {"workload": WORKLOAD_DESC[name], "elements": int(mesh.n_elems), "nodes": int(mesh.n_nodes),
           "nnz_blocks": int(g.nnz), "variant": args.variant, "precision": args.precision,
           "ms_per_step": round(ms, 4), "elements_per_s": round(mesh.n_elems / (ms * 1e-3), 1),
           "phases_ms": {"element": round(ph[0], 4), "block_value_kernel": round(ph[1], 4),
                         "total": round(ph[2], 4)},
           "element_phase": {"algorithmic_bytes": int(eb), "ms": round(ph[0], 4),
                             "effective_GBps": round(eb / (ph[0] * 1e-3) / 1e9, 1),
                             "frac_of_peak": round(eb / (ph[0] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
           "graph_build_ms": round(graph_ms, 2), "first_call_ms": round(first_ms, 2),
           "upper_triangle_layout": sym}
    if args.variant == "rowsym":
        out["roofline"] = sym_roofline(g, sym, B, s_c, s_v, ph[1], copy_gbps,
                                       f"k_segsum_sym<9>{'' if s_c == 8 else ',mixed'}@{name}")
    elif args.variant == "rowowner":
        kb = reduce_bytes(g, B, s_c, s_v)
        a = kb / (ph[1] * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": "k_segsum<9>", "achieved": round(a, 1), "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": round(a / PEAK_HBM_GBS, 4),
                           "traffic": traffic_from_profile(f"k_segsum<9>@{name}", "segsum.h"),
                           "algorithmic_bytes": int(kb), "kernel_ms": round(ph[1], 4)}
    del vals, rhs
    variants = {}
    for vname in variant_names:
        for pname, (p, o) in PRECISIONS.items():
            vv, rr, ss = dm.assemble(g, variant=fea.VARIANTS[vname], precision=p, out_dtype=o)
            dm.assemble(g, variant=fea.VARIANTS[vname], precision=p, out_dtype=o, vals=vv, rhs=rr, status=ss)
            med = phase_medians(np, g, lambda t: dm.assemble(g, variant=fea.VARIANTS[vname], precision=p,
                                                             out_dtype=o, vals=vv, rhs=rr, status=ss,
                                                             timing=t), 5)
            sc = 8 if p == fea.FP64 else 4
            rec = {"total_ms": round(med[2], 4), "element_ms": round(med[0], 4),
                   "block_value_kernel_ms": round(med[1], 4),
                   "elements_per_s": round(mesh.n_elems / (med[2] * 1e-3), 1),
                   "status_ok": int(ss.item()) == -1}
            key = f"{vname}_{pname}"
            if vname == "rowsym":
                rec["roofline"] = sym_roofline(g, sym, B, sc, sc, med[1], copy_gbps,
                                               f"k_segsum_sym<9>{'' if sc == 8 else ',mixed'}@{name}")
            elif vname == "rowowner":
                kb = reduce_bytes(g, B, sc, sc)
                a = kb / (med[1] * 1e-3) / 1e9
                rec["roofline"] = {"bound": "hbm", "kernel": "k_segsum<9>" + ("" if sc == 8 else ",mixed"),
                                   "achieved": round(a, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                   "frac": round(a / PEAK_HBM_GBS, 4),
                                   "traffic": traffic_from_profile(
                                       f"k_segsum<9>{'' if sc == 8 else ',mixed'}@{name}", "segsum.h"),
                                   "algorithmic_bytes": int(kb)}
            elif vname in ("colour", "atomic"):
                # fused element kernels: the whole scatter happens in them
                eb2 = element_bytes(g, B, sc, 8, conn_len, mesh.n_nodes, mesh.n_elems, vname)
                a = eb2 / (med[0] * 1e-3) / 1e9
                tr = traffic_from_profile(f"{vname}_{pname}@{name}", "elem.h")
                rec["scatter"] = {"kernels": f"k_element<family, elasticity, {vname}>", "algorithmic_bytes": int(eb2),
                                  "effective_GBps": round(a, 1), "frac_of_peak": round(a / PEAK_HBM_GBS, 4),
                                  "counter_bytes": tr,
                                  "counter_GBps": round(tr / (med[0] * 1e-3) / 1e9, 1) if tr else None}
            variants[key] = rec
            del vv, rr, ss
    if variants:
        out["variants"] = variants
    torch.cuda.synchronize()
    return out, dm, g


def persistent_vs_one_mesh(fea, torch, np, dm, g, reps=7):
    """The one-mesh upper-triangle assembly against the same mesh through
    the persistent batched kernels (type-sorted queue), FP64 and mixed:
    median of reps calls each, alternating, timed with events around the
    whole call."""
    b = fea.Batch([dm], model=fea.ELASTIC)
    out = {}
    for pname, p, o in (("fp64", fea.FP64, fea.F64), ("mixed", fea.MIXED, fea.F32)):
        v, r, s = b.outputs(o)
        b.assemble(precision=p, out_dtype=o, vals=v, rhs=r, status=s, variant=fea.ROWSYM)
        gv, gr, gs = dm.assemble(g, variant=fea.ROWSYM, precision=p, out_dtype=o)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tp, to = [], []
        for _ in range(reps):
            e0.record()
            b.assemble(precision=p, out_dtype=o, vals=v, rhs=r, status=s, variant=fea.ROWSYM)
            e1.record()
            torch.cuda.synchronize()
            tp.append(e0.elapsed_time(e1))
            e0.record()
            dm.assemble(g, variant=fea.ROWSYM, precision=p, out_dtype=o, vals=gv, rhs=gr, status=gs)
            e1.record()
            torch.cuda.synchronize()
            to.append(e0.elapsed_time(e1))
        mp, mo = float(np.median(tp)), float(np.median(to))
        out[pname] = {"persistent_ms": round(mp, 3), "one_mesh_ms": round(mo, 3), "ratio": round(mp / mo, 3),
                      "status_ok": bool((s.cpu() == -1).all()) and int(gs.item()) == -1}
        del v, r, s, gv, gr, gs
    b.destroy()
    return out


def cpu_baseline_leg(fea, torch, np, mesh, name):
    """The only part of this benchmark that runs the oracle. (1) CPU
    baseline: the C oracle (FP64, -O3) on a bounded sample of the workload,
    ten z-layers of cells taken from the middle of its bands in its
    40/30/20/10 hex8/tet4/pen6/pyr5 proportion, timed as sequential
    Algorithm 1 and as its OpenMP atomic (Algorithm 4) and colour (Algorithm
    5) analogues on every host thread, median of five runs each; the best
    is reported, extrapolated to the whole mesh by its elements/s (same
    per-element work mix). (2) Accuracy: the GPU's FP64 and mixed
    upper-triangle assemblies of a four-layer sample (one layer per band)
    against the oracle, and the mixed error against its bound gamma_L T."""
    import oracle
    import meshgen as mg
    n = mesh.n_cells
    bands = mg.split_bands(n)
    starts = np.concatenate([[0], np.cumsum([l for _, l in bands])])
    take = (4, 3, 2, 1)

    def mid_layers(k, cnt):
        lo, hi = int(starts[k]), int(starts[k + 1])
        m0 = (lo + hi) // 2 - cnt // 2
        return list(range(m0, m0 + cnt))

    layers = sum((mid_layers(k, c) for k, c in enumerate(take)), [])
    sample = mg.layer_sample(mesh, layers)
    og = oracle.mesh_graph(sample)
    colour, nc = oracle.colour_greedy(sample.n_nodes, sample.conn_ptr, sample.conn)
    buckets = oracle.colour_buckets(colour, nc)
    runs = {}
    for kind in ("sequential", "atomic", "colour"):
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            if kind == "sequential":
                oracle.assemble(sample, og, model=oracle.ELASTIC)
            else:
                oracle.assemble_parallel(sample, og, kind, buckets=buckets if kind == "colour" else None)
            ts.append(time.perf_counter() - t0)
        runs[kind] = float(np.median(ts))
        print(f"[bench] cpu {kind}: {runs[kind]:.2f} s", file=sys.stderr, flush=True)
    best = min(runs, key=runs.get)
    rate = sample.n_elems / runs[best]
    threads = oracle.threads()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cpu = {"value": round(rate, 1), "unit": "elements/s", "cores": threads if best != "sequential" else 1,
           "kind": "oracle",
           "sample": (f"{sample.n_elems} elements of {name}: cell layers {layers} (4/3/2/1 layers from the middle "
                      f"of the hex8/tet4/pen6/pyr5 bands, the workload's family mix); FP64 C oracle at -O3, graph "
                      f"excluded, median of 5 runs per variant, best variant '{best}'; whole-mesh time "
                      f"extrapolated at this rate: {mesh.n_elems / rate:.1f} s"),
           "variants_s": {k: round(v, 3) for k, v in runs.items()},
           "variants_elements_per_s": {k: round(sample.n_elems / v, 1) for k, v in runs.items()},
           "omp_threads": threads, "nproc": os.cpu_count(), "cpu_model": model,
           "omp_proc_bind": os.environ.get("OMP_PROC_BIND", "")}
    # accuracy of the GPU forms against the oracle on a smaller sample
    acc_layers = sum((mid_layers(k, 1) for k in range(4)), [])
    am = mg.layer_sample(mesh, acc_layers)
    ag = oracle.mesh_graph(am)
    ov, orhs, tv, tr = oracle.assemble(am, ag, model=oracle.ELASTIC, with_terms=True)
    dma = fea.DeviceMesh(am, device="cuda:0")
    ga = dma.graph()
    scale = np.repeat(_row_max(np, ov, ag.row_ptr), 9)
    L = max({0: 1, 1: 8, 2: 6, 3: 8}[int(t)] for t in np.unique(am.types)) + 12
    gam = L * 2.0 ** -24 / (1 - L * 2.0 ** -24)
    accuracy = {"sample": f"{am.n_elems} elements of {name}: cell layers {acc_layers} (one per band)",
                "fp32_bound": f"|v32 - v64| <= gamma_L T + 1e-12 rowscale, L = {L}"}
    for pname, (p, o) in PRECISIONS.items():
        v, r, s = dma.assemble(ga, variant=fea.ROWSYM, precision=p, out_dtype=o)
        torch.cuda.synchronize()
        v = v.cpu().numpy().astype(np.float64)
        r = r.cpu().numpy().astype(np.float64)
        err = np.abs(v - ov)
        rec = {"status_ok": int(s.item()) == -1,
               "max_row_scaled": float((err / scale).max()),
               "median_row_scaled": float(np.median(err / scale)),
               "rhs_max_rel": float(np.abs(r - orhs).max() / np.abs(orhs).max())}
        if pname == "mixed":
            bound = gam * tv + 1e-12 * scale
            ratio = err / bound
            rec.update({"max_err_over_bound": float(ratio.max()), "median_err_over_bound": float(np.median(ratio)),
                        "max_abs_err": float(err.max()), "median_abs_err": float(np.median(err))})
        accuracy[pname] = rec
    ga.destroy()
    del dma
    torch.cuda.empty_cache()
    return cpu, accuracy


def _row_max(np, vals, row_ptr):
    """max_j |A(i, j)| of every block row i, broadcast to its blocks."""
    a = np.abs(vals.reshape(-1, 9)).max(axis=1)
    nr = np.diff(row_ptr)
    rm = np.zeros(row_ptr.size - 1)
    nz = nr > 0
    rm[nz] = np.maximum.reduceat(a, row_ptr[:-1][nz])
    out = np.repeat(rm, nr)
    out[out == 0] = 1.0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hybrid256", choices=["hybrid256", "hybrid96"])
    ap.add_argument("--variant", default="rowsym")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the other scatter forms")
    ap.add_argument("--no-small", action="store_true", help="skip the hybrid96 companion workload")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the subgrid-scale, batched, heterogeneous-cost and persistent workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy three times (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(assembly would shard by element slabs or whole meshes, with no communication "
              "between GPUs).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen as mg
    import paper_1805_03949_amd as fea

    t0 = time.time()
    mesh = workload_mesh(mg, args.workload)
    print(f"[bench] {args.workload}: {mesh.n_elems} elements in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    copy_gbps = copy_bandwidth(torch)
    head_variants = [] if args.no_variants else (["rowsym"] if args.workload == "hybrid256" else
                                                 ["rowsym", "rowowner", "rowgather", "tilecolour", "atomic",
                                                  "colour"])
    head, dm, g = one_mesh_workload(fea, torch, np, mesh, args.workload, args, head_variants, copy_gbps)

    extras = {}
    print("[bench] subgrid scale", file=sys.stderr, flush=True)
    sub, _ = subscale_workload(fea, mg, torch, np, mesh, dm, g, name=args.workload)
    g.destroy()
    del dm, g
    torch.cuda.empty_cache()

    if args.workload == "hybrid256" and not args.no_small:
        print("[bench] hybrid96", file=sys.stderr, flush=True)
        small = workload_mesh(mg, "hybrid96")
        sargs = argparse.Namespace(**{**vars(args), "steps": 20, "warmup": 3})
        sv = [] if args.no_variants else ["rowsym", "rowowner", "rowgather", "tilecolour", "atomic", "colour"]
        extras["hybrid96"], sdm, sg = one_mesh_workload(fea, torch, np, small, "hybrid96", sargs, sv, copy_gbps)
        if not args.no_extras:
            extras["hybrid96"]["persistent_vs_one_mesh"] = persistent_vs_one_mesh(fea, torch, np, sdm, sg)
        sg.destroy()
        del sdm, sg
        torch.cuda.empty_cache()

    if not args.no_extras:
        print("[bench] batched workload", file=sys.stderr, flush=True)
        extras["batched"] = batched_workload(fea, mg, torch)
        torch.cuda.empty_cache()
        print("[bench] heterogeneous workload", file=sys.stderr, flush=True)
        extras["heterogeneous"] = heterogeneous_workload(fea, mg, torch, np)
        torch.cuda.empty_cache()
        if args.workload == "hybrid256":
            print("[bench] persistent form of the large workload", file=sys.stderr, flush=True)
            extras["large_persistent"] = large_workload(fea, mg, torch, np, mesh=mesh)
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        if args.workload == "hybrid256":
            cpu, extras["accuracy"] = cpu_baseline_leg(fea, torch, np, mesh, args.workload)
        else:
            import oracle
            og = oracle.mesh_graph(mesh)
            t0 = time.perf_counter()
            oracle.assemble(mesh, og, model=oracle.ELASTIC)
            cpu_s = time.perf_counter() - t0
            cpu = {"value": round(mesh.n_elems / cpu_s, 1), "unit": "elements/s", "cores": 1, "kind": "oracle",
                   "sample": f"the whole workload ({mesh.n_elems} elements), FP64 C oracle, sequential "
                             f"Algorithm 1 order, graph build excluded; {cpu_s:.1f} s"}

    value = head["elements_per_s"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "elements": head["elements"], "nodes": head["nodes"],
                   "nnz_blocks": head["nnz_blocks"], "variant": args.variant, "precision": args.precision,
                   "out_dtype": "f64" if args.precision == "fp64" else "f32"},
        "roofline": head.get("roofline"),
        "cpu_baseline": cpu,
        "headline": head,
        "subscale": sub,
        "copy_GBps": copy_gbps,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
