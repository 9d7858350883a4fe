"""Benchmark: finite-element assembly on one MI355X.

A step is one fea_assemble call over the whole workload (element quadrature
for every element plus the race-free scatter into the 3x3 block matrix and
the right-hand side), with the mesh, graph and outputs resident in HBM.
The graph build is timed once and reported separately.

Workload (default): linear elasticity on a 96^3-cell hybrid mesh, four
z-bands of 24 cell layers (hex8 / pen6 / tet4 / pyr5), E = 1, nu per element
U[0.2, 0.35], body force (0, 0, -1); 3,317,760 elements, 1,133,857 nodes.

Prints one JSON line. Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--variant rowsym]
                  [--precision fp64|mixed] [--no-cpu] [--no-variants]
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
    every block value (upper and transposed lower) written once."""
    return ulen * B * B * s_c + (nup + 1) * 8 + nup * 8 + nnz * B * B * s_v


def element_bytes(g, B, s_c, s_v, conn_len, n_nodes, n_elems, variant, sym=None):
    """Algorithmic bytes of the element phase: node coordinates once, the
    connectivity and per-element data once, and its outputs once (the slot
    contributions for row-owner; for the upper-triangle form the tile sums
    plus its tile entries (2 bytes), tile-block ends and slots (6 bytes) and
    tile ranges (16 bytes); for row-gather the final values, plus the
    pair-ordered node lists, lane bytes and segment bounds it reads)."""
    inputs = n_nodes * 24 + conn_len * 4 + n_elems * (8 + 4 + 8 + 16 + 8 * B)
    if variant == "rowowner":
        return inputs + g.map_len * B * B * s_c + conn_len * B * s_c
    if variant == "rowsym":
        return (inputs + sym["tile_blocks"] * (B * B * s_c + 6) + sym["entries"] * 2 + sym["tiles"] * 16
                + conn_len * B * s_c)
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
    (FMA = 2): per node J (9 FMA) and, unless the family is affine (tet4),
    the mixed second derivatives of x (9) and grad / mixed second
    derivatives of u (3B + 3B); then J^-1 with its determinant and w detJ
    (43), the second-derivative transform and the operator (282 for
    elasticity, 56 for Poisson; tet4: none), the volume sum (1) and tau r
    (B)."""
    per_node = 18 + (0 if t == 0 else 18 + 12 * B)
    post = 0 if t == 0 else (282 if B == 3 else 56)
    return SUB_NN[t] * per_node + 43 + post + 1 + B


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


def subscale_workload(fea, mg, torch, np, mesh, dm, g, reps=20):
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
    res = {"workload": "hybrid96 elasticity, smooth displacement field, FP64", "ms": round(ms, 4),
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
            "persistent_kernel_ms_tuned_tiles": round(tuned_ms, 4),
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


def large_workload(fea, mg, torch, np, cells=256):
    """53.9M-element hybrid mesh (40/30/20/10 hex/tet/pen/pyr layers) through
    the persistent path in the upper-triangle form (plain FP64 against mixed
    precision with the learned schedule; row-owner FP64 for reference), then
    one-mesh assemblies in the row-gather and upper-triangle forms."""
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
    out["mixed_queue_learned"] = run(fea.MIXED)
    best = min(out["mixed_static_learned"]["total_ms"], out["mixed_queue_learned"]["total_ms"])
    out["speedup_learned_mixed_vs_fp64"] = round(out["fp64_type_sorted"]["total_ms"] / best, 4)
    b.destroy()
    torch.cuda.empty_cache()

    # the same mesh through the fused row-gather form (no workspace) and the
    # upper-triangle row-owner form
    g = dm.graph()
    for vname in ("rowgather", "rowsym"):
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


def heterogeneous_workload(fea, mg, torch, np, cells=128):
    """Hybrid split mesh (40/30/20/10 hex/tet/pen/pyr layers) where 30% of
    8^3-cell bricks use the neo-Hookean tangent: the cost model is trained
    on the recorded cycles and orders the queue; compared with the
    type-sorted order and the Gauss-point-weight order, and the learned
    mixed-precision form with the plain FP64 form."""
    mesh = mg.heterogeneous(cells, seed=4)
    dm = fea.DeviceMesh(mesh)
    b = fea.Batch([dm], model=fea.ELASTIC, use_nh=True)

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

    out = {"workload": f"hetero{cells}-elasticity (30% neo-Hookean bricks, 40/30/20/10 hex/tet/pen/pyr)",
           "elements": int(mesh.n_elems), "items": int(b.n_items), "workers": 0,
           "variant": "rowsym (persistent kernel)"}
    out["fp64_type_sorted_rowowner"], _, _ = run(fea.FP64, variant=fea.ROWOWNER)
    fp64_ts, v64, st64 = run(fea.FP64)
    out["fp64_type_sorted"] = fp64_ts
    mix_ts, vmx, stm = run(fea.MIXED)
    out["mixed_type_sorted"] = mix_ts
    # training data: log-cycles of every item, averaged over five
    # type-sorted mixed runs (single runs are noisy: concurrent workgroups
    # share the caches and memory channels)
    vals, rhs, st = b.outputs(fea.F32)
    logs = []
    for _ in range(5):
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=vals, rhs=rhs, status=st, variant=fea.ROWSYM)
        c, _, _ = b.cycles()
        logs.append(fea.CostModel.log_cycles(c))
    target = torch.stack(logs).mean(dim=0).contiguous()
    del vals, rhs, st
    feats = b.features(fp64_geometry=False)
    cm = fea.CostModel(seed=7)
    cm.fit_norm(feats)
    t0 = time.perf_counter()
    hist = cm.train(feats, target, steps=600, lr=3e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    pred = cm.predict(feats)
    t = target.cpu().numpy().astype(np.float64)
    p = pred.cpu().numpy().astype(np.float64)
    gp = np.log(b.items[:, 3] * np.array([1, 8, 6, 8])[b.items[:, 1]])

    def r2(x, y):
        x = x - x.mean()
        y = y - y.mean()
        return float((x @ y) ** 2 / ((x @ x) * (y @ y)))

    # static split of the whole mesh into 8 contiguous parts (the sharding
    # of a mesh over 8 GPUs): cut the type-sorted items where the running
    # weight crosses k/8 of the total, then rate each split by the
    # measured cycles of its parts (load balance = mean / max part cost)
    cyc = np.exp(t)

    def split_lb(wts, parts=8):
        cs = np.cumsum(wts)
        cut = np.searchsorted(cs - 0.5 * wts, cs[-1] * np.arange(1, parts) / parts)
        sums = np.array([c.sum() for c in np.split(cyc, cut)])
        return round(float(sums.mean() / sums.max()), 4)

    out["static_split_8_load_balance"] = {
        "elements": split_lb(b.items[:, 3].astype(np.float64)),
        "gauss_points": split_lb(np.exp(gp)),
        "learned": split_lb(np.exp(p)),
        "measured_cycles": split_lb(cyc)}
    out["cost_model"] = {"train_steps": 600, "train_s": round(train_s, 3),
                         "loss_first": round(float(hist[0].item()), 5), "loss_last": round(float(hist[-1].item()), 5),
                         "r2_learned_vs_measured": round(r2(p, t), 4),
                         "r2_gauss_point_weight_vs_measured": round(r2(gp, t), 4)}
    # dynamic queue, largest predicted cost first
    b.order(fea.GP_WEIGHT)
    out["mixed_queue_gp_weight_lpt"], _, _ = run(fea.MIXED)
    b.order(fea.LEARNED, pred)
    out["mixed_queue_learned_lpt"], _, _ = run(fea.MIXED)
    # static partitions of the type-sorted items, one range per workgroup
    b.partition(fea.TYPE_SORTED)
    out["mixed_static_by_elements"], _, _ = run(fea.MIXED)
    b.partition(fea.GP_WEIGHT)
    out["mixed_static_by_gauss_points"], _, _ = run(fea.MIXED)
    b.partition(fea.LEARNED, pred)
    out["mixed_static_learned"], vl, stl = run(fea.MIXED)
    b.partition(fea.LEARNED, pred)
    out["fp64_static_learned"], _, _ = run(fea.FP64)
    b.order(fea.TYPE_SORTED)
    out["workers"] = b.workers()
    best_learned = min(out["mixed_queue_learned_lpt"]["total_ms"], out["mixed_static_learned"]["total_ms"])
    out["speedup_learned_mixed_vs_fp64_type_sorted"] = round(fp64_ts["total_ms"] / best_learned, 4)
    out["speedup_learned_static_vs_gauss_point_static"] = round(
        out["mixed_static_by_gauss_points"]["total_ms"] / out["mixed_static_learned"]["total_ms"], 4)
    out["speedup_learned_vs_type_sorted_queue_mixed"] = round(mix_ts["total_ms"] / best_learned, 4)
    d = (vl.double() - v64).norm() / v64.norm()
    out["mixed_vs_fp64_rel_frobenius"] = float(d.item())
    out["status_ok"] = bool((st64.cpu() == -1).all()) and bool((stl.cpu() == -1).all())
    # the same mesh (neo-Hookean bricks included) in the row-gather and
    # upper-triangle row-owner forms
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
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=96)
    ap.add_argument("--variant", default="rowsym")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 256^3 workload")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and heterogeneous-cost workloads")
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
    mesh = mg.hybrid_bands(args.cells, seed=2)
    print(f"[bench] mesh {mesh.n_elems} elements in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dm = fea.DeviceMesh(mesh, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = dm.graph()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3

    prec = fea.FP64 if args.precision == "fp64" else fea.MIXED
    outd = fea.F64 if prec == fea.FP64 else fea.F32
    var = fea.VARIANTS[args.variant]
    B = 3
    s_c = 8 if prec == fea.FP64 else 4
    s_v = 8 if outd == fea.F64 else 4
    conn_len = int(mesh.conn_ptr[-1])

    vals, rhs, st = dm.assemble(g, variant=var, precision=prec, out_dtype=outd)

    def step(timing=False):
        dm.assemble(g, variant=var, precision=prec, out_dtype=outd, vals=vals, rhs=rhs, status=st,
                    timing=timing)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert int(st.item()) == -1, "an element was rejected"
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    print(f"[bench] {args.steps} steps, {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    # phase durations from HIP events recorded by the library on its stream
    phases, classes = [], []
    for _ in range(max(5, min(args.steps, 20))):
        step(timing=True)
        phases.append(g.last_timing())
        if args.variant == "rowgather":
            classes.append(g.last_class_timing())
    ph = np.median(np.array(phases), axis=0)
    elem_ms, second_ms = float(ph[0]), float(ph[1])
    # sizes of the upper-triangle layout (built by its first assembly)
    vs, rs, ss = dm.assemble(g, variant=fea.ROWSYM)
    del vs, rs, ss
    sym = g.sym_sizes()
    ulen, nup = sym["tile_blocks"], sym["upper_blocks"]
    eb = element_bytes(g, B, s_c, s_v, conn_len, mesh.n_nodes, mesh.n_elems, args.variant, sym)
    copy_gbps = copy_bandwidth(torch)
    class_ms = None
    if args.variant == "rowgather":
        # dominant kernel: the row-tile class kernel that takes longest; its
        # bound is FP64 (vector ALU) arithmetic, not HBM
        cm = np.median(np.array(classes), axis=0)
        class_ms = {n: round(float(v), 4) for n, v in zip(GATHER_FAMILIES, cm)}
        flops, executed = gather_class_flops(mesh, np)
        c = int(np.argmax(cm))
        kernel, k_ms, k_work = f"k_gather<{GATHER_FAMILIES[c]}>", float(cm[c]), flops[c]
        achieved = k_work / (k_ms * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if prec == fea.FP64 else PEAK_FP32_TFLOPS
        roofline = {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 2), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                    "traffic": traffic_from_profile(kernel, "gather.hip"),
                    "algorithmic_flops": int(k_work), "kernel_ms": round(k_ms, 4),
                    "executed_flops": int(executed[c]),
                    "executed_TFLOPs": round(executed[c] / (k_ms * 1e-3) / 1e12, 2),
                    "note": "algorithmic: per-element element-matrix flops exploiting the sparsity of B, "
                            "1/n of an element per (row, element) pair; executed: the kernel's own "
                            "operations, geometry recomputed per pair"}
    elif args.variant in ("rowowner", "rowsym"):
        if args.variant == "rowowner":
            kernel, k_bytes = "k_segsum<9>", reduce_bytes(g, B, s_c, s_v)
        else:
            kernel, k_bytes = "k_segsum<9,sym>", sym_reduce_bytes(ulen, nup, g.nnz, B, s_c, s_v)
        k_ms = second_ms
        achieved = k_bytes / (k_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                    "traffic": traffic_from_profile(kernel + ("" if prec == fea.FP64 else ",mixed"), "segsum.h"),
                    "algorithmic_bytes": int(k_bytes), "kernel_ms": round(k_ms, 4),
                    "copy_GBps": copy_gbps, "frac_of_copy": round(achieved / copy_gbps, 4)}
    else:
        kernel, k_ms, k_bytes = f"{args.variant} element phase", elem_ms, eb
        achieved = k_bytes / (k_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                    "traffic": None, "algorithmic_bytes": int(k_bytes), "kernel_ms": round(k_ms, 4)}

    variants = {}
    if not args.no_variants:
        for vname in ("rowgather", "rowsym", "tilecolour", "rowowner", "atomic", "colour"):
            for pname, p, o in (("fp64", fea.FP64, fea.F64), ("mixed", fea.MIXED, fea.F32)):
                vv, rr, ss = dm.assemble(g, variant=fea.VARIANTS[vname], precision=p, out_dtype=o)
                dm.assemble(g, variant=fea.VARIANTS[vname], precision=p, out_dtype=o, vals=vv, rhs=rr, status=ss)
                ts = []
                for _ in range(5):
                    dm.assemble(g, variant=fea.VARIANTS[vname], precision=p, out_dtype=o, vals=vv, rhs=rr,
                                status=ss, timing=True)
                    ts.append(g.last_timing())
                med = np.median(np.array(ts), axis=0)
                variants[f"{vname}_{pname}"] = {"total_ms": round(float(med[2]), 4),
                                                "element_ms": round(float(med[0]), 4),
                                                "block_value_kernel_ms": round(float(med[1]), 4),
                                                "elements_per_s": round(mesh.n_elems / (float(med[2]) * 1e-3), 1)}
                del vv, rr, ss
        torch.cuda.synchronize()
        # HBM rooflines of the block-value kernels of the two-phase forms
        for vkey, kname, sc in (("rowowner_fp64", "k_segsum<9>", 8), ("rowowner_mixed", "k_segsum<9>,mixed", 4),
                                ("rowsym_fp64", "k_segsum<9,sym>", 8), ("rowsym_mixed", "k_segsum<9,sym>,mixed", 4)):
            ro = variants[vkey]
            rb = (reduce_bytes(g, B, sc, sc) if vkey.startswith("rowowner")
                  else sym_reduce_bytes(ulen, nup, g.nnz, B, sc, sc))
            ra = rb / (ro["block_value_kernel_ms"] * 1e-3) / 1e9
            variants[vkey]["roofline"] = {
                "bound": "hbm", "kernel": kname, "achieved": round(ra, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(ra / PEAK_HBM_GBS, 4),
                "traffic": traffic_from_profile(kname, "segsum.h"),
                "algorithmic_bytes": int(rb), "copy_GBps": copy_gbps, "frac_of_copy": round(ra / copy_gbps, 4)}

    print("[bench] subgrid scale", file=sys.stderr, flush=True)
    sub, sub_u = subscale_workload(fea, mg, torch, np, mesh, dm, g)

    extras = {}
    if not args.no_extras:
        del vals, rhs
        torch.cuda.empty_cache()
        print("[bench] batched workload", file=sys.stderr, flush=True)
        extras["batched"] = batched_workload(fea, mg, torch)
        torch.cuda.empty_cache()
        print("[bench] heterogeneous workload", file=sys.stderr, flush=True)
        extras["heterogeneous"] = heterogeneous_workload(fea, mg, torch, np)
        torch.cuda.empty_cache()
        if not args.no_large:
            print("[bench] large workload", file=sys.stderr, flush=True)
            extras["large"] = large_workload(fea, mg, torch, np)
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        import oracle
        og = oracle.mesh_graph(mesh)
        t0 = time.perf_counter()
        oracle.assemble(mesh, og, model=oracle.ELASTIC)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(mesh.n_elems / cpu_s, 1), "unit": "elements/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the whole workload ({mesh.n_elems} elements), FP64 C oracle, sequential "
                         f"Algorithm 1 order, graph build excluded; {cpu_s:.1f} s"}
        t0 = time.perf_counter()
        oracle.subscale(mesh, sub_u.cpu().numpy(), model=oracle.ELASTIC)
        sub_s = time.perf_counter() - t0
        sub["cpu_baseline"] = {"value": round(mesh.n_elems / sub_s, 1), "unit": "elements/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the whole subgrid-scale workload, FP64 C oracle; {sub_s:.1f} s"}

    # scatter HBM rate of the two-phase (row-owner) form: its block-value
    # kernel (the right-hand-side reduction runs before it, inside the
    # element phase of the timing)
    scatter = {"kernel": "k_segsum<9>", "copy_GBps": copy_gbps,
               "note": "row-owner form, block-value kernel (workspace sorted by destination block)"}
    if args.variant == "rowowner":
        t2 = second_ms
    elif "rowowner_" + args.precision in variants:
        t2 = variants["rowowner_" + args.precision]["block_value_kernel_ms"]
    else:
        t2 = None
    if t2:
        rb = reduce_bytes(g, B, s_c, s_v)
        eff = rb / (t2 * 1e-3) / 1e9
        scatter.update({"algorithmic_bytes": int(rb), "effective_GBps": round(eff, 1),
                        "frac_of_peak": round(eff / PEAK_HBM_GBS, 4), "frac_of_copy": round(eff / copy_gbps, 4),
                        "ms": round(t2, 4)})
    tr = traffic_from_profile("k_segsum<9>" + ("" if prec == fea.FP64 else ",mixed"), "segsum.h")
    if tr and t2:
        scatter["counter_GBps"] = round(tr / (t2 * 1e-3) / 1e9, 1)

    value = mesh.n_elems / (ms_per_step * 1e-3)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fea.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"hybrid{args.cells}-elasticity (hex8/pen6/tet4/pyr5 z-bands, 3x3 BSR)",
                   "elements": mesh.n_elems, "nodes": mesh.n_nodes, "nnz_blocks": g.nnz,
                   "variant": args.variant, "precision": args.precision,
                   "out_dtype": "f64" if outd == fea.F64 else "f32"},
        "roofline": roofline,
        "scatter": scatter,
        "gather_class_ms": class_ms,
        "element_phase": {"algorithmic_bytes": int(eb), "ms": round(elem_ms, 4),
                          "effective_GBps": round(eb / (elem_ms * 1e-3) / 1e9, 1)},
        "phases_ms": {"element": round(elem_ms, 4), "block_value_kernel": round(second_ms, 4),
                      "total": round(float(ph[2]), 4)},
        "graph_build_ms": round(graph_ms, 2),
        "variants": variants,
        "subscale": sub,
        **extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
