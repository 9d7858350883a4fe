"""GPU tests of the cost model kernels against the FP64 NumPy oracle, of the
work-item features, the tile autotuner and the queue schedules."""
import os
import tempfile

import numpy as np
import pytest

import meshgen as mg
import oracle
from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1805_03949_amd as fea  # noqa: E402


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 12)) * rng.uniform(0.5, 3.0, 12) + rng.uniform(-2, 2, 12)
    t = np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2] - 0.2 * X[:, 5] + 2.0
    return X.astype(np.float32), t.astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_forward_and_gradient_match_fp64_oracle():
    X, t = _data(1000)
    cm = fea.CostModel(seed=11)
    mean, scale = X.mean(axis=0), X.std(axis=0)
    cm.set_norm(mean, scale)
    theta = cm.params().astype(np.float64)
    Xd, td = _dev(X), _dev(t)
    y = cm.predict(Xd).cpu().numpy()
    y_ref, _ = mlp.forward(theta, X.astype(np.float64), mean.astype(np.float32).astype(np.float64),
                           scale.astype(np.float32).astype(np.float64))
    assert np.abs(y - y_ref).max() <= 1e-4 * max(1.0, np.abs(y_ref).max())
    g, loss = cm.grad(Xd, td)
    g = g.cpu().numpy()
    l_ref, g_ref = mlp.loss_grad(theta, X.astype(np.float64), t.astype(np.float64),
                                 mean.astype(np.float64), scale.astype(np.float64))
    assert abs(float(loss.item()) - l_ref) <= 1e-4 * l_ref
    assert np.abs(g - g_ref).max() <= 2e-4 * np.abs(g_ref).max()


def test_adam_step_matches_oracle_and_is_deterministic():
    X, t = _data(700, seed=2)
    Xd, td = _dev(X), _dev(t)
    cm = fea.CostModel(seed=12)
    cm.fit_norm(Xd)
    theta0 = cm.params().astype(np.float64)
    g, _ = cm.grad(Xd, td)
    g = g.cpu().numpy().astype(np.float64)
    cm.train(Xd, td, steps=1, lr=1e-3)
    theta1 = cm.params().astype(np.float64)
    ref, _, _ = mlp.adam_step(theta0, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    assert np.abs(theta1 - ref).max() <= 1e-6
    # same init and data: identical parameters after training
    a = fea.CostModel(seed=5)
    b = fea.CostModel(seed=5)
    for c in (a, b):
        c.fit_norm(Xd)
        c.train(Xd, td, steps=20, lr=1e-3)
    assert a.params().tobytes() == b.params().tobytes()


def test_norm_fit_and_training_reduce_loss_and_checkpoint():
    X, t = _data(4000, seed=3)
    Xd, td = _dev(X), _dev(t)
    cm = fea.CostModel(seed=13)
    cm.fit_norm(Xd)
    hist = cm.train(Xd, td, steps=400, lr=3e-3).cpu().numpy()
    assert hist[-1] < 0.1 * hist[0]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "cost.bin")
        cm.save(path)
        other = fea.CostModel(seed=99)
        other.load(path)
        assert other.params().tobytes() == cm.params().tobytes()
        y1 = cm.predict(Xd).cpu().numpy()
        y2 = other.predict(Xd).cpu().numpy()
        assert y1.tobytes() == y2.tobytes()
        with open(path, "r+b") as f:
            f.write(b"XXXX")
        with pytest.raises(fea.FeaError):
            other.load(path)


def test_item_features_against_mesh_data_and_oracle_volumes():
    mesh = mg.heterogeneous(12, seed=31, brick=3, jitter=0.15)
    dm = fea.DeviceMesh(mesh)
    b = fea.Batch([dm], model=fea.ELASTIC, tile=[40, 30, 21, 12], use_nh=True)
    F = b.features(fp64_geometry=True).cpu().numpy()
    perm = np.argsort(mesh.types, kind="stable")
    seg = np.concatenate([[0], np.cumsum(np.bincount(mesh.types, minlength=4))])
    # element volumes from the oracle: Poisson rhs with f = 1 sums to the volume
    vols = np.zeros(mesh.n_elems)
    for e in range(mesh.n_elems):
        X = np.stack([mesh.x, mesh.y, mesh.z], 1)[mesh.conn[mesh.conn_ptr[e]:mesh.conn_ptr[e + 1]]]
        _, fe = oracle.element(int(mesh.types[e]), X, model=oracle.POISSON, f=np.ones(1))
        vols[e] = fe.sum()
    for i, (m, fam, begin, count) in enumerate(b.items):
        els = perm[seg[fam] + begin: seg[fam] + begin + count]
        f = F[i]
        assert np.array_equal(f[:4], np.eye(4)[fam])
        assert abs(f[4] - mesh.nh_flag[els].mean()) < 1e-6
        assert abs(f[5] - np.log2(count)) < 1e-6
        nodes = np.concatenate([mesh.conn[mesh.conn_ptr[e]:mesh.conn_ptr[e + 1]] for e in els])
        span = (nodes.max() - nodes.min() + 1) / (count * fea_nodes(fam))
        assert abs(f[6] - np.log2(span)) < 1e-4
        assert abs(f[7] - mesh.nu[els].mean()) < 1e-5
        assert f[8] >= -1e-6 and f[9] >= f[8] - 1e-6
        assert abs(f[10] - np.log10(vols[els].mean())) < 1e-4
        assert f[11] == 1.0


def fea_nodes(fam):
    return (4, 5, 6, 8)[fam]


def test_autotune_picks_candidates_and_persists():
    meshes = [mg.cube_mesh(6, np.random.default_rng(s).integers(0, 4, 216).astype(np.uint8), jitter=0.2,
                           seed=s) for s in range(3)]
    dms = [fea.DeviceMesh(m) for m in meshes]
    b = fea.Batch(dms, model=fea.ELASTIC)
    v0, r0, _ = b.assemble(precision=fea.MIXED, out_dtype=fea.F32)
    ref = (v0.cpu().numpy().tobytes(), r0.cpu().numpy().tobytes())
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tiles.txt")
        tile = b.autotune(precision=fea.MIXED, out_dtype=fea.F32, reps=3, table_path=path)
        epb = (25, 17, 12, 7)
        for t in range(4):
            assert tile[t] % epb[t] == 0 and tile[t] // epb[t] in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32)
        assert list(fea.tile_table_load(path, fea.ELASTIC, fea.MIXED)) == list(tile)
        with pytest.raises(fea.FeaError):
            fea.tile_table_load(path, fea.POISSON, fea.FP64)
    v, r, _ = b.assemble(precision=fea.MIXED, out_dtype=fea.F32)
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref


def test_schedules_order_items_and_keep_results():
    mesh = mg.heterogeneous(16, seed=41, brick=4)
    dm = fea.DeviceMesh(mesh)
    b = fea.Batch([dm], model=fea.ELASTIC, use_nh=True)
    v0, r0, _ = b.assemble()
    ref = (v0.cpu().numpy().tobytes(), r0.cpu().numpy().tobytes())
    b.order(fea.GP_WEIGHT)
    v, r, _ = b.assemble()
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref
    c, _, _ = b.cycles()
    target = fea.CostModel.log_cycles(c)
    assert np.allclose(target.cpu().numpy(), np.log(c.cpu().numpy().astype(np.float64)), rtol=1e-6)
    cm = fea.CostModel(seed=1)
    feats = b.features()
    cm.fit_norm(feats)
    cm.train(feats, target, steps=200, lr=3e-3)
    pred = cm.predict(feats)
    b.order(fea.LEARNED, pred)
    # the queue order is the oracle's longest-predicted-first order (ties by index)
    from oracle import sched
    assert np.array_equal(b.get_order(), sched.lpt_order(pred.cpu().numpy()))
    gpw = b.items[:, 3] * np.array([1, 8, 6, 8])[b.items[:, 1]]
    b.order(fea.GP_WEIGHT)
    assert np.array_equal(b.get_order(), sched.lpt_order(gpw))
    b.order(fea.LEARNED, pred)
    v, r, _ = b.assemble()
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref
    # cost classes: the oracle's class order, and the same results
    b.order(fea.LEARNED_CLASSES, pred)
    assert np.array_equal(b.get_order(), sched.class_order(pred.cpu().numpy(), b.items[:, 1]))
    v, r, _ = b.assemble()
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref
    with pytest.raises(fea.FeaError):
        b.order(fea.LEARNED, None)
    with pytest.raises(fea.FeaError):
        b.order(fea.LEARNED_CLASSES, None)
    bad = pred.clone()
    bad[bad.numel() // 2] = float("nan")
    for sch in (fea.LEARNED, fea.LEARNED_CLASSES):
        with pytest.raises(fea.FeaError):
            b.order(sch, bad)
    with pytest.raises(fea.FeaError):
        b.partition(fea.LEARNED, bad)
    b.order(fea.TYPE_SORTED)
    assert np.array_equal(b.get_order(), np.arange(b.n_items))


def test_static_partitions_keep_results_and_ranges():
    mesh = mg.heterogeneous(16, seed=42, brick=4)
    dm = fea.DeviceMesh(mesh)
    b = fea.Batch([dm], model=fea.ELASTIC, use_nh=True)
    v0, r0, _ = b.assemble()
    ref = (v0.cpu().numpy().tobytes(), r0.cpu().numpy().tobytes())
    c, _, _ = b.cycles()
    target = fea.CostModel.log_cycles(c)
    cm = fea.CostModel(seed=3)
    feats = b.features()
    cm.fit_norm(feats)
    cm.train(feats, target, steps=100, lr=3e-3)
    pred = cm.predict(feats)
    for weights in (fea.TYPE_SORTED, fea.GP_WEIGHT, fea.LEARNED):
        b.partition(weights, pred if weights == fea.LEARNED else None)
        v, r, st = b.assemble()
        assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref
        _, w, _ = b.cycles()
        w = w.cpu().numpy()
        # every workgroup of a family's launch ran one contiguous range of
        # that family's type-sorted items
        fam = b.items[:, 1]
        for t in range(4):
            assert np.all(np.diff(w[fam == t]) >= 0), t
    b.order(fea.TYPE_SORTED)
    v, r, _ = b.assemble()
    assert (v.cpu().numpy().tobytes(), r.cpu().numpy().tobytes()) == ref


def _log_cycles(b, runs=3):
    v, r, s = b.outputs(fea.F32)
    logs = []
    for _ in range(runs):
        b.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=v, rhs=r, status=s, variant=fea.ROWSYM)
        c, _, _ = b.cycles()
        logs.append(fea.CostModel.log_cycles(c))
    return torch.stack(logs).mean(dim=0).contiguous()


def test_learned_cost_model_on_a_held_out_mesh():
    """The paper's premise (abstract; Section 4.1): element cost is not known
    a priori and Gauss-point weights balance poorly. Trained on the measured
    cycles of one heterogeneous mesh, the model is judged on another (other
    neo-Hookean bricks, other displacement field) by the paper's metric, the
    load balance sum t_i / (n max t_i) of a partition: an 8-way static split
    of the held-out mesh by its predictions is far better balanced (by
    measured cycles) than one by Gauss points. Per-item r^2 against single
    items' cycles (noisy: concurrent workgroups share caches and memory
    channels) and the persistent kernel's times under each queue order are
    reported, not asserted."""
    from oracle import sched
    train = mg.heterogeneous(48, seed=51, brick=8)
    test = mg.heterogeneous(48, seed=52, brick=8)
    print(f"[case] hetero48 train/held-out: {train.n_elems} elements", flush=True)
    bt = fea.Batch([fea.DeviceMesh(train)], model=fea.ELASTIC, use_nh=True)
    cm = fea.CostModel(seed=9)
    ft = bt.features(fp64_geometry=False)
    cm.fit_norm(ft)
    cm.train(ft, _log_cycles(bt), steps=300, lr=3e-3)
    bh = fea.Batch([fea.DeviceMesh(test)], model=fea.ELASTIC, use_nh=True)
    pred = cm.predict(bh.features(fp64_geometry=False)).cpu().numpy().astype(np.float64)
    meas = _log_cycles(bh).cpu().numpy().astype(np.float64)
    gp = np.log(bh.items[:, 3] * np.array([1, 8, 6, 8])[bh.items[:, 1]])

    def r2(x, y):
        x, y = x - x.mean(), y - y.mean()
        return float((x @ y) ** 2 / ((x @ x) * (y @ y)))

    cyc = np.exp(meas)

    def split_lb(w, parts=8):
        cs = np.cumsum(w)
        cut = np.searchsorted(cs - 0.5 * w, cs[-1] * np.arange(1, parts) / parts)
        return sched.load_balance([c.sum() for c in np.split(cyc, cut)])

    r2l, r2g = r2(pred, meas), r2(gp, meas)
    lbl, lbg = split_lb(np.exp(pred)), split_lb(np.exp(gp))
    times = {}
    v, r, s = bh.outputs(fea.F32)
    for name, setup in (("type_sorted", lambda: bh.order(fea.TYPE_SORTED)),
                        ("gp_weight_lpt", lambda: bh.order(fea.GP_WEIGHT)),
                        ("learned_lpt", lambda: bh.order(fea.LEARNED, torch.from_numpy(pred.astype(np.float32)).cuda())),
                        ("learned_classes", lambda: bh.order(fea.LEARNED_CLASSES,
                                                             torch.from_numpy(pred.astype(np.float32)).cuda())),
                        ("learned_static", lambda: bh.partition(fea.LEARNED,
                                                                torch.from_numpy(pred.astype(np.float32)).cuda()))):
        setup()
        ts = []
        for _ in range(5):
            bh.assemble(precision=fea.MIXED, out_dtype=fea.F32, vals=v, rhs=r, status=s, variant=fea.ROWSYM,
                        timing=True)
            ts.append(bh.last_ms())
        times[name] = float(np.median(ts))
    print(f"[held-out] r2 learned {r2l:.3f} gp {r2g:.3f}; 8-way split LB learned {lbl:.3f} gp {lbg:.3f}; "
          f"persistent kernel ms {times}", flush=True)
    assert lbl >= 0.85 and lbl > lbg + 0.2, (lbl, lbg)
