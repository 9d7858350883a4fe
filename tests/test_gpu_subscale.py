"""GPU parity of the element-wise subgrid scale (fea_subscale) against the CPU
oracle, through the C ABI.

Tolerance: every Gauss-point value is tau_e (f_e + L(u_h)); the second
derivatives in L come from sums of size |u| (reference coordinates) that
cancel, then two products with J^-1, and tau_e ~ h_e^2 / (4k) undoes the
1/h^2 of J^-1 J^-T. The rounding error of a value is therefore a small
multiple (the operation count times cond(J)^2, both < 100 on these meshes)
of eps times tau_e |f_e| + (lam_e + 2 mu_e) / (4 k_e) max_a |u_a|, and the
test allows 1e-11 times that scale (with |out| standing in for tau_e |f_e|
plus the L part). A wrong term, sign, index or transpose changes values at
O(1) of that scale."""
import ctypes

import numpy as np
import pytest

import meshgen as mg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1805_03949_amd as fea  # noqa: E402


def _mesh(name):
    if name == "bands8_jitter":
        return mg.hybrid_bands(8, seed=21, jitter=0.2)
    if name == "mix6_jitter":
        ct = np.random.default_rng(22).integers(0, 4, 6 ** 3).astype(np.uint8)
        return mg.cube_mesh(6, ct, jitter=0.25, seed=23)
    if name == "hetero16":
        return mg.heterogeneous(16, seed=24, brick=4, jitter=0.1)
    # 5^3 cells of one family: 750 tet4 / 750 pyr5 / 250 pen6 / 125 hex8
    # elements, none a multiple of its workgroup's 256 / 32 / 42 / 32
    fam = {"tet_ragged": mg.TET4, "pyr_ragged": mg.PYR5, "pen_ragged": mg.PEN6, "hex_ragged": mg.HEX8}[name]
    return mg.cube_mesh(5, np.full(125, fam, dtype=np.uint8), jitter=0.2, seed=25)


MESHES = ["bands8_jitter", "mix6_jitter", "hetero16", "tet_ragged", "pyr_ragged", "pen_ragged", "hex_ragged"]
_cache = {}


def case(name):
    if name not in _cache:
        m = _mesh(name)
        m.source[:, 0] = np.random.default_rng(5).uniform(0.5, 1.5, m.n_elems)
        print(f"[case] {name}: E={m.n_elems} N={m.n_nodes}", flush=True)
        dm = fea.DeviceMesh(m, device="cuda:0")
        _cache[name] = (m, dm, dm.graph())
    return _cache[name]


def _scale(m, u, B, gp_ptr, model):
    """Per Gauss point: (lam + 2 mu) / (4 k) max_a |u_a| over the element."""
    un = np.abs(u.reshape(-1, B)).max(axis=1)
    ue = np.maximum.reduceat(un[m.conn], m.conn_ptr[:-1])
    if model == oracle.POISSON:
        c = np.full(m.n_elems, 0.25)
    else:
        E, nu = m.young, m.nu
        lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
        c = (lam + 2 * mu) / (4 * mu)
    return np.repeat(c * ue, np.diff(gp_ptr))


def check(m, dm, g, u, model):
    B = 1 if model == oracle.POISSON else 3
    gp_ref, ref = oracle.subscale(m, u, model=model)
    n_pts, gp_ptr = g.gauss_points()
    assert n_pts == ref.shape[0]
    assert np.array_equal(gp_ptr.cpu().numpy(), gp_ref)
    out, st = dm.subscale(g, torch.from_numpy(u).to(dm.x.device), model=model)
    torch.cuda.synchronize()
    assert int(st.item()) == -1
    got = out.cpu().numpy()
    assert got.shape == ref.shape
    tol = 1e-11 * (np.abs(ref) + _scale(m, u, B, gp_ref, model)[:, None])
    err = np.abs(got - ref)
    assert (err <= tol).all(), (float((err / tol).max()), int(np.argmax((err / tol).max(axis=1))))
    return got, ref


@pytest.mark.parametrize("model", [oracle.POISSON, oracle.ELASTIC])
@pytest.mark.parametrize("name", MESHES)
def test_subscale_fp64_parity(name, model):
    m, dm, g = case(name)
    B = 1 if model == oracle.POISSON else 3
    u = mg.smooth_field(m, B, seed=7, noise=0.3)
    check(m, dm, g, u, model)


def test_subscale_linear_field_is_tau_f():
    """A linear field is reproduced exactly by every element, so L(u_h) = 0
    and each element's Gauss points all hold tau_e f_e (the GPU path checked
    against this property directly, not only against the oracle)."""
    m, dm, g = case("mix6_jitter")
    X = np.stack([m.x, m.y, m.z], axis=1)
    u = (X @ np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.2], [0.1, 0.0, -0.3]]).T).reshape(-1)
    out, st = dm.subscale(g, torch.from_numpy(u).cuda(), model=fea.ELASTIC)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    gp = g.gauss_points()[1].cpu().numpy()
    for e in range(0, m.n_elems, 7):
        blk = got[gp[e]:gp[e + 1]]
        tau_f = blk[0]
        # tau_e > 0 times f_e, the same at every Gauss point of the element
        np.testing.assert_allclose(blk, np.tile(tau_f, (len(blk), 1)), rtol=0, atol=1e-12 * np.abs(tau_f).max())
        f = m.source[e]
        nz = f != 0
        ratio = tau_f[nz] / f[nz]
        assert np.all(ratio > 0) and np.ptp(ratio) <= 1e-12 * ratio.max()
        assert np.abs(tau_f[~nz]).max(initial=0.0) <= 1e-12 * ratio.max()


def test_subscale_is_bitwise_repeatable():
    m, dm, g = case("bands8_jitter")
    u = torch.from_numpy(mg.smooth_field(m, 3, seed=8, noise=0.3)).cuda()
    a, _ = dm.subscale(g, u)
    b, _ = dm.subscale(g, u)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_subscale_inverted_element_sets_status():
    m = mg.cube_mesh(3, np.full(27, mg.HEX8, dtype=np.uint8))
    e = 13
    c = m.conn.copy()
    p0 = m.conn_ptr[e]
    c[p0:p0 + 4], c[p0 + 4:p0 + 8] = m.conn[p0 + 4:p0 + 8].copy(), m.conn[p0:p0 + 4].copy()
    m.conn = c
    with pytest.raises(oracle.MeshError) as ei:
        oracle.subscale(m, np.zeros(3 * m.n_nodes))
    assert ei.value.elem == e
    dm = fea.DeviceMesh(m)
    g = dm.graph()
    _, st = dm.subscale(g, torch.zeros(3 * m.n_nodes, dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    assert int(st.item()) == e


def test_subscale_empty_mesh():
    d = "cuda:0"
    types = torch.empty(0, dtype=torch.uint8, device=d)
    cp = torch.zeros(1, dtype=torch.int64, device=d)
    conn = torch.empty(0, dtype=torch.int32, device=d)
    g = fea.Graph(10, types, cp, conn)
    n, gp_ptr = g.gauss_points()
    assert n == 0 and gp_ptr.cpu().tolist() == [0]
    x = torch.zeros(10, dtype=torch.float64, device=d)
    out, st = fea.subscale(g, x, x, x, x, torch.empty(0, dtype=torch.float64, device=d), model=fea.POISSON)
    torch.cuda.synchronize()
    assert out.numel() == 0 and int(st.item()) == -1


def test_subscale_rejects_neo_hookean_and_bad_model():
    m, dm, g = case("tet_ragged")
    u = torch.zeros(3 * m.n_nodes, dtype=torch.float64, device="cuda:0")
    n, _ = g.gauss_points()
    out = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
    P = ctypes.c_void_p
    for mat in (fea.Material(fea.ELASTIC, P(dm.young.data_ptr()), P(dm.nu.data_ptr()),
                             P(dm.nh_flag.data_ptr()), None, 0),
                fea.Material(5, None, None, None, None, 0),
                fea.Material(fea.ELASTIC, None, None, None, None, 0)):  # nu missing
        rc = fea._lib.fea_subscale(g.handle, P(dm.x.data_ptr()), P(dm.y.data_ptr()), P(dm.z.data_ptr()),
                                   ctypes.byref(mat), P(u.data_ptr()), P(dm.source.data_ptr()),
                                   fea._stream(None), P(out.data_ptr()), None)
        assert rc == fea.FEA_EINVAL


def test_batched_subscale_equals_one_mesh_bitwise():
    """The batched form (persistent workgroups fed by per-family queues of
    its own items) computes each element exactly as the one-mesh form:
    outputs are equal bit for bit, mesh by mesh, and stay so when the
    assembly's tile sizes change."""
    meshes = mg.batched(n_meshes=5, seed=31, n_range=(3, 7), jitter=0.2, first_seed=900)
    dms = []
    for k, m in enumerate(meshes):
        m.u = mg.smooth_field(m, 3, seed=40 + k, noise=0.3)
        dms.append(fea.DeviceMesh(m))
    b = fea.Batch(dms, model=fea.ELASTIC)
    off = b.gauss_points()
    refs = []
    for dm in dms:
        g = dm.graph()
        out, st = dm.subscale(g, dm.u)
        torch.cuda.synchronize()
        assert int(st.item()) == -1
        refs.append(out.cpu().numpy())
    assert int(off[-1]) == sum(r.shape[0] for r in refs)
    for tiles in (None, [25, 17, 12, 7]):
        if tiles is not None:
            b.set_tiles(tiles)
        out, st = b.subscale()
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == -1).all()
        got = out.cpu().numpy()
        for k, r in enumerate(refs):
            assert np.array_equal(got[off[k]:off[k + 1]], r), (tiles, k)
    # oracle agreement of one mesh of the batch
    _, oref = oracle.subscale(meshes[2], meshes[2].u, model=oracle.ELASTIC)
    np.testing.assert_allclose(got[off[2]:off[3]], oref, rtol=1e-11, atol=1e-11 * np.abs(oref).max())


def test_batched_subscale_rejects_neo_hookean_batches():
    m = mg.heterogeneous(8, seed=6, brick=2, jitter=0.1)
    dm = fea.DeviceMesh(m)
    b = fea.Batch([dm], model=fea.ELASTIC, use_nh=True)
    with pytest.raises(fea.FeaError) as ei:
        b.subscale()
    assert ei.value.code == fea.FEA_EINVAL


def test_batched_subscale_of_an_empty_batch():
    b = fea.Batch([], model=fea.ELASTIC)
    assert b.gauss_points().tolist() == [0]
    out, st = b.subscale()
    torch.cuda.synchronize()
    assert out.shape == (0, 3) and st.numel() == 0
