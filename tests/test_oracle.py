"""Pins for the CPU oracle: it is checked against what the mathematics fixes
(closed forms, invariants, brute force, an independent dense formulation),
never against itself or the GPU library."""
import itertools

import numpy as np
import pytest

import meshgen as mg
import oracle
from oracle import dense

TET4, PYR5, PEN6, HEX8 = 0, 1, 2, 3

REF_NODES = {
    TET4: np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float),
    HEX8: np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                    [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], float),
    PEN6: np.array([[0, 0, -1], [1, 0, -1], [0, 1, -1], [0, 0, 1], [1, 0, 1], [0, 1, 1]], float),
    PYR5: np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1], [0, 0, 1]], float),
}
REF_VOLUME = {TET4: 1 / 6, HEX8: 8.0, PEN6: 1.0, PYR5: 8.0}


def random_ref_point(t, rng):
    if t == TET4:
        p = rng.dirichlet(np.ones(4))
        return p[1:]
    if t == PEN6:
        p = rng.dirichlet(np.ones(3))
        return np.array([p[1], p[2], rng.uniform(-1, 1)])
    return rng.uniform(-1, 1, 3)


# ---------------------------------------------------------------- reference elements

@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_partition_of_unity_and_kronecker(t):
    rng = np.random.default_rng(0)
    for _ in range(20):
        N, dN = oracle.shape(t, random_ref_point(t, rng))
        assert abs(N.sum() - 1) < 1e-14
        assert np.abs(dN.sum(axis=0)).max() < 1e-14
    for b, xb in enumerate(REF_NODES[t]):
        N, _ = oracle.shape(t, xb)
        np.testing.assert_allclose(N, np.eye(len(N))[b], atol=1e-15)


@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_shape_gradients_central_difference(t):
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(10):
        xi = random_ref_point(t, rng) * 0.9
        _, dN = oracle.shape(t, xi)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            fd = (oracle.shape(t, xi + e)[0] - oracle.shape(t, xi - e)[0]) / (2 * h)
            np.testing.assert_allclose(dN[:, j], fd, atol=1e-9)


@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_rule_weights_and_exactness(t):
    pts, w = oracle.rule(t)
    assert len(w) == {TET4: 1, PYR5: 8, PEN6: 6, HEX8: 8}[t]
    assert abs(w.sum() - REF_VOLUME[t]) < 1e-14
    if t in (HEX8, PYR5):
        # 2-point Gauss per axis is exact for x^2 y^2 z^2 over [-1,1]^3: (2/3)^3
        assert abs((w * (pts ** 2).prod(axis=1)).sum() - (2 / 3) ** 3) < 1e-14
    if t == PEN6:
        # integral of r^2 over the triangle (1/12) times integral of t^2 (2/3)
        assert abs((w * pts[:, 0] ** 2 * pts[:, 2] ** 2).sum() - (1 / 12) * (2 / 3)) < 1e-14
        assert abs((w * pts[:, 0] * pts[:, 1]).sum() - (1 / 24) * 2) < 1e-14
    if t == TET4:
        # a linear function is integrated exactly: int r over the unit tet = 1/24
        assert abs((w * pts[:, 0]).sum() - 1 / 24) < 1e-15


# ---------------------------------------------------------------- closed forms

def _box_hex(hx, hy, hz, x0=(0.3, -0.2, 0.1)):
    s = REF_NODES[HEX8]
    return np.array(x0) + (s + 1) / 2 * np.array([hx, hy, hz])


def _k1(h):
    return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h


def _m1(h):
    return h * np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])


C1D = np.array([[-0.5, -0.5], [0.5, 0.5]])   # int phi'_a phi_b on an interval


def test_hex8_poisson_box_closed_form():
    hx, hy, hz = 0.7, 1.3, 0.4
    K, fe = oracle.element(HEX8, _box_hex(hx, hy, hz), model=oracle.POISSON)
    bits = ((REF_NODES[HEX8] + 1) / 2).astype(int)
    h = (hx, hy, hz)
    Kx = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            v = 0.0
            for d in range(3):
                term = 1.0
                for e in range(3):
                    M = _k1(h[e]) if e == d else _m1(h[e])
                    term *= M[bits[a, e], bits[b, e]]
                v += term
            Kx[a, b] = v
    np.testing.assert_allclose(K, Kx, rtol=0, atol=1e-14)
    np.testing.assert_allclose(fe, np.full(8, hx * hy * hz / 8), atol=1e-15)


def test_hex8_poisson_unit_cube_values():
    K, _ = oracle.element(HEX8, _box_hex(1, 1, 1), model=oracle.POISSON)
    assert abs(K[0, 0] - 1 / 3) < 1e-15
    assert abs(K[0, 1]) < 1e-15            # edge neighbour
    assert abs(K[0, 2] + 1 / 12) < 1e-15   # face diagonal
    assert abs(K[0, 6] + 1 / 12) < 1e-15   # body diagonal


def test_hex8_elasticity_box_closed_form():
    hx, hy, hz = 0.5, 0.8, 1.1
    young, nu = 2.0, 0.27
    lam = young * nu / ((1 + nu) * (1 - 2 * nu))
    mu = young / (2 * (1 + nu))
    K, _ = oracle.element(HEX8, _box_hex(hx, hy, hz), young=young, nu=nu)
    bits = ((REF_NODES[HEX8] + 1) / 2).astype(int)
    h = (hx, hy, hz)

    def integ(a, b, i, j):
        """int dN_a/dx_i dN_b/dx_j over the box, by tensor products."""
        v = 1.0
        for d in range(3):
            A, B = bits[a, d], bits[b, d]
            if d == i and d == j:
                v *= _k1(h[d])[A, B]
            elif d == i:
                v *= C1D[A, B]
            elif d == j:
                v *= C1D[B, A]
            else:
                v *= _m1(h[d])[A, B]
        return v

    Kx = np.zeros((24, 24))
    for a in range(8):
        for b in range(8):
            dot = sum(integ(a, b, k, k) for k in range(3))
            for i in range(3):
                for j in range(3):
                    Kx[3 * a + i, 3 * b + j] = (lam * integ(a, b, i, j) + mu * integ(a, b, j, i)
                                                + (mu * dot if i == j else 0.0))
    np.testing.assert_allclose(K, Kx, rtol=0, atol=1e-14)


def _barycentric_gradients(X):
    """Gradients of the P1 barycentric functions of a tetrahedron (linear solve)."""
    M = np.hstack([np.ones((4, 1)), X])
    Minv = np.linalg.inv(M)
    return Minv[1:, :].T, abs(np.linalg.det(M)) / 6.0


def test_tet4_closed_forms():
    rng = np.random.default_rng(3)
    Xr = REF_NODES[TET4]
    K, fe = oracle.element(TET4, Xr, model=oracle.POISSON)
    Kx = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6
    np.testing.assert_allclose(K, Kx, atol=1e-15)
    np.testing.assert_allclose(fe, np.full(4, 1 / 24), atol=1e-16)
    for _ in range(5):
        X = Xr + rng.uniform(-0.15, 0.15, (4, 3))
        Gb, V = _barycentric_gradients(X)
        K, fe = oracle.element(TET4, X, model=oracle.POISSON)
        np.testing.assert_allclose(K, V * Gb @ Gb.T, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(fe, np.full(4, V / 4), rtol=1e-13)
        # elasticity: V * B^T D B with a hand-built Voigt B
        B = dense.voigt_B(Gb)
        D = dense.voigt_D(1.0, 0.3)
        K, fe = oracle.element(TET4, X, young=1.0, nu=0.3)
        np.testing.assert_allclose(K, V * B.T @ D @ B, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(fe.reshape(4, 3), np.tile([0, 0, -V / 4], (4, 1)), atol=1e-15)


def test_pen6_right_prism_closed_form():
    Lz = 0.6
    tri = np.array([[0.1, 0.2], [0.9, 0.3], [0.4, 1.0]])
    X = np.array([[tri[k, 0], tri[k, 1], z] for z in (0.0, Lz) for k in range(3)])
    K, fe = oracle.element(PEN6, X, model=oracle.POISSON)
    M = np.hstack([np.ones((3, 1)), tri])
    A = abs(np.linalg.det(M)) / 2
    G = np.linalg.inv(M)[1:, :].T
    k_tri = A * G @ G.T
    m_tri = A / 12 * np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]])
    Kx = np.kron(_m1(Lz), k_tri) + np.kron(_k1(Lz), m_tri)
    np.testing.assert_allclose(K, Kx, rtol=0, atol=1e-14)
    np.testing.assert_allclose(fe, np.full(6, A * Lz / 6), atol=1e-15)


def test_pyr5_square_pyramid_rhs_and_volume():
    side, height = 0.8, 0.5
    X = np.array([[0, 0, 0], [side, 0, 0], [side, side, 0], [0, side, 0],
                  [side / 2, side / 2, height]])
    _, fe = oracle.element(PYR5, X, model=oracle.POISSON)
    V = side * side * height / 3
    np.testing.assert_allclose(fe[4], V / 4, rtol=1e-14)
    np.testing.assert_allclose(fe[:4], np.full(4, 3 * V / 16), rtol=1e-14)
    assert abs(fe.sum() - V) < 1e-15


# ---------------------------------------------------------------- meshes / graph

def small_meshes():
    out = {}
    out["hex_jitter"] = mg.tiny_mesh(np.full((3, 3, 3), HEX8), jitter=0.2, seed=5)
    out["hex_jitter"].source[:, 0] = 1.0     # Poisson source f = 1 in column 0
    out["bands"] = mg.hybrid_bands(4, seed=6)
    ct = np.random.default_rng(7).integers(0, 4, (3, 3, 3))
    out["random_mix_jitter"] = mg.tiny_mesh(ct, jitter=0.25, seed=8)
    return out


def brute_force_pattern(mesh):
    rows = [set() for _ in range(mesh.n_nodes)]
    for e in range(mesh.n_elems):
        nodes = mesh.conn[mesh.conn_ptr[e]:mesh.conn_ptr[e + 1]]
        for a in nodes:
            for b in nodes:
                rows[a].add(int(b))
    return rows


@pytest.mark.parametrize("name", ["hex_jitter", "bands", "random_mix_jitter"])
def test_graph_brute_force(name):
    m = small_meshes()[name]
    g = oracle.mesh_graph(m)
    rows = brute_force_pattern(m)
    for i in range(m.n_nodes):
        cols = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert list(cols) == sorted(rows[i])
        assert i in cols
    # e2nnz points at the right (row, col), and the inverse map is its inverse
    rowof = np.repeat(np.arange(m.n_nodes), np.diff(g.row_ptr))
    for e in range(m.n_elems):
        nodes = m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]]
        nn = len(nodes)
        for a, b in itertools.product(range(nn), range(nn)):
            k = g.e2nnz[g.map_ptr[e] + a * nn + b]
            assert rowof[k] == nodes[a] and g.col[k] == nodes[b]
    slot_elem = np.repeat(np.arange(m.n_elems), np.diff(g.map_ptr))
    for k in range(g.nnz):
        sl = g.inv[g.inv_ptr[k]:g.inv_ptr[k + 1]]
        assert np.all(g.e2nnz[sl] == k)
        assert np.all(np.diff(slot_elem[sl]) > 0)
    assert g.inv_ptr[-1] == m.map_len()
    assert np.array_equal(np.sort(g.inv), np.arange(m.map_len()))


def test_hex_grid_nnz_closed_form():
    for n in (2, 5):
        m = mg.tiny_mesh(np.full((n, n, n), HEX8), dofs=1)
        g = oracle.mesh_graph(m)
        assert g.nnz == (3 * (n + 1) - 2) ** 3


def test_invalid_connectivity_is_reported():
    m = small_meshes()["bands"]
    bad = m.conn.copy()
    e = 17
    bad[m.conn_ptr[e] + 1] = bad[m.conn_ptr[e]]          # repeated node
    with pytest.raises(oracle.MeshError) as ei:
        oracle.graph(m.n_nodes, m.types, m.conn_ptr, bad)
    assert ei.value.elem == e
    bad = m.conn.copy()
    bad[m.conn_ptr[40]] = m.n_nodes                       # out of range
    with pytest.raises(oracle.MeshError) as ei:
        oracle.graph(m.n_nodes, m.types, m.conn_ptr, bad)
    assert ei.value.elem == 40
    t = m.types.copy()
    t[3] = 9                                              # unknown type
    with pytest.raises(oracle.MeshError) as ei:
        oracle.graph(m.n_nodes, t, m.conn_ptr, m.conn)
    assert ei.value.elem == 3


def test_inverted_element_is_reported():
    m = mg.tiny_mesh(np.full((2, 2, 2), TET4))
    g = oracle.mesh_graph(m)
    e = 5
    c = m.conn.copy()
    c[m.conn_ptr[e] + 1], c[m.conn_ptr[e] + 2] = c[m.conn_ptr[e] + 2], c[m.conn_ptr[e] + 1]
    m.conn = c
    with pytest.raises(oracle.MeshError) as ei:
        oracle.assemble(m, oracle.mesh_graph(m))
    assert ei.value.elem == e
    del g


def test_greedy_colouring_valid_and_first_fit():
    m = small_meshes()["random_mix_jitter"]
    col, nc = oracle.colour_greedy(m.n_nodes, m.conn_ptr, m.conn)
    assert nc == col.max() + 1
    elems_of = [[] for _ in range(m.n_nodes)]
    for e in range(m.n_elems):
        for v in m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]]:
            elems_of[v].append(e)
    for e in range(m.n_elems):
        nb = {o for v in m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]] for o in elems_of[v] if o != e}
        assert all(col[o] != col[e] for o in nb)
        earlier = {int(col[o]) for o in nb if o < e}
        assert col[e] == min(set(range(len(earlier) + 1)) - earlier)


# ---------------------------------------------------------------- invariants

def _dense(m, model):
    g = oracle.mesh_graph(m)
    vals, rhs = oracle.assemble(m, g, model=model)
    B = 1 if model == oracle.POISSON else 3
    return oracle.to_dense(g, vals, B, m.n_nodes), rhs, g


@pytest.mark.parametrize("name", ["hex_jitter", "bands", "random_mix_jitter"])
def test_cross_oracle_dense_voigt(name):
    m = small_meshes()[name]
    for model in (oracle.POISSON, oracle.ELASTIC):
        A, b, _ = _dense(m, model)
        Ad, bd = dense.assemble_dense(m, poisson=(model == oracle.POISSON))
        scale = np.abs(Ad).max()
        assert np.abs(A - Ad).max() <= 1e-13 * scale
        assert np.abs(b - bd).max() <= 1e-13 * np.abs(bd).max()


def test_volume_and_rhs_sum():
    m = small_meshes()["hex_jitter"]       # conforming jittered hexes: volume 1
    A, b, _ = _dense(m, oracle.POISSON)
    assert abs(b.sum() - 1.0) < 1e-13
    m = small_meshes()["bands"]            # unjittered hybrid: volume 1
    A, b, _ = _dense(m, oracle.ELASTIC)
    np.testing.assert_allclose(b.reshape(-1, 3).sum(axis=0), [0, 0, -1.0], atol=1e-13)


@pytest.mark.parametrize("name", ["hex_jitter", "bands", "random_mix_jitter"])
def test_poisson_row_sums_and_symmetry(name):
    m = small_meshes()[name]
    A, _, _ = _dense(m, oracle.POISSON)
    scale = np.abs(A).max()
    assert np.abs(A.sum(axis=1)).max() < 1e-14 * 64 * scale
    assert np.abs(A - A.T).max() < 1e-15 * 8 * scale


@pytest.mark.parametrize("name", ["hex_jitter", "bands", "random_mix_jitter"])
def test_elasticity_rigid_modes_and_symmetry(name):
    m = small_meshes()[name]
    A, _, _ = _dense(m, oracle.ELASTIC)
    X = np.stack([m.x, m.y, m.z], axis=1)
    modes = []
    for i in range(3):
        t = np.zeros_like(X)
        t[:, i] = 1.0
        modes.append(t.ravel())
    for w in np.eye(3):
        modes.append(np.cross(w, X).ravel())
    scale = np.abs(A).max()
    for r in modes:
        assert np.abs(A @ r).max() < 1e-13 * scale * np.abs(r).max()
    assert np.abs(A - A.T).max() < 1e-14 * scale
    # and nothing else: exactly six zero eigenvalues
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert np.sum(np.abs(ev) < 1e-10 * scale) == 6


@pytest.mark.parametrize("ctype", [HEX8, TET4, PYR5, PEN6])
def test_patch_test_linear_field(ctype):
    m = mg.tiny_mesh(np.full((3, 3, 3), ctype), jitter=0.2, seed=11)
    m.nu[:] = 0.3
    X = np.stack([m.x, m.y, m.z], axis=1)
    interior = ~m.boundary
    G = np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.2], [0.1, 0.0, -0.3]])
    u = X @ G.T + np.array([0.1, 0.2, 0.3])
    A, _, _ = _dense(m, oracle.ELASTIC)
    r = (A @ u.ravel()).reshape(-1, 3)
    assert np.abs(r[interior]).max() < 1e-13 * np.abs(A).max()
    Ap, _, _ = _dense(m, oracle.POISSON)
    rp = Ap @ (X @ np.array([0.7, -0.3, 0.2]))
    assert np.abs(rp[interior]).max() < 1e-13 * np.abs(Ap).max()


def test_patch_test_conforming_prism_tet_interface():
    ct = np.zeros((4, 4, 4), dtype=np.uint8)
    ct[:2] = PEN6
    ct[2:] = TET4
    m = mg.tiny_mesh(ct, jitter=0.15, seed=12)
    m.nu[:] = 0.25
    X = np.stack([m.x, m.y, m.z], axis=1)
    A, _, _ = _dense(m, oracle.ELASTIC)
    u = X @ np.array([[0.2, 0.1, 0], [0, -0.3, 0.1], [0.1, 0.2, 0.3]]).T
    r = (A @ u.ravel()).reshape(-1, 3)
    assert np.abs(r[~m.boundary]).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_covariance(t):
    rng = np.random.default_rng(20 + t)
    X = REF_NODES[t] * 0.3 + rng.uniform(-0.03, 0.03, REF_NODES[t].shape)
    K, fe = oracle.element(t, X, young=1.3, nu=0.31)
    Kt, fet = oracle.element(t, X + np.array([5.0, -2.0, 1.0]), young=1.3, nu=0.31)
    np.testing.assert_allclose(Kt, K, atol=1e-12 * np.abs(K).max())
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    R = q * np.sign(np.linalg.det(q))
    Kr, _ = oracle.element(t, X @ R.T, young=1.3, nu=0.31)
    nn = len(X)
    Rb = np.kron(np.eye(nn), R)
    np.testing.assert_allclose(Kr, Rb @ K @ Rb.T, atol=1e-13 * np.abs(K).max())
    s = 2.5
    Kp, fp = oracle.element(t, X, model=oracle.POISSON)
    Ks, fs = oracle.element(t, X * s, model=oracle.POISSON)
    np.testing.assert_allclose(Ks, s * Kp, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(fs, s ** 3 * fp, rtol=1e-13)


# ---------------------------------------------------------------- neo-Hookean

@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_neo_hookean_reduces_to_linear_at_identity(t):
    rng = np.random.default_rng(30 + t)
    X = REF_NODES[t] * 0.2 + rng.uniform(-0.02, 0.02, REF_NODES[t].shape)
    Kl, _ = oracle.element(t, X, young=1.0, nu=0.3)
    Kn, _ = oracle.element(t, X, young=1.0, nu=0.3, nh=True, u=np.zeros_like(X))
    np.testing.assert_allclose(Kn, Kl, atol=1e-15 * 10 * np.abs(Kl).max())


@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_neo_hookean_tangent_is_derivative_of_internal_force(t):
    rng = np.random.default_rng(40 + t)
    X = REF_NODES[t] * 0.2 + rng.uniform(-0.02, 0.02, REF_NODES[t].shape)
    u = rng.uniform(-0.02, 0.02, X.shape)
    young, nu = 1.0, 0.32
    K, _ = oracle.element(t, X, young=young, nu=nu, nh=True, u=u)
    nn = len(X)
    h = 1e-7
    fd = np.zeros((3 * nn, 3 * nn))
    for c in range(3 * nn):
        du = np.zeros(3 * nn)
        du[c] = h
        fp = oracle.element_fint(t, X, young, nu, (u.ravel() + du).reshape(nn, 3))
        fm = oracle.element_fint(t, X, young, nu, (u.ravel() - du).reshape(nn, 3))
        fd[:, c] = (fp - fm) / (2 * h)
    assert np.abs(K - fd).max() <= 1e-6 * np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    for i in range(3):
        tr = np.zeros((nn, 3))
        tr[:, i] = 1.0
        assert np.abs(K @ tr.ravel()).max() <= 1e-13 * np.abs(K).max()


def test_neo_hookean_internal_force_zero_at_rest():
    X = REF_NODES[HEX8] * 0.2
    f = oracle.element_fint(HEX8, X, 1.0, 0.3, np.zeros((8, 3)))
    assert np.abs(f).max() < 1e-16


# ---------------------------------------------------------------- FP32 bound companion

def test_term_sums_bound_values():
    m = small_meshes()["random_mix_jitter"]
    g = oracle.mesh_graph(m)
    v, r, tv, tr = oracle.assemble(m, g, with_terms=True)
    assert np.all(tv >= np.abs(v) * (1 - 1e-12))
    assert np.all(tr >= np.abs(r) * (1 - 1e-12))
    # Poisson diagonal entries are sums of non-negative terms: T == value
    vp, _, tvp, _ = oracle.assemble(m, g, model=oracle.POISSON, with_terms=True)
    diag = [np.searchsorted(g.col[g.row_ptr[i]:g.row_ptr[i + 1]], i) + g.row_ptr[i]
            for i in range(m.n_nodes)]
    np.testing.assert_allclose(tvp[diag], vp[diag], rtol=1e-14)


def _lame(young, nu):
    return young * nu / ((1 + nu) * (1 - 2 * nu)), young / (2 * (1 + nu))


def _tet_term_closed_form(G, V, lam, mu, c, s):
    """|term| sums of a one-point tet4 element with gradient rows G (barycentric,
    from a linear solve) and volume V, for the tangent lam_eff |G_ai G_bj| +
    |c| |G_aj G_bi| + mu d_ij sum_k |G_ak G_bk|, where the deformation
    F = s I scales every pushed gradient by 1/s (s = 1, c = mu: linear)."""
    A = np.abs(G)
    T = np.zeros((12, 12))
    for a in range(4):
        for b in range(4):
            dot = (A[a] * A[b]).sum()
            for i in range(3):
                for j in range(3):
                    T[3 * a + i, 3 * b + j] = V * (lam * A[a, i] * A[b, j] / s ** 2
                                                   + abs(c) * A[a, j] * A[b, i] / s ** 2
                                                   + (mu * dot if i == j else 0.0))
    return T


def test_term_sums_tet4_closed_form_from_above():
    """T pinned from above on a perturbed tet4 (one Gauss point, weight 1/6,
    det J = 6V): Poisson V sum_k |G_ak G_bk|, elasticity V (lam |G_ai G_bj| +
    mu |G_aj G_bi| + d_ij mu sum_k |G_ak G_bk|), right-hand side V/4 |f_i|.
    A T too large by any factor fails here, not only one too small."""
    rng = np.random.default_rng(41)
    young, nu = 1.3, 0.31
    lam, mu = _lame(young, nu)
    for _ in range(4):
        X = REF_NODES[TET4] + rng.uniform(-0.2, 0.2, (4, 3))
        G, V = _barycentric_gradients(X)
        _, _, Tp, Tfp = oracle.element(TET4, X, model=oracle.POISSON, with_terms=True)
        np.testing.assert_allclose(Tp, V * np.abs(G) @ np.abs(G).T, rtol=1e-13)
        np.testing.assert_allclose(Tfp, np.full(4, V / 4), rtol=1e-13)
        f = np.array([0.3, -2.0, 0.7])
        _, _, T, Tf = oracle.element(TET4, X, young=young, nu=nu, f=f, with_terms=True)
        np.testing.assert_allclose(T, _tet_term_closed_form(G, V, lam, mu, mu, 1.0), rtol=1e-13)
        np.testing.assert_allclose(Tf.reshape(4, 3), np.tile(V / 4 * np.abs(f), (4, 1)), rtol=1e-13)


@pytest.mark.parametrize("eps", [0.0, 0.1, -0.12, 0.35])
def test_term_sums_neo_hookean_tet4_dilation(eps):
    """Neo-Hookean T, its three tangent parts summed in absolute value, on a
    tet4 under the uniform dilation u = eps X: F = (1 + eps) I, so
    F^-1 = I / (1 + eps) and ln det F = 3 ln(1 + eps), and T is the linear
    closed form with lam and |mu - lam ln J| scaled by (1 + eps)^-2. eps = 0
    is the identity (T equals the linear T); eps = 0.35 makes
    mu - lam ln J negative, which only its absolute value survives."""
    rng = np.random.default_rng(42)
    young, nu = 1.0, 0.3
    lam, mu = _lame(young, nu)
    X = REF_NODES[TET4] + rng.uniform(-0.15, 0.15, (4, 3))
    G, V = _barycentric_gradients(X)
    s = 1.0 + eps
    c = mu - lam * 3 * np.log(s)
    if eps == 0.35:
        assert c < 0
    _, _, T, _ = oracle.element(TET4, X, young=young, nu=nu, nh=True, u=eps * X, with_terms=True)
    np.testing.assert_allclose(T, _tet_term_closed_form(G, V, lam, mu, c, s), rtol=1e-12)
    if eps == 0.0:
        _, _, Tl, _ = oracle.element(TET4, X, young=young, nu=nu, with_terms=True)
        np.testing.assert_allclose(T, Tl, rtol=1e-14)


@pytest.mark.parametrize("t", [PYR5, PEN6, HEX8])
def test_term_sums_neo_hookean_equal_linear_at_rest(t):
    """At u = 0 every neo-Hookean tangent part reduces to its linear
    counterpart (F = I, ln det F = 0), so the two T agree for every family."""
    rng = np.random.default_rng(50 + t)
    X = REF_NODES[t] * 0.2 + rng.uniform(-0.02, 0.02, REF_NODES[t].shape)
    _, _, Tl, _ = oracle.element(t, X, young=1.0, nu=0.3, with_terms=True)
    _, _, Tn, _ = oracle.element(t, X, young=1.0, nu=0.3, nh=True, u=np.zeros_like(X), with_terms=True)
    np.testing.assert_allclose(Tn, Tl, rtol=1e-13)


def test_term_sums_hex8_box_closed_form():
    """Eight Gauss points: on an axis-aligned box every product term
    dN_a/dx_i dN_b/dx_j keeps one sign inside the element, so its sum of
    absolute values over the exact rule is the absolute value of its
    integral, a product of 1D stiffness, mass and coupling matrices:
    T = lam |I_ij| + mu |I_ji| + d_ij mu sum_k |I_kk| (Poisson: sum_k |I_kk|)."""
    hx, hy, hz = 0.6, 1.1, 0.45
    young, nu = 1.7, 0.29
    lam, mu = _lame(young, nu)
    X = _box_hex(hx, hy, hz)
    bits = ((REF_NODES[HEX8] + 1) / 2).astype(int)
    h = (hx, hy, hz)

    def integ(a, b, i, j):
        v = 1.0
        for d in range(3):
            A, B = bits[a, d], bits[b, d]
            if d == i and d == j:
                v *= _k1(h[d])[A, B]
            elif d == i:
                v *= C1D[A, B]
            elif d == j:
                v *= C1D[B, A]
            else:
                v *= _m1(h[d])[A, B]
        return v

    Tx = np.zeros((24, 24))
    Tpx = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            adot = sum(abs(integ(a, b, k, k)) for k in range(3))
            Tpx[a, b] = adot
            for i in range(3):
                for j in range(3):
                    Tx[3 * a + i, 3 * b + j] = (lam * abs(integ(a, b, i, j)) + mu * abs(integ(a, b, j, i))
                                                + (mu * adot if i == j else 0.0))
    _, _, T, _ = oracle.element(HEX8, X, young=young, nu=nu, with_terms=True)
    np.testing.assert_allclose(T, Tx, rtol=1e-13, atol=1e-15)
    _, _, Tp, _ = oracle.element(HEX8, X, model=oracle.POISSON, with_terms=True)
    np.testing.assert_allclose(Tp, Tpx, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- paper fixture

def test_table2_load_balance_golden():
    """Element-count load balance (average/maximum, Section 4.1) from Table 2."""
    from oracle import sched
    rows = np.loadtxt(__file__.replace("test_oracle.py", "golden/table2_chunks.txt"))
    for row in rows:
        chunk = row[0]
        for p, (mx, mn, avg) in zip((256, 512, 1024), row[1:].reshape(3, 3)):
            # the average chunk count times chunk size times partitions is the mesh size
            if chunk == 100:
                assert abs(avg * chunk * p - 17.7e6) / 17.7e6 < 0.01
            assert mn <= avg <= mx
    r100 = rows[0][1:].reshape(3, 3)
    # non-weighted LB = average / maximum
    lbs = [avg / mx for mx, _, avg in r100]
    np.testing.assert_allclose(lbs, [0.345, 0.252, 0.247], atol=1e-3)
    assert abs(sched.load_balance([1.0, 2.0, 3.0]) - 6.0 / 9.0) < 1e-15


# ---------------------------------------------------------------- residual
def _with_u(m, seed, amp=0.03):
    rng = np.random.default_rng(seed)
    X = np.stack([m.x, m.y, m.z], axis=1)
    k, ph = rng.integers(1, 3, size=(3, 3)), rng.uniform(0, 2 * np.pi, size=3)
    u = amp * np.stack([np.sin(2 * np.pi * X @ k[i] + ph[i]) for i in range(3)], axis=1)
    m.u = u.reshape(-1).copy()
    return m


def test_parts_of_a_partition_sum_to_the_whole():
    """Assembly is a sum over elements (Algorithm 1), so the matrices and
    right-hand sides of the parts of any partition of the elements, each
    assembled as a mesh of its own and mapped back to the mesh's node ids,
    add up to the whole mesh's: the identity a split of the elements over
    several GPUs (each summing partial rows) rests on."""
    from tests.helpers import fp64_errors, scatter_part
    m = mg.heterogeneous(8, seed=4, brick=4)
    assert m.nh_flag.any() and not m.nh_flag.all()
    g = oracle.mesh_graph(m)
    v, r = oracle.assemble(m, g)
    part = np.random.default_rng(0).integers(0, 3, m.n_elems)
    acc, accr = np.zeros_like(v), np.zeros_like(r)
    for p in range(3):
        sub, nodes = mg.submesh(m, np.nonzero(part == p)[0], return_nodes=True)
        sg = oracle.mesh_graph(sub)
        sv, sr = oracle.assemble(sub, sg)
        scatter_part(np.asarray(g.row_ptr), np.asarray(g.col), nodes, np.asarray(sg.row_ptr), np.asarray(sg.col),
                     sv, 3, acc, sr, accr)
    ev, er = fp64_errors(acc, v, np.asarray(g.row_ptr), 3, accr, r)
    assert ev < 1e-13 and er < 1e-13, (ev, er)
    # a part left out is missed
    acc2 = acc.copy()
    sub, nodes = mg.submesh(m, np.nonzero(part == 0)[0], return_nodes=True)
    sg = oracle.mesh_graph(sub)
    sv, _ = oracle.assemble(sub, sg)
    scatter_part(np.asarray(g.row_ptr), np.asarray(g.col), nodes, np.asarray(sg.row_ptr), np.asarray(sg.col),
                 -sv, 3, acc2)
    assert fp64_errors(acc2, v, np.asarray(g.row_ptr), 3)[0] > 1e-3


def test_residual_at_rest_is_the_external_force():
    """f_int(0) = 0 for both materials (P(I) = 0, K u = 0): the residual at
    u = 0 is exactly the assembled right-hand side."""
    m = mg.heterogeneous(8, seed=5, brick=2, jitter=0.1)
    m.u = np.zeros_like(m.u)
    og = oracle.mesh_graph(m)
    _, rhs = oracle.assemble(m, og, model=oracle.ELASTIC)
    assert np.array_equal(oracle.residual(m), rhs)


def test_residual_of_a_linear_solid_is_f_minus_A_u():
    """Linear elasticity: f_int = K u, so the residual equals f - A u with
    the assembled global matrix."""
    m = _with_u(mg.hybrid_bands(4, seed=3, jitter=0.2), seed=4)
    og = oracle.mesh_graph(m)
    vals, rhs = oracle.assemble(m, og, model=oracle.ELASTIC, use_nh=False)
    A = oracle.to_dense(og, vals, 3, m.n_nodes)
    ref = rhs - A @ m.u
    r = oracle.residual(m, use_nh=False)
    assert np.abs(r - ref).max() <= 1e-12 * np.abs(A).max() * np.abs(m.u).max() * 10


def test_residual_internal_forces_sum_to_zero():
    """Every element's internal force sums to zero over its nodes (the shape
    functions sum to one), so the residual's total is the external force's."""
    m = mg.heterogeneous(8, seed=6, brick=2, jitter=0.1)
    og = oracle.mesh_graph(m)
    _, rhs = oracle.assemble(m, og, model=oracle.ELASTIC)
    r = oracle.residual(m)
    assert not np.allclose(r, rhs)  # the displacement field is not zero
    scale = np.abs(r).sum()
    for i in range(3):
        assert abs(r[i::3].sum() - rhs[i::3].sum()) <= 1e-12 * scale


# ---------------------------------------------------------------- subgrid scale
# The element-wise subgrid scale (Section 2.1.3), read for Poisson and linear
# elasticity: tau_e (f + L(u_h)) at every Gauss point, tau_e = V_e^(2/3)/(4k).

# physical volume of the element whose nodes sit at REF_NODES[t]
PHYS_VOLUME = {TET4: 1 / 6, PYR5: 8 / 3, PEN6: 1.0, HEX8: 8.0}


def _ref_map(t, xi):
    """Position of reference point xi in the element with nodes REF_NODES[t]:
    the identity for tet4, pen6 and hex8, the collapsed-hexahedron map for
    the pyramid (base at z = -1, apex at z = 1)."""
    r, s, z = xi
    if t == PYR5:
        return np.array([r * (1 - z) / 2, s * (1 - z) / 2, z])
    return np.array([r, s, z])


def _field(t, p, k):
    """Value and exact Hessian at p of a field that the family's shape
    functions represent exactly on the REF_NODES element (k picks one of
    three variants). tet4: linear only (zero Hessian)."""
    p1, p2, p3 = p
    c = [(1.0, 2.0, -1.0, 3.0), (-0.5, 1.0, 2.0, -1.0), (2.0, -1.5, 0.5, 1.0)][k]
    H = np.zeros((3, 3))
    if t == HEX8:   # multilinear
        v = c[0] * p1 * p2 + c[1] * p2 * p3 + c[2] * p1 * p3 + c[3] * p1 * p2 * p3
        H[0, 1] = c[0] + c[3] * p3
        H[1, 2] = c[1] + c[3] * p1
        H[0, 2] = c[2] + c[3] * p2
    elif t == PEN6:  # linear in (p1, p2) times linear in p3
        v = c[0] * p1 * p3 + c[1] * p2 * p3
        H[0, 2] = c[0]
        H[1, 2] = c[1]
    elif t == PYR5:  # the pyramid's rational mode p1 p2 / (1 - p3), 0 at the apex
        d = 1.0 - p3
        v = c[0] * p1 * p2 / d if d > 0 else 0.0
        if d > 0:  # Gauss points lie below the apex
            H[0, 1] = c[0] / d
            H[0, 2] = c[0] * p2 / d ** 2
            H[1, 2] = c[0] * p1 / d ** 2
            H[2, 2] = 2 * c[0] * p1 * p2 / d ** 3
    else:
        v = 0.0
    v += c[1] * p1 - c[2] * p2 + c[3] * p3 + c[0]
    return v, H + np.triu(H, 1).T


@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_subscale_closed_form_on_affine_images(t):
    """Affine image x = A p + b of the reference-node element (A not
    symmetric), field u(x) = phi(A^-1 (x - b)) with phi exactly
    representable: the physical Hessian is A^-T H_p A^-1 at every Gauss
    point, the volume |det A| times the reference volume."""
    rng = np.random.default_rng(40 + t)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    b = rng.standard_normal(3)
    Ai = np.linalg.inv(A)
    Xr = REF_NODES[t]
    X = Xr @ A.T + b
    pts, _ = oracle.rule(t)
    V = abs(np.linalg.det(A)) * PHYS_VOLUME[t]
    young, nu = 1.7, 0.28
    lam = young * nu / ((1 + nu) * (1 - 2 * nu))
    mu = young / (2 * (1 + nu))
    # Poisson
    u = np.array([_field(t, p, 0)[0] for p in Xr])
    got = oracle.element_subscale(t, X, u, model=oracle.POISSON, f=np.array([0.7]))
    tau = V ** (2 / 3) / 4
    for q, xi in enumerate(pts):
        Hx = Ai.T @ _field(t, _ref_map(t, xi), 0)[1] @ Ai
        assert abs(got[q, 0] - tau * (0.7 + np.trace(Hx))) <= 1e-13 * tau * (1 + np.abs(Hx).max())
    # elasticity: component i uses variant i
    u3 = np.array([[_field(t, p, i)[0] for i in range(3)] for p in Xr])
    f = np.array([0.1, -0.2, -1.0])
    got = oracle.element_subscale(t, X, u3, model=oracle.ELASTIC, young=young, nu=nu, f=f)
    tau = V ** (2 / 3) / (4 * mu)
    for q, xi in enumerate(pts):
        H = [Ai.T @ _field(t, _ref_map(t, xi), i)[1] @ Ai for i in range(3)]
        L = np.array([mu * np.trace(H[i]) + (lam + mu) * sum(H[k][i, k] for k in range(3)) for i in range(3)])
        scale = tau * (1 + (lam + mu) * max(np.abs(h).max() for h in H))
        np.testing.assert_allclose(got[q], tau * (f + L), rtol=0, atol=1e-13 * scale)
    if t != TET4:  # the closed forms are not trivially zero
        assert np.abs(got / tau - f).max() > 0.1


@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_subscale_of_linear_fields_on_distorted_elements(t):
    """Isoparametric elements reproduce linear fields, so L(u_h) = 0 on any
    valid element: at every Gauss point the subgrid scale is tau_e f. On a
    non-affine element this needs the geometric term of the second
    derivatives to cancel the reference ones exactly. V_e is taken from the
    element right-hand side (sum_a f_a = V_e f for f = 1)."""
    rng = np.random.default_rng(50 + t)
    X = REF_NODES[t] * 0.3 + rng.uniform(-0.04, 0.04, REF_NODES[t].shape)
    _, fe = oracle.element(t, X, model=oracle.POISSON, f=np.ones(1))
    V = fe.sum()
    G = rng.standard_normal((3, 3))
    u3 = X @ G.T + rng.standard_normal(3)
    f = np.array([0.3, 0.5, -1.0])
    young, nu = 2.1, 0.33
    mu = young / (2 * (1 + nu))
    got = oracle.element_subscale(t, X, u3, model=oracle.ELASTIC, young=young, nu=nu, f=f)
    tau = V ** (2 / 3) / (4 * mu)
    lam_mu = young * nu / ((1 + nu) * (1 - 2 * nu)) + mu
    # rounding of second derivatives of size |G| / h^2 amplified by lam + mu
    np.testing.assert_allclose(got, np.tile(tau * f, (len(got), 1)), rtol=0,
                               atol=1e-12 * tau * lam_mu * np.abs(G).max() / 0.3 ** 2)
    up = X @ G[0] + 0.4
    got = oracle.element_subscale(t, X, up, model=oracle.POISSON, f=np.array([2.0]))
    np.testing.assert_allclose(got[:, 0], V ** (2 / 3) / 4 * 2.0, rtol=1e-11)
    if t != TET4:  # the reference second derivatives alone do not vanish
        D2 = oracle.shape2(t, oracle.rule(t)[0][0])
        assert np.abs(np.einsum("ajl,a->jl", D2, up)).max() > 1e-3


@pytest.mark.parametrize("t", [TET4, PYR5, PEN6, HEX8])
def test_shape_second_derivatives_central_difference(t):
    rng = np.random.default_rng(60 + t)
    h = 1e-5
    for _ in range(3):
        xi = random_ref_point(t, rng) * 0.9
        D2 = oracle.shape2(t, xi)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            fd = (oracle.shape(t, xi + e)[1] - oracle.shape(t, xi - e)[1]) / (2 * h)
            np.testing.assert_allclose(D2[:, j, :], fd, atol=1e-8)


def test_subscale_mesh_layout_on_a_hex_grid():
    """Axis-aligned cubes and a global multilinear field: each element's
    interpolant is the field itself, so every Gauss point holds the exact
    tau_e (f_e + div sigma(u)) at its own position; Gauss points are laid
    out element by element in element order."""
    m = mg.tiny_mesh(np.full((3, 3, 3), HEX8), jitter=0.0, seed=13)
    rng = np.random.default_rng(7)
    m.young[:] = rng.uniform(1.0, 2.0, m.n_elems)
    m.nu[:] = rng.uniform(0.2, 0.35, m.n_elems)
    m.source = rng.standard_normal((m.n_elems, 3))
    X = np.stack([m.x, m.y, m.z], axis=1)
    x, y, z = X.T
    u = np.stack([x * y + 2 * x * y * z, y * z - x * z, x * z + 3 * x * y], axis=1)
    gp_ptr, got = oracle.subscale(m, u.reshape(-1), model=oracle.ELASTIC)
    assert np.array_equal(gp_ptr, 8 * np.arange(m.n_elems + 1))
    pts, _ = oracle.rule(HEX8)
    for e in range(m.n_elems):
        nodes = m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]]
        lo, hi = X[nodes].min(0), X[nodes].max(0)
        V = np.prod(hi - lo)
        E, nu = m.young[e], m.nu[e]
        lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
        tau = V ** (2 / 3) / (4 * mu)
        for q, xi in enumerate(pts):
            # the cube's nodes follow the reference order, so x = lo + (xi + 1)/2 (hi - lo)
            px, py, pz = lo + (xi + 1) / 2 * (hi - lo)
            # div u = y + 2yz + z + x; Lap u = 0 for multilinear components
            gdiv = np.array([1.0, 1.0 + 2 * pz, 1.0 + 2 * py])
            L = (lam + mu) * gdiv
            np.testing.assert_allclose(got[gp_ptr[e] + q], tau * (m.source[e] + L), rtol=1e-12,
                                       atol=1e-12 * tau * (lam + mu))


def test_subscale_mesh_volumes_and_scalar_field():
    """Unjittered hybrid bands: every element of a family has the same
    volume (h^3 for hex8, h^3/2 for pen6, h^3/6 for tet4 and pyr5); with a
    linear field L(u_h) = 0 and each Gauss point holds tau_e f_e."""
    n = 4
    m = mg.hybrid_bands(n, seed=3, jitter=0.0)
    h = 1.0 / n
    vol = {HEX8: h ** 3, PEN6: h ** 3 / 2, TET4: h ** 3 / 6, PYR5: h ** 3 / 6}
    X = np.stack([m.x, m.y, m.z], axis=1)
    m.source[:, 0] = np.random.default_rng(8).uniform(0.5, 1.5, m.n_elems)
    nq = {TET4: 1, PYR5: 8, PEN6: 6, HEX8: 8}
    up = X @ np.array([0.3, -0.7, 1.1]) + 0.2
    gp_ptr, got = oracle.subscale(m, up, model=oracle.POISSON)
    assert np.array_equal(np.diff(gp_ptr), [nq[int(t)] for t in m.types])
    for e in range(m.n_elems):
        tau = vol[int(m.types[e])] ** (2 / 3) / 4
        np.testing.assert_allclose(got[gp_ptr[e]:gp_ptr[e + 1], 0], tau * m.source[e, 0], rtol=1e-12)


# ---------------------------------------------------------------- parallel timing variants

@pytest.mark.parametrize("variant", ["atomic", "colour"])
def test_parallel_variants_equal_sequential_up_to_rounding(variant):
    """The OpenMP timing variants (Algorithm 4 atomics, Algorithm 5 colour
    sweeps) compute Algorithm 1's sums in another order: equal up to
    rounding, for linear elasticity, the neo-Hookean tangent and Poisson."""
    m = mg.heterogeneous(8, seed=71, brick=2, jitter=0.15)
    g = oracle.mesh_graph(m)
    for model, nh in ((oracle.ELASTIC, False), (oracle.ELASTIC, True), (oracle.POISSON, False)):
        v0, r0 = oracle.assemble(m, g, model=model, use_nh=nh)
        v1, r1 = oracle.assemble_parallel(m, g, variant, model=model, use_nh=nh)
        assert np.abs(v1 - v0).max() <= 1e-13 * np.abs(v0).max()
        assert np.abs(r1 - r0).max() <= 1e-13 * np.abs(r0).max()
    if variant == "colour":
        # the buckets hold every element once, and a colour's elements share no node
        colour, nc = oracle.colour_greedy(m.n_nodes, m.conn_ptr, m.conn)
        cptr, celems = oracle.colour_buckets(colour, nc)
        assert np.array_equal(np.sort(celems), np.arange(m.n_elems))
        for c in range(nc):
            es = celems[cptr[c]:cptr[c + 1]]
            nodes = np.concatenate([m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]] for e in es])
            assert np.unique(nodes).size == nodes.size
