"""CPU checks of the benchmark's work accounting (no GPU): the roofline's
flop and byte figures are sums that must add up."""
import numpy as np

import bench
import meshgen as mg


def test_class_flops_add_up_to_the_per_element_figures():
    m = mg.hybrid_bands(8, seed=2)
    alg, exe = bench.gather_class_flops(m, np)
    # every (row, element) pair carries 1/n of its element: the classes
    # together hold every element exactly once
    total = sum(bench.ELEMENT_FLOPS[t] for t in m.types)
    assert abs(sum(alg) - total) <= 1e-9 * total
    per_pair = [bench.gather_pair_flops(t) for t in range(4)]
    assert abs(sum(exe) - sum(per_pair[t] * bench.NODES[t] for t in m.types)) <= 1e-6 * sum(exe)
    # one-family bands: the four one-family classes hold most of the work
    assert sum(alg[:4]) > 0.6 * total


def test_pair_flop_formula_by_hand():
    # tet4: one Gauss point, four nodes: 1 * (18*4 + 77) + 4 * (33 + 33) + 4 * 9
    assert bench.gather_pair_flops(0) == 149 + 264 + 36
    # hex8: 8 * (18*8 + 77) + 8 * (8*33 + 33) + 8 * 9
    assert bench.gather_pair_flops(3) == 8 * 221 + 8 * 297 + 72


def test_reduce_bytes_definition():
    class G:
        map_len, nnz = 84_492_288, 22_156_129
    b = bench.reduce_bytes(G, 3, 8, 8)
    assert b == 84_492_288 * 72 + (22_156_129 + 1) * 8 + 22_156_129 * 72


def test_element_bytes_of_the_upper_triangle_form():
    """Element-phase bytes of the upper-triangle form: the inputs, then per
    tile-block its b^2 tile sums and 6 bytes of slot and end, 2 bytes per
    entry and 16 per tile; with 1x1 blocks also one right-hand-side value
    per element node, with 3x3 blocks none (the diagonal tile sums carry
    it)."""
    class G:
        map_len, nnz = 1000, 400
    sym = {"tile_blocks": 300, "entries": 500, "tiles": 20}
    N, E, L = 100, 40, 240
    for B, s_c in ((3, 8), (3, 4), (1, 8)):
        inputs = N * 24 + L * 4 + E * (8 + 4 + 8 + 16 + 8 * B)
        want = inputs + 300 * (B * B * s_c + 6) + 500 * 2 + 20 * 16 + (L * B * s_c if B == 1 else 0)
        assert bench.element_bytes(G, B, s_c, s_c, L, N, E, "rowsym", sym) == want
    # the row-owner form writes every slot and every right-hand-side entry
    assert bench.element_bytes(G, 3, 8, 8, L, N, E, "rowowner") == \
        N * 24 + L * 4 + E * (8 + 4 + 8 + 16 + 24) + 1000 * 72 + L * 24


def _tile_blocks_brute_force(m):
    """Tile entries and distinct (tile, upper block) pairs, element by
    element in type-sorted order with Python sets."""
    order = sorted(range(m.n_elems), key=lambda e: int(m.types[e]))
    seen, ent, tile0 = set(), 0, 0
    for t in range(4):
        elems = [e for e in order if m.types[e] == t]
        n = bench.NODES[t]
        epb = 256 // (n * (n + 1) // 2)
        for r, e in enumerate(elems):
            nodes = [int(v) for v in m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]]]
            for a in range(n):
                for b in range(a, n):
                    ent += 1 + (a != b and nodes[a] == nodes[b])
                    seen.add((tile0 + r // epb, min(nodes[a], nodes[b]), max(nodes[a], nodes[b])))
        tile0 += (len(elems) + epb - 1) // epb
    return ent, len(seen)


def test_sym_tile_blocks_match_brute_force():
    m = mg.hybrid_bands(4, seed=2)
    assert bench.sym_tile_blocks(m, np) == _tile_blocks_brute_force(m)
    ent, tb = bench.sym_tile_blocks(m, np)
    # distinct nodes per element: n(n+1)/2 entries each; tiles share blocks
    assert ent == sum(bench.NODES[t] * (bench.NODES[t] + 1) // 2 for t in m.types)
    assert tb < ent


def test_sym_reduce_bytes_definition():
    # 10 upper blocks, 15 blocks in all: 5 diagonal blocks, so 5 rows whose
    # right-hand side (3 values) the 3x3 diagonal tile sums carry
    b = bench.sym_reduce_bytes(100, 10, 15, 3, 4, 8)
    assert b == 100 * 9 * 4 + 11 * 8 + 10 * 8 + 15 * 9 * 8 + 5 * 3 * 8
    assert bench.sym_reduce_bytes(100, 10, 15, 1, 4, 8) == 100 * 4 + 11 * 8 + 10 * 8 + 15 * 8


def test_subscale_work_counts_every_element_and_node_once():
    """The subgrid scale's algorithmic bytes and flops: per element its id,
    node ids, material, source, Gauss-point offset and outputs, per node its
    coordinates and field once; flops per Gauss point by family. A brute
    force over the elements must give the same sums."""
    m = mg.hybrid_bands(6, seed=2)
    byts, flops = bench.subscale_work(m, 3, np)
    nn = {0: 4, 1: 5, 2: 6, 3: 8}
    nq = {0: 1, 1: 8, 2: 6, 3: 8}
    b2 = m.n_nodes * (24 + 24)
    f2 = 0
    for t in m.types:
        t = int(t)
        b2 += 4 + 4 * nn[t] + 16 + 24 + 8 + 24 * nq[t]
        f2 += nq[t] * bench.subscale_flops_per_point(t, 3)
    assert byts == b2 and flops == f2
    # per Gauss point, by hand: tet4 reads J only (18 per node); the others
    # form one polynomial coefficient per field (hex8 / pyramid: 8 additions
    # and a scaling; pen6: at most 5 operations) and evaluate its first and
    # mixed second derivatives (hex8 / pyramid 9 FMA, pen6 4 FMA), then 282
    # (elasticity) or 56 (Poisson) after them
    assert bench.subscale_flops_per_point(0, 3) == 4 * 18 + 43 + 1 + 3
    assert bench.subscale_flops_per_point(3, 3) == 6 * (9 + 18) + 43 + 282 + 1 + 3
    assert bench.subscale_flops_per_point(2, 3) == 6 * (5 + 8) + 43 + 282 + 1 + 3
    assert bench.subscale_flops_per_point(1, 1) == 4 * (9 + 18) + 43 + 56 + 1 + 1


def test_layer_sample_keeps_the_elements_of_its_layers():
    """The CPU baseline's sample: the elements of the chosen cell layers,
    with their own coordinates, materials and node order."""
    m = mg.hybrid_split(12, seed=5)
    layers = [1, 6, 9, 11]
    s = mg.layer_sample(m, layers)
    epl = {t: 144 * n for t, n in enumerate((6, 6, 2, 1))}   # elements per layer by family
    # layer offsets from the band definition
    bands = mg.split_bands(12)
    lt = np.concatenate([np.full(l, t) for t, l in bands])
    start = np.concatenate([[0], np.cumsum([epl[int(t)] for t in lt])])
    elems = np.concatenate([np.arange(start[L], start[L + 1]) for L in layers])
    assert s.n_elems == elems.size
    assert np.array_equal(s.types, m.types[elems])
    for k in range(0, elems.size, 97):
        e = elems[k]
        on = m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]]
        sn = s.conn[s.conn_ptr[k]:s.conn_ptr[k + 1]]
        assert np.array_equal(m.x[on], s.x[sn]) and np.array_equal(m.z[on], s.z[sn])
        assert s.nu[k] == m.nu[e]
    assert np.unique(s.conn).size == s.n_nodes
    s2, nodes = mg.layer_sample(m, layers, return_nodes=True)
    assert np.array_equal(s2.conn, s.conn)
    assert np.all(np.diff(nodes) > 0) and nodes.size == s.n_nodes
    assert np.array_equal(m.x[nodes], s.x) and np.array_equal(m.z[nodes], s.z)
    # the sample's connectivity is the mesh's, renumbered
    k = elems[::131]
    for e, kk in zip(k, np.searchsorted(elems, k)):
        assert np.array_equal(nodes[s.conn[s.conn_ptr[kk]:s.conn_ptr[kk + 1]]], m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]])


def test_submesh_copies_its_elements_and_renumbers_their_nodes():
    """A part of a partition of the elements as a mesh of its own: its
    elements in the order given, every per-element and per-node input
    copied, nodes renumbered in ascending order of their mesh ids."""
    m = mg.heterogeneous(8, seed=4, brick=4)
    rng = np.random.default_rng(1)
    elems = rng.permutation(m.n_elems)[: m.n_elems // 3]
    s, nodes = mg.submesh(m, elems, return_nodes=True)
    assert s.n_elems == elems.size and np.all(np.diff(nodes) > 0)
    assert np.array_equal(s.types, m.types[elems]) and np.array_equal(s.nh_flag, m.nh_flag[elems])
    assert np.array_equal(s.young, m.young[elems]) and np.array_equal(s.nu, m.nu[elems])
    assert np.array_equal(s.source, m.source[elems])
    assert np.array_equal(s.x, m.x[nodes]) and np.array_equal(s.y, m.y[nodes]) and np.array_equal(s.z, m.z[nodes])
    assert np.array_equal(s.u.reshape(-1, 3), m.u.reshape(-1, 3)[nodes])
    assert np.array_equal(s.boundary, m.boundary[nodes])
    # every node of the part is used, and the connectivity maps back
    assert np.unique(s.conn).size == s.n_nodes == nodes.size
    for k in range(0, elems.size, 7):
        e = elems[k]
        assert np.array_equal(nodes[s.conn[s.conn_ptr[k]:s.conn_ptr[k + 1]]], m.conn[m.conn_ptr[e]:m.conn_ptr[e + 1]])


def test_static_split_cuts():
    """The 8-part static split of the cost-model study: contiguous parts
    covering every item, each within one item's weight of an even share."""
    rng = np.random.default_rng(3)
    for n, parts in ((1000, 8), (37, 8), (8, 8), (500, 3)):
        w = rng.lognormal(0.0, 1.0, n)
        cut = bench.static_split_cuts(np, w, parts)
        assert cut.size == parts - 1 and np.all(np.diff(cut) >= 0) and cut[0] >= 0 and cut[-1] <= n
        pieces = np.split(np.arange(n), cut)
        assert np.array_equal(np.concatenate(pieces), np.arange(n))
        share = w.sum() / parts
        for p in pieces:
            assert abs(w[p].sum() - share) <= w.max() + 1e-9
    # equal weights: equal parts
    cut = bench.static_split_cuts(np, np.ones(800), 8)
    assert np.array_equal(cut, np.arange(100, 800, 100))


def test_row_max_by_hand():
    vals = np.arange(27, dtype=np.float64) - 13.0     # 3 blocks
    row_ptr = np.array([0, 2, 2, 3])
    rm = bench._row_max(np, vals, row_ptr)
    assert list(rm) == [13.0, 13.0, 13.0]
