"""Seeded synthetic hybrid meshes for finite-element assembly.

This module only builds *inputs*: node coordinates, element connectivity,
per-element material and source values, and (for the hyperelastic workload) a
nodal displacement field. It contains no quadrature, no shape function and no
element matrix arithmetic, so the CPU oracle and the GPU library can both be
fed from it without sharing any of the assembly method.

Meshes tile the unit cube [0,1]^3 with n^3 cells of size h = 1/n. Every cell
becomes one of four element families, matching the hybrid meshes of the
paper's two test cases (Section 2, respiratory and Iter meshes: prisms,
tetrahedra, pyramids and hexahedra):

  HEX8  1 trilinear hexahedron per cell
  PEN6  2 prisms per cell; the z-faces are split along the c000-c110 diagonal
  TET4  6 tetrahedra per cell (Kuhn / Freudenthal split along c000-c111)
  PYR5  6 pyramids per cell, one per face, apex at an added cell-centre node

The prism split diagonal matches the z-face diagonal of the Kuhn tetrahedra,
so prism/tetrahedron interfaces are conforming; hexahedron/prism and
tetrahedron/pyramid interfaces share nodes but are nonconforming.

Node numbering: corner (i, j, k) has id i + (n+1)*(j + (n+1)*k); the centre
nodes of pyramid cells follow, in cell order. Elements are numbered cell by
cell (cell id ci + n*(cj + n*ck)), the sub-elements of a cell consecutively.
"""
from __future__ import annotations

import dataclasses
import numpy as np

TET4, PYR5, PEN6, HEX8 = 0, 1, 2, 3
NODES_PER_TYPE = np.array([4, 5, 6, 8], dtype=np.int64)
TYPE_NAMES = ("tet4", "pyr5", "pen6", "hex8")

# Cell corner labels: 0:c000 1:c100 2:c110 3:c010 4:c001 5:c101 6:c111 7:c011
# (cXYZ = corner at offsets X,Y,Z in {0,1}); label 8 is the cell-centre node.
_CORNER_OFFSETS = np.array(
    [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)

# Local connectivity templates, positively oriented for the reference
# elements (hex: (-1,-1,-1),(1,-1,-1),(1,1,-1),(-1,1,-1) then the top face;
# prism: triangle (0,0),(1,0),(0,1) at t=-1 then t=+1; tet: (0,0,0),(1,0,0),
# (0,1,0),(0,0,1); pyramid: base counter-clockwise seen from the apex).
_TEMPLATES = {
    HEX8: [[0, 1, 2, 3, 4, 5, 6, 7]],
    PEN6: [[0, 1, 2, 4, 5, 6], [0, 2, 3, 4, 6, 7]],
    TET4: [[0, 1, 2, 6], [0, 2, 3, 6], [0, 5, 1, 6],
           [0, 4, 5, 6], [0, 3, 7, 6], [0, 7, 4, 6]],
    PYR5: [[0, 1, 2, 3, 8], [4, 7, 6, 5, 8], [0, 4, 5, 1, 8],
           [3, 2, 6, 7, 8], [0, 3, 7, 4, 8], [1, 5, 6, 2, 8]],
}

# Corner tetrahedra (vertex, then three element neighbours) used by the
# mesh-quality test that rejects a jittered node placement. This is a
# geometric acceptance test on node positions only; it is not the quadrature.
_CORNER_TETS = {
    TET4: [(0, 1, 2, 3)],
    HEX8: [(0, 1, 3, 4), (1, 2, 0, 5), (2, 3, 1, 6), (3, 0, 2, 7),
           (4, 7, 5, 0), (5, 4, 6, 1), (6, 5, 7, 2), (7, 6, 4, 3)],
    PEN6: [(0, 1, 2, 3), (1, 2, 0, 4), (2, 0, 1, 5),
           (3, 5, 4, 0), (4, 3, 5, 1), (5, 4, 3, 2)],
    PYR5: [(0, 1, 3, 4), (1, 2, 0, 4), (2, 3, 1, 4), (3, 0, 2, 4)],
}

SUBELEMS = np.array([len(_TEMPLATES[t]) for t in range(4)], dtype=np.int64)


@dataclasses.dataclass
class Mesh:
    """A hybrid mesh plus per-element material/source data (host, numpy)."""
    n_cells: int                 # cells per axis
    x: np.ndarray                # [N] float64
    y: np.ndarray
    z: np.ndarray
    types: np.ndarray            # [E] uint8 (TET4, PYR5, PEN6, HEX8)
    conn_ptr: np.ndarray         # [E+1] int64
    conn: np.ndarray             # [sum n_e] int32
    young: np.ndarray            # [E] float64 (Young's modulus)
    nu: np.ndarray               # [E] float64 (Poisson ratio)
    source: np.ndarray           # [E, b] float64 (per-element constant source)
    nh_flag: np.ndarray          # [E] uint8 (1 = neo-Hookean tangent)
    u: np.ndarray                # [3N] float64 nodal displacement (node-major)
    boundary: np.ndarray         # [N] bool, node on the cube surface
    redraws: int = 0             # number of rejected jitter draws

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.types.shape[0])

    def type_counts(self):
        return np.bincount(self.types, minlength=4)

    def map_len(self) -> int:
        """Number of element-matrix blocks, sum over elements of n_e^2."""
        return int((NODES_PER_TYPE[self.types] ** 2).sum())


def _corner_id(n, ci, cj, ck):
    m = n + 1
    return ci + m * (cj + m * ck)


def _cell_nodes(n, cell_ids, centre_ids):
    """[ncells, 9] node ids of the 8 corners and the centre (or -1)."""
    ck = cell_ids // (n * n)
    cj = (cell_ids // n) % n
    ci = cell_ids % n
    out = np.empty((cell_ids.shape[0], 9), dtype=np.int64)
    for lab, (dx, dy, dz) in enumerate(_CORNER_OFFSETS):
        out[:, lab] = _corner_id(n, ci + dx, cj + dy, ck + dz)
    out[:, 8] = centre_ids
    return out


def build_connectivity(n, cell_types):
    """Expand per-cell types into elements (cell-major order).

    Returns (types[E] u8, conn_ptr[E+1] i64, conn i32, n_nodes, elem_cell[E]).
    """
    cell_types = np.asarray(cell_types, dtype=np.uint8).reshape(-1)
    ncell = n ** 3
    assert cell_types.shape[0] == ncell
    n_corner = (n + 1) ** 3
    is_pyr = cell_types == PYR5
    centre = np.full(ncell, -1, dtype=np.int64)
    centre[is_pyr] = n_corner + np.arange(int(is_pyr.sum()), dtype=np.int64)
    n_nodes = n_corner + int(is_pyr.sum())

    sub = SUBELEMS[cell_types]                       # elements per cell
    elem_start = np.zeros(ncell + 1, dtype=np.int64)
    np.cumsum(sub, out=elem_start[1:])
    E = int(elem_start[-1])
    types = np.empty(E, dtype=np.uint8)
    elem_cell = np.empty(E, dtype=np.int64)
    nn_elem = np.empty(E, dtype=np.int64)
    for t in range(4):
        cells = np.nonzero(cell_types == t)[0]
        for s in range(SUBELEMS[t]):
            eid = elem_start[cells] + s
            types[eid] = t
            elem_cell[eid] = cells
            nn_elem[eid] = NODES_PER_TYPE[t]
    conn_ptr = np.zeros(E + 1, dtype=np.int64)
    np.cumsum(nn_elem, out=conn_ptr[1:])
    conn = np.empty(int(conn_ptr[-1]), dtype=np.int32)
    for t in range(4):
        cells = np.nonzero(cell_types == t)[0]
        if cells.size == 0:
            continue
        cn = _cell_nodes(n, cells, centre[cells])
        for s, tmpl in enumerate(_TEMPLATES[t]):
            eid = elem_start[cells] + s
            base = conn_ptr[eid]
            for a, lab in enumerate(tmpl):
                conn[base + a] = cn[:, lab]
    return types, conn_ptr, conn, n_nodes, elem_cell


def _base_coords(n, n_nodes, cell_types):
    m = n + 1
    h = 1.0 / n
    idx = np.arange(m ** 3, dtype=np.int64)
    i = idx % m
    j = (idx // m) % m
    k = idx // (m * m)
    x = np.empty(n_nodes)
    y = np.empty(n_nodes)
    z = np.empty(n_nodes)
    x[: m ** 3] = i * h
    y[: m ** 3] = j * h
    z[: m ** 3] = k * h
    bnd = np.zeros(n_nodes, dtype=bool)
    bnd[: m ** 3] = (i == 0) | (i == n) | (j == 0) | (j == n) | (k == 0) | (k == n)
    pc = np.nonzero(np.asarray(cell_types).reshape(-1) == PYR5)[0]
    if pc.size:
        ck = pc // (n * n)
        cj = (pc // n) % n
        ci = pc % n
        x[m ** 3:] = (ci + 0.5) * h
        y[m ** 3:] = (cj + 0.5) * h
        z[m ** 3:] = (ck + 0.5) * h
    return x, y, z, bnd


def corner_tet_volumes(x, y, z, types, conn_ptr, conn, subset=None):
    """Minimum signed corner-tetrahedron volume per element (6x volume),
    for all elements or for the element ids in `subset` (in that order)."""
    ids = np.arange(types.shape[0]) if subset is None else np.asarray(subset)
    out = np.full(ids.shape[0], np.inf)
    st = types[ids]
    for t in range(4):
        sel = np.nonzero(st == t)[0]
        if sel.size == 0:
            continue
        base = conn_ptr[ids[sel]]
        for (v, p, q, r) in _CORNER_TETS[t]:
            a = conn[base + v]
            b = conn[base + p]
            c = conn[base + q]
            d = conn[base + r]
            ux, uy, uz = x[b] - x[a], y[b] - y[a], z[b] - z[a]
            vx, vy, vz = x[c] - x[a], y[c] - y[a], z[c] - z[a]
            wx, wy, wz = x[d] - x[a], y[d] - y[a], z[d] - z[a]
            tri = ux * (vy * wz - vz * wy) - uy * (vx * wz - vz * wx) + uz * (vx * wy - vy * wx)
            out[sel] = np.minimum(out[sel], tri)
    return out


def cube_mesh(n, cell_types, jitter=0.0, seed=0, dofs=3, nu_range=(0.2, 0.35),
              young=1.0, source=None, quality=0.06):
    """Build a mesh of the unit cube.

    n          cells per axis
    cell_types [n^3] per-cell element family (cell order)
    jitter     interior nodes move by U[-jitter*h, jitter*h] per coordinate;
               a placement whose elements fail the corner-tetrahedron test
               (6x signed volume below quality*h^3) is redrawn for the
               interior nodes of the failing elements
    dofs       1 (scalar Poisson source) or 3 (elasticity body force)
    """
    rng = np.random.default_rng(seed)
    types, conn_ptr, conn, n_nodes, _ = build_connectivity(n, cell_types)
    x, y, z, bnd = _base_coords(n, n_nodes, cell_types)
    h = 1.0 / n
    redraws = 0
    if jitter > 0.0:
        interior = np.nonzero(~bnd)[0]
        d = rng.uniform(-jitter * h, jitter * h, size=(interior.size, 3))
        x0, y0, z0 = x.copy(), y.copy(), z.copy()
        x[interior] += d[:, 0]
        y[interior] += d[:, 1]
        z[interior] += d[:, 2]
        q = corner_tet_volumes(x, y, z, types, conn_ptr, conn)
        bad = np.nonzero(q <= quality * h ** 3)[0]
        elem_of_pos = np.repeat(np.arange(types.shape[0]), np.diff(conn_ptr))
        for _ in range(200):
            if bad.size == 0:
                break
            starts = conn_ptr[bad]
            lens = conn_ptr[bad + 1] - starts
            pos = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + \
                np.arange(int(lens.sum()))
            nodes = np.unique(conn[pos])
            nodes = nodes[~bnd[nodes]]
            redraws += int(nodes.size)
            d = rng.uniform(-jitter * h, jitter * h, size=(nodes.size, 3))
            x[nodes] = x0[nodes] + d[:, 0]
            y[nodes] = y0[nodes] + d[:, 1]
            z[nodes] = z0[nodes] + d[:, 2]
            moved = np.zeros(x.shape[0], dtype=bool)
            moved[nodes] = True
            touched = np.unique(elem_of_pos[moved[conn]])
            qt = corner_tet_volumes(x, y, z, types, conn_ptr, conn, subset=touched)
            bad = touched[qt <= quality * h ** 3]
        else:
            raise RuntimeError("jitter redraw did not converge")
    E = types.shape[0]
    nu = rng.uniform(nu_range[0], nu_range[1], size=E)
    if source is None:
        source = (1.0,) if dofs == 1 else (0.0, 0.0, -1.0)
    src = np.tile(np.asarray(source, dtype=np.float64), (E, 1))
    return Mesh(n_cells=n, x=x, y=y, z=z, types=types, conn_ptr=conn_ptr,
                conn=conn, young=np.full(E, float(young)), nu=nu, source=src,
                nh_flag=np.zeros(E, dtype=np.uint8), u=np.zeros(3 * n_nodes),
                boundary=bnd, redraws=redraws)


def band_cell_types(n, bands):
    """Per-cell types from bottom-to-top z-bands [(type, n_layers), ...]."""
    assert sum(l for _, l in bands) == n
    layer_type = np.concatenate([np.full(l, t, dtype=np.uint8) for t, l in bands])
    return np.repeat(layer_type, n * n)


# ---------------------------------------------------------------- workloads

def poisson_hex(n=16, jitter=0.2, seed=1):
    """Scalar Poisson on hex8 cells, interior nodes jittered, source f = 1."""
    return cube_mesh(n, np.full(n ** 3, HEX8, dtype=np.uint8), jitter=jitter,
                     seed=seed, dofs=1)


def hybrid_bands(n=96, seed=2, jitter=0.0):
    """Four equal z-bands, bottom to top: hex8, pen6, tet4, pyr5."""
    q = n // 4
    bands = [(HEX8, q), (PEN6, q), (TET4, q), (PYR5, n - 3 * q)]
    return cube_mesh(n, band_cell_types(n, bands), jitter=jitter, seed=seed)


def split_bands(n):
    """40% hex8 / 30% tet4 / 20% pen6 / 10% pyr5 of the cell layers."""
    nh = round(0.4 * n)
    nt = round(0.3 * n)
    npn = round(0.2 * n)
    return [(HEX8, nh), (TET4, nt), (PEN6, npn), (PYR5, n - nh - nt - npn)]


def hybrid_split(n=256, seed=5, jitter=0.0):
    """Large hybrid mesh with the 40/30/20/10 hex/tet/pen/pyr layer split."""
    return cube_mesh(n, band_cell_types(n, split_bands(n)), jitter=jitter, seed=seed)


def batched(n_meshes=64, seed=3, n_range=(8, 48), jitter=0.25, first_seed=3000):
    """Independent meshes of random size with a random per-cell type mix.

    Mesh m: n ~ U{n_range}; type fractions ~ Dirichlet(1,1,1,1); each cell
    draws its type iid from those fractions; interior jitter +-jitter*h.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_range[0], n_range[1] + 1, size=n_meshes)
    meshes = []
    for m in range(n_meshes):
        r = np.random.default_rng(first_seed + m)
        frac = r.dirichlet(np.ones(4))
        n = int(sizes[m])
        ct = r.choice(4, size=n ** 3, p=frac).astype(np.uint8)
        meshes.append(cube_mesh(n, ct, jitter=jitter, seed=first_seed + m))
    return meshes


def heterogeneous(n=128, seed=4, nh_fraction=0.3, brick=8, grad_bound=0.1,
                  jitter=0.0):
    """Hybrid split mesh where a random set of bricks uses the neo-Hookean
    tangent at a smooth displacement field; the rest is linear elastic.

    The displacement is u(X) = A * sum_m a_m sin(2 pi k_m . X + phi_m) with
    k_m in {1,2}^3, a_m ~ U[-1,1]^3, phi_m ~ U[0, 2 pi); A scales the
    analytic gradient bound A * sum_m |a_m| 2 pi |k_m| to grad_bound.
    """
    mesh = cube_mesh(n, band_cell_types(n, split_bands(n)), jitter=jitter, seed=seed)
    rng = np.random.default_rng(seed + 100)
    nb = n // brick
    n_bricks = nb ** 3
    chosen = rng.permutation(n_bricks)[: int(round(nh_fraction * n_bricks))]
    brick_nh = np.zeros(n_bricks, dtype=bool)
    brick_nh[chosen] = True
    _, _, _, _, elem_cell = build_connectivity(n, band_cell_types(n, split_bands(n)))
    ck = elem_cell // (n * n)
    cj = (elem_cell // n) % n
    ci = elem_cell % n
    bid = (ci // brick) + nb * ((cj // brick) + nb * (ck // brick))
    mesh.nh_flag = brick_nh[bid].astype(np.uint8)
    mesh.u = _sine_field(mesh, rng, 3, grad_bound)
    return mesh


def _sine_field(mesh, rng, components, grad_bound):
    """u(X) = A sum_{m<3} a_m sin(2 pi k_m . X + phi_m), k_m in {1,2}^3,
    a_m ~ U[-1,1]^components, phi_m ~ U[0, 2 pi), A scaling the analytic
    gradient bound to grad_bound; node-major, components values per node."""
    k = rng.integers(1, 3, size=(3, 3)).astype(np.float64)
    a = rng.uniform(-1.0, 1.0, size=(3, components))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=3)
    scale = sum(np.linalg.norm(a[m]) * 2 * np.pi * np.linalg.norm(k[m]) for m in range(3))
    A = grad_bound / scale
    X = np.stack([mesh.x, mesh.y, mesh.z], axis=1)
    u = np.zeros((mesh.n_nodes, components))
    for m in range(3):
        u += A * np.outer(np.sin(2 * np.pi * X @ k[m] + phi[m]), a[m])
    return u.reshape(-1).copy()


def smooth_field(mesh, components=3, seed=0, grad_bound=0.1, noise=0.0):
    """A seeded nodal field for element loops that read one (the subgrid
    scale): the smooth sine field above, plus, if noise > 0, independent
    normal nodal values of that standard deviation times the mean cell size
    (a field that is not smooth on the mesh scale)."""
    rng = np.random.default_rng(seed)
    u = _sine_field(mesh, rng, components, grad_bound)
    if noise > 0:
        h = 1.0 / max(getattr(mesh, "n_cells", 1), 1)
        u = u + noise * h * rng.standard_normal(u.shape[0])
    return u


def tiny_mesh(cell_types_grid, jitter=0.0, seed=0, dofs=3):
    """Small mesh from an explicit (n,n,n) array of cell types (tests)."""
    ct = np.asarray(cell_types_grid, dtype=np.uint8)
    n = ct.shape[0]
    assert ct.shape == (n, n, n)
    # cell order: ci fastest -> array indexed [ck, cj, ci]
    return cube_mesh(n, ct.reshape(-1), jitter=jitter, seed=seed, dofs=dofs)


def submesh(mesh, elems, return_nodes=False):
    """The elements `elems` (ids in `mesh`, kept in the order given) as a
    mesh of their own: nodes renumbered in ascending order of their ids in
    `mesh`, coordinates, materials, sources, flags and displacements
    copied. Used for the parts of a partition of the elements, each
    assembled on its own. return_nodes: also return the ids in `mesh` of
    the submesh's nodes (ascending)."""
    elems = np.asarray(elems, dtype=np.int64)
    lens = mesh.conn_ptr[elems + 1] - mesh.conn_ptr[elems]
    pos = np.repeat(mesh.conn_ptr[elems] - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + \
        np.arange(int(lens.sum()))
    old = mesh.conn[pos].astype(np.int64)
    nodes, conn = np.unique(old, return_inverse=True)
    conn_ptr = np.zeros(elems.size + 1, dtype=np.int64)
    np.cumsum(lens, out=conn_ptr[1:])
    u = mesh.u.reshape(-1, 3)[nodes].reshape(-1).copy()
    sub = Mesh(n_cells=mesh.n_cells, x=mesh.x[nodes].copy(), y=mesh.y[nodes].copy(), z=mesh.z[nodes].copy(),
               types=mesh.types[elems].copy(), conn_ptr=conn_ptr, conn=conn.reshape(-1).astype(np.int32),
               young=mesh.young[elems].copy(), nu=mesh.nu[elems].copy(), source=mesh.source[elems].copy(),
               nh_flag=mesh.nh_flag[elems].copy(), u=u, boundary=mesh.boundary[nodes].copy(),
               redraws=0)
    return (sub, nodes) if return_nodes else sub


def layer_sample(mesh, layers, return_nodes=False):
    """The elements of the given z-layers of cells of a band mesh (every cell
    of a layer has one family), as a mesh of their own (submesh). Used to
    time work on a bounded part of a large mesh with its family mix, and to
    check whole rows of it. return_nodes: also return the ids in `mesh` of
    the sample's nodes (ascending)."""
    n = mesh.n_cells
    lay = n * n
    # element offset of every layer: a layer holds n^2 cells of one family
    start = np.zeros(n + 1, dtype=np.int64)
    for L in range(n):
        start[L + 1] = start[L] + lay * SUBELEMS[int(mesh.types[start[L]])]
    assert start[-1] == mesh.n_elems, "not a band mesh"
    elems = np.concatenate([np.arange(start[L], start[L + 1]) for L in sorted(layers)])
    return submesh(mesh, elems, return_nodes=return_nodes)
