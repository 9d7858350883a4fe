"""Comparison helpers for the parity tests (no assembly arithmetic here)."""
import numpy as np

U32 = 2.0 ** -24
GAUSS_POINTS = {0: 1, 1: 8, 2: 6, 3: 8}


def row_scale(ref_vals, row_ptr, B):
    """max_j |A_ref(i, j)| for every scalar row i, broadcast to the blocks."""
    nnz = ref_vals.size // (B * B)
    a = np.abs(ref_vals.reshape(nnz, B, B)).max(axis=2)          # [nnz, B]
    rows = np.diff(row_ptr)
    starts = row_ptr[:-1][rows > 0]
    rmax = np.zeros((row_ptr.size - 1, B))
    rmax[rows > 0] = np.maximum.reduceat(a, starts, axis=0)
    row_of = np.repeat(np.arange(row_ptr.size - 1), rows)
    return np.repeat(rmax[row_of][:, :, None], B, axis=2).reshape(-1)


def fp64_errors(v, ref, row_ptr, B, rhs=None, ref_rhs=None):
    """Row-scaled max error of vals and max|rhs|-scaled error of rhs."""
    sc = row_scale(ref, row_ptr, B)
    sc[sc == 0] = 1.0
    ev = float(np.max(np.abs(v - ref) / sc)) if v.size else 0.0
    er = 0.0
    if rhs is not None and rhs.size:
        er = float(np.max(np.abs(rhs - ref_rhs)) / max(np.abs(ref_rhs).max(), 1e-300))
    return ev, er


def gamma(L):
    return L * U32 / (1.0 - L * U32)


def fp32_bound_L(types):
    """Roundings per chain for the mixed path: FP32 inputs (3 factors), two
    products, up to three additions per Gauss point, one accumulation per
    Gauss point, the FP64 sums across elements and the final FP32 output,
    with margin: L = (Gauss points) + 12, the largest over the mesh."""
    present = np.unique(types)
    return max(GAUSS_POINTS[int(t)] for t in present) + 12


def within_fp32_bound(v, ref, T, L, floor=None):
    """Max of |v - ref| / (gamma_L T + floor) (must be <= 1).

    The mixed path computes the geometry (J, det J, J^-1, gradients) in
    FP64, so on top of the FP32 rounding bound it carries the FP64 error of
    that geometry; `floor` is the FP64 tolerance (1e-12 of the row scale),
    which matters only where every term is exactly zero (axis-aligned
    elements whose exact gradients have zero components)."""
    bound = gamma(L) * T
    if floor is not None:
        bound = bound + floor
    tiny = np.finfo(np.float64).tiny
    return float(np.max(np.abs(v.astype(np.float64) - ref) / np.maximum(bound, tiny))) if v.size else 0.0


def scatter_part(row_ptr, col, nodes, part_row_ptr, part_col, part_vals, B, acc, part_rhs=None, acc_rhs=None):
    """Adds the matrix of a part of a mesh (a mesh of its own, node i of the
    part being node nodes[i] of the mesh) into the mesh's value array `acc`
    (pattern row_ptr, col), and its right-hand side into `acc_rhs`. Every
    block of the part must exist in the mesh's pattern."""
    N = row_ptr.size - 1
    keys = np.repeat(np.arange(N, dtype=np.int64), np.diff(row_ptr)) * N + col.astype(np.int64)
    prow = np.repeat(np.arange(part_row_ptr.size - 1, dtype=np.int64), np.diff(part_row_ptr))
    pkeys = nodes[prow].astype(np.int64) * N + nodes[part_col].astype(np.int64)
    pos = np.searchsorted(keys, pkeys)
    assert np.all(pos < keys.size) and np.array_equal(keys[pos], pkeys)
    np.add.at(acc.reshape(-1, B * B), pos, np.asarray(part_vals, dtype=np.float64).reshape(-1, B * B))
    if part_rhs is not None:
        np.add.at(acc_rhs.reshape(-1, B), nodes, np.asarray(part_rhs, dtype=np.float64).reshape(-1, B))
    return acc
