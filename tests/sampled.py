"""Oracle values for sampled rows of a large mesh, computed one element at a
time (test infrastructure: the whole-mesh oracle would take too long at the
benchmark sizes). For node i, row i of A is the sum, over the elements that
contain i in ascending order, of the element-matrix rows of i; its absolute
term sums give the FP32 bound."""
import numpy as np

import oracle


def incident_elements(mesh, nodes):
    """{node: ascending element ids containing it} for the given nodes."""
    want = np.zeros(mesh.n_nodes, dtype=bool)
    want[np.asarray(nodes)] = True
    pos = np.nonzero(want[mesh.conn])[0]
    elems = np.searchsorted(mesh.conn_ptr, pos, side="right") - 1
    out = {int(n): [] for n in nodes}
    for p, e in zip(pos, elems):
        out[int(mesh.conn[p])].append(int(e))
    return {n: sorted(v) for n, v in out.items()}


def oracle_rows(mesh, nodes, model=oracle.ELASTIC, use_nh=True, residual=False):
    """{node: (cols, blocks[ncol, B, B], terms[ncol, B, B], rhs[B], rhs_terms[B])}.
    residual: rhs is the Newton residual f_ext - f_int(mesh.u) (elasticity):
    f_int the neo-Hookean internal force where flagged, K^e u^e elsewhere;
    rhs_terms then holds the larger of |f_ext| and |f_int| per component
    (the scale of a residual whose two parts partly cancel)."""
    B = 1 if model == oracle.POISSON else 3
    X = np.stack([mesh.x, mesh.y, mesh.z], axis=1)
    U = mesh.u.reshape(-1, 3)
    inc = incident_elements(mesh, nodes)
    out = {}
    for i, elems in inc.items():
        acc, tacc = {}, {}
        rhs = np.zeros(B)
        trhs = np.zeros(B)
        for e in elems:
            nodes_e = mesh.conn[mesh.conn_ptr[e]:mesh.conn_ptr[e + 1]]
            a = int(np.nonzero(nodes_e == i)[0][0])
            nh = bool(use_nh and model == oracle.ELASTIC and mesh.nh_flag[e])
            K, fe, T, Tf = oracle.element(int(mesh.types[e]), X[nodes_e], model=model,
                                          young=float(mesh.young[e]), nu=float(mesh.nu[e]),
                                          f=mesh.source[e, :B], u=U[nodes_e], nh=nh,
                                          with_terms=True)
            for b, j in enumerate(nodes_e):
                blk = K[a * B:(a + 1) * B, b * B:(b + 1) * B]
                tb = T[a * B:(a + 1) * B, b * B:(b + 1) * B]
                acc[int(j)] = acc.get(int(j), 0.0) + blk
                tacc[int(j)] = tacc.get(int(j), 0.0) + tb
            if residual:
                if nh:
                    fint = oracle.element_fint(int(mesh.types[e]), X[nodes_e], float(mesh.young[e]),
                                               float(mesh.nu[e]), U[nodes_e])
                else:
                    Kl, _ = oracle.element(int(mesh.types[e]), X[nodes_e], model=model,
                                           young=float(mesh.young[e]), nu=float(mesh.nu[e]), f=mesh.source[e, :B])
                    fint = Kl @ U[nodes_e].reshape(-1)
                fa, ia = fe[a * B:(a + 1) * B], fint[a * B:(a + 1) * B]
                rhs += fa - ia
                trhs += np.maximum(np.abs(fa), np.abs(ia))
            else:
                rhs += fe[a * B:(a + 1) * B]
                trhs += Tf[a * B:(a + 1) * B]
        cols = np.array(sorted(acc))
        out[i] = (cols, np.array([acc[c] for c in cols]), np.array([tacc[c] for c in cols]), rhs, trhs)
    return out


def _host(a, lo, hi):
    """a[lo:hi] as a NumPy array (a may be a device tensor: only the slice moves)."""
    part = a[lo:hi]
    return part.cpu().numpy() if hasattr(part, "cpu") else part


def check_rows(mesh, rows, row_ptr, col, vals, rhs, B, fp32_L=None):
    """Max row-scaled FP64 error (or max ratio to the FP32 bound) over the rows."""
    from tests.helpers import gamma
    worst = 0.0
    for i, (cols, blocks, terms, r_ref, r_terms) in rows.items():
        k0, k1 = int(row_ptr[i]), int(row_ptr[i + 1])
        assert np.array_equal(col[k0:k1], cols), i
        got = _host(vals, k0 * B * B, k1 * B * B).astype(np.float64).reshape(-1, B, B)
        scale = np.abs(blocks).max(axis=(0, 2))[None, :, None]     # per scalar row
        if fp32_L is None:
            worst = max(worst, float(np.max(np.abs(got - blocks) / scale)))
        else:
            bound = gamma(fp32_L) * terms + 1e-12 * scale
            worst = max(worst, float(np.max(np.abs(got - blocks) / bound)))
        rg = _host(rhs, i * B, (i + 1) * B).astype(np.float64)
        if fp32_L is None:
            worst = max(worst, float(np.max(np.abs(rg - r_ref)) / max(np.abs(r_ref).max(), 1e-300)))
        else:
            rb = gamma(fp32_L) * r_terms + 1e-12 * np.abs(r_ref).max()
            worst = max(worst, float(np.max(np.abs(rg - r_ref) / np.maximum(rb, 1e-300))))
    return worst
