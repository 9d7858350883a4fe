"""Second, independent formulation of the element arithmetic -- TEST ONLY.

Dense Voigt form for tiny meshes: strains [exx, eyy, ezz, gyz, gxz, gxy]
(engineering shear), D = lam * m m^T + mu * diag(2,2,2,1,1,1), element
K = sum_q w detJ B^T D B, assembled into a dense matrix by plain loops in
element order (Algorithm 1). Shape functions are built differently from
fea_oracle.c (hexahedron as a tensor product of 1D hat functions, pyramid by
merging the four top hexahedron functions into the apex, prism as triangle
barycentrics times a 1D hat), the Jacobian is inverted with a linear solve,
and Gauss-Legendre points come from numpy. Agreement with fea_oracle.c on
random distorted elements therefore checks the C oracle's indexing, signs and
transposes, not just its rounding.
"""
from __future__ import annotations

import numpy as np

TET4, PYR5, PEN6, HEX8 = 0, 1, 2, 3


def _hat(s, x):
    """1D linear Lagrange function on [-1,1] for node s = -1 or +1, and derivative."""
    return 0.5 * (1.0 + s * x), 0.5 * s


_HEX_CORNERS = [(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1),
                (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)]


def _hex(xi):
    N = np.zeros(8)
    dN = np.zeros((8, 3))
    for a, (sx, sy, sz) in enumerate(_HEX_CORNERS):
        fx, gx = _hat(sx, xi[0])
        fy, gy = _hat(sy, xi[1])
        fz, gz = _hat(sz, xi[2])
        N[a] = fx * fy * fz
        dN[a] = (gx * fy * fz, fx * gy * fz, fx * fy * gz)
    return N, dN


def shape(etype, xi):
    if etype == HEX8:
        return _hex(xi)
    if etype == PYR5:
        Nh, dNh = _hex(xi)
        N = np.concatenate([Nh[:4], [Nh[4:].sum()]])
        dN = np.vstack([dNh[:4], dNh[4:].sum(axis=0, keepdims=True)])
        return N, dN
    if etype == PEN6:
        r, s, t = xi
        lam = np.array([1 - r - s, r, s])
        dlam = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
        N = np.zeros(6)
        dN = np.zeros((6, 3))
        for layer, sz in enumerate((-1, 1)):
            f, g = _hat(sz, t)
            for k in range(3):
                a = 3 * layer + k
                N[a] = lam[k] * f
                dN[a] = (dlam[k, 0] * f, dlam[k, 1] * f, lam[k] * g)
        return N, dN
    if etype == TET4:
        r, s, t = xi
        N = np.array([1 - r - s - t, r, s, t])
        dN = np.vstack([-np.ones(3), np.eye(3)])
        return N, dN
    raise ValueError(etype)


def rule(etype):
    gp, gw = np.polynomial.legendre.leggauss(2)
    if etype in (HEX8, PYR5):
        pts = [(gp[i], gp[j], gp[k]) for k in range(2) for j in range(2) for i in range(2)]
        w = [gw[i] * gw[j] * gw[k] for k in range(2) for j in range(2) for i in range(2)]
        return np.array(pts), np.array(w)
    if etype == PEN6:
        tri = [(1 / 6, 1 / 6), (2 / 3, 1 / 6), (1 / 6, 2 / 3)]
        pts = [(r, s, gp[k]) for k in range(2) for (r, s) in tri]
        w = [gw[k] / 6.0 for k in range(2) for _ in tri]
        return np.array(pts), np.array(w)
    if etype == TET4:
        return np.array([[0.25, 0.25, 0.25]]), np.array([1.0 / 6.0])
    raise ValueError(etype)


def _grad(etype, X, xi):
    N, dN = shape(etype, xi)
    Jt = dN.T @ X                 # Jt[j, i] = d x_i / d xi_j
    detJ = np.linalg.det(Jt)
    G = np.linalg.solve(Jt, dN.T).T   # G[a, i] = dN_a / dx_i
    return N, G, detJ


def voigt_B(G):
    nn = G.shape[0]
    B = np.zeros((6, 3 * nn))
    for a in range(nn):
        dx, dy, dz = G[a]
        B[:, 3 * a:3 * a + 3] = [[dx, 0, 0], [0, dy, 0], [0, 0, dz],
                                 [0, dz, dy], [dz, 0, dx], [dy, dx, 0]]
    return B


def voigt_D(young, nu):
    lam = young * nu / ((1 + nu) * (1 - 2 * nu))
    mu = young / (2 * (1 + nu))
    m = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    return lam * np.outer(m, m) + mu * np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])


def element(etype, X, poisson=False, young=1.0, nu=0.3, f=None):
    X = np.asarray(X, dtype=np.float64)
    pts, w = rule(etype)
    nn = X.shape[0]
    if poisson:
        K = np.zeros((nn, nn))
        fe = np.zeros(nn)
        fv = 1.0 if f is None else float(np.asarray(f).reshape(-1)[0])
        for q in range(len(w)):
            N, G, d = _grad(etype, X, pts[q])
            K += w[q] * d * (G @ G.T)
            fe += w[q] * d * N * fv
        return K, fe
    D = voigt_D(young, nu)
    fv = np.array([0.0, 0.0, -1.0]) if f is None else np.asarray(f, dtype=np.float64)
    K = np.zeros((3 * nn, 3 * nn))
    fe = np.zeros(3 * nn)
    for q in range(len(w)):
        N, G, d = _grad(etype, X, pts[q])
        B = voigt_B(G)
        K += w[q] * d * (B.T @ D @ B)
        fe += w[q] * d * np.kron(N, fv)
    return K, fe


def assemble_dense(mesh, poisson=False):
    """Dense global matrix and RHS, elements in ascending order (tiny meshes)."""
    B = 1 if poisson else 3
    n = mesh.n_nodes * B
    A = np.zeros((n, n))
    b = np.zeros(n)
    X = np.stack([mesh.x, mesh.y, mesh.z], axis=1)
    for e in range(mesh.n_elems):
        nodes = mesh.conn[mesh.conn_ptr[e]:mesh.conn_ptr[e + 1]]
        K, fe = element(int(mesh.types[e]), X[nodes], poisson=poisson,
                        young=float(mesh.young[e]), nu=float(mesh.nu[e]),
                        f=mesh.source[e, :B])
        dofs = (nodes[:, None] * B + np.arange(B)[None, :]).reshape(-1)
        A[np.ix_(dofs, dofs)] += K
        b[dofs] += fe
    return A, b
