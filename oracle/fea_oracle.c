/*
 * fea_oracle.c -- plain, slow, FP64 CPU oracle for finite-element assembly.
 *
 * TEST INFRASTRUCTURE ONLY. This file is used by the test suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark. The GPU library
 * never includes, links or calls it, and it shares no code with the GPU
 * library: shape functions, quadrature rules, element matrices, sparsity
 * pattern, element-to-nonzero map and inverse map are all written out here
 * from their definitions.
 *
 * What it computes (paper: Section 2.1.1, Algorithm 1 "assembly of a generic
 * matrix A and vector b"): for every element e in ascending order, compute
 * the element matrix A^e and right-hand side b^e, then add them into the
 * global sparse matrix A and vector b. The paper does not state the element
 * integrand (it cites the formulation), so the element arithmetic is the
 * textbook isoparametric one:
 *   - reference elements tet4 / pyr5 (collapsed hexahedron) / pen6 / hex8,
 *   - Gauss rules: tet 1 point, prism 3x2 points, hex and pyramid 2x2x2,
 *     matching the paper's remark that tetrahedra carry fewer Gauss points
 *     (Section 4.1, element weight = number of Gauss points),
 *   - J = sum_a x_a (x) grad_xi N_a, grad N_a = J^-T grad_xi N_a,
 *   - Poisson: K_ab = sum_q w detJ grad N_a . grad N_b, f_a = sum_q w detJ N_a f,
 *   - linear elasticity (3 dof/node, 3x3 blocks, row-major):
 *       K_(a,i)(b,j) = sum_q w detJ [lam dN_a/dx_i dN_b/dx_j
 *                      + mu dN_a/dx_j dN_b/dx_i + mu delta_ij grad N_a.grad N_b]
 *   - compressible neo-Hookean tangent (Section 2.2: first Piola-Kirchhoff
 *     stress P, Newton-Raphson with A = Jacobian):
 *       F = I + sum_a u_a (x) grad N_a,  P = mu (F - F^-T) + lam ln(det F) F^-T,
 *       AA_iJjL = mu d_ij d_JL + (mu - lam ln J) Finv_Jj Finv_Li + lam Finv_Ji Finv_Lj,
 *       K_(a,i)(b,j) = sum_q w detJ sum_JL dN_a/dX_J AA_iJjL dN_b/dX_L.
 * It also evaluates, element by element with nothing assembled, the
 * subgrid scale of Section 2.1.3 read for these problems (the strong
 * residual f + L(u_h) at every Gauss point scaled by an element constant;
 * or_element_subscale states the reading).
 * Alongside the values it assembles T, the same sums taken over the
 * absolute value of every product term (for the neo-Hookean tangent, of
 * each of its three parts separately); a computation in a lower precision
 * with L roundings per chain must satisfy |v_low - v| <= gamma_L T.
 *
 * Sparsity pattern (compressed sparse rows of node blocks): row i holds
 * every node j that shares an element with node i (diagonal included),
 * columns strictly ascending, zero-based. e2nnz[map_ptr[e] + a*n_e + b] is
 * the block index of (conn[e][a], conn[e][b]). The inverse map lists, for
 * each block, the slots that land in it, in ascending element order.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_TET4 = 0, OR_PYR5 = 1, OR_PEN6 = 2, OR_HEX8 = 3 };
enum { OR_POISSON = 0, OR_ELASTIC = 1 };

static const int or_nodes_of[4] = {4, 5, 6, 8};

int or_nodes(int type) { return (type >= 0 && type < 4) ? or_nodes_of[type] : -1; }

/* ------------------------------------------------------------------ *
 * Reference elements: shape functions and their xi-gradients.         *
 * ------------------------------------------------------------------ */
static const double hex_sign[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

/* Fills N[a] and dN[a][j] = dN_a/dxi_j at reference point xi. */
int or_shape(int type, const double *xi, double *N, double *dN)
{
    double r = xi[0], s = xi[1], t = xi[2];
    int a;
    switch (type) {
    case OR_TET4:
        N[0] = 1.0 - r - s - t; N[1] = r; N[2] = s; N[3] = t;
        for (a = 0; a < 12; ++a) dN[a] = 0.0;
        dN[0] = -1.0; dN[1] = -1.0; dN[2] = -1.0;
        dN[3 + 0] = 1.0;
        dN[6 + 1] = 1.0;
        dN[9 + 2] = 1.0;
        return 4;
    case OR_HEX8:
        for (a = 0; a < 8; ++a) {
            double sx = hex_sign[a][0], sy = hex_sign[a][1], sz = hex_sign[a][2];
            double fx = 1.0 + sx * r, fy = 1.0 + sy * s, fz = 1.0 + sz * t;
            N[a] = fx * fy * fz / 8.0;
            dN[3 * a + 0] = sx * fy * fz / 8.0;
            dN[3 * a + 1] = fx * sy * fz / 8.0;
            dN[3 * a + 2] = fx * fy * sz / 8.0;
        }
        return 8;
    case OR_PEN6: {
        /* triangle (0,0),(1,0),(0,1) times the interval t in [-1,1] */
        double L[3] = {1.0 - r - s, r, s};
        double dLr[3] = {-1.0, 1.0, 0.0}, dLs[3] = {-1.0, 0.0, 1.0};
        for (a = 0; a < 6; ++a) {
            int k = a % 3;
            double g = (a < 3) ? 0.5 * (1.0 - t) : 0.5 * (1.0 + t);
            double dg = (a < 3) ? -0.5 : 0.5;
            N[a] = L[k] * g;
            dN[3 * a + 0] = dLr[k] * g;
            dN[3 * a + 1] = dLs[k] * g;
            dN[3 * a + 2] = L[k] * dg;
        }
        return 6;
    }
    case OR_PYR5:
        /* collapsed hexahedron: the four top nodes merge into the apex */
        for (a = 0; a < 4; ++a) {
            double sx = hex_sign[a][0], sy = hex_sign[a][1];
            double fx = 1.0 + sx * r, fy = 1.0 + sy * s, fz = 1.0 - t;
            N[a] = fx * fy * fz / 8.0;
            dN[3 * a + 0] = sx * fy * fz / 8.0;
            dN[3 * a + 1] = fx * sy * fz / 8.0;
            dN[3 * a + 2] = -fx * fy / 8.0;
        }
        N[4] = 0.5 * (1.0 + t);
        dN[12] = 0.0; dN[13] = 0.0; dN[14] = 0.5;
        return 5;
    }
    return -1;
}

/* Gauss rule: points (xi fastest; prism: triangle point fastest) and weights. */
int or_rule(int type, double *pts, double *w)
{
    const double g = 1.0 / sqrt(3.0);
    int q = 0, i, j, k;
    switch (type) {
    case OR_TET4:
        pts[0] = pts[1] = pts[2] = 0.25;
        w[0] = 1.0 / 6.0;
        return 1;
    case OR_HEX8:
    case OR_PYR5:
        for (k = 0; k < 2; ++k)
            for (j = 0; j < 2; ++j)
                for (i = 0; i < 2; ++i) {
                    pts[3 * q + 0] = i ? g : -g;
                    pts[3 * q + 1] = j ? g : -g;
                    pts[3 * q + 2] = k ? g : -g;
                    w[q] = 1.0;
                    ++q;
                }
        return 8;
    case OR_PEN6: {
        const double tr[3][2] = {{1.0 / 6.0, 1.0 / 6.0}, {2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}};
        for (k = 0; k < 2; ++k)
            for (i = 0; i < 3; ++i) {
                pts[3 * q + 0] = tr[i][0];
                pts[3 * q + 1] = tr[i][1];
                pts[3 * q + 2] = k ? g : -g;
                w[q] = 1.0 / 6.0;
                ++q;
            }
        return 6;
    }
    }
    return -1;
}

/* ------------------------------------------------------------------ *
 * Small dense linear algebra (3x3).                                   *
 * ------------------------------------------------------------------ */
static double det3(const double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* inverse by the adjugate; returns the determinant */
static double inv3(const double A[3][3], double B[3][3])
{
    double d = det3(A);
    B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
    B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
    B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
    return d;
}

/* Geometry at one point: detJ and physical gradients G[a][i] = dN_a/dx_i. */
static double point_geometry(int nn, const double *X, const double *dN, double G[8][3])
{
    double J[3][3], Ji[3][3];
    int a, i, j;
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (a = 0; a < nn; ++a) acc += X[3 * a + i] * dN[3 * a + j];
            J[i][j] = acc;
        }
    double d = det3(J);
    if (!(d > 0.0)) return d;
    inv3(J, Ji);
    for (a = 0; a < nn; ++a)
        for (i = 0; i < 3; ++i) {
            double acc = 0.0;
            for (j = 0; j < 3; ++j) acc += Ji[j][i] * dN[3 * a + j];
            G[a][i] = acc;
        }
    return d;
}

static void lame(double young, double nu, double *lam, double *mu)
{
    *lam = young * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    *mu = young / (2.0 * (1.0 + nu));
}

/*
 * One element. X[a*3+i]: node coordinates; u[a*3+i]: nodal displacement
 * (used only when nh != 0); f: per-element source (1 or 3 values).
 * model: OR_POISSON (1 dof/node) or OR_ELASTIC (3 dof/node; nh selects the
 * neo-Hookean tangent). Outputs, in block order (a, b, i, j):
 *   Ke[((a*nn + b)*B + i)*B + j], fe[a*B + i],
 * and, if Tk/Tf are not NULL, the absolute-term sums of the same entries.
 * Returns 0, or 1 + q when detJ <= 0 at Gauss point q.
 */
int or_element(int type, int model, int nh, const double *X, double young, double nu,
               const double *u, const double *f, double *Ke, double *fe,
               double *Tk, double *Tf)
{
    double pts[8 * 3], w[8], N[8], dN[24], G[8][3];
    int nn = or_nodes(type);
    int nq = or_rule(type, pts, w);
    int B = (model == OR_POISSON) ? 1 : 3;
    int a, b, i, j, q, k, J, L;
    double lam = 0.0, mu = 0.0;
    if (nn < 0) return -1;
    if (model != OR_POISSON) lame(young, nu, &lam, &mu);
    memset(Ke, 0, sizeof(double) * nn * nn * B * B);
    memset(fe, 0, sizeof(double) * nn * B);
    if (Tk) memset(Tk, 0, sizeof(double) * nn * nn * B * B);
    if (Tf) memset(Tf, 0, sizeof(double) * nn * B);

    for (q = 0; q < nq; ++q) {
        or_shape(type, &pts[3 * q], N, dN);
        double detJ = point_geometry(nn, X, dN, G);
        if (!(detJ > 0.0)) return 1 + q;
        double wd = w[q] * detJ;

        for (a = 0; a < nn; ++a)
            for (i = 0; i < B; ++i) {
                double t = wd * N[a] * f[i];
                fe[a * B + i] += t;
                if (Tf) Tf[a * B + i] += fabs(t);
            }

        if (model == OR_POISSON) {
            for (a = 0; a < nn; ++a)
                for (b = 0; b < nn; ++b) {
                    double acc = 0.0, tac = 0.0;
                    for (k = 0; k < 3; ++k) {
                        double t = wd * G[a][k] * G[b][k];
                        acc += t;
                        tac += fabs(t);
                    }
                    Ke[a * nn + b] += acc;
                    if (Tk) Tk[a * nn + b] += tac;
                }
        } else if (!nh) {
            for (a = 0; a < nn; ++a)
                for (b = 0; b < nn; ++b) {
                    double dot = 0.0, tdot = 0.0;
                    for (k = 0; k < 3; ++k) {
                        double t = wd * mu * G[a][k] * G[b][k];
                        dot += t;
                        tdot += fabs(t);
                    }
                    for (i = 0; i < 3; ++i)
                        for (j = 0; j < 3; ++j) {
                            double t1 = wd * lam * G[a][i] * G[b][j];
                            double t2 = wd * mu * G[a][j] * G[b][i];
                            double v = t1 + t2 + (i == j ? dot : 0.0);
                            Ke[((a * nn + b) * 3 + i) * 3 + j] += v;
                            if (Tk)
                                Tk[((a * nn + b) * 3 + i) * 3 + j] +=
                                    fabs(t1) + fabs(t2) + (i == j ? tdot : 0.0);
                        }
                }
        } else {
            /* deformation gradient with respect to the mesh coordinates */
            double F[3][3], Fi[3][3], AA[3][3][3][3];
            for (i = 0; i < 3; ++i)
                for (J = 0; J < 3; ++J) {
                    double acc = (i == J) ? 1.0 : 0.0;
                    for (a = 0; a < nn; ++a) acc += u[3 * a + i] * G[a][J];
                    F[i][J] = acc;
                }
            double JF = inv3(F, Fi);
            if (!(JF > 0.0)) return 1 + q;
            double lnJ = log(JF);
            for (i = 0; i < 3; ++i)
                for (J = 0; J < 3; ++J)
                    for (j = 0; j < 3; ++j)
                        for (L = 0; L < 3; ++L)
                            AA[i][J][j][L] = mu * (i == j) * (J == L)
                                           + (mu - lam * lnJ) * Fi[J][j] * Fi[L][i]
                                           + lam * Fi[J][i] * Fi[L][j];
            for (a = 0; a < nn; ++a)
                for (b = 0; b < nn; ++b)
                    for (i = 0; i < 3; ++i)
                        for (j = 0; j < 3; ++j) {
                            double acc = 0.0, tac = 0.0;
                            for (J = 0; J < 3; ++J)
                                for (L = 0; L < 3; ++L) {
                                    double g2 = wd * G[a][J] * G[b][L];
                                    acc += g2 * AA[i][J][j][L];
                                    /* |terms|: the tangent's three parts separately */
                                    tac += fabs(g2) * (mu * (i == j) * (J == L)
                                                       + fabs((mu - lam * lnJ) * Fi[J][j] * Fi[L][i])
                                                       + fabs(lam * Fi[J][i] * Fi[L][j]));
                                }
                            Ke[((a * nn + b) * 3 + i) * 3 + j] += acc;
                            if (Tk) Tk[((a * nn + b) * 3 + i) * 3 + j] += tac;
                        }
        }
    }
    return 0;
}

/* Internal force of the neo-Hookean element, fint[a*3+i] = sum_q w detJ P_iJ dN_a/dX_J. */
int or_element_fint(int type, const double *X, double young, double nu, const double *u,
                    double *fint)
{
    double pts[8 * 3], w[8], N[8], dN[24], G[8][3], F[3][3], Fi[3][3], P[3][3];
    int nn = or_nodes(type), nq = or_rule(type, pts, w), a, i, J, q;
    double lam, mu;
    lame(young, nu, &lam, &mu);
    memset(fint, 0, sizeof(double) * nn * 3);
    for (q = 0; q < nq; ++q) {
        or_shape(type, &pts[3 * q], N, dN);
        double detJ = point_geometry(nn, X, dN, G);
        if (!(detJ > 0.0)) return 1 + q;
        for (i = 0; i < 3; ++i)
            for (J = 0; J < 3; ++J) {
                double acc = (i == J) ? 1.0 : 0.0;
                for (a = 0; a < nn; ++a) acc += u[3 * a + i] * G[a][J];
                F[i][J] = acc;
            }
        double JF = inv3(F, Fi);
        if (!(JF > 0.0)) return 1 + q;
        double lnJ = log(JF);
        for (i = 0; i < 3; ++i)
            for (J = 0; J < 3; ++J)
                P[i][J] = mu * (F[i][J] - Fi[J][i]) + lam * lnJ * Fi[J][i];
        for (a = 0; a < nn; ++a)
            for (i = 0; i < 3; ++i) {
                double acc = 0.0;
                for (J = 0; J < 3; ++J) acc += P[i][J] * G[a][J];
                fint[3 * a + i] += w[q] * detJ * acc;
            }
    }
    return 0;
}

/* Newton residual b = f_ext - f_int(u) of the solid (Section 2.2: Newton
 * iterations on the internal force; A is its Jacobian): for every element
 * in ascending order, its body-force vector minus its internal force --
 * the neo-Hookean one, sum_q w detJ P grad N_a, where nh_flag is set, else
 * the linear-elastic one, K^e u^e with this file's element matrix -- added
 * into rhs[3 * n_nodes]. Returns 0, or -(1 + e) for a rejected element. */
int64_t or_residual(int64_t n_nodes, int64_t n_elems, const uint8_t *types, const int64_t *conn_ptr,
                    const int32_t *conn, const double *x, const double *y, const double *z,
                    const double *young, const double *nu, const uint8_t *nh_flag, const double *u,
                    const double *source, double *rhs)
{
    double X[24], U[24], Ke[64 * 9], fe[24], fint[24];
    int64_t e;
    memset(rhs, 0, sizeof(double) * (size_t)(n_nodes * 3));
    for (e = 0; e < n_elems; ++e) {
        int nn = or_nodes(types[e]), a, b, i, j;
        double E = young ? young[e] : 1.0;
        for (a = 0; a < nn; ++a) {
            int32_t v = conn[conn_ptr[e] + a];
            X[3 * a + 0] = x[v]; X[3 * a + 1] = y[v]; X[3 * a + 2] = z[v];
            for (i = 0; i < 3; ++i) U[3 * a + i] = u[3 * (int64_t)v + i];
        }
        if (or_element(types[e], OR_ELASTIC, 0, X, E, nu[e], U, &source[e * 3], Ke, fe, NULL, NULL))
            return -(1 + e);
        if (nh_flag && nh_flag[e]) {
            if (or_element_fint(types[e], X, E, nu[e], U, fint)) return -(1 + e);
        } else {
            for (a = 0; a < nn; ++a)
                for (i = 0; i < 3; ++i) {
                    double acc = 0.0;
                    for (b = 0; b < nn; ++b)
                        for (j = 0; j < 3; ++j) acc += Ke[((a * nn + b) * 3 + i) * 3 + j] * U[3 * b + j];
                    fint[3 * a + i] = acc;
                }
        }
        for (a = 0; a < nn; ++a) {
            int32_t r = conn[conn_ptr[e] + a];
            for (i = 0; i < 3; ++i) rhs[(int64_t)r * 3 + i] += fe[3 * a + i] - fint[3 * a + i];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ *
 * Subgrid scale: an element loop with no assembly.                    *
 * ------------------------------------------------------------------ */

/* Second reference derivatives at xi: D2[(a*3 + j)*3 + l] = d2 N_a / dxi_j dxi_l,
 * all nine entries, from the shape functions of or_shape differentiated
 * twice. */
int or_shape2(int type, const double *xi, double *D2)
{
    double r = xi[0], s = xi[1], t = xi[2];
    int a, j, l;
    switch (type) {
    case OR_TET4:
        /* linear: every second derivative vanishes */
        for (a = 0; a < 36; ++a) D2[a] = 0.0;
        return 4;
    case OR_HEX8:
        for (a = 0; a < 8; ++a) {
            double sx = hex_sign[a][0], sy = hex_sign[a][1], sz = hex_sign[a][2];
            double f[3] = {1.0 + sx * r, 1.0 + sy * s, 1.0 + sz * t};
            double d[3] = {sx, sy, sz}; /* d f_j / d xi_j; d2 f_j / d xi_j^2 = 0 */
            for (j = 0; j < 3; ++j)
                for (l = 0; l < 3; ++l) {
                    double v;
                    if (j == l) {
                        v = 0.0;
                    } else {
                        int m = 3 - j - l; /* the third direction */
                        v = d[j] * d[l] * f[m] / 8.0;
                    }
                    D2[(a * 3 + j) * 3 + l] = v;
                }
        }
        return 8;
    case OR_PEN6: {
        /* N = L_k(r, s) g(t): L linear in (r, s), g linear in t */
        double L[3] = {1.0 - r - s, r, s};
        double dL[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
        for (a = 0; a < 6; ++a) {
            int k = a % 3;
            double dg = (a < 3) ? -0.5 : 0.5;
            double H[3][3];
            H[0][0] = 0.0; H[1][1] = 0.0; H[0][1] = H[1][0] = 0.0;
            H[0][2] = H[2][0] = dL[k][0] * dg;
            H[1][2] = H[2][1] = dL[k][1] * dg;
            H[2][2] = L[k] * 0.0;
            for (j = 0; j < 3; ++j)
                for (l = 0; l < 3; ++l) D2[(a * 3 + j) * 3 + l] = H[j][l];
        }
        return 6;
    }
    case OR_PYR5:
        for (a = 0; a < 4; ++a) {
            double sx = hex_sign[a][0], sy = hex_sign[a][1];
            double fx = 1.0 + sx * r, fy = 1.0 + sy * s, fz = 1.0 - t;
            double H[3][3];
            H[0][0] = 0.0; H[1][1] = 0.0; H[2][2] = 0.0;
            H[0][1] = H[1][0] = sx * sy * fz / 8.0;
            H[0][2] = H[2][0] = -sx * fy / 8.0;
            H[1][2] = H[2][1] = -fx * sy / 8.0;
            for (j = 0; j < 3; ++j)
                for (l = 0; l < 3; ++l) D2[(a * 3 + j) * 3 + l] = H[j][l];
        }
        for (j = 0; j < 9; ++j) D2[36 + j] = 0.0; /* apex (1 + t) / 2 */
        return 5;
    }
    return -1;
}

/*
 * Subgrid scale of one element (Section 2.1.3: the subgrid scale comes from
 * an element-wise equation, utilde = tau^-1 (R u + b) with a diagonal tau
 * and a rectangular R, in a plain loop over elements, no system formed).
 * Read for the problems assembled here: at Gauss point q,
 *   utilde_q = tau_e (f_e + L(u_h)(x_q)),
 * L(u) = Laplacian of u (Poisson, -Lap u = f) or div sigma(u) =
 * mu Lap u + (lam + mu) grad div u (linear elasticity), u_h = sum_a N_a u_a,
 * tau_e = h_e^2 / (4 k), h_e = V_e^(1/3), V_e = sum_q w_q detJ_q, k = 1
 * (Poisson) or mu_e (elasticity). The paper's diagonal matrix is 1/tau_e on
 * every (Gauss point, component); R u + b is the strong residual.
 * Physical second derivatives of u_h follow from differentiating
 * u(x(xi)) twice: H_xi = J^T H_x J + sum_k (du/dx_k) H_xi(x_k), so
 * H_x = J^-T (H_xi(u) - sum_k (du/dx_k) H_xi(x_k)) J^-1.
 * U[a*B + c]: nodal values; out[q*B + c]. Returns 0, or 1 + q when
 * detJ <= 0 at Gauss point q.
 */
int or_element_subscale(int type, int model, const double *X, double young, double nu,
                        const double *U, const double *f, double *out)
{
    double pts[8 * 3], w[8], N[8], dN[24], D2[72], G[8][3], Ji[3][3], Jm[3][3];
    double r[8][3];
    int nn = or_nodes(type), nq = or_rule(type, pts, w), B = (model == OR_POISSON) ? 1 : 3;
    int a, c, i, j, k, l, m, q;
    double lam = 0.0, mu = 1.0, V = 0.0;
    if (model != OR_POISSON) lame(young, nu, &lam, &mu);
    for (q = 0; q < nq; ++q) {
        or_shape(type, &pts[3 * q], N, dN);
        or_shape2(type, &pts[3 * q], D2);
        double detJ = point_geometry(nn, X, dN, G);
        if (!(detJ > 0.0)) return 1 + q;
        for (i = 0; i < 3; ++i)
            for (j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (a = 0; a < nn; ++a) acc += X[3 * a + i] * dN[3 * a + j];
                Jm[i][j] = acc;
            }
        inv3(Jm, Ji);
        V += w[q] * detJ;
        double gu[3][3], Hx_geo[3][3][3], H[3][3][3];
        /* du_c/dx_k */
        for (c = 0; c < B; ++c)
            for (k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (a = 0; a < nn; ++a) acc += U[a * B + c] * G[a][k];
                gu[c][k] = acc;
            }
        /* second xi-derivatives of the geometry x_k(xi) */
        for (k = 0; k < 3; ++k)
            for (j = 0; j < 3; ++j)
                for (l = 0; l < 3; ++l) {
                    double acc = 0.0;
                    for (a = 0; a < nn; ++a) acc += X[3 * a + k] * D2[(a * 3 + j) * 3 + l];
                    Hx_geo[k][j][l] = acc;
                }
        for (c = 0; c < B; ++c) {
            double M[3][3];
            for (j = 0; j < 3; ++j)
                for (l = 0; l < 3; ++l) {
                    double acc = 0.0;
                    for (a = 0; a < nn; ++a) acc += U[a * B + c] * D2[(a * 3 + j) * 3 + l];
                    for (k = 0; k < 3; ++k) acc -= gu[c][k] * Hx_geo[k][j][l];
                    M[j][l] = acc;
                }
            /* H = J^-T M J^-1 */
            for (i = 0; i < 3; ++i)
                for (m = 0; m < 3; ++m) {
                    double acc = 0.0;
                    for (j = 0; j < 3; ++j)
                        for (l = 0; l < 3; ++l) acc += Ji[j][i] * M[j][l] * Ji[l][m];
                    H[c][i][m] = acc;
                }
        }
        if (B == 1) {
            r[q][0] = f[0] + (H[0][0][0] + H[0][1][1] + H[0][2][2]);
        } else {
            for (i = 0; i < 3; ++i) {
                double lap = H[i][0][0] + H[i][1][1] + H[i][2][2];
                double gdiv = H[0][i][0] + H[1][i][1] + H[2][i][2];
                r[q][i] = f[i] + (mu * lap + (lam + mu) * gdiv);
            }
        }
    }
    double h = cbrt(V);
    double tau = h * h / (4.0 * (model == OR_POISSON ? 1.0 : mu));
    for (q = 0; q < nq; ++q)
        for (c = 0; c < B; ++c) out[q * B + c] = tau * r[q][c];
    return 0;
}

/* Subgrid scale of every element, in element order: element e's Gauss
 * points at gp_ptr[e] .. gp_ptr[e+1] (gp_ptr[0] = 0, its Gauss-point counts
 * summed), out[(gp_ptr[e] + q) * B + c]. u: nodal field, B values per node
 * (node-major). Returns 0, or -(1 + e) for a rejected element. */
int64_t or_subscale(int64_t n_elems, const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                    const double *x, const double *y, const double *z, int model, const double *young,
                    const double *nu, const double *u, const double *source, int64_t *gp_ptr, double *out)
{
    double X[24], U[24], pts[24], w[8];
    int B = (model == OR_POISSON) ? 1 : 3;
    int64_t e;
    gp_ptr[0] = 0;
    for (e = 0; e < n_elems; ++e) gp_ptr[e + 1] = gp_ptr[e] + or_rule(types[e], pts, w);
    for (e = 0; e < n_elems; ++e) {
        int nn = or_nodes(types[e]), a, c;
        for (a = 0; a < nn; ++a) {
            int32_t v = conn[conn_ptr[e] + a];
            X[3 * a + 0] = x[v]; X[3 * a + 1] = y[v]; X[3 * a + 2] = z[v];
            for (c = 0; c < B; ++c) U[a * B + c] = u[(int64_t)v * B + c];
        }
        if (or_element_subscale(types[e], model, X, young ? young[e] : 1.0, nu ? nu[e] : 0.0, U,
                                &source[e * B], &out[gp_ptr[e] * B]))
            return -(1 + e);
    }
    return 0;
}

/* ------------------------------------------------------------------ *
 * Sparsity pattern, element-to-nonzero map and inverse map.           *
 * ------------------------------------------------------------------ */
static int cmp_i32(const void *p, const void *q)
{
    int32_t a = *(const int32_t *)p, b = *(const int32_t *)q;
    return (a > b) - (a < b);
}

/* node -> incident elements (ascending), as a CSR; caller frees. */
static int node_elements(int64_t n_nodes, int64_t n_elems, const int64_t *conn_ptr,
                         const int32_t *conn, int64_t **ptr_out, int64_t **lst_out)
{
    int64_t *ptr = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int64_t *cur, *lst, e, k;
    if (!ptr) return -1;
    for (e = 0; e < n_elems; ++e)
        for (k = conn_ptr[e]; k < conn_ptr[e + 1]; ++k) ptr[conn[k] + 1]++;
    for (k = 0; k < n_nodes; ++k) ptr[k + 1] += ptr[k];
    lst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ptr[n_nodes] + 1));
    cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    if (!lst || !cur) { free(ptr); free(lst); free(cur); return -1; }
    memcpy(cur, ptr, sizeof(int64_t) * (size_t)n_nodes);
    for (e = 0; e < n_elems; ++e)
        for (k = conn_ptr[e]; k < conn_ptr[e + 1]; ++k) lst[cur[conn[k]]++] = e;
    free(cur);
    *ptr_out = ptr;
    *lst_out = lst;
    return 0;
}

/* Collects row i's sorted unique columns into buf (returns the count). */
static int64_t row_columns(int64_t i, const int64_t *nptr, const int64_t *nlst,
                           const int64_t *conn_ptr, const int32_t *conn, int32_t *buf)
{
    int64_t m = 0, p, k, out = 0;
    for (p = nptr[i]; p < nptr[i + 1]; ++p) {
        int64_t e = nlst[p];
        for (k = conn_ptr[e]; k < conn_ptr[e + 1]; ++k) buf[m++] = conn[k];
    }
    qsort(buf, (size_t)m, sizeof(int32_t), cmp_i32);
    for (p = 0; p < m; ++p)
        if (out == 0 || buf[p] != buf[out - 1]) buf[out++] = buf[p];
    return out;
}

/*
 * Pass 1: row_ptr[n_nodes+1] (block rows) and map_ptr[n_elems+1].
 * Validates the mesh; returns 0, or -(1 + e) for the first bad element e
 * (node id out of range, a node repeated inside the element, unknown type,
 * or a conn_ptr range that does not match the type).
 */
int64_t or_graph_rows(int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                      const int64_t *conn_ptr, const int32_t *conn,
                      int64_t *row_ptr, int64_t *map_ptr)
{
    int64_t e, i, k, l, *nptr, *nlst;
    int32_t *buf;
    for (e = 0; e < n_elems; ++e) {
        int nn = or_nodes(types[e]);
        if (nn < 0 || conn_ptr[e + 1] - conn_ptr[e] != nn) return -(1 + e);
        for (k = conn_ptr[e]; k < conn_ptr[e + 1]; ++k) {
            if (conn[k] < 0 || conn[k] >= n_nodes) return -(1 + e);
            for (l = conn_ptr[e]; l < k; ++l)
                if (conn[l] == conn[k]) return -(1 + e);
        }
    }
    map_ptr[0] = 0;
    for (e = 0; e < n_elems; ++e) {
        int64_t nn = conn_ptr[e + 1] - conn_ptr[e];
        map_ptr[e + 1] = map_ptr[e] + nn * nn;
    }
    if (node_elements(n_nodes, n_elems, conn_ptr, conn, &nptr, &nlst)) return -(1 + n_elems) - 1;
    int64_t maxc = 0;
    for (i = 0; i < n_nodes; ++i) {
        int64_t c = 0, p;
        for (p = nptr[i]; p < nptr[i + 1]; ++p) c += conn_ptr[nlst[p] + 1] - conn_ptr[nlst[p]];
        if (c > maxc) maxc = c;
    }
    buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxc + 1));
    row_ptr[0] = 0;
    for (i = 0; i < n_nodes; ++i)
        row_ptr[i + 1] = row_ptr[i] + row_columns(i, nptr, nlst, conn_ptr, conn, buf);
    free(buf);
    free(nptr);
    free(nlst);
    return 0;
}

/* Pass 2: col[nnz], e2nnz[map_len], inv_ptr[nnz+1], inv[map_len]. */
int or_graph_fill(int64_t n_nodes, int64_t n_elems, const int64_t *conn_ptr,
                  const int32_t *conn, const int64_t *row_ptr, const int64_t *map_ptr,
                  int32_t *col, int32_t *e2nnz, int64_t *inv_ptr, int32_t *inv)
{
    int64_t e, i, k, *nptr, *nlst, *cur;
    int32_t *buf;
    int64_t nnz = row_ptr[n_nodes];
    if (node_elements(n_nodes, n_elems, conn_ptr, conn, &nptr, &nlst)) return -1;
    int64_t maxc = 0;
    for (i = 0; i < n_nodes; ++i) {
        int64_t c = 0, p;
        for (p = nptr[i]; p < nptr[i + 1]; ++p) c += conn_ptr[nlst[p] + 1] - conn_ptr[nlst[p]];
        if (c > maxc) maxc = c;
    }
    buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxc + 1));
    for (i = 0; i < n_nodes; ++i) {
        int64_t m = row_columns(i, nptr, nlst, conn_ptr, conn, buf);
        memcpy(&col[row_ptr[i]], buf, sizeof(int32_t) * (size_t)m);
    }
    free(buf);
    free(nptr);
    free(nlst);
    /* e2nnz by binary search of column conn[b] in row conn[a] */
    for (e = 0; e < n_elems; ++e) {
        int64_t nn = conn_ptr[e + 1] - conn_ptr[e], a, b;
        for (a = 0; a < nn; ++a) {
            int32_t r = conn[conn_ptr[e] + a];
            for (b = 0; b < nn; ++b) {
                int32_t c = conn[conn_ptr[e] + b];
                int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1, found = -1;
                while (lo <= hi) {
                    int64_t mid = lo + (hi - lo) / 2;
                    if (col[mid] == c) { found = mid; break; }
                    if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
                }
                if (found < 0) return -2;
                e2nnz[map_ptr[e] + a * nn + b] = (int32_t)found;
            }
        }
    }
    /* inverse map: count per block, prefix, then fill in slot order,
       which is ascending element order */
    int64_t map_len = map_ptr[n_elems], s;
    memset(inv_ptr, 0, sizeof(int64_t) * (size_t)(nnz + 1));
    for (s = 0; s < map_len; ++s) inv_ptr[e2nnz[s] + 1]++;
    for (k = 0; k < nnz; ++k) inv_ptr[k + 1] += inv_ptr[k];
    cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz + 1));
    memcpy(cur, inv_ptr, sizeof(int64_t) * (size_t)nnz);
    for (s = 0; s < map_len; ++s) inv[cur[e2nnz[s]]++] = (int32_t)s;
    free(cur);
    return 0;
}

/* Greedy first-fit colouring in element order: each element takes the
   smallest colour not used by an earlier element sharing one of its nodes. */
int or_colour_greedy(int64_t n_nodes, int64_t n_elems, const int64_t *conn_ptr,
                     const int32_t *conn, int16_t *colour)
{
    int64_t *nptr, *nlst, e, k, p;
    unsigned char used[4096];
    int ncol = 0;
    if (node_elements(n_nodes, n_elems, conn_ptr, conn, &nptr, &nlst)) return -1;
    for (e = 0; e < n_elems; ++e) {
        memset(used, 0, sizeof(used));
        for (k = conn_ptr[e]; k < conn_ptr[e + 1]; ++k) {
            int32_t v = conn[k];
            for (p = nptr[v]; p < nptr[v + 1]; ++p) {
                int64_t o = nlst[p];
                if (o < e) used[colour[o]] = 1;
            }
        }
        int c = 0;
        while (c < 4095 && used[c]) ++c;
        colour[e] = (int16_t)c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(nptr);
    free(nlst);
    return ncol;
}

/* ------------------------------------------------------------------ *
 * Assembly, Algorithm 1: elements in ascending order.                 *
 * ------------------------------------------------------------------ */
/*
 * model: OR_POISSON (B = 1, source[e]) or OR_ELASTIC (B = 3, source[3e+i],
 * nh_flag[e] != 0 selects the neo-Hookean tangent at displacement u[3*node+i];
 * nh_flag may be NULL). vals[nnz*B*B] and rhs[n_nodes*B] are overwritten;
 * tvals/trhs (may be NULL) receive the absolute-term sums.
 * Returns 0, or -(1 + e) for the first element with detJ <= 0 (or det F <= 0).
 */
int64_t or_assemble(int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                    const int64_t *conn_ptr, const int32_t *conn, const double *x,
                    const double *y, const double *z, int model, const double *young,
                    const double *nu, const uint8_t *nh_flag, const double *u,
                    const double *source, const int64_t *row_ptr, const int64_t *map_ptr,
                    const int32_t *e2nnz, double *vals, double *rhs, double *tvals,
                    double *trhs)
{
    int B = (model == OR_POISSON) ? 1 : 3;
    int64_t nnz = row_ptr[n_nodes], e;
    double X[24], U[24], Ke[64 * 9], fe[24], Tk[64 * 9], Tf[24];
    memset(vals, 0, sizeof(double) * (size_t)(nnz * B * B));
    memset(rhs, 0, sizeof(double) * (size_t)(n_nodes * B));
    if (tvals) memset(tvals, 0, sizeof(double) * (size_t)(nnz * B * B));
    if (trhs) memset(trhs, 0, sizeof(double) * (size_t)(n_nodes * B));
    for (e = 0; e < n_elems; ++e) {
        int nn = or_nodes(types[e]), a, b, i, j;
        int nh = (model != OR_POISSON && nh_flag && nh_flag[e]) ? 1 : 0;
        for (a = 0; a < nn; ++a) {
            int32_t v = conn[conn_ptr[e] + a];
            X[3 * a + 0] = x[v]; X[3 * a + 1] = y[v]; X[3 * a + 2] = z[v];
            if (nh)
                for (i = 0; i < 3; ++i) U[3 * a + i] = u[3 * (int64_t)v + i];
        }
        if (or_element(types[e], model, nh, X, young ? young[e] : 1.0, nu ? nu[e] : 0.0, U,
                       &source[e * B], Ke, fe, tvals ? Tk : NULL, trhs ? Tf : NULL))
            return -(1 + e);
        for (a = 0; a < nn; ++a) {
            int32_t r = conn[conn_ptr[e] + a];
            for (b = 0; b < nn; ++b) {
                int64_t blk = e2nnz[map_ptr[e] + a * nn + b];
                for (i = 0; i < B; ++i)
                    for (j = 0; j < B; ++j) {
                        int64_t o = ((int64_t)(a * nn + b) * B + i) * B + j;
                        vals[blk * B * B + i * B + j] += Ke[o];
                        if (tvals) tvals[blk * B * B + i * B + j] += Tk[o];
                    }
            }
            for (i = 0; i < B; ++i) {
                rhs[(int64_t)r * B + i] += fe[a * B + i];
                if (trhs) trhs[(int64_t)r * B + i] += Tf[a * B + i];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ *
 * Parallel timing variants of Algorithm 1 (the CPU baseline).         *
 * ------------------------------------------------------------------ */

/* Threads the OpenMP variants use (1 without OpenMP). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* A^e and b^e of element e and their scatter, in a thread's own buffers:
 * atomic != 0 adds with atomic updates. Returns 0 or -(1 + e). */
static int64_t omp_element(int64_t e, const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                           const double *x, const double *y, const double *z, int model, const double *young,
                           const double *nu, const uint8_t *nh_flag, const double *u, const double *source,
                           const int64_t *map_ptr, const int32_t *e2nnz, double *vals, double *rhs, int atomic)
{
    double X[24], U[24], Ke[64 * 9], fe[24];
    int B = (model == OR_POISSON) ? 1 : 3;
    int nn = or_nodes(types[e]), a, b, i, j;
    int nh = (model != OR_POISSON && nh_flag && nh_flag[e]) ? 1 : 0;
    for (a = 0; a < nn; ++a) {
        int32_t v = conn[conn_ptr[e] + a];
        X[3 * a + 0] = x[v]; X[3 * a + 1] = y[v]; X[3 * a + 2] = z[v];
        if (nh)
            for (i = 0; i < 3; ++i) U[3 * a + i] = u[3 * (int64_t)v + i];
    }
    if (or_element(types[e], model, nh, X, young ? young[e] : 1.0, nu ? nu[e] : 0.0, U, &source[e * B], Ke, fe,
                   NULL, NULL))
        return -(1 + e);
    for (a = 0; a < nn; ++a) {
        int32_t r = conn[conn_ptr[e] + a];
        for (b = 0; b < nn; ++b) {
            int64_t blk = e2nnz[map_ptr[e] + a * nn + b];
            for (i = 0; i < B; ++i)
                for (j = 0; j < B; ++j) {
                    double *d = &vals[blk * B * B + i * B + j];
                    double v = Ke[((int64_t)(a * nn + b) * B + i) * B + j];
                    if (atomic) {
#ifdef _OPENMP
#pragma omp atomic update
#endif
                        *d += v;
                    } else {
                        *d += v;
                    }
                }
        }
        for (i = 0; i < B; ++i) {
            double *d = &rhs[(int64_t)r * B + i];
            if (atomic) {
#ifdef _OPENMP
#pragma omp atomic update
#endif
                *d += fe[a * B + i];
            } else {
                *d += fe[a * B + i];
            }
        }
    }
    return 0;
}

/*
 * Algorithm 1 with the element loop shared by OpenMP threads, for timing
 * (same arguments as or_assemble, no |term| sums):
 *   variant 1: every element in parallel, A^e and b^e added with atomic
 *              updates (the paper's Algorithm 4);
 *   variant 2: colour by colour, the elements of one colour in parallel
 *              with plain updates (Algorithm 5): colour c's elements are
 *              celems[cptr[c] .. cptr[c+1]), and no two of them share a node.
 * Sums are taken in a thread-dependent order, so the result equals
 * or_assemble's up to rounding. Returns 0, or -(1 + e) for a rejected
 * element (the smallest such e among those that were run).
 */
int64_t or_assemble_omp(int variant, int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                        const int64_t *conn_ptr, const int32_t *conn, const double *x, const double *y,
                        const double *z, int model, const double *young, const double *nu,
                        const uint8_t *nh_flag, const double *u, const double *source, const int64_t *row_ptr,
                        const int64_t *map_ptr, const int32_t *e2nnz, const int64_t *cptr,
                        const int32_t *celems, int n_colours, double *vals, double *rhs)
{
    int B = (model == OR_POISSON) ? 1 : 3;
    int64_t nnz = row_ptr[n_nodes], bad = 0;
    memset(vals, 0, sizeof(double) * (size_t)(nnz * B * B));
    memset(rhs, 0, sizeof(double) * (size_t)(n_nodes * B));
    if (variant == 1) {
        int64_t e;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256) reduction(min : bad)
#endif
        for (e = 0; e < n_elems; ++e) {
            int64_t rc = omp_element(e, types, conn_ptr, conn, x, y, z, model, young, nu, nh_flag, u, source,
                                     map_ptr, e2nnz, vals, rhs, 1);
            if (rc < bad) bad = rc;
        }
    } else if (variant == 2) {
        int c;
        for (c = 0; c < n_colours; ++c) {
            int64_t k;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256) reduction(min : bad)
#endif
            for (k = cptr[c]; k < cptr[c + 1]; ++k) {
                int64_t rc = omp_element(celems[k], types, conn_ptr, conn, x, y, z, model, young, nu, nh_flag,
                                         u, source, map_ptr, e2nnz, vals, rhs, 0);
                if (rc < bad) bad = rc;
            }
        }
    } else {
        return -(1 + n_elems);
    }
    return bad;
}
