// Element-wise subgrid scale (Section 2.1.3): the subscale comes from an
// equation posed element by element -- the strong residual at the Gauss
// points times a diagonal stabilisation matrix -- evaluated in a plain loop
// over the elements with no system formed and nothing scattered. Read for
// the problems this library assembles:
//   utilde_q = tau_e (f_e + L(u_h)(x_q)),   tau_e = V_e^(2/3) / (4 k),
// L the Laplacian (Poisson, -Lap u = f, k = 1) or div sigma(u) =
// mu Lap u + (lam + mu) grad div u (linear elasticity, k = mu_e), u_h the
// interpolated nodal field, V_e = sum_q w_q detJ_q.
//
// Physical second derivatives: differentiating u(x(xi)) twice gives
//   H_xi(u) = J^T H_x(u) J + sum_k (du/dx_k) H_xi(x_k),
// so H_x(u) = J^-T M J^-1 with M = H_xi(u) - sum_k (du/dx_k) H_xi(x_k).
// Every shape function here is linear in each reference coordinate taken
// alone (tet4 linear, hex8 and the collapsed-hexahedron pyramid
// multilinear, pen6 linear in (r, s) times linear in t), so the pure
// second reference derivatives vanish and M has only its three mixed
// entries (xi eta, xi zeta, eta zeta). For tet4 all of them vanish:
// L(u_h) = 0 identically and u is not read.
//
// Work layout: one launch per element family over its type-sorted
// elements; one lane per (element, Gauss point), NQ consecutive lanes per
// element, 256 / NQ elements per workgroup. The element's first NN lanes
// each gather one node's coordinates and field values into LDS (one
// dependent load chain per lane instead of one per node: gathers walked
// node by node left the kernel waiting on memory latency). Over the
// reference element every field is a polynomial with as many coefficients
// as the family has Gauss points (hex8 and the pyramid: the eight
// monomials of the trilinear hexahedron; pen6: A(r, s) + t B(r, s) with A,
// B linear), so lane q forms coefficient q of every field from the node
// values, the coefficients replace the node values in LDS, and each lane
// evaluates J, grad_xi u and the mixed second reference derivatives at its
// Gauss point from them (a few FMAs per field instead of a sum over the
// nodes: about 5% faster, the lanes holding fewer registers). tet4, one
// lane per element and no second derivatives, sums its four nodes
// directly. The element volume is summed over the element's Gauss points
// in ascending order through LDS, and each lane writes its B values at
// the element's Gauss-point offset.
#include <algorithm>
#include <climits>

#include "elem.h"

namespace fea {

// Gauss coordinate of the two-point rule, as in the reference tables.
constexpr double kGauss = 0.57735026918962576451;

struct SubArgs {
    const double *x, *y, *z;
    const double *u;       // B values per node, node-major
    const double *young;   // per element, NULL = 1
    const double *nu;      // per element (elasticity)
    const double *source;  // B values per element
    const int32_t *perm;   // this family's element ids (type-sorted order)
    const int32_t *pnodes; // their node ids, NN per element
    const int64_t *gp_ptr; // Gauss-point offsets in element order
    int64_t n;             // elements in this launch
    double *out;           // out[(gp_ptr[e] + q) * B + c]
    int32_t *status;       // smallest element id with detJ <= 0
};

// SubArgs as the batched kernel reads them from its table: every pointer
// typed as addressing global memory, so that the compiler keeps global
// instead of flat accesses (see ElemArgsGlobal).
#define FEA_G(T) T __attribute__((address_space(1))) *
struct SubArgsGlobal {
    FEA_G(const double) x;
    FEA_G(const double) y;
    FEA_G(const double) z;
    FEA_G(const double) u;
    FEA_G(const double) young;
    FEA_G(const double) nu;
    FEA_G(const double) source;
    FEA_G(const int32_t) perm;
    FEA_G(const int32_t) pnodes;
    FEA_G(const int64_t) gp_ptr;
    int64_t n;
    FEA_G(double) out;
    FEA_G(int32_t) status;
};
#undef FEA_G
static_assert(sizeof(SubArgsGlobal) == sizeof(SubArgs) && offsetof(SubArgsGlobal, status) == offsetof(SubArgs, status),
              "SubArgsGlobal mirrors SubArgs");

__device__ __forceinline__ SubArgs from_global(const SubArgsGlobal &g)
{
    SubArgs a;
    a.x = (const double *)g.x;
    a.y = (const double *)g.y;
    a.z = (const double *)g.z;
    a.u = (const double *)g.u;
    a.young = (const double *)g.young;
    a.nu = (const double *)g.nu;
    a.source = (const double *)g.source;
    a.perm = (const int32_t *)g.perm;
    a.pnodes = (const int32_t *)g.pnodes;
    a.gp_ptr = (const int64_t *)g.gp_ptr;
    a.n = g.n;
    a.out = (double *)g.out;
    a.status = (int32_t *)g.status;
    return a;
}

// LDS of one workgroup. Strides padded to 2 (mod 4) doubles: the 8 Gauss
// points or elements that a wave reads at once then start in distinct
// 16-byte bank slots (hex8's 48-double element records aliased every
// second element).
template <int T, int MODEL>
struct SubSmem {
    static constexpr int NN = Fam<T>::NN, NQ = Fam<T>::NQ, EPW = 256 / NQ;
    static constexpr int B = MODEL == FEA_POISSON ? 1 : 3;
    static constexpr int NV = 3 + B;                                    // node values
    static constexpr int SQ = NN * 3 + ((2 - (NN * 3) % 4) + 4) % 4;    // per Gauss point of a table
    // per element: its nodes' values, then (same space) its NQ coefficients
    static constexpr int NR = NN > NQ ? NN : NQ;
    static constexpr int SE = NR * NV + ((2 - (NR * NV) % 4) + 4) % 4;
    double sDN[T == 0 ? NQ * SQ : 1];  // reference gradients (tet4; the others use coefficients)
    double sWq[NQ];
    double sWd[256];
    double sNode[(T == 0 ? 1 : EPW) * SE];  // node coordinates and field values
};

// Reference tables of family T into LDS (the caller synchronises).
template <int T, int MODEL>
__device__ inline void sub_tables(SubSmem<T, MODEL> &S)
{
    using Sm = SubSmem<T, MODEL>;
    constexpr int NN = Sm::NN, NQ = Sm::NQ, SQ = Sm::SQ;
    const int tid = threadIdx.x;
    if constexpr (T == 0) {
        for (int i = tid; i < NQ * NN * 3; i += 256) {
            const int q = i / (NN * 3), a = (i / 3) % NN, j = i % 3;
            S.sDN[q * SQ + a * 3 + j] = c_ref.dN[T][q][a][j];
        }
    }
    if (tid < NQ) S.sWq[tid] = c_ref.w[T][tid];
}

// First and mixed second reference derivatives of field f at Gauss point q
// of family T (pyr5, pen6, hex8) from the element's NQ polynomial
// coefficients c[m * NV + f] (see sub_group): d[j] = df/dxi_j, m2 = the
// mixed pairs (0, 1), (0, 2), (1, 2).
template <int T, int NV>
__device__ inline void sub_eval(const double *c, const int f, const int q, double d[3], double m2[3])
{
    if constexpr (T == 2) {
        // A(r, s) + t B(r, s): coefficients A0, A1, A2, B0, B1, B2
        constexpr double tr[3][2] = {{1.0 / 6, 1.0 / 6}, {2.0 / 3, 1.0 / 6}, {1.0 / 6, 2.0 / 3}};
        const double r = tr[q % 3][0], sc = tr[q % 3][1], t = q < 3 ? -kGauss : kGauss;
        const double A1 = c[1 * NV + f], A2 = c[2 * NV + f], B0 = c[3 * NV + f], B1 = c[4 * NV + f],
                     B2 = c[5 * NV + f];
        d[0] = A1 + t * B1;
        d[1] = A2 + t * B2;
        d[2] = B0 + B1 * r + B2 * sc;
        m2[0] = 0.0;
        m2[1] = B1;
        m2[2] = B2;
    } else {
        // sum_m c_m xi^m, m a bit mask of the coordinates
        const double x0 = (q & 1) ? kGauss : -kGauss, x1 = (q & 2) ? kGauss : -kGauss, x2 = (q & 4) ? kGauss : -kGauss;
        const double c1 = c[1 * NV + f], c2 = c[2 * NV + f], c3 = c[3 * NV + f], c4 = c[4 * NV + f],
                     c5 = c[5 * NV + f], c6 = c[6 * NV + f], c7 = c[7 * NV + f];
        m2[0] = c3 + c7 * x2;
        m2[1] = c5 + c7 * x1;
        m2[2] = c6 + c7 * x0;
        d[0] = c1 + c3 * x1 + m2[1] * x2;
        d[1] = c2 + c3 * x0 + m2[2] * x2;
        d[2] = c4 + c5 * x0 + m2[2] * x1;
    }
}

// One group of up to EPW consecutive elements of a family, type-sorted
// positions p0 .. min(p0 + EPW, pend). Every lane of the workgroup calls it;
// it starts with a barrier (the previous group's readers of S are done)
// and lanes without an element only take part in the barriers.
template <int T, int MODEL>
__device__ void sub_group(const SubArgs &A, int64_t p0, int64_t pend, SubSmem<T, MODEL> &S)
{
    using Sm = SubSmem<T, MODEL>;
    constexpr int NN = Sm::NN, NQ = Sm::NQ, EPW = Sm::EPW, B = Sm::B, NV = Sm::NV, SQ = Sm::SQ, SE = Sm::SE;
    const double *sDN = S.sDN, *sWq = S.sWq;
    double *sWd = S.sWd, *sNode = S.sNode;
    const int tid = threadIdx.x;
    __syncthreads();
    const int el = tid / NQ, q = tid - el * NQ;
    const int64_t p = p0 + el;
    const bool act = el < EPW && p < pend;
    const int32_t e = act ? A.perm[p] : 0;
    double wd = 0.0, kmat = 1.0;  // w_q detJ; tau's material constant k
    double r[B];
#pragma unroll
    for (int c = 0; c < B; ++c) r[c] = 0.0;
    if constexpr (T != 0) {
        if (act && q < NN) {
            const int32_t v = A.pnodes[p * NN + q];
            double *rec = sNode + el * SE + q * NV;
            rec[0] = A.x[v];
            rec[1] = A.y[v];
            rec[2] = A.z[v];
#pragma unroll
            for (int c = 0; c < B; ++c) rec[3 + c] = A.u[(int64_t)v * B + c];
        }
        __syncthreads();  // every lane, active or not
    }
    double J[3][3] = {}, Dx[3][3] = {};
    if constexpr (T == 0) {
        if (act) {
            // tet4: constant gradients, no second derivatives
            const int32_t *pn = A.pnodes + p * NN;
#pragma unroll 1
            for (int a = 0; a < NN; ++a) {
                const int32_t v = pn[a];
                const double X[3] = {A.x[v], A.y[v], A.z[v]};
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double dn = sDN[q * SQ + a * 3 + j];
#pragma unroll
                    for (int i = 0; i < 3; ++i) J[i][j] += X[i] * dn;
                }
            }
        }
    } else {
        // Every field f (coordinates, then the field's B components) is,
        // over the reference element, a polynomial with NQ coefficients:
        // hex8 and the collapsed-hexahedron pyramid sum_m c_m xi^m over the
        // eight monomials m of {1, xi0, xi1, xi0 xi1, xi2, ...} (m read as
        // a bit mask of the coordinates), pen6 A(r, s) + t B(r, s) with A
        // and B linear. Lane q of an element forms coefficient q of every
        // field from the node values, the coefficients replace the node
        // values in LDS, and each lane evaluates the first and mixed second
        // reference derivatives at its Gauss point from them.
        double cf[NV];
        if (act) {
            const double *nv = sNode + el * SE;
#pragma unroll
            for (int f = 0; f < NV; ++f) cf[f] = 0.0;
            if constexpr (T == 2) {
                // P_k = (v_k + v_k+3) / 2, Q_k = (v_k+3 - v_k) / 2; coefficients
                // A0 = P0, A1 = P1 - P0, A2 = P2 - P0, B0 = Q0, B1 = Q1 - Q0, B2 = Q2 - Q0
                const int k = q % 3, top = q / 3;
#pragma unroll
                for (int f = 0; f < NV; ++f) {
                    const double v0 = nv[0 * NV + f], v3 = nv[3 * NV + f];
                    const double vk = nv[k * NV + f], vk3 = nv[(k + 3) * NV + f];
                    const double c0 = top ? 0.5 * (v3 - v0) : 0.5 * (v0 + v3);
                    const double ck = top ? 0.5 * (vk3 - vk) : 0.5 * (vk + vk3);
                    cf[f] = k == 0 ? c0 : ck - c0;
                }
            } else {
                // c_m = 1/8 sum_a s_m(a) v_a, s_m(a) the product of node a's
                // corner signs over the coordinates in m; the pyramid's apex
                // stands for the four collapsed top corners
                constexpr int PLUS[8] = {0, 1, 3, 2, 4, 5, 7, 6};  // corner a: bit d set where its sign is +
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    const int node = (T == 1 && a > 4) ? 4 : a;
                    const bool neg = __builtin_popcount(q & ~PLUS[a] & 7) & 1;
#pragma unroll
                    for (int f = 0; f < NV; ++f) {
                        const double v = nv[node * NV + f];
                        cf[f] += neg ? -v : v;
                    }
                }
#pragma unroll
                for (int f = 0; f < NV; ++f) cf[f] *= 0.125;
            }
        }
        __syncthreads();  // every lane has read the node values
        if (act) {
#pragma unroll
            for (int f = 0; f < NV; ++f) sNode[el * SE + q * NV + f] = cf[f];
        }
        __syncthreads();
        if (act) {
            const double *c = sNode + el * SE;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double d[3], m2[3];
                sub_eval<T, NV>(c, i, q, d, m2);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    J[i][j] = d[j];
                    Dx[i][j] = m2[j];
                }
            }
        }
    }
    if (act) {
        // J^-1 by the adjugate
        double Ji[3][3];
        Ji[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        Ji[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        Ji[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        Ji[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        Ji[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        Ji[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        Ji[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        Ji[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        Ji[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * Ji[0][0] + J[0][1] * Ji[1][0] + J[0][2] * Ji[2][0];
        if (!(det > 0.0)) atomicMin(A.status, e);
        const double id = 1.0 / det;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Ji[i][j] *= id;
        wd = sWq[q] * det;

        double lam = 0.0, mu = 1.0;
        if constexpr (MODEL != FEA_POISSON) {
            const double E = A.young ? A.young[e] : 1.0, nu = A.nu[e];
            lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
            mu = E / (2.0 * (1.0 + nu));
            kmat = mu;
        }
#pragma unroll
        for (int c = 0; c < B; ++c) r[c] = A.source[(int64_t)e * B + c];
        if constexpr (T != 0) {
            constexpr int PJ[3] = {0, 0, 1}, PL[3] = {1, 2, 2};  // mixed pairs (j, l)
            // M^c on the mixed pairs: H_xi(u_c) - sum_k du_c/dx_k H_xi(x_k)
            double M[B][3];
#pragma unroll
            for (int c = 0; c < B; ++c) {
                // grad_xi u_c and its mixed second derivatives, one field at
                // a time
                double Gu[3], Du[3], g[3];
                sub_eval<T, NV>(sNode + el * SE, 3 + c, q, Gu, Du);
#pragma unroll
                for (int k = 0; k < 3; ++k) g[k] = Gu[0] * Ji[0][k] + Gu[1] * Ji[1][k] + Gu[2] * Ji[2][k];
#pragma unroll
                for (int m = 0; m < 3; ++m) M[c][m] = Du[m] - (g[0] * Dx[0][m] + g[1] * Dx[1][m] + g[2] * Dx[2][m]);
            }
            // Lap u_c = tr(J^-T M^c J^-1) = 2 sum_m M^c_m (J^-1 J^-T)_(j_m, l_m)
            double S[3];
#pragma unroll
            for (int m = 0; m < 3; ++m)
                S[m] = Ji[PJ[m]][0] * Ji[PL[m]][0] + Ji[PJ[m]][1] * Ji[PL[m]][1] + Ji[PJ[m]][2] * Ji[PL[m]][2];
            if constexpr (MODEL == FEA_POISSON) {
                r[0] += 2.0 * (M[0][0] * S[0] + M[0][1] * S[1] + M[0][2] * S[2]);
            } else {
                // (grad div u)_i = sum_k (H_x u_k)_ik = sum_j Ji[j][i] W_j with
                // W_j = sum_k sum_l M^k_jl Ji[l][k] (M^k symmetric, zero diagonal)
                double W[3];
                W[0] = W[1] = W[2] = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    W[0] += M[k][0] * Ji[1][k] + M[k][1] * Ji[2][k];
                    W[1] += M[k][0] * Ji[0][k] + M[k][2] * Ji[2][k];
                    W[2] += M[k][1] * Ji[0][k] + M[k][2] * Ji[1][k];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double lap = 2.0 * (M[i][0] * S[0] + M[i][1] * S[1] + M[i][2] * S[2]);
                    const double gdiv = Ji[0][i] * W[0] + Ji[1][i] * W[1] + Ji[2][i] * W[2];
                    r[i] += mu * lap + (lam + mu) * gdiv;
                }
            }
        }
    }
    // every lane reaches the barrier, active or not
    sWd[tid] = wd;
    __syncthreads();
    if (act) {
        double V = 0.0;
#pragma unroll
        for (int k = 0; k < NQ; ++k) V += sWd[el * NQ + k];
        const double h = cbrt(V);
        const double tau = h * h / (4.0 * kmat);
        double *o = A.out + (A.gp_ptr[e] + q) * B;
#pragma unroll
        for (int c = 0; c < B; ++c) o[c] = tau * r[c];
    }
}

template <int T, int MODEL>
__global__ void __launch_bounds__(256) k_subscale(SubArgs A)
{
    __shared__ SubSmem<T, MODEL> S;
    sub_tables(S);
    sub_group(A, (int64_t)blockIdx.x * SubSmem<T, MODEL>::EPW, A.n, S);
}

// Batched form: persistent workgroups of one family dequeue work items
// (mesh, family, first type-sorted position, count) from the batch's queue
// of that family and run the item's elements group by group with the
// arguments of the item's mesh, margs[mesh] (its view of family T). Every
// workgroup reaches the exit test after each item.
template <int T, int MODEL>
__global__ void __launch_bounds__(256) k_subscale_batch(const SubArgs *__restrict__ margs, const int4 *items,
                                                        const int32_t *order, int32_t n_items, int32_t *head)
{
    constexpr int EPW = SubSmem<T, MODEL>::EPW;
    __shared__ SubSmem<T, MODEL> S;
    __shared__ int32_t s_item;
    sub_tables(S);
    for (;;) {
        __syncthreads();  // every lane has read the previous item
        if (threadIdx.x == 0) {
            const int32_t q = atomicAdd(head, 1);
            s_item = q < n_items ? order[q] : -1;
        }
        __syncthreads();
        const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
        if (it < 0) break;
        const int4 w = items[it];
        const int32_t m = __builtin_amdgcn_readfirstlane(w.x);
        const int64_t first = __builtin_amdgcn_readfirstlane(w.z), count = __builtin_amdgcn_readfirstlane(w.w);
        const SubArgs A = from_global(reinterpret_cast<const SubArgsGlobal *>(margs)[m]);
        for (int64_t g0 = 0; g0 < count; g0 += EPW) sub_group(A, first + g0, first + count, S);
    }
}

__global__ void k_sub_status_init(int32_t *s) { *s = INT_MAX; }
__global__ void k_sub_status_final(int32_t *s)
{
    if (*s == INT_MAX) *s = -1;
}

// Gauss points per element, in element order, from the type segmentation.
template <int T>
__global__ void k_gp_counts(const int32_t *perm, int64_t n, uint8_t *cnt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) cnt[perm[i]] = (uint8_t)Fam<T>::NQ;
}

struct SubTmp {
    void *p = nullptr;
    ~SubTmp() { dfree(p); }
};

static int gauss_points_prepare(fea_graph *g, hipStream_t s)
{
    if (g->gpready) return FEA_OK;
    int rc;
    const int64_t E = g->n_elems;
    if (!g->gp_ptr && (rc = dalloc((void **)&g->gp_ptr, sizeof(int64_t) * (E + 1)))) return rc;
    int64_t n_gp = 0;
    for (int t = 0; t < 4; ++t) {
        const int nq = t == 0 ? 1 : (t == 2 ? 6 : 8);
        n_gp += (g->seg[t + 1] - g->seg[t]) * nq;
    }
    if (E > 0) {
        SubTmp cnt, tmp;
        if ((rc = dalloc(&cnt.p, (size_t)E))) return rc;
        if ((rc = dalloc(&tmp.p, sizeof(int64_t) * (scan_tmp_elems(E) + 64)))) return rc;
        uint8_t *c = (uint8_t *)cnt.p;
        const int64_t n0 = g->seg[1] - g->seg[0], n1 = g->seg[2] - g->seg[1], n2 = g->seg[3] - g->seg[2],
                      n3 = g->seg[4] - g->seg[3];
        if (n0) k_gp_counts<0><<<grid_for(n0, 256), 256, 0, s>>>(g->perm + g->seg[0], n0, c);
        if (n1) k_gp_counts<1><<<grid_for(n1, 256), 256, 0, s>>>(g->perm + g->seg[1], n1, c);
        if (n2) k_gp_counts<2><<<grid_for(n2, 256), 256, 0, s>>>(g->perm + g->seg[2], n2, c);
        if (n3) k_gp_counts<3><<<grid_for(n3, 256), 256, 0, s>>>(g->perm + g->seg[3], n3, c);
        if ((rc = scan_to_ptr_u8(c, E, g->gp_ptr, (int64_t *)tmp.p, s))) return rc;
        FEA_HIP(hipGetLastError());
        // the temporaries are freed on return: wait for their readers
        FEA_HIP(hipStreamSynchronize(s));
    } else {
        FEA_HIP(hipMemsetAsync(g->gp_ptr, 0, sizeof(int64_t), s));
        FEA_HIP(hipStreamSynchronize(s));
    }
    g->n_gp = n_gp;
    g->gpready = true;
    return FEA_OK;
}

template <int T, int MODEL>
static void launch_sub(const fea_graph *g, SubArgs a, hipStream_t s)
{
    constexpr int EPW = 256 / Fam<T>::NQ;
    a.n = g->seg[T + 1] - g->seg[T];
    if (a.n == 0) return;
    a.perm = g->perm + g->seg[T];
    a.pnodes = g->pnodes + g->node_base[T];
    k_subscale<T, MODEL><<<grid_for(a.n, EPW), 256, 0, s>>>(a);
}

template <int MODEL>
static void run_sub(const fea_graph *g, const SubArgs &a, hipStream_t s)
{
    // the costliest family first, so the cheap launches fill the tail
    launch_sub<1, MODEL>(g, a, s);
    launch_sub<3, MODEL>(g, a, s);
    launch_sub<2, MODEL>(g, a, s);
    launch_sub<0, MODEL>(g, a, s);
}

}  // namespace fea

using namespace fea;

extern "C" int fea_graph_gauss_points(const fea_graph *gc, int64_t *n_points, int64_t *gp_ptr, hipStream_t stream)
{
    clear_error();
    fea_graph *g = const_cast<fea_graph *>(gc);
    if (!g) return set_error(FEA_EINVAL, "graph is required");
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev != g->device) return set_error(FEA_EINVAL, "graph lives on device %d, current is %d", g->device, dev);
    int rc = gauss_points_prepare(g, stream);
    if (rc) return rc;
    if (n_points) *n_points = g->n_gp;
    if (gp_ptr)
        FEA_HIP(hipMemcpyAsync(gp_ptr, g->gp_ptr, sizeof(int64_t) * (g->n_elems + 1), hipMemcpyDeviceToDevice,
                               stream));
    return FEA_OK;
}

extern "C" int fea_subscale(const fea_graph *gc, const double *x, const double *y, const double *z,
                            const fea_material *mat, const double *u, const double *source,
                            hipStream_t stream, double *out, int32_t *status)
{
    clear_error();
    fea_graph *g = const_cast<fea_graph *>(gc);
    if (!g || !mat) return set_error(FEA_EINVAL, "graph and material are required");
    if (mat->model != FEA_POISSON && mat->model != FEA_ELASTIC)
        return set_error(FEA_EINVAL, "unknown model %d", mat->model);
    if (mat->nh_flag) return set_error(FEA_EINVAL, "the subgrid scale is defined for the linear models only");
    if (g->n_elems > 0) {
        if (!x || !y || !z || !u || !source || !out) return set_error(FEA_EINVAL, "NULL array argument");
        if (mat->model == FEA_ELASTIC && !mat->nu) return set_error(FEA_EINVAL, "nu is required");
    }
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev != g->device) return set_error(FEA_EINVAL, "graph lives on device %d, current is %d", g->device, dev);
    int rc;
    if ((rc = ensure_tables()) || (rc = gauss_points_prepare(g, stream))) return rc;

    int32_t *st = status;
    if (!st) {
        static thread_local int32_t *own[64] = {nullptr};
        if (!own[dev] && (rc = dalloc((void **)&own[dev], sizeof(int32_t)))) return rc;
        st = own[dev];
    }
    k_sub_status_init<<<1, 1, 0, stream>>>(st);
    if (g->n_elems > 0) {
        SubArgs a = {};
        a.x = x; a.y = y; a.z = z;
        a.u = u;
        a.young = mat->young;
        a.nu = mat->nu;
        a.source = source;
        a.gp_ptr = g->gp_ptr;
        a.out = out;
        a.status = st;
        if (mat->model == FEA_POISSON)
            run_sub<FEA_POISSON>(g, a, stream);
        else
            run_sub<FEA_ELASTIC>(g, a, stream);
    }
    k_sub_status_final<<<1, 1, 0, stream>>>(st);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

// ------------------------------------------------------------------ //
// Batched subgrid scale: the batch's work items from its device queues. //
// ------------------------------------------------------------------ //
namespace fea {

__global__ void k_sub_batch_begin(int32_t *head, int32_t *status, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < 4) head[i] = 0;
    if (i < n) status[i] = INT_MAX;
}

__global__ void k_sub_batch_end(int32_t *status, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && status[i] == INT_MAX) status[i] = -1;
}

// Resident workgroups of the batched kernel of family T on a device.
template <int T, int MODEL>
static int sub_batch_workers(int dev, int64_t *out)
{
    static int64_t cache[64] = {0};
    if (dev < 0 || dev >= 64) return set_error(FEA_EINVAL, "device index %d unsupported", dev);
    if (!cache[dev]) {
        int per = 0, cus = 0;
        FEA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_subscale_batch<T, MODEL>, 256, 0));
        FEA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cache[dev] = (int64_t)std::max(per, 1) * std::max(cus, 1);
    }
    *out = cache[dev];
    return FEA_OK;
}

template <int T>
static int launch_sub_batch(const BatchView &v, const SubArgs *d_args, hipStream_t s)
{
    const int64_t n = v.foff[T + 1] - v.foff[T];
    if (n == 0) return FEA_OK;
    int64_t w = 0;
    int rc = sub_batch_workers<T, FEA_ELASTIC>(v.device, &w);
    if (rc) return rc;
    const unsigned grid = (unsigned)std::min<int64_t>(n, w);
    k_subscale_batch<T, FEA_ELASTIC><<<grid, 256, 0, s>>>(d_args + (size_t)T * v.n_meshes, v.items,
                                                          v.order + v.foff[T], (int32_t)n, v.head + T);
    return FEA_OK;
}

// Gauss-point layouts of every mesh of a batch; off[m] = first Gauss point
// of mesh m in the concatenated output (off[n_meshes] = total).
static int batch_gauss_offsets(const BatchView &v, hipStream_t s, std::vector<int64_t> &off)
{
    off.assign((size_t)v.n_meshes + 1, 0);
    for (int m = 0; m < v.n_meshes; ++m) {
        int rc = gauss_points_prepare(v.graphs[m], s);
        if (rc) return rc;
        off[m + 1] = off[m] + v.graphs[m]->n_gp;
    }
    return FEA_OK;
}

}  // namespace fea

namespace fea {

// The subgrid scale's work items: per family, runs of 4 element groups
// (1024 tet4, 128 pyr5, 168 pen6, 128 hex8 elements) of one mesh, so that
// only a mesh's last item of a family has a partial group; the order lists
// them family by family (mesh, then position), as the queues expect.
static int sub_items_prepare(BatchView &v)
{
    if (*v.items_owner) return FEA_OK;
    const int per[4] = {4 * 256, 4 * 32, 4 * 42, 4 * 32};
    std::vector<int32_t> items;
    std::vector<int32_t> order;
    int64_t foff[5] = {0, 0, 0, 0, 0};
    for (int t = 0; t < 4; ++t) {
        foff[t] = (int64_t)order.size();
        for (int m = 0; m < v.n_meshes; ++m) {
            const fea_graph *g = v.graphs[m];
            const int64_t n = g->seg[t + 1] - g->seg[t];
            for (int64_t s0 = 0; s0 < n; s0 += per[t]) {
                order.push_back((int32_t)(items.size() / 4));
                items.push_back(m);
                items.push_back(t);
                items.push_back((int32_t)s0);
                items.push_back((int32_t)std::min<int64_t>(per[t], n - s0));
            }
        }
    }
    foff[4] = (int64_t)order.size();
    const size_t ni = order.size();
    int rc;
    int4 *d_items = nullptr;
    int32_t *d_order = nullptr;
    if ((rc = dalloc((void **)&d_items, sizeof(int4) * std::max<size_t>(ni, 1)))) return rc;
    if ((rc = dalloc((void **)&d_order, sizeof(int32_t) * std::max<size_t>(ni, 1)))) {
        dfree(d_items);
        return rc;
    }
    if (ni) {
        hipError_t e1 = hipMemcpy(d_items, items.data(), sizeof(int4) * ni, hipMemcpyHostToDevice);
        hipError_t e2 = hipMemcpy(d_order, order.data(), sizeof(int32_t) * ni, hipMemcpyHostToDevice);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            dfree(d_items);
            dfree(d_order);
            return set_error(FEA_EHIP, "uploading the subgrid-scale items failed");
        }
    }
    *v.items_owner = d_items;
    *v.order_owner = d_order;
    for (int t = 0; t < 5; ++t) v.foff_owner[t] = foff[t];
    v.items = d_items;
    v.order = d_order;
    for (int t = 0; t < 5; ++t) v.foff[t] = foff[t];
    return FEA_OK;
}

}  // namespace fea

extern "C" int fea_batch_gauss_points(fea_batch *b, int64_t *offsets, hipStream_t stream)
{
    clear_error();
    if (!b) return set_error(FEA_EINVAL, "batch is required");
    BatchView v;
    int rc = batch_view(b, &v);
    if (rc) return rc;
    std::vector<int64_t> off;
    if ((rc = batch_gauss_offsets(v, stream, off))) return rc;
    if (offsets) std::copy(off.begin(), off.end(), offsets);
    return FEA_OK;
}

extern "C" int fea_batch_subscale(fea_batch *b, hipStream_t stream, double *out, int32_t *status)
{
    clear_error();
    if (!b) return set_error(FEA_EINVAL, "batch is required");
    BatchView v;
    int rc = batch_view(b, &v);
    if (rc) return rc;
    if (v.model != FEA_ELASTIC) return set_error(FEA_EINVAL, "the batched subgrid scale is built for FEA_ELASTIC");
    if (!status && v.n_meshes > 0) return set_error(FEA_EINVAL, "status (one int32 per mesh) is required");
    for (int m = 0; m < v.n_meshes; ++m) {
        const fea_mesh_desc &d = v.desc[m];
        if (d.nh_flag) return set_error(FEA_EINVAL, "mesh %d: the subgrid scale is defined for linear elasticity only", m);
        if (d.n_elems > 0 && (!d.u || !d.nu || !d.source || !d.x || !d.y || !d.z))
            return set_error(FEA_EINVAL, "mesh %d: u, nu, source and coordinates are required", m);
    }
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev != v.device) return set_error(FEA_EINVAL, "batch lives on device %d, current is %d", v.device, dev);
    if ((rc = ensure_tables())) return rc;
    std::vector<int64_t> off;
    if ((rc = batch_gauss_offsets(v, stream, off))) return rc;
    if (off.back() > 0 && !out) return set_error(FEA_EINVAL, "NULL output");
    if ((rc = sub_items_prepare(v))) return rc;
    // per-(family, mesh) arguments, rebuilt when the outputs change
    const size_t na = (size_t)4 * std::max(v.n_meshes, 1);
    if (!(v.args_key[0] == out && v.args_key[1] == status && *v.args)) {
        std::vector<SubArgs> h(na);
        for (int t = 0; t < 4; ++t)
            for (int m = 0; m < v.n_meshes; ++m) {
                const fea_mesh_desc &d = v.desc[m];
                const fea_graph *g = v.graphs[m];
                SubArgs a = {};
                a.x = d.x; a.y = d.y; a.z = d.z;
                a.u = d.u;
                a.young = d.young;
                a.nu = d.nu;
                a.source = d.source;
                a.perm = g->perm + g->seg[t];
                a.pnodes = g->pnodes + g->node_base[t];
                a.gp_ptr = g->gp_ptr;
                a.n = g->seg[t + 1] - g->seg[t];
                a.out = out + off[m] * 3;
                a.status = status + m;
                h[(size_t)t * v.n_meshes + m] = a;
            }
        // a kernel still in flight may read the previous table
        FEA_HIP(hipStreamSynchronize(stream));
        if (*v.args_cap < na) {
            dfree(*v.args);
            *v.args = nullptr;
            *v.args_cap = 0;
            if ((rc = dalloc(v.args, sizeof(SubArgs) * na))) return rc;
            *v.args_cap = na;
        }
        FEA_HIP(hipMemcpy(*v.args, h.data(), sizeof(SubArgs) * na, hipMemcpyHostToDevice));
        v.args_key[0] = out;
        v.args_key[1] = status;
    }
    const SubArgs *d_args = (const SubArgs *)*v.args;
    const int nb = (int)grid_for(std::max(v.n_meshes, 4), 256);
    k_sub_batch_begin<<<nb, 256, 0, stream>>>(v.head, status, v.n_meshes);
    if ((rc = launch_sub_batch<1>(v, d_args, stream)) || (rc = launch_sub_batch<3>(v, d_args, stream)) ||
        (rc = launch_sub_batch<2>(v, d_args, stream)) || (rc = launch_sub_batch<0>(v, d_args, stream)))
        return rc;
    k_sub_batch_end<<<nb, 256, 0, stream>>>(status, v.n_meshes);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}
