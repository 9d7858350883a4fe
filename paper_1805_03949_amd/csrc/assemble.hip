// Element quadrature and scatter kernels (paper Section 2.1.1, Algorithm 1;
// race treatments of Section 3.2: Algorithm 4 ATOMIC, Algorithm 5 colouring).
//
// Element arithmetic (isoparametric, Gauss quadrature):
//   J = sum_a x_a (x) dN_a/dxi, G_a = J^-T dN_a/dxi, wd = w_q detJ
//   Poisson     K_ab    += wd G_a.G_b,            f_a   += wd N_a f
//   elasticity  K_ab,ij += wd [lam h_a,i h_b,j + c2 h_a,j h_b,i
//                              + mu delta_ij G_a.G_b],  f_a,i += wd N_a f_i
// with h = G and c2 = mu for linear elasticity, and for the compressible
// neo-Hookean tangent (Section 2.2, A = Jacobian of the first Piola-Kirchhoff
// stress) F = I + sum_a u_a (x) G_a, h_a = F^-T-applied gradient
// (h_a,j = sum_J G_a,J Finv_Jj) and c2 = mu - lam ln det F. That factored
// form is algebraically identical to contracting the 81-entry tangent
// AA_iJjL = mu d_ij d_JL + (mu - lam lnJ) Finv_Jj Finv_Li + lam Finv_Ji Finv_Lj.
//
// Work layout: one 256-thread workgroup holds EPB = 256 / n^2 elements of
// one family; geometry runs one thread per (element, Gauss point) and
// writes gradients to LDS; the element matrix runs one thread per
// (element, block a-b), each accumulating its b x b block over the Gauss
// points; the right-hand side one thread per (element, node).
#include <climits>
#include <cstring>
#include <mutex>

#include "fea_internal.h"

namespace fea {

struct RefTables {
    double N[4][8][8];      // [family][gauss point][node]
    double dN[4][8][8][3];  // [family][gauss point][node][reference direction]
    double w[4][8];
};

__constant__ RefTables c_ref;

template <int T>
struct Fam {
    static constexpr int NN = 4 + T + (T == 3);
    static constexpr int NQ = T == 0 ? 1 : (T == 2 ? 6 : 8);
};

// Reference shape functions and Gauss rules (host side, uploaded once per
// device). hex8 / pyr5: 2x2x2 Gauss, xi fastest; pen6: 3-point triangle
// rule (weights 1/6) x 2-point Gauss in t, triangle point fastest; tet4:
// one point at the centroid, weight 1/6. The pyramid is the hexahedron with
// its top face collapsed into the apex.
static void shape_host(int t, const double p[3], double N[8], double dN[8][3])
{
    static const int sg[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                 {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
    if (t == 3 || t == 1) {
        double h[8], dh[8][3];
        for (int a = 0; a < 8; ++a) {
            double fx = 0.5 * (1 + sg[a][0] * p[0]), fy = 0.5 * (1 + sg[a][1] * p[1]),
                   fz = 0.5 * (1 + sg[a][2] * p[2]);
            h[a] = fx * fy * fz;
            dh[a][0] = 0.5 * sg[a][0] * fy * fz;
            dh[a][1] = 0.5 * sg[a][1] * fx * fz;
            dh[a][2] = 0.5 * sg[a][2] * fx * fy;
        }
        int nb = t == 3 ? 8 : 4;
        for (int a = 0; a < nb; ++a) {
            N[a] = h[a];
            for (int j = 0; j < 3; ++j) dN[a][j] = dh[a][j];
        }
        if (t == 1) {
            N[4] = h[4] + h[5] + h[6] + h[7];
            for (int j = 0; j < 3; ++j) dN[4][j] = dh[4][j] + dh[5][j] + dh[6][j] + dh[7][j];
        }
    } else if (t == 2) {
        double L[3] = {1 - p[0] - p[1], p[0], p[1]};
        double dL[3][2] = {{-1, -1}, {1, 0}, {0, 1}};
        for (int a = 0; a < 6; ++a) {
            int k = a % 3;
            double s = a < 3 ? -1.0 : 1.0;
            double g = 0.5 * (1 + s * p[2]);
            N[a] = L[k] * g;
            dN[a][0] = dL[k][0] * g;
            dN[a][1] = dL[k][1] * g;
            dN[a][2] = 0.5 * s * L[k];
        }
    } else {
        N[0] = 1 - p[0] - p[1] - p[2];
        N[1] = p[0];
        N[2] = p[1];
        N[3] = p[2];
        for (int a = 0; a < 4; ++a)
            for (int j = 0; j < 3; ++j) dN[a][j] = (a == 0) ? -1.0 : (a - 1 == j ? 1.0 : 0.0);
    }
}

static void build_tables(RefTables *R)
{
    memset(R, 0, sizeof(*R));
    const double g = 0.57735026918962576451;  // 1/sqrt(3)
    for (int t = 0; t < 4; ++t) {
        double pts[8][3], w[8];
        int nq = 0;
        if (t == 0) {
            pts[0][0] = pts[0][1] = pts[0][2] = 0.25;
            w[0] = 1.0 / 6.0;
            nq = 1;
        } else if (t == 2) {
            const double tr[3][2] = {{1.0 / 6, 1.0 / 6}, {2.0 / 3, 1.0 / 6}, {1.0 / 6, 2.0 / 3}};
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 3; ++i, ++nq) {
                    pts[nq][0] = tr[i][0];
                    pts[nq][1] = tr[i][1];
                    pts[nq][2] = k ? g : -g;
                    w[nq] = 1.0 / 6.0;
                }
        } else {
            for (int k = 0; k < 2; ++k)
                for (int j = 0; j < 2; ++j)
                    for (int i = 0; i < 2; ++i, ++nq) {
                        pts[nq][0] = i ? g : -g;
                        pts[nq][1] = j ? g : -g;
                        pts[nq][2] = k ? g : -g;
                        w[nq] = 1.0;
                    }
        }
        for (int q = 0; q < nq; ++q) {
            double N[8] = {0}, dN[8][3] = {{0}};
            shape_host(t, pts[q], N, dN);
            R->w[t][q] = w[q];
            for (int a = 0; a < 8; ++a) {
                R->N[t][q][a] = N[a];
                for (int j = 0; j < 3; ++j) R->dN[t][q][a][j] = dN[a][j];
            }
        }
    }
}

static int ensure_tables()
{
    static std::mutex mtx;
    static bool done[64] = {false};
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(FEA_EINVAL, "device index %d unsupported", dev);
    std::lock_guard<std::mutex> lock(mtx);
    if (done[dev]) return FEA_OK;
    RefTables R;
    build_tables(&R);
    FEA_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_ref), &R, sizeof(R), 0, hipMemcpyHostToDevice));
    done[dev] = true;
    return FEA_OK;
}

struct ElemArgs {
    const double *x, *y, *z;
    const int64_t *conn_ptr;
    const int32_t *conn;
    const int32_t *elems;  // element ids handled by this launch
    int64_t n;             // number of ids
    const int64_t *map_ptr;
    const int32_t *e2nnz;
    const int32_t *e2pos;  // row-owner: destination position of every slot
    const int32_t *rpos;   // row-owner: destination position of every conn entry
    const double *young, *nu;
    const uint8_t *nh_flag;
    const double *u;
    const double *source;
    double *vals;    // FP64 target of ATOMIC / COLOUR
    double *rhs;
    void *contrib;   // ROWOWNER slot workspace (compute type)
    void *rcontrib;  // ROWOWNER right-hand-side workspace
    int32_t *status;
};

enum { V_ROWOWNER = 0, V_ATOMIC = 1, V_COLOUR = 2 };

__device__ inline double det3(const double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// inverse through the adjugate
__device__ inline void inv3(const double J[3][3], double d, double Ji[3][3])
{
    double r = 1.0 / d;
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * r;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * r;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * r;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
}

// The hardware hands workgroup b to XCD b % 8. Renumbering tiles so that
// each XCD receives one contiguous range keeps neighbouring elements (which
// share nodes, coordinates and destination cache lines) in the same L2.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nblk)
{
    const int64_t q = nblk >> 3, rem = nblk & 7, x = b & 7, r = b >> 3;
    return x * q + (x < rem ? x : rem) + r;
}

template <int T, int MODEL, int VAR, typename CT>
__global__ void __launch_bounds__(256) k_element(ElemArgs A)
{
    constexpr int NN = Fam<T>::NN, NQ = Fam<T>::NQ, P = NN * NN;
    constexpr int EPB = 256 / P;
    constexpr bool ELAS = MODEL != FEA_POISSON;
    constexpr int B = ELAS ? 3 : 1;
    constexpr int BB = B * B;
    constexpr int EU = ELAS ? EPB : 1;
    constexpr bool RO = VAR == V_ROWOWNER;

    __shared__ double sX[EPB][NN][3];
    __shared__ double sU[EU][NN][3];
    __shared__ CT sG[EPB][NQ][NN][3];   // physical gradients
    __shared__ CT sH[EU][NQ][NN][3];    // neo-Hookean: gradients pushed through F^-T
    __shared__ CT sC[EPB][NQ][4];       // wd, and for neo-Hookean wd*lam, wd*c2, wd*mu
    __shared__ double sLM[EU][2];       // lam, mu
    __shared__ int32_t sE[EPB];
    __shared__ int sNH[EPB];
    __shared__ int64_t sM[EPB];         // first slot of each element
    __shared__ int64_t sCP[EPB];        // first conn position of each element
    __shared__ double sDN[NQ][NN][3];   // reference gradients of this family
    __shared__ double sNr[NQ][NN];      // reference shape functions

    const int tid = threadIdx.x;
    const int64_t first = xcd_tile(blockIdx.x, gridDim.x) * EPB;

    for (int i = tid; i < NQ * NN; i += 256) {
        const int q = i / NN, a = i % NN;
        sNr[q][a] = c_ref.N[T][q][a];
        sDN[q][a][0] = c_ref.dN[T][q][a][0];
        sDN[q][a][1] = c_ref.dN[T][q][a][1];
        sDN[q][a][2] = c_ref.dN[T][q][a][2];
    }

    if (tid < EPB) {
        int64_t i = first + tid;
        int32_t e = i < A.n ? A.elems[i] : -1;
        sE[tid] = e;
        sM[tid] = e >= 0 ? A.map_ptr[e] : 0;
        sCP[tid] = e >= 0 ? A.conn_ptr[e] : 0;
        sNH[tid] = (ELAS && e >= 0 && A.nh_flag) ? (int)A.nh_flag[e] : 0;
        if constexpr (ELAS) {
            double E = (e >= 0 && A.young) ? A.young[e] : 1.0, nu = e >= 0 ? A.nu[e] : 0.25;
            sLM[tid][0] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
            sLM[tid][1] = E / (2.0 * (1.0 + nu));
        }
    }
    __syncthreads();

    if (tid < EPB * NN) {
        int el = tid / NN, a = tid % NN;
        int32_t e = sE[el];
        if (e >= 0) {
            int32_t v = A.conn[sCP[el] + a];
            sX[el][a][0] = A.x[v];
            sX[el][a][1] = A.y[v];
            sX[el][a][2] = A.z[v];
            if constexpr (ELAS) {
                bool nh = sNH[el] != 0;
                for (int k = 0; k < 3; ++k) sU[el][a][k] = nh ? A.u[3 * (int64_t)v + k] : 0.0;
            }
        }
    }
    __syncthreads();

    // geometry: one thread per (element, Gauss point), in FP64
    if (tid < EPB * NQ) {
        int el = tid / NQ, q = tid % NQ;
        int32_t e = sE[el];
        if (e >= 0) {
            double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
            for (int a = 0; a < NN; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) J[i][j] += sX[el][a][i] * sDN[q][a][j];
            double d = det3(J);
            if (!(d > 0.0)) atomicMin(A.status, e);
            double Ji[3][3];
            inv3(J, d, Ji);
            double G[NN][3];
#pragma unroll
            for (int a = 0; a < NN; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    G[a][i] = Ji[0][i] * sDN[q][a][0] + Ji[1][i] * sDN[q][a][1] + Ji[2][i] * sDN[q][a][2];
                    sG[el][q][a][i] = (CT)G[a][i];
                }
            double wd = c_ref.w[T][q] * d;
            sC[el][q][0] = (CT)wd;
            if constexpr (ELAS) {
                if (sNH[el]) {
                    const double lam = sLM[el][0], mu = sLM[el][1];
                    double F[3][3];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
                            for (int a = 0; a < NN; ++a) acc += sU[el][a][i] * G[a][j];
                            F[i][j] = acc;
                        }
                    double jf = det3(F);
                    if (!(jf > 0.0)) atomicMin(A.status, e);
                    double Fi[3][3];
                    inv3(F, jf, Fi);
#pragma unroll
                    for (int a = 0; a < NN; ++a)
#pragma unroll
                        for (int j = 0; j < 3; ++j)
                            sH[el][q][a][j] =
                                (CT)(G[a][0] * Fi[0][j] + G[a][1] * Fi[1][j] + G[a][2] * Fi[2][j]);
                    sC[el][q][1] = (CT)(wd * lam);
                    sC[el][q][2] = (CT)(wd * (mu - lam * log(jf)));
                    sC[el][q][3] = (CT)(wd * mu);
                }
            }
        }
    }
    __syncthreads();

    // element matrix: one thread per (element, block a-b)
    if (tid < EPB * P) {
        int el = tid / P, p = tid % P, a = p / NN, b = p % NN;
        int32_t e = sE[el];
        if (e >= 0) {
            // destination of this block, fetched before the contraction
            const int64_t dest = RO ? (int64_t)A.e2pos[sM[el] + p] : (int64_t)A.e2nnz[sM[el] + p];
            CT K[BB];
            if constexpr (!ELAS) {
                CT acc = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    CT dot = sG[el][q][a][0] * sG[el][q][b][0] + sG[el][q][a][1] * sG[el][q][b][1] +
                             sG[el][q][a][2] * sG[el][q][b][2];
                    acc += sC[el][q][0] * dot;
                }
                K[0] = acc;
            } else if (!sNH[el]) {
                // linear: K = lam S + mu S^T + mu tr(S) I, S = sum_q wd G_a (x) G_b
                CT S[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) S[c] = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    CT w = sC[el][q][0];
                    CT ga[3] = {w * sG[el][q][a][0], w * sG[el][q][a][1], w * sG[el][q][a][2]};
                    CT gb[3] = {sG[el][q][b][0], sG[el][q][b][1], sG[el][q][b][2]};
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) S[i * 3 + j] += ga[i] * gb[j];
                }
                const CT lam = (CT)sLM[el][0], mu = (CT)sLM[el][1];
                const CT tr = S[0] + S[4] + S[8];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        CT v = lam * S[i * 3 + j] + mu * S[j * 3 + i];
                        if (i == j) v += mu * tr;
                        K[i * 3 + j] = v;
                    }
            } else {
                // neo-Hookean: K_ij = sum_q c1 h_a,i h_b,j + c2 h_a,j h_b,i + c0 d_ij G_a.G_b
                CT T1[9], T2[9], dsum = 0;
#pragma unroll
                for (int c = 0; c < 9; ++c) T1[c] = T2[c] = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    CT c1 = sC[el][q][1], c2 = sC[el][q][2], c0 = sC[el][q][3];
                    CT ha[3] = {sH[el][q][a][0], sH[el][q][a][1], sH[el][q][a][2]};
                    CT hb[3] = {sH[el][q][b][0], sH[el][q][b][1], sH[el][q][b][2]};
                    CT dot = sG[el][q][a][0] * sG[el][q][b][0] + sG[el][q][a][1] * sG[el][q][b][1] +
                             sG[el][q][a][2] * sG[el][q][b][2];
                    dsum += c0 * dot;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            CT hh = ha[i] * hb[j];
                            T1[i * 3 + j] += c1 * hh;
                            T2[i * 3 + j] += c2 * hh;
                        }
                }
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        CT v = T1[i * 3 + j] + T2[j * 3 + i];
                        if (i == j) v += dsum;
                        K[i * 3 + j] = v;
                    }
            }
            if constexpr (RO) {
                // row-owner: the workspace is sorted by destination block
                CT *dst = (CT *)A.contrib + dest * BB;
#pragma unroll
                for (int c = 0; c < BB; ++c) dst[c] = K[c];
            } else {
                double *dst = A.vals + dest * BB;
#pragma unroll
                for (int c = 0; c < BB; ++c) {
                    if constexpr (VAR == V_ATOMIC)
                        unsafeAtomicAdd(dst + c, (double)K[c]);
                    else
                        dst[c] += (double)K[c];
                }
            }
        }
    }

    // right-hand side: one thread per (element, node)
    if (tid < EPB * NN) {
        int el = tid / NN, a = tid % NN;
        int32_t e = sE[el];
        if (e >= 0) {
            CT f[B];
#pragma unroll
            for (int i = 0; i < B; ++i) f[i] = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                CT wn = sC[el][q][0] * (CT)sNr[q][a];
#pragma unroll
                for (int i = 0; i < B; ++i) f[i] += wn * (CT)A.source[(int64_t)e * B + i];
            }
            if constexpr (RO) {
                CT *dst = (CT *)A.rcontrib + (int64_t)A.rpos[sCP[el] + a] * B;
#pragma unroll
                for (int i = 0; i < B; ++i) dst[i] = f[i];
            } else {
                int64_t v = A.conn[sCP[el] + a];
                double *dst = A.rhs + v * B;
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    if constexpr (VAR == V_ATOMIC)
                        unsafeAtomicAdd(dst + i, (double)f[i]);
                    else
                        dst[i] += (double)f[i];
                }
            }
        }
    }

}

// Row-owner second phase. The workspace holds every block's contributions
// contiguously, in ascending element order (the order of Algorithm 1), so
// block k's value is a plain sum over its segment: a streaming pass with
// the result independent of how the element phase was scheduled.
template <int W, typename CT, typename OT>
__global__ void __launch_bounds__(256) k_reduce_seg(int64_t nseg, const int64_t *seg_ptr,
                                                    const CT *data, OT *out)
{
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nseg * W) return;
    int64_t k = t / W;
    int c = (int)(t - k * W);
    double s = 0.0;
    const int64_t e = seg_ptr[k + 1];
    const CT *d = data + c;
    // four loads in flight per step; the additions stay in ascending order
    for (int64_t j = seg_ptr[k]; j < e; j += 4) {
        CT v0 = d[j * W];
        CT v1 = j + 1 < e ? d[(j + 1) * W] : (CT)0;
        CT v2 = j + 2 < e ? d[(j + 2) * W] : (CT)0;
        CT v3 = j + 3 < e ? d[(j + 3) * W] : (CT)0;
        s += (double)v0;
        if (j + 1 < e) s += (double)v1;
        if (j + 2 < e) s += (double)v2;
        if (j + 3 < e) s += (double)v3;
    }
    out[t] = (OT)s;
}

__global__ void k_fill_f64(double *p, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_to_f32(const double *in, float *out, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

__global__ void k_status_init(int32_t *s) { *s = INT_MAX; }
__global__ void k_status_final(int32_t *s)
{
    if (*s == INT_MAX) *s = -1;
}

template <int T, int MODEL, int VAR, typename CT>
static void launch_fam(const ElemArgs &a, hipStream_t s)
{
    constexpr int P = Fam<T>::NN * Fam<T>::NN;
    constexpr int EPB = 256 / P;
    if (a.n <= 0) return;
    k_element<T, MODEL, VAR, CT><<<grid_for(a.n, EPB), 256, 0, s>>>(a);
}

template <int MODEL, int VAR, typename CT>
static void launch_type(int t, const ElemArgs &a, hipStream_t s)
{
    switch (t) {
    case 0: launch_fam<0, MODEL, VAR, CT>(a, s); break;
    case 1: launch_fam<1, MODEL, VAR, CT>(a, s); break;
    case 2: launch_fam<2, MODEL, VAR, CT>(a, s); break;
    default: launch_fam<3, MODEL, VAR, CT>(a, s); break;
    }
}

static int ensure_ws(void **p, size_t *have, size_t need)
{
    if (*have >= need && *p) return FEA_OK;
    dfree(*p);
    *p = nullptr;
    *have = 0;
    int rc = dalloc(p, need);
    if (rc) return rc;
    *have = need;
    return FEA_OK;
}

static inline void mark(fea_graph *g, int i, const fea_options *o, hipStream_t s)
{
    if (o->timing) (void)hipEventRecord(g->ev[i], s);
}

template <int MODEL, typename CT>
static int run(fea_graph *g, ElemArgs a, const fea_options *o, hipStream_t s, void *vals, void *rhs)
{
    constexpr int B = MODEL == FEA_POISSON ? 1 : 3;
    constexpr int BB = B * B;
    const int64_t nv = g->nnz * BB, nr = g->n_nodes * B;
    const bool f32 = o->out_dtype == FEA_F32;
    int rc;
    if (o->variant == FEA_ROWOWNER) {
        if ((rc = ensure_ws(&g->contrib, &g->contrib_bytes, sizeof(CT) * (size_t)g->map_len * BB))) return rc;
        if ((rc = ensure_ws(&g->rcontrib, &g->rcontrib_bytes, sizeof(CT) * (size_t)g->conn_len * B))) return rc;
        a.contrib = g->contrib;
        a.rcontrib = g->rcontrib;
        mark(g, 0, o, s);
        for (int t = 0; t < 4; ++t) {
            a.elems = g->perm + g->seg[t];
            a.n = g->seg[t + 1] - g->seg[t];
            launch_type<MODEL, V_ROWOWNER, CT>(t, a, s);
        }
        mark(g, 1, o, s);
        if (f32) {
            if (nv) k_reduce_seg<BB, CT, float><<<grid_for(nv, 256), 256, 0, s>>>(g->nnz, g->inv_ptr, (const CT *)g->contrib, (float *)vals);
            mark(g, 2, o, s);
            if (nr) k_reduce_seg<B, CT, float><<<grid_for(nr, 256), 256, 0, s>>>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (float *)rhs);
        } else {
            if (nv) k_reduce_seg<BB, CT, double><<<grid_for(nv, 256), 256, 0, s>>>(g->nnz, g->inv_ptr, (const CT *)g->contrib, (double *)vals);
            mark(g, 2, o, s);
            if (nr) k_reduce_seg<B, CT, double><<<grid_for(nr, 256), 256, 0, s>>>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (double *)rhs);
        }
        mark(g, 3, o, s);
        FEA_HIP(hipGetLastError());
        return FEA_OK;
    }
    // ATOMIC and COLOUR accumulate in FP64, directly in the output when it is
    // FP64, else in a workspace converted at the end.
    double *tv, *tr;
    if (f32) {
        if ((rc = ensure_ws((void **)&g->acc64, &g->acc64_bytes, sizeof(double) * (size_t)(nv + nr)))) return rc;
        tv = g->acc64;
        tr = g->acc64 + nv;
    } else {
        tv = (double *)vals;
        tr = (double *)rhs;
    }
    mark(g, 0, o, s);
    if (nv) k_fill_f64<<<grid_for(nv, 256), 256, 0, s>>>(tv, nv, 0.0);
    if (nr) k_fill_f64<<<grid_for(nr, 256), 256, 0, s>>>(tr, nr, 0.0);
    a.vals = tv;
    a.rhs = tr;
    if (o->variant == FEA_ATOMIC) {
        for (int t = 0; t < 4; ++t) {
            a.elems = g->perm + g->seg[t];
            a.n = g->seg[t + 1] - g->seg[t];
            launch_type<MODEL, V_ATOMIC, CT>(t, a, s);
        }
    } else {
        const int nc = g->n_colours;
        for (int c = 0; c < nc; ++c)
            for (int t = 0; t < 4; ++t) {
                int64_t b = g->cseg[(size_t)t * (nc + 1) + c], e = g->cseg[(size_t)t * (nc + 1) + c + 1];
                a.elems = g->cperm + b;
                a.n = e - b;
                launch_type<MODEL, V_COLOUR, CT>(t, a, s);
            }
    }
    mark(g, 1, o, s);
    if (f32 && nv) k_to_f32<<<grid_for(nv, 256), 256, 0, s>>>(tv, (float *)vals, nv);
    mark(g, 2, o, s);
    if (f32 && nr) k_to_f32<<<grid_for(nr, 256), 256, 0, s>>>(tr, (float *)rhs, nr);
    mark(g, 3, o, s);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

}  // namespace fea

using namespace fea;

extern "C" int fea_assemble(const fea_graph *gc, const double *x, const double *y, const double *z,
                            const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                            const fea_material *mat, const double *source, const fea_options *opt,
                            hipStream_t stream, void *vals, void *rhs, int32_t *status)
{
    clear_error();
    fea_graph *g = const_cast<fea_graph *>(gc);
    fea_options dflt = {0, 0, 0, 0};
    const fea_options *o = opt ? opt : &dflt;
    if (!g || !mat) return set_error(FEA_EINVAL, "graph and material are required");
    if (o->precision < 0 || o->precision > 1 || o->variant < 0 || o->variant > 2 ||
        o->out_dtype < 0 || o->out_dtype > 1)
        return set_error(FEA_EINVAL, "bad option (precision %d, variant %d, out_dtype %d)",
                         o->precision, o->variant, o->out_dtype);
    if (mat->model != FEA_POISSON && mat->model != FEA_ELASTIC)
        return set_error(FEA_EINVAL, "unknown model %d", mat->model);
    if (g->n_elems > 0) {
        if (!x || !y || !z || !types || !conn_ptr || !conn || !source)
            return set_error(FEA_EINVAL, "NULL array argument");
        if (mat->model == FEA_ELASTIC && !mat->nu) return set_error(FEA_EINVAL, "nu is required");
        if (mat->nh_flag && !mat->u) return set_error(FEA_EINVAL, "u is required with nh_flag");
    }
    if ((g->nnz > 0 && !vals) || (g->n_nodes > 0 && !rhs))
        return set_error(FEA_EINVAL, "NULL output argument");
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev != g->device) return set_error(FEA_EINVAL, "graph lives on device %d, current is %d", g->device, dev);
    int rc = ensure_tables();
    if (rc) return rc;
    if (o->timing) {
        for (hipEvent_t &e : g->ev)
            if (!e) FEA_HIP(hipEventCreate(&e));
    }
    g->timed = false;

    int32_t *st = status;
    if (!st) {
        static thread_local int32_t *own[64] = {nullptr};
        if (!own[dev] && (rc = dalloc((void **)&own[dev], sizeof(int32_t)))) return rc;
        st = own[dev];
    }
    k_status_init<<<1, 1, 0, stream>>>(st);

    ElemArgs a = {};
    a.x = x; a.y = y; a.z = z;
    a.conn_ptr = conn_ptr;
    a.conn = conn;
    a.map_ptr = g->map_ptr;
    a.e2nnz = g->e2nnz;
    a.e2pos = g->e2pos;
    a.rpos = g->rpos;
    a.young = mat->young;
    a.nu = mat->nu;
    a.nh_flag = mat->model == FEA_ELASTIC ? mat->nh_flag : nullptr;
    a.u = mat->u;
    a.source = source;
    a.status = st;

    if (g->n_elems > 0) {
        if (mat->model == FEA_POISSON)
            rc = o->precision == FEA_FP64 ? run<FEA_POISSON, double>(g, a, o, stream, vals, rhs)
                                          : run<FEA_POISSON, float>(g, a, o, stream, vals, rhs);
        else
            rc = o->precision == FEA_FP64 ? run<FEA_ELASTIC, double>(g, a, o, stream, vals, rhs)
                                          : run<FEA_ELASTIC, float>(g, a, o, stream, vals, rhs);
        if (rc) return rc;
    } else {
        const int B = mat->model == FEA_POISSON ? 1 : 3;
        const int64_t words = (o->out_dtype == FEA_F32 ? 1 : 2);
        const int64_t nv = g->nnz * B * B * words, nr = g->n_nodes * B * words;
        if (nv) k_zero_u32<<<grid_for(nv, 256), 256, 0, stream>>>((uint32_t *)vals, nv);
        if (nr) k_zero_u32<<<grid_for(nr, 256), 256, 0, stream>>>((uint32_t *)rhs, nr);
    }
    k_status_final<<<1, 1, 0, stream>>>(st);
    FEA_HIP(hipGetLastError());
    g->timed = o->timing && g->n_elems > 0;
    return FEA_OK;
}

extern "C" int fea_last_timing(const fea_graph *g, float *ms)
{
    clear_error();
    if (!g || !ms) return set_error(FEA_EINVAL, "graph and ms are required");
    if (!g->timed) return set_error(FEA_EINVAL, "no timed fea_assemble call on this graph");
    FEA_HIP(hipEventSynchronize(g->ev[3]));
    FEA_HIP(hipEventElapsedTime(&ms[0], g->ev[0], g->ev[1]));
    FEA_HIP(hipEventElapsedTime(&ms[1], g->ev[1], g->ev[2]));
    FEA_HIP(hipEventElapsedTime(&ms[2], g->ev[0], g->ev[3]));
    return FEA_OK;
}
