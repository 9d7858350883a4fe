// Element quadrature device code shared by the one-launch-per-family
// kernels and the persistent batched kernel.
//
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
#pragma once
#include <climits>
#include <cstddef>
#include <cstring>
#include <mutex>

#include "fea_internal.h"

namespace fea {

struct RefTables {
    double N[4][8][8];      // [family][gauss point][node]
    double dN[4][8][8][3];  // [family][gauss point][node][reference direction]
    double w[4][8];
};

// one copy per translation unit, uploaded by that unit's ensure_tables()
static __constant__ RefTables c_ref;

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

// Gauss rule of family t (points as above); returns the number of points.
static int rule_host(int t, double pts[8][3], double w[8])
{
    const double g = 0.57735026918962576451;  // 1/sqrt(3)
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
    return nq;
}

static void build_tables(RefTables *R)
{
    memset(R, 0, sizeof(*R));
    for (int t = 0; t < 4; ++t) {
        double pts[8][3], w[8];
        const int nq = rule_host(t, pts, w);
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
    // row-owner, indexed by the launch-local element index i (type-sorted
    // order): node ids [i][a], destination of slot (a,b) [i][a*n+b] and of
    // the right-hand-side entry of node a [i][a] in the sorted workspaces
    const int32_t *pnodes;
    const int32_t *pdest;
    const int32_t *prdest;
    const double *young, *nu;
    const uint8_t *nh_flag;
    const double *u;
    const double *source;
    double *vals;    // FP64 target of ATOMIC / COLOUR
    double *rhs;
    void *contrib;   // ROWOWNER slot workspace (compute type)
    void *rcontrib;  // right-hand-side workspace (ROWOWNER, TILECOL; ROWSYM with 1x1 blocks)
    int32_t *status;
    // upper-triangle form, indexed by the launch-local tile index: entry and
    // tile-block ranges, entries (lane << 1 | transposed), tile-block entry
    // ends and workspace slots
    const int64_t *tent_ptr;
    const int64_t *ttb_ptr;
    const uint16_t *tent;
    const uint16_t *tb_eend;
    const int32_t *tb_slot;
    // tile-coloured form: the launch's tiles (launch-local tile indices,
    // ntiles of them), every tile-block's block and every block's lower
    // partner (-1 if none)
    const int32_t *tiles;
    int64_t ntiles;
    const int32_t *tb_blk;
    const int32_t *lpart;
};

// The element arguments as the persistent kernels read them from their
// argument table: the same layout as ElemArgs, with every pointer typed as
// addressing global memory. Pointers loaded as plain (generic) pointers are
// accessed with flat instructions, which also count against the LDS wait
// counter, so that every wait for LDS data would wait for outstanding
// global loads and stores too; pointers typed global keep global
// instructions, as kernel arguments do.
#define FEA_G(T) T __attribute__((address_space(1))) *
struct ElemArgsGlobal {
    FEA_G(const double) x;
    FEA_G(const double) y;
    FEA_G(const double) z;
    FEA_G(const int64_t) conn_ptr;
    FEA_G(const int32_t) conn;
    FEA_G(const int32_t) elems;
    int64_t n;
    FEA_G(const int64_t) map_ptr;
    FEA_G(const int32_t) e2nnz;
    FEA_G(const int32_t) pnodes;
    FEA_G(const int32_t) pdest;
    FEA_G(const int32_t) prdest;
    FEA_G(const double) young;
    FEA_G(const double) nu;
    FEA_G(const uint8_t) nh_flag;
    FEA_G(const double) u;
    FEA_G(const double) source;
    FEA_G(double) vals;
    FEA_G(double) rhs;
    FEA_G(void) contrib;
    FEA_G(void) rcontrib;
    FEA_G(int32_t) status;
    FEA_G(const int64_t) tent_ptr;
    FEA_G(const int64_t) ttb_ptr;
    FEA_G(const uint16_t) tent;
    FEA_G(const uint16_t) tb_eend;
    FEA_G(const int32_t) tb_slot;
    FEA_G(const int32_t) tiles;
    int64_t ntiles;
    FEA_G(const int32_t) tb_blk;
    FEA_G(const int32_t) lpart;
};
#undef FEA_G
static_assert(sizeof(ElemArgsGlobal) == sizeof(ElemArgs), "ElemArgsGlobal mirrors ElemArgs");
static_assert(offsetof(ElemArgsGlobal, lpart) == offsetof(ElemArgs, lpart), "ElemArgsGlobal mirrors ElemArgs");
static_assert(offsetof(ElemArgsGlobal, ntiles) == offsetof(ElemArgs, ntiles), "ElemArgsGlobal mirrors ElemArgs");
static_assert(offsetof(ElemArgsGlobal, n) == offsetof(ElemArgs, n), "ElemArgsGlobal mirrors ElemArgs");

// ElemArgs from an argument-table entry (its pointers converted from the
// global address space, so that the compiler keeps global accesses).
__device__ __forceinline__ ElemArgs from_global(const ElemArgsGlobal &g)
{
    ElemArgs a;
    a.x = (const double *)g.x;
    a.y = (const double *)g.y;
    a.z = (const double *)g.z;
    a.conn_ptr = (const int64_t *)g.conn_ptr;
    a.conn = (const int32_t *)g.conn;
    a.elems = (const int32_t *)g.elems;
    a.n = g.n;
    a.map_ptr = (const int64_t *)g.map_ptr;
    a.e2nnz = (const int32_t *)g.e2nnz;
    a.pnodes = (const int32_t *)g.pnodes;
    a.pdest = (const int32_t *)g.pdest;
    a.prdest = (const int32_t *)g.prdest;
    a.young = (const double *)g.young;
    a.nu = (const double *)g.nu;
    a.nh_flag = (const uint8_t *)g.nh_flag;
    a.u = (const double *)g.u;
    a.source = (const double *)g.source;
    a.vals = (double *)g.vals;
    a.rhs = (double *)g.rhs;
    a.contrib = (void *)g.contrib;
    a.rcontrib = (void *)g.rcontrib;
    a.status = (int32_t *)g.status;
    a.tent_ptr = (const int64_t *)g.tent_ptr;
    a.ttb_ptr = (const int64_t *)g.ttb_ptr;
    a.tent = (const uint16_t *)g.tent;
    a.tb_eend = (const uint16_t *)g.tb_eend;
    a.tb_slot = (const int32_t *)g.tb_slot;
    a.tiles = (const int32_t *)g.tiles;
    a.ntiles = g.ntiles;
    a.tb_blk = (const int32_t *)g.tb_blk;
    a.lpart = (const int32_t *)g.lpart;
    return a;
}

// V_ROWSYM: the row-owner scatter on the upper triangle. A symmetric
// element matrix has block (b, a) equal to block (a, b) transposed, so one
// thread per local pair a <= b computes block (a, b); the workgroup's tile
// of elements then sums, per distinct upper block it touches, its lanes'
// blocks (transposed where node a > node b) in ascending lane order and
// writes one value per (tile, block) to the workspace; the reduction adds
// the tile sums of each upper block and writes lower blocks as transposes.
// V_TILECOL: the same tiles and tile sums, coloured so that the tiles of a
// colour share no node (and so no block); a tile adds its sums, and their
// transposes for the lower partners, straight into FP64 block values, one
// colour at a time (the commutative tile accumulation of Algorithm 7).
enum { V_ROWOWNER = 0, V_ATOMIC = 1, V_COLOUR = 2, V_ROWSYM = 3, V_TILECOL = 4 };

// Kernel model codes: FEA_POISSON, FEA_ELASTIC (linear elements only) and
// M_ELASTIC_NH (some elements use the neo-Hookean tangent; only these
// kernels carry the displacement and pushed-gradient LDS arrays).
constexpr int M_ELASTIC_NH = 2;
// M_ELASTIC_RES: as M_ELASTIC_NH, and the right-hand side is the Newton
// residual f_ext - f_int(u) (its own instantiations: the internal-force
// code would otherwise raise every neo-Hookean kernel's register count)
constexpr int M_ELASTIC_RES = 3;


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
// The thread index as a value the compiler cannot treat as loop-invariant:
// inside a persistent loop this keeps per-thread index arithmetic from being
// hoisted out of the loop and held in registers across iterations.
__device__ inline int opaque_tid()
{
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}

__device__ inline int64_t xcd_tile(int64_t b, int64_t nblk)
{
    const int64_t q = nblk >> 3, rem = nblk & 7, x = b & 7, r = b >> 3;
    return x * q + (x < rem ? x : rem) + r;
}

// Gradients of one element at its Gauss points, optionally padded by one
// value (see ElemSmem).
template <typename CT, int NQ, int NN, bool PAD>
struct GradRecT {
    CT v[NQ][NN][3];
};
template <typename CT, int NQ, int NN>
struct GradRecT<CT, NQ, NN, true> {
    CT v[NQ][NN][3];
    CT pad;
};

template <int T, int MODEL, int VAR, typename CT_>
struct ElemDims {
    using CT = CT_;
    static constexpr int NN = Fam<T>::NN, NQ = Fam<T>::NQ, P = NN * NN;
    // threads per element: all n*n blocks, or the n(n+1)/2 pairs a <= b
    static constexpr int PW = (VAR == V_ROWSYM || VAR == V_TILECOL) ? NN * (NN + 1) / 2 : P;
    static constexpr int EPB = 256 / PW;
    static constexpr bool ELAS = MODEL != FEA_POISSON;
    static constexpr bool NHK = MODEL == M_ELASTIC_NH || MODEL == M_ELASTIC_RES;
    static constexpr int B = ELAS ? 3 : 1;
    static constexpr int BB = B * B;
    static constexpr int EU = NHK ? EPB : 1;
    static constexpr bool RO = VAR == V_ROWOWNER || VAR == V_ROWSYM || VAR == V_TILECOL;

    static constexpr bool SYM = VAR == V_ROWSYM || VAR == V_TILECOL;  // tile sums
    static constexpr bool TCOL = VAR == V_TILECOL;
    static_assert(!SYM || EPB == sym_epb(T), "tile size of the upper-triangle layout");
    // a tile holds one entry per lane (the graph rejects an element that
    // repeats a node, and the layout builder checks the count), and so at
    // most as many tile-blocks
    static constexpr int MAXENT = EPB * PW;
    static constexpr int NC = NHK ? 4 : 1;
    // Row-owner stores staged in LDS so that BB consecutive threads write one
    // block's BB contiguous values. Measured per family on MI355X: a gain
    // everywhere except FP64 pyramids of the neo-Hookean kernel, where the
    // extra LDS costs more occupancy than it saves. The upper-triangle form
    // always stages (its tile sums read the staged blocks).
    static constexpr bool STAGE = RO && (SYM || sizeof(CT) == 4 || T != 1 || !NHK);
    // physical gradients sG[EPB][NQ][NN][3], neo-Hookean gradients pushed
    // through F^-T sH[EU][NQ][NN][3], staged blocks sK[EPB * PW * BB].
    // Per-element gradient records are padded by one value where their size
    // is a multiple of the 64 LDS banks (hex8: 192 values): the lanes of a
    // wave span two elements, whose same-position reads would otherwise
    // fall in the same banks (36% of LDS cycles lost to conflicts).
    using GradRec = GradRecT<CT, NQ, NN, (NQ * NN * 3 * (int)sizeof(CT) / 4) % 64 == 0>;
    static constexpr int NG = EPB * (int)(sizeof(GradRec) / sizeof(CT)), NHG = EU * (int)(sizeof(GradRec) / sizeof(CT)),
                         NK = STAGE ? EPB * PW * BB : 1;
    // Upper-triangle form: the staged blocks overwrite the gradients (one
    // barrier more, after every lane has read them) where the gradient
    // records are large enough for the shared space to decide occupancy,
    // and always in FP64; FP32 tet4 blocks get a space of their own.
    static constexpr bool ALIAS = SYM && ((NG + NHG) * (int)sizeof(CT) > 4096 || sizeof(CT) == 8);
    static constexpr int NBUF = ALIAS ? (NG + NHG > NK ? NG + NHG : NK) : NG + NHG + NK;
    static constexpr int KOFF = ALIAS ? 0 : NG + NHG;  // where sK starts in buf
    // FP64 upper-triangle form: the per-element inputs, Gauss-point
    // coefficients and reference tables are dead once the blocks are
    // staged, and share the staged blocks' space beyond the gradients where
    // they fit
    static constexpr int SRC = SYM ? EPB : 1, NLM = ELAS ? EPB : 1;
    static constexpr int PRE_BYTES =
        (EPB * NN * 3 + EU * NN * 3 + NLM * 2 + SRC * B + NQ * NN * 3 + NQ * NN) * 8 +
        EPB * NQ * NC * (int)sizeof(CT) + 2 * EPB * 4;
    static constexpr bool PRE_ALIAS =
        ALIAS && sizeof(CT) == 8 && (NG + NHG) * (int)sizeof(CT) + PRE_BYTES <= NBUF * (int)sizeof(CT);
};

// The LDS arrays that the upper-triangle form may overlay on the staged
// blocks, apart or overlaid.
template <typename D>
struct ElemPreArrays {
    using CT = typename D::CT;
    double sX[D::EPB][D::NN][3];
    double sU[D::EU][D::NN][3];
    double sLM[D::NLM][2];        // lam, mu of every element (elasticity)
    double sSrc[D::SRC][D::B];    // source of every element (upper-triangle form)
    double sDN[D::NQ][D::NN][3];  // reference gradients of this family
    double sNr[D::NQ][D::NN];     // reference shape functions
    CT sC[D::EPB][D::NQ][D::NC];  // wd, and for neo-Hookean wd*lam, wd*c2, wd*mu
    int32_t sE[D::EPB];
    int sNH[D::EPB];
};
template <typename D, bool OVERLAY = D::PRE_ALIAS>
struct ElemPre : ElemPreArrays<D> {
    alignas(16) typename D::CT buf[D::NBUF];
};
template <typename D>
struct ElemPre<D, true> {
    using CT = typename D::CT;
    union {
        alignas(16) CT buf[D::NBUF];
        struct {
            CT pre_gradients_[D::NG + D::NHG];
            double sX[D::EPB][D::NN][3];
            double sU[D::EU][D::NN][3];
            double sLM[D::NLM][2];
            double sSrc[D::SRC][D::B];
            double sDN[D::NQ][D::NN][3];
            double sNr[D::NQ][D::NN];
            CT sC[D::EPB][D::NQ][D::NC];
            int32_t sE[D::EPB];
            int sNH[D::EPB];
        };
    };
};

template <int T, int MODEL, int VAR, typename CT>
struct ElemSmem : ElemDims<T, MODEL, VAR, CT>, ElemPre<ElemDims<T, MODEL, VAR, CT>> {
    using D = ElemDims<T, MODEL, VAR, CT>;
    int64_t sM[D::RO ? 1 : D::EPB];   // first slot of each element
    int64_t sCP[D::RO ? 1 : D::EPB];  // first conn position of each element
    int32_t sD[D::STAGE && !D::SYM ? D::EPB * D::PW : 1];
    uint16_t sEnt[D::SYM ? D::MAXENT : 1];   // the tile's entries
    uint16_t sEend[D::SYM ? D::MAXENT : 1];  // and tile-block ends
    int32_t sSlot[D::SYM ? D::MAXENT : 1];   // workspace slot (tile-coloured: block) of every tile-block
    int32_t sLp[D::TCOL ? D::MAXENT : 1];    // tile-coloured: lower partner of every tile-block's block
};

// Waves per SIMD that the LDS of one 256-thread workgroup (one wave per
// SIMD) and the extra bytes of a kernel leave room for on a 160 KB CU, at
// most 8: the occupancy a kernel's register budget should not undercut.
template <typename Smem>
constexpr int lds_waves(int extra = 0)
{
    const int w = (160 * 1024) / (int)(sizeof(Smem) + extra);
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// Minimum waves per SIMD asked of the element kernels: the FP64
// linear-elastic upper-triangle instances at their LDS occupancy (tet4,
// pen6 and hex8 eight waves: 64 VGPRs, which their one-tile code fits
// without spills, and their persistent code too; pyr5 six); in the
// persistent kernels also the FP64 neo-Hookean tet4 instance at five (96
// VGPRs instead of 102, no spills; hetero128 kernel 5.47 -> 5.27 ms); the
// others unbounded (a bound there spills, the FP32 hex8 and the other
// neo-Hookean instances included, and a seven-wave bound on the persistent
// pen6 and hex8 code as well: measured with the compiler's resource
// report).
template <int T, int MODEL, int VAR, typename CT>
constexpr int persistent_min_waves()
{
    using S = ElemSmem<T, MODEL, VAR, CT>;
    if (MODEL == FEA_ELASTIC && S::SYM && sizeof(CT) == 8) return lds_waves<S>(16);
    if (MODEL == M_ELASTIC_NH && S::SYM && T == 0 && sizeof(CT) == 8) return 5;
    return 1;
}

template <int T, int MODEL, int VAR, typename CT>
constexpr int one_tile_min_waves()
{
    using S = ElemSmem<T, MODEL, VAR, CT>;
    return (MODEL == FEA_ELASTIC && S::SYM && sizeof(CT) == 8) ? lds_waves<S>() : 1;
}

// Reference shape functions and gradients of family T into LDS.
template <int T, int MODEL, int VAR, typename CT>
__device__ inline void elem_ref_tables(ElemSmem<T, MODEL, VAR, CT> &S, const int tid)
{
    constexpr int NN = Fam<T>::NN, NQ = Fam<T>::NQ;
    for (int i = tid; i < NQ * NN; i += 256) {
        const int q = i / NN, a = i % NN;
        S.sNr[q][a] = c_ref.N[T][q][a];
        S.sDN[q][a][0] = c_ref.dN[T][q][a][0];
        S.sDN[q][a][1] = c_ref.dN[T][q][a][1];
        S.sDN[q][a][2] = c_ref.dN[T][q][a][2];
    }
}

// Lame parameters of element e into LDS (elasticity).
__device__ inline void elem_lame(const ElemArgs &A, int32_t e, double lm[2])
{
    const double E = (e >= 0 && A.young) ? A.young[e] : 1.0, nu = e >= 0 ? A.nu[e] : 0.25;
    lm[0] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    lm[1] = E / (2.0 * (1.0 + nu));
}

// Geometry: one thread per (element, Gauss point), in FP64. Reads sX, sU,
// sE, sNH, sLM and the reference tables; writes the physical gradients (and
// the neo-Hookean pushed gradients) and the Gauss-point coefficients.
template <int T, int MODEL, int VAR, typename CT>
__device__ inline void elem_geometry(const ElemArgs &A, ElemSmem<T, MODEL, VAR, CT> &S, const int tid)
{
    using Smem = ElemSmem<T, MODEL, VAR, CT>;
    constexpr int NN = Fam<T>::NN, NQ = Fam<T>::NQ, EPB = Smem::EPB;
    constexpr bool NHK = Smem::NHK;
    using GradRec = typename Smem::GradRec;
    GradRec *sG = reinterpret_cast<GradRec *>(S.buf);
    GradRec *sH = reinterpret_cast<GradRec *>(S.buf + Smem::NG);
    if constexpr (!NHK && EPB * NQ <= 4 * 21) {
        // Three lanes per (element, Gauss point), 21 such groups per wave
        // (lane 63 idle, so that a group never spans two waves): lane r of a
        // group forms row r of J, the rows are exchanged across the group's
        // lanes, each lane inverts J and writes the gradients of nodes
        // r, r + 3, ... Same operations per value as one lane per point,
        // spread over up to four waves instead of one or two.
        const int lane = tid & 63, r = lane % 3;
        const int grp = (tid >> 6) * 21 + lane / 3;
        if (lane < 63 && grp < EPB * NQ) {
            const int el = grp / NQ, q = grp % NQ;
            const int32_t e = S.sE[el];
            if (e >= 0) {
                double Jr[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < NN; ++a)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Jr[j] += S.sX[el][a][r] * S.sDN[q][a][j];
                const int g0 = lane - r;
                double J[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) J[i][j] = __shfl(Jr[j], g0 + i);
                const double d = det3(J);
                if (r == 0 && !(d > 0.0)) atomicMin(A.status, e);
                double Ji[3][3];
                inv3(J, d, Ji);
#pragma unroll
                for (int a = r; a < NN; a += 3)
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        sG[el].v[q][a][i] =
                            (CT)(Ji[0][i] * S.sDN[q][a][0] + Ji[1][i] * S.sDN[q][a][1] + Ji[2][i] * S.sDN[q][a][2]);
                if (r == 0) S.sC[el][q][0] = (CT)(c_ref.w[T][q] * d);
            }
        }
        return;
    }
    if (tid < EPB * NQ) {
        int el = tid / NQ, q = tid % NQ;
        int32_t e = S.sE[el];
        if (e >= 0) {
            double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
            for (int a = 0; a < NN; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) J[i][j] += S.sX[el][a][i] * S.sDN[q][a][j];
            double d = det3(J);
            if (!(d > 0.0)) atomicMin(A.status, e);
            double Ji[3][3];
            inv3(J, d, Ji);
            double G[NN][3];
#pragma unroll
            for (int a = 0; a < NN; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    G[a][i] = Ji[0][i] * S.sDN[q][a][0] + Ji[1][i] * S.sDN[q][a][1] + Ji[2][i] * S.sDN[q][a][2];
                    sG[el].v[q][a][i] = (CT)G[a][i];
                }
            double wd = c_ref.w[T][q] * d;
            S.sC[el][q][0] = (CT)wd;
            if constexpr (NHK) {
                if (S.sNH[el]) {
                    const double lam = S.sLM[el][0], mu = S.sLM[el][1];
                    double F[3][3];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
                            for (int a = 0; a < NN; ++a) acc += S.sU[el][a][i] * G[a][j];
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
                            sH[el].v[q][a][j] =
                                (CT)(G[a][0] * Fi[0][j] + G[a][1] * Fi[1][j] + G[a][2] * Fi[2][j]);
                    S.sC[el][q][1] = (CT)(wd * lam);
                    S.sC[el][q][2] = (CT)(wd * (mu - lam * log(jf)));
                    S.sC[el][q][3] = (CT)(wd * mu);
                }
            }
        }
    }
}

// Block (a, b) of element el of the tile, from the gradients in LDS.
template <int T, int MODEL, int VAR, typename CT>
__device__ inline void elem_block(const ElemSmem<T, MODEL, VAR, CT> &S, const int el, const int a, const int b,
                                  CT *K)
{
    using Smem = ElemSmem<T, MODEL, VAR, CT>;
    constexpr int NQ = Fam<T>::NQ;
    constexpr bool ELAS = Smem::ELAS, NHK = Smem::NHK;
    using GradRec = typename Smem::GradRec;
    const GradRec *sG = reinterpret_cast<const GradRec *>(S.buf);
    const GradRec *sH = reinterpret_cast<const GradRec *>(S.buf + Smem::NG);
    if constexpr (!ELAS) {
        CT acc = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            CT dot = sG[el].v[q][a][0] * sG[el].v[q][b][0] + sG[el].v[q][a][1] * sG[el].v[q][b][1] +
                     sG[el].v[q][a][2] * sG[el].v[q][b][2];
            acc += S.sC[el][q][0] * dot;
        }
        K[0] = acc;
    } else if (!NHK || !S.sNH[el]) {
        // linear: K = lam S + mu S^T + mu tr(S) I, S = sum_q wd G_a (x) G_b
        CT Sm[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) Sm[c] = 0;
#pragma unroll 2
        for (int q = 0; q < NQ; ++q) {
            CT w = S.sC[el][q][0];
            CT ga[3] = {w * sG[el].v[q][a][0], w * sG[el].v[q][a][1], w * sG[el].v[q][a][2]};
            CT gb[3] = {sG[el].v[q][b][0], sG[el].v[q][b][1], sG[el].v[q][b][2]};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) Sm[i * 3 + j] += ga[i] * gb[j];
        }
        const CT lam = (CT)S.sLM[el][0], mu = (CT)S.sLM[el][1];
        const CT tr = Sm[0] + Sm[4] + Sm[8];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                CT v = lam * Sm[i * 3 + j] + mu * Sm[j * 3 + i];
                if (i == j) v += mu * tr;
                K[i * 3 + j] = v;
            }
    } else if constexpr (NHK) {
        // neo-Hookean: K_ij = sum_q c1 h_a,i h_b,j + c2 h_a,j h_b,i + c0 d_ij G_a.G_b
        CT T1[9], T2[9], dsum = 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) T1[c] = T2[c] = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            CT c1 = S.sC[el][q][1], c2 = S.sC[el][q][2], c0 = S.sC[el][q][3];
            CT ha[3] = {sH[el].v[q][a][0], sH[el].v[q][a][1], sH[el].v[q][a][2]};
            CT hb[3] = {sH[el].v[q][b][0], sH[el].v[q][b][1], sH[el].v[q][b][2]};
            CT dot = sG[el].v[q][a][0] * sG[el].v[q][b][0] + sG[el].v[q][a][1] * sG[el].v[q][b][1] +
                     sG[el].v[q][a][2] * sG[el].v[q][b][2];
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
}

// Right-hand side of node a of element el: the body force (src, B values),
// minus, for the Newton residual, the internal force.
template <int T, int MODEL, int VAR, typename CT>
__device__ inline void elem_rhs(const ElemSmem<T, MODEL, VAR, CT> &S, const int el, const int a, const double *src,
                                CT *f)
{
    using Smem = ElemSmem<T, MODEL, VAR, CT>;
    constexpr int NN = Fam<T>::NN, NQ = Fam<T>::NQ, B = Smem::B;
    constexpr bool RES = MODEL == M_ELASTIC_RES && sizeof(CT) == 8;
    using GradRec = typename Smem::GradRec;
    const GradRec *sG = reinterpret_cast<const GradRec *>(S.buf);
    const GradRec *sH = reinterpret_cast<const GradRec *>(S.buf + Smem::NG);
#pragma unroll
    for (int i = 0; i < B; ++i) f[i] = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        CT wn = S.sC[el][q][0] * (CT)S.sNr[q][a];
#pragma unroll
        for (int i = 0; i < B; ++i) f[i] += wn * (CT)src[i];
    }
    if constexpr (RES) {
        // f -= f_int_a = sum_q w detJ P grad N_a. Neo-Hookean:
        // P grad N_a = mu F grad N_a + (lam ln J - mu) F^-T grad N_a,
        // with F grad N_a = grad N_a + sum_b u_b (grad N_b . grad N_a)
        // and h_a = F^-T grad N_a from the tangent's records.
        // Linear: sigma = lam tr(H) I + mu (H + H^T), H = sum_b u_b (x) grad N_b.
        const bool nh = S.sNH[el] != 0;
        const double lam = S.sLM[el][0], mu = S.sLM[el][1];
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            const double ga[3] = {sG[el].v[q][a][0], sG[el].v[q][a][1], sG[el].v[q][a][2]};
            double uh[3] = {0.0, 0.0, 0.0};  // sum_b u_b (G_b . G_a)
            double hu[3] = {0.0, 0.0, 0.0};  // sum_b (u_b . G_a) G_b
            double trh = 0.0;                // sum_b u_b . G_b
            // both loops rolled: unrolled, every node's gradient and
            // displacement is hoisted into registers for the whole kernel
            // (residual instances at 133-188 VGPRs)
#pragma unroll 1
            for (int b = 0; b < NN; ++b) {
                const double gb[3] = {sG[el].v[q][b][0], sG[el].v[q][b][1], sG[el].v[q][b][2]};
                const double ub[3] = {S.sU[el][b][0], S.sU[el][b][1], S.sU[el][b][2]};
                const double gg = gb[0] * ga[0] + gb[1] * ga[1] + gb[2] * ga[2];
                const double ug = ub[0] * ga[0] + ub[1] * ga[1] + ub[2] * ga[2];
                trh += ub[0] * gb[0] + ub[1] * gb[1] + ub[2] * gb[2];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    uh[i] += ub[i] * gg;
                    hu[i] += ug * gb[i];
                }
            }
            if (nh) {
                const double c0 = S.sC[el][q][3], c2 = S.sC[el][q][2];
#pragma unroll
                for (int i = 0; i < 3; ++i) f[i] -= c0 * (ga[i] + uh[i]) - c2 * (double)sH[el].v[q][a][i];
            } else {
                const double wd = S.sC[el][q][0];
#pragma unroll
                for (int i = 0; i < 3; ++i) f[i] -= wd * (lam * trh * ga[i] + mu * (uh[i] + hu[i]));
            }
        }
    }
}

// Row-owner, atomic and colour forms: the EPB elements A.elems[first ..
// first + EPB) (ids beyond A.n are skipped) with the calling workgroup's 256
// threads and LDS S; one thread per block (a, b) of every element.
template <int T, int MODEL, int VAR, typename CT>
__device__ void elem_tile_full(const ElemArgs &A, int64_t first, ElemSmem<T, MODEL, VAR, CT> &S, const int tid)
{
    using Smem = ElemSmem<T, MODEL, VAR, CT>;
    constexpr int NN = Fam<T>::NN, P = NN * NN;
    constexpr int PW = Smem::PW, EPB = Smem::EPB, B = Smem::B, BB = Smem::BB;
    constexpr bool ELAS = Smem::ELAS, NHK = Smem::NHK, RO = Smem::RO, STAGE = Smem::STAGE;
    CT *sK = S.buf + Smem::NG + Smem::NHG;
    __syncthreads();  // the previous tile's readers of S are done
    elem_ref_tables(S, tid);

    // element data (threads below EPB) and, for the row-owner layout, node
    // data (the next EPB*NN threads) are fetched in the same phase
    if (tid < EPB) {
        int64_t i = first + tid;
        int32_t e = i < A.n ? A.elems[i] : -1;
        S.sE[tid] = e;
        if constexpr (!RO) {
            S.sM[tid] = e >= 0 ? A.map_ptr[e] : 0;
            S.sCP[tid] = e >= 0 ? A.conn_ptr[e] : 0;
        }
        S.sNH[tid] = (ELAS && e >= 0 && A.nh_flag) ? (int)A.nh_flag[e] : 0;
        if constexpr (ELAS) elem_lame(A, e, S.sLM[tid]);
    }
    if constexpr (RO) {
        if (tid >= EPB && tid < EPB + EPB * NN) {
            const int k = tid - EPB, el = k / NN, a = k % NN;
            const int64_t i = first + el;
            if (i < A.n) {
                const int32_t v = A.pnodes[i * NN + a];
                S.sX[el][a][0] = A.x[v];
                S.sX[el][a][1] = A.y[v];
                S.sX[el][a][2] = A.z[v];
                if constexpr (NHK) {
                    for (int c = 0; c < 3; ++c) S.sU[el][a][c] = A.u[3 * (int64_t)v + c];
                }
            }
        }
        __syncthreads();
    } else {
        __syncthreads();
        if (tid < EPB * NN) {
            int el = tid / NN, a = tid % NN;
            int32_t e = S.sE[el];
            if (e >= 0) {
                int32_t v = A.conn[S.sCP[el] + a];
                S.sX[el][a][0] = A.x[v];
                S.sX[el][a][1] = A.y[v];
                S.sX[el][a][2] = A.z[v];
                if constexpr (NHK) {
                    bool nh = S.sNH[el] != 0 || MODEL == M_ELASTIC_RES;
                    for (int c = 0; c < 3; ++c) S.sU[el][a][c] = nh ? A.u[3 * (int64_t)v + c] : 0.0;
                }
            }
        }
        __syncthreads();
    }

    elem_geometry(A, S, tid);
    __syncthreads();

    // element matrix: one thread per (element, block a-b)
    if (tid < EPB * PW) {
        const int el = tid / PW, w = tid % PW;
        const int a = w / NN, b = w % NN;
        const int p = a * NN + b;
        int32_t e = S.sE[el];
        // destination of this block, fetched before the contraction
        const int64_t dest = e < 0 ? -1
                             : RO  ? (int64_t)A.pdest[(first + el) * P + p]
                                   : (int64_t)A.e2nnz[S.sM[el] + p];
        if (dest >= 0) {
            CT K[BB];
            elem_block(S, el, a, b, K);
            if constexpr (STAGE) {
                S.sD[el * P + p] = (int32_t)dest;
#pragma unroll
                for (int c = 0; c < BB; ++c) sK[(el * P + p) * BB + c] = K[c];
            } else if constexpr (RO) {
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
        int32_t e = S.sE[el];
        if (e >= 0) {
            double src[B];
#pragma unroll
            for (int i = 0; i < B; ++i) src[i] = A.source[(int64_t)e * B + i];
            CT f[B];
            elem_rhs(S, el, a, src, f);
            if constexpr (RO) {
                CT *dst = (CT *)A.rcontrib + (int64_t)A.prdest[(first + el) * NN + a] * B;
#pragma unroll
                for (int i = 0; i < B; ++i) dst[i] = f[i];
            } else {
                int64_t v = A.conn[S.sCP[el] + a];
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

    if constexpr (STAGE) {
        __syncthreads();
        CT *out = (CT *)A.contrib;
        for (int idx = tid; idx < EPB * PW * BB; idx += 256) {
            const int blk = idx / BB;
            if (first + blk / PW < A.n) out[(int64_t)S.sD[blk] * BB + (idx - blk * BB)] = sK[idx];
        }
    }
}

// Upper-triangle form (V_ROWSYM) and its tile-coloured variant (V_TILECOL):
// tile first / EPB, one thread per local pair a <= b of every element.
// Every global load of the tile -- node ids, coordinates, right-hand-side
// destinations (where b has a workspace of its own), element data and
// source, the tile's entries, tile-block ends and slots (tile-coloured:
// blocks and their lower partners) -- is
// issued in the first phase, so that a tile waits for two dependent load
// latencies (range -> entries, node id -> coordinates) before its
// arithmetic, and none after it.
template <int T, int MODEL, int VAR, typename CT>
__device__ void elem_tile_sym(const ElemArgs &A, int64_t first, ElemSmem<T, MODEL, VAR, CT> &S, const int tid)
{
    using Smem = ElemSmem<T, MODEL, VAR, CT>;
    constexpr int NN = Fam<T>::NN;
    constexpr int PW = Smem::PW, EPB = Smem::EPB, B = Smem::B, BB = Smem::BB;
    constexpr bool ELAS = Smem::ELAS, NHK = Smem::NHK, TCOL = Smem::TCOL, ALIAS = Smem::ALIAS;
    // 3x3 blocks of the upper-triangle form: the right-hand side of node a
    // of an element rides in the strictly lower entries (3, 6, 7) of the
    // element's diagonal block (a, a), which symmetry makes redundant; the
    // tile sums then add it with the block values, and the block-value
    // kernel writes it out (no right-hand-side workspace, no reduction of
    // its own)
    constexpr bool RHSD = !TCOL && B == 3;
    CT *sK = S.buf + Smem::KOFF;
    __syncthreads();  // the previous tile's readers of S are done
    elem_ref_tables(S, tid);
    const int64_t tl = first / EPB;
    const int64_t e0 = A.tent_ptr[tl], d0 = A.ttb_ptr[tl];
    const int ne = (int)(A.tent_ptr[tl + 1] - e0), nd = (int)(A.ttb_ptr[tl + 1] - d0);
    int32_t rdest = 0;  // right-hand-side destination of (element, node) tid
    if (tid < EPB * NN) {
        const int el = tid / NN, a = tid % NN;
        const int64_t i = first + el;
        if (i < A.n) {
            const int32_t v = A.pnodes[i * NN + a];
            if constexpr (!RHSD) rdest = A.prdest[i * NN + a];
            S.sX[el][a][0] = A.x[v];
            S.sX[el][a][1] = A.y[v];
            S.sX[el][a][2] = A.z[v];
            if constexpr (NHK) {
                for (int c = 0; c < 3; ++c) S.sU[el][a][c] = A.u[3 * (int64_t)v + c];
            }
        }
    } else if (tid < EPB * NN + EPB) {
        const int el = tid - EPB * NN;
        const int64_t i = first + el;
        const int32_t e = i < A.n ? A.elems[i] : -1;
        S.sE[el] = e;
        S.sNH[el] = (ELAS && e >= 0 && A.nh_flag) ? (int)A.nh_flag[e] : 0;
        if constexpr (ELAS) elem_lame(A, e, S.sLM[el]);
#pragma unroll
        for (int c = 0; c < B; ++c) S.sSrc[el][c] = e >= 0 ? A.source[(int64_t)e * B + c] : 0.0;
    }
    for (int i = tid; i < ne; i += 256) S.sEnt[i] = A.tent[e0 + i];
    for (int i = tid; i < nd; i += 256) {
        S.sEend[i] = A.tb_eend[d0 + i];
        if constexpr (TCOL) {
            const int32_t k = A.tb_blk[d0 + i];
            S.sSlot[i] = k;
            S.sLp[i] = A.lpart[k];
        } else {
            S.sSlot[i] = A.tb_slot[d0 + i];
        }
    }
    __syncthreads();

    elem_geometry(A, S, tid);
    __syncthreads();

    // blocks: one thread per (element, pair a <= b); right-hand side: one
    // thread per (element, node)
    CT Ks[BB];
#pragma unroll
    for (int c = 0; c < BB; ++c) Ks[c] = 0;
    bool diag = false;
    // the block's staged entries; on a diagonal lane with RHSD the
    // strictly lower ones belong to the right-hand side
    auto stage = [&] {
#pragma unroll
        for (int c = 0; c < BB; ++c)
            if (!(RHSD && diag && (c == 3 || c == 6 || c == 7))) sK[tid * BB + c] = Ks[c];
    };
    if (tid < EPB * PW) {
        const int el = tid / PW, w = tid % PW;
        // w-th pair of the row-major upper triangle
        int a = 0, r = w;
#pragma unroll
        for (int k = 0; k < NN - 1; ++k) {
            const bool step = r >= NN - a;
            r -= step ? NN - a : 0;
            a += step ? 1 : 0;
        }
        const int b = a + r;
        diag = a == b;
        if (S.sE[el] >= 0) {
            elem_block(S, el, a, b, Ks);
            if (!RHSD && diag) {
                // a diagonal block is symmetric; copying its upper entries
                // makes it so bitwise (the products G_i (w G_j) and
                // G_j (w G_i) round differently), and with it A (with
                // RHSD the block-value kernel writes the copies)
#pragma unroll
                for (int i = 0; i < B; ++i)
#pragma unroll
                    for (int j = i + 1; j < B; ++j) Ks[j * B + i] = Ks[i * B + j];
            }
        }
        if constexpr (!ALIAS) stage();
    }
    CT f[B];
    int flane = -1;  // RHSD: the diagonal lane that carries f
    if (tid < EPB * NN) {
        const int el = tid / NN, a = tid % NN;
        if (S.sE[el] >= 0) {
            elem_rhs(S, el, a, S.sSrc[el], f);
            if constexpr (RHSD) {
                flane = el * PW + a * NN - a * (a - 1) / 2;  // pair (a, a)
            } else {
                CT *dst = (CT *)A.rcontrib + (int64_t)rdest * B;
#pragma unroll
                for (int i = 0; i < B; ++i) dst[i] = f[i];
            }
        }
    }
    if constexpr (ALIAS) {
        __syncthreads();  // every lane has read the gradients that sK overwrites
        if (tid < EPB * PW) stage();
    }
    if constexpr (RHSD) {
        if (flane >= 0) {
            sK[flane * BB + 3] = f[0];
            sK[flane * BB + 6] = f[1];
            sK[flane * BB + 7] = f[2];
        }
    }
    __syncthreads();

    // tile sums, the block's entries added in ascending lane (element)
    // order, in FP64: either one thread per tile-block adding all BB
    // components, or one thread per (tile-block, component), which walks
    // the block's entry list BB times but spreads a tile's sums over more
    // threads. Measured on MI355X (element phase, ms, FP64, hybrid256 /
    // hybrid96): per component everywhere 24.56 / 1.62, per block for pen6
    // and hex8 24.70 / 1.67, per block everywhere 26.2 / 1.71; FP32 staged
    // blocks: per block in every family (per component for tet4 and pyr5
    // was slightly slower). Both give bitwise the same sums.
    CT *out = (CT *)A.contrib;
    constexpr bool PER_BLOCK = sizeof(CT) == 4;
    if constexpr (PER_BLOCK) {
        for (int d = tid; d < nd; d += 256) {
            double acc[BB];
#pragma unroll
            for (int c = 0; c < BB; ++c) acc[c] = 0.0;
            const int q1 = S.sEend[d];
            for (int q = d ? S.sEend[d - 1] : 0; q < q1; ++q) {
                const int u = S.sEnt[q];
                const CT *k = sK + (u >> 1) * BB;
                CT v[BB];
#pragma unroll
                for (int c = 0; c < BB; ++c) v[c] = k[c];
                const bool tr = (u & 1) != 0;
#pragma unroll
                for (int c = 0; c < BB; ++c) acc[c] += (double)(tr ? v[(c % B) * B + c / B] : v[c]);
            }
            const int64_t blk = S.sSlot[d];
            if constexpr (TCOL) {
                // blk is the block; no other tile of this colour touches it
                // or its partner
                const int64_t l = S.sLp[d];
#pragma unroll
                for (int c = 0; c < BB; ++c) A.vals[blk * BB + c] += acc[c];
                if (l >= 0) {
#pragma unroll
                    for (int c = 0; c < BB; ++c) A.vals[l * BB + (c % B) * B + c / B] += acc[c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < BB; ++c) out[blk * BB + c] = (CT)acc[c];
            }
        }
    } else {
        for (int idx = tid; idx < nd * BB; idx += 256) {
            const int d = idx / BB, c = idx - d * BB, ct = (c % B) * B + c / B;
            double acc = 0.0;
            for (int q = d ? S.sEend[d - 1] : 0; q < S.sEend[d]; ++q) {
                const int u = S.sEnt[q];
                acc += (double)sK[(u >> 1) * BB + ((u & 1) ? ct : c)];
            }
            const int64_t blk = S.sSlot[d];
            if constexpr (TCOL) {
                const int64_t l = S.sLp[d];
                A.vals[blk * BB + c] += acc;
                if (l >= 0) A.vals[l * BB + ct] += acc;
            } else {
                out[blk * BB + c] = (CT)acc;
            }
        }
    }
}

// One tile of elements in the form VAR.
template <int T, int MODEL, int VAR, typename CT>
__device__ inline void elem_tile(const ElemArgs &A, int64_t first, ElemSmem<T, MODEL, VAR, CT> &S,
                                 const int tid = threadIdx.x)
{
    if constexpr (ElemSmem<T, MODEL, VAR, CT>::SYM)
        elem_tile_sym(A, first, S, tid);
    else
        elem_tile_full(A, first, S, tid);
}

}  // namespace fea
