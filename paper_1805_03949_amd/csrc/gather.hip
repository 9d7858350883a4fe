// Fused owner-computes assembly (FEA_ROWGATHER).
//
// Row i of A is the sum, over the elements that contain node i taken in
// ascending element order (the order of Algorithm 1), of the element-matrix
// rows of i; the same holds for entry i of b. A workgroup owns a tile of
// consecutive rows. For every (row, incident element) pair of the tile it
// recomputes the element's geometry at the Gauss points (one thread per pair
// and point, FP64), then the pair's strip of blocks K_ab, a the row node and
// b every node of the element (one thread per pair and b), keeps the strips
// in LDS and forms every block of its rows as the ascending-order sum of that
// block's contributions (one thread per block and block row). A and b are
// written once, with no workspace and no atomics: the paper's full-row
// distribution (Section 3.1, halo elements computed by every owner) at the
// scale of a workgroup.
//
// The price is that an element's geometry is recomputed once per incident
// row: FP64 arithmetic replaces the round trip of every element block through
// HBM that bounds the row-owner form.
//
// Tiles are built once per graph and come in five classes: rows whose
// elements all belong to one family (tet4, pyr5, pen6, hex8), with every loop
// bound known at compile time, and rows on family interfaces. Workgroups are
// persistent: each walks a run of tiles of one XCD's share and loads the next
// tile's data while it computes the current one. One-family tiles take their
// Gauss points in chunks (records of one chunk in LDS, partial sums in
// registers). A batched form runs the tiles of many meshes in one launch per
// class; neo-Hookean kernels add F^-1 and the tangent coefficients to the
// records.
#include <algorithm>
#include <cstddef>
#include <vector>

#include "elem.h"

namespace fea {

constexpr int GT = 256;              // threads of an interface-tile workgroup
// Threads per workgroup of the one-family classes (tet4, pyr5, pen6, hex8):
// at most one strip lane per thread, so a tile holds TPB / nodes pairs.
// Measured on MI355X: 128-thread workgroups (twice as many, half-size
// tiles) are no faster for pyr5/hex8 and slower for pen6.
constexpr int G_TPB[4] = {256, 256, 256, 256};
__host__ __device__ inline int gather_tpb(int c) { return c == 4 ? GT : G_TPB[c]; }
constexpr int G_MIXED = 4;           // tile class of rows touching several families
constexpr int G_RMAX = 64;           // rows per tile
constexpr int G_PMAX_MIXED = 64;     // (row, element) pairs per interface tile
constexpr int G_GMAX_MIXED = 384;    // Gauss points per interface tile

__host__ __device__ inline int gauss_of(int t) { return t == 0 ? 1 : (t == 2 ? 6 : 8); }

// Pairs a tile of rows of one family may hold (at most TPB / nodes: one
// strip lane per thread), and Gauss points a tile of class c may hold.
__host__ __device__ inline int gather_pmax(int c)
{
    return c == G_MIXED ? G_PMAX_MIXED : gather_tpb(c) / nodes_of(c);
}
__host__ __device__ inline int gather_gmax(int c)
{
    return c == G_MIXED ? G_GMAX_MIXED : gather_pmax(c) * gauss_of(c);
}

template <int C, int MODEL, typename CT>
struct GatherSmem {
    static constexpr bool MIX = C == G_MIXED;
    static constexpr int FAMILY = C;
    static constexpr int NN = MIX ? 8 : Fam<C>::NN;
    static constexpr int NQ = MIX ? 8 : Fam<C>::NQ;
    static constexpr int TPB = MIX ? GT : G_TPB[MIX ? 0 : C];
    static constexpr int PMAX = MIX ? G_PMAX_MIXED : TPB / NN;
    static_assert(PMAX * NN <= TPB || MIX, "one strip lane per thread");
    using CTy = CT;
    static constexpr bool NHK = MODEL == M_ELASTIC_NH;
    // One-family tiles take their Gauss points in NCH chunks of QC: the
    // geometry records of one chunk at a time live in LDS (the strips keep
    // their partial sums in registers). Linear 6- and 8-point families: two
    // chunks; neo-Hookean (larger records): two points per chunk.
    static constexpr int NCH = MIX ? 1 : (NQ < 6 ? 1 : (NHK ? NQ / 2 : 2));
    static constexpr int QC = NQ / NCH;
    static_assert(NQ % NCH == 0 && NCH <= 4, "whole chunks");
    // Records of pair p start at p * GS: an odd stride (5 for 4 points)
    // keeps the records that one wave's lanes read at the same point in
    // distinct LDS banks (a stride of 4 or 8 maps every fourth pair to one).
    static constexpr int GS = (QC == 2 || QC == 4 || QC == 8) ? QC + 1 : QC;
    static constexpr int GMAX = MIX ? G_GMAX_MIXED : PMAX * GS;
    static constexpr int NT = MIX ? 4 : 1;
    static constexpr int B = MODEL == FEA_POISSON ? 1 : 3;
    static constexpr int BB = B * B;
    // accumulators of a strip lane: S, or T1, T2 and the gradient dot sum
    static constexpr int ACC = NHK ? 19 : BB;

    double sJi[GMAX][9];      // inverse Jacobian at each (pair, Gauss point)
    CT sGa[GMAX][3];          // physical gradient of the row node there
                              // (linear elasticity: times the weight, wd G_a)
    CT sWd[GMAX];             // weight times det J
    // neo-Hookean pairs: F^-1, the row node's gradient pushed through it
    // (h_a,j = sum_J G_a,J Finv_Jj) and wd lam, wd (mu - lam ln det F), wd mu
    double sFi[NHK ? GMAX : 1][9];
    CT sHa[NHK ? GMAX : 1][3];
    CT sCc[NHK ? GMAX : 1][3];
    // one slot per lane: the node's coordinates (and displacement) until the
    // geometry is done, then the lane's block
    union LaneSlot {
        double x[NHK ? 6 : 3];
        CT k[BB];
    };
    static constexpr int LMAX = MIX ? GT : PMAX * NN;
    LaneSlot sL[LMAX];
    union {                   // same element type: pair p's entries of the
        double sF[PMAX][B];   // two views coincide (source of the pair's
        double sR[PMAX][B];   // element, then its right-hand-side contribution)
    };
    double sDN[NT][8][8][3];  // reference gradients [family][point][node]
    double sN[NT][8][8];
    double sW[NT][8];
    double sLM[PMAX][2];      // lam, mu of each pair's element
    int32_t sNH[NHK ? PMAX : 1];  // neo-Hookean flag of each pair's element
    int32_t sE[PMAX];
    int32_t sA[PMAX];         // local index of the row node in the element
    int32_t sT[MIX ? PMAX : 1];
    int32_t sLane[MIX ? PMAX + 1 : 1];  // first lane of each pair
    int32_t sGeo[MIX ? PMAX + 1 : 1];   // first Gauss-point record of each pair
    uint8_t sLP[MIX ? GT : 1];          // pair of each lane
    uint8_t sGP[MIX ? GMAX : 1];        // pair of each Gauss-point record
    int32_t sSL[MIX ? PMAX : 1];        // place of each pair's first lane and
    int32_t sSG[MIX ? PMAX : 1];        // first record in the family-sorted orders
    uint8_t sLI[MIX ? GT : 1];          // lanes in family-sorted order
    uint16_t sGI[MIX ? GMAX : 1];       // records in family-sorted order
    uint16_t sRP[G_RMAX + 1]; // first pair of each row
    uint16_t sIP[TPB + 1];    // first contribution of each block
    uint8_t sD[TPB];          // lane of each contribution, ascending element per block
};

struct GatherArgs {
    const double *x, *y, *z;
    const uint8_t *types;
    const double *young, *nu;
    const double *source;
    int32_t *status;
    const int64_t *n2e_ptr, *inv_ptr;
    const int32_t *n2e;
    const uint8_t *n2a;
    const int32_t *gnodes;
    const uint8_t *desc;
    const uint8_t *nh_flag;  // neo-Hookean kernels: per element
    const double *u;         // and displacements, 3 per node
    int64_t vals_off, rhs_off;  // first value of this mesh in vals and rhs
    int32_t mesh;               // index of this mesh's status entry
    // launch: tile records, outputs, status entries (one per mesh)
    const int32_t *tiles;
    void *vals, *rhs;
    int out_f32;
};

// GatherArgs as the batched kernels read them from the mesh table: every
// pointer typed as addressing global memory, so that the compiler keeps
// global instead of flat accesses (flat ones also count against the LDS
// wait counter).
#define FEA_G(T) T __attribute__((address_space(1))) *
struct GatherArgsGlobal {
    FEA_G(const double) x;
    FEA_G(const double) y;
    FEA_G(const double) z;
    FEA_G(const uint8_t) types;
    FEA_G(const double) young;
    FEA_G(const double) nu;
    FEA_G(const double) source;
    FEA_G(int32_t) status;
    FEA_G(const int64_t) n2e_ptr;
    FEA_G(const int64_t) inv_ptr;
    FEA_G(const int32_t) n2e;
    FEA_G(const uint8_t) n2a;
    FEA_G(const int32_t) gnodes;
    FEA_G(const uint8_t) desc;
    FEA_G(const uint8_t) nh_flag;
    FEA_G(const double) u;
    int64_t vals_off, rhs_off;
    int32_t mesh;
    FEA_G(const int32_t) tiles;
    FEA_G(void) vals;
    FEA_G(void) rhs;
    int out_f32;
};
#undef FEA_G
static_assert(sizeof(GatherArgsGlobal) == sizeof(GatherArgs) &&
                  offsetof(GatherArgsGlobal, tiles) == offsetof(GatherArgs, tiles) &&
                  offsetof(GatherArgsGlobal, out_f32) == offsetof(GatherArgs, out_f32),
              "GatherArgsGlobal mirrors GatherArgs");

__device__ __forceinline__ GatherArgs from_global(const GatherArgsGlobal &g)
{
    GatherArgs a;
    a.x = (const double *)g.x;
    a.y = (const double *)g.y;
    a.z = (const double *)g.z;
    a.types = (const uint8_t *)g.types;
    a.young = (const double *)g.young;
    a.nu = (const double *)g.nu;
    a.source = (const double *)g.source;
    a.status = (int32_t *)g.status;
    a.n2e_ptr = (const int64_t *)g.n2e_ptr;
    a.inv_ptr = (const int64_t *)g.inv_ptr;
    a.n2e = (const int32_t *)g.n2e;
    a.n2a = (const uint8_t *)g.n2a;
    a.gnodes = (const int32_t *)g.gnodes;
    a.desc = (const uint8_t *)g.desc;
    a.nh_flag = (const uint8_t *)g.nh_flag;
    a.u = (const double *)g.u;
    a.vals_off = g.vals_off;
    a.rhs_off = g.rhs_off;
    a.mesh = g.mesh;
    a.tiles = (const int32_t *)g.tiles;
    a.vals = (void *)g.vals;
    a.rhs = (void *)g.rhs;
    a.out_f32 = g.out_f32;
    return a;
}

// J, det J, J^-1 and the row node's gradient at Gauss point q of pair p
// (coordinates at lanes x0 ..), with the expressions of the element kernels
// (same rounding in FP64).
template <int F, typename Sm>
__device__ inline void g_geometry(Sm &S, int32_t *status, int p, int x0, int q, int g, int tf)
{
    using CT = typename Sm::CTy;
    constexpr int MODEL = Sm::B == 1 ? FEA_POISSON : FEA_ELASTIC;
    constexpr int NN = Fam<F>::NN;
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int a = 0; a < NN; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) J[i][j] += S.sL[x0 + a].x[i] * S.sDN[tf][q][a][j];
    const double d = det3(J);
    if (!(d > 0.0)) atomicMin(status, S.sE[p]);
    double Ji[3][3];
    inv3(J, d, Ji);
    const int a = S.sA[p];
    const double da0 = S.sDN[tf][q][a][0], da1 = S.sDN[tf][q][a][1], da2 = S.sDN[tf][q][a][2];
    const double wd = S.sW[tf][q] * d;
    const CT w = (CT)wd;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const CT ga = (CT)(Ji[0][i] * da0 + Ji[1][i] * da1 + Ji[2][i] * da2);
        S.sGa[g][i] = (MODEL == FEA_POISSON || Sm::NHK) ? ga : w * ga;
#pragma unroll
        for (int j = 0; j < 3; ++j) S.sJi[g][i * 3 + j] = Ji[i][j];
    }
    S.sWd[g] = w;
    if constexpr (Sm::NHK) {
        if (S.sNH[p]) {
            // F = I + sum_c u_c (x) G_c, then F^-1, the pushed row gradient
            // and the tangent coefficients (the element kernels' expressions)
            double G[NN][3];
#pragma unroll
            for (int c = 0; c < NN; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    G[c][i] = Ji[0][i] * S.sDN[tf][q][c][0] + Ji[1][i] * S.sDN[tf][q][c][1] +
                              Ji[2][i] * S.sDN[tf][q][c][2];
            double Fd[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
                    for (int c = 0; c < NN; ++c) acc += S.sL[x0 + c].x[3 + i] * G[c][j];
                    Fd[i][j] = acc;
                }
            const double jf = det3(Fd);
            if (!(jf > 0.0)) atomicMin(status, S.sE[p]);
            double Fi[3][3];
            inv3(Fd, jf, Fi);
            const double ga0 = Ji[0][0] * da0 + Ji[1][0] * da1 + Ji[2][0] * da2;
            const double ga1 = Ji[0][1] * da0 + Ji[1][1] * da1 + Ji[2][1] * da2;
            const double ga2 = Ji[0][2] * da0 + Ji[1][2] * da1 + Ji[2][2] * da2;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                S.sHa[g][j] = (CT)(ga0 * Fi[0][j] + ga1 * Fi[1][j] + ga2 * Fi[2][j]);
#pragma unroll
                for (int i = 0; i < 3; ++i) S.sFi[g][i * 3 + j] = Fi[i][j];
            }
            const double lam = S.sLM[p][0], mu = S.sLM[p][1];
            S.sCc[g][0] = (CT)(wd * lam);
            S.sCc[g][1] = (CT)(wd * (mu - lam * log(jf)));
            S.sCc[g][2] = (CT)(wd * mu);
        }
    }
}

// Accumulates, into acc, the Gauss points Q0 .. Q0 + QN - 1 of block K_ab
// of pair p (a its row node) for element node b: Poisson wd G_a.G_b, else
// S = wd G_a (x) G_b. Point q's record is g0 + q - Q0.
template <int F, int Q0, int QN, typename Sm, typename CT>
__device__ inline void g_strip_acc(Sm &S, CT *acc, int b, int g0, int tf, int nh)
{
#pragma unroll
    for (int q = Q0; q < Q0 + QN; ++q) {
        const int g = g0 + q - Q0;
        const double *Ji = S.sJi[g];
        const double d0 = S.sDN[tf][q][b][0], d1 = S.sDN[tf][q][b][1], d2 = S.sDN[tf][q][b][2];
        CT gb[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) gb[j] = (CT)(Ji[j] * d0 + Ji[3 + j] * d1 + Ji[6 + j] * d2);
        if constexpr (Sm::B == 1) {
            const CT dot = S.sGa[g][0] * gb[0] + S.sGa[g][1] * gb[1] + S.sGa[g][2] * gb[2];
            acc[0] += S.sWd[g] * dot;
        } else if (!Sm::NHK || !nh) {
            CT ga[3] = {S.sGa[g][0], S.sGa[g][1], S.sGa[g][2]};
            if constexpr (Sm::NHK) {
                const CT w = S.sWd[g];
#pragma unroll
                for (int i = 0; i < 3; ++i) ga[i] = w * ga[i];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) acc[i * 3 + j] += ga[i] * gb[j];
        } else if constexpr (Sm::NHK) {
            // T1 += c1 h_a (x) h_b, T2 += c2 h_a (x) h_b, dsum += c0 G_a.G_b
            const double *Fi = S.sFi[g];
            double gd[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) gd[j] = Ji[j] * d0 + Ji[3 + j] * d1 + Ji[6 + j] * d2;
            CT hb[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) hb[j] = (CT)(gd[0] * Fi[j] + gd[1] * Fi[3 + j] + gd[2] * Fi[6 + j]);
            const CT c1 = S.sCc[g][0], c2 = S.sCc[g][1], c0 = S.sCc[g][2];
            const CT ha[3] = {S.sHa[g][0], S.sHa[g][1], S.sHa[g][2]};
            const CT dot = S.sGa[g][0] * gb[0] + S.sGa[g][1] * gb[1] + S.sGa[g][2] * gb[2];
            acc[18] += c0 * dot;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const CT hh = ha[i] * hb[j];
                    acc[i * 3 + j] += c1 * hh;
                    acc[9 + i * 3 + j] += c2 * hh;
                }
        }
    }
}

// Lane l's block from its accumulated sums: Poisson as is, elasticity
// K = lam S + mu S^T + mu tr(S) I with the pair's Lame parameters.
template <typename Sm, typename CT>
__device__ inline void g_strip_out(Sm &S, const CT *acc, int p, int l)
{
    if constexpr (Sm::B == 1) {
        S.sL[l].k[0] = acc[0];
    } else if (Sm::NHK && S.sNH[p]) {
        // K_ij = T1_ij + T2_ji + delta_ij dsum
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                CT v = acc[i * 3 + j] + acc[9 + j * 3 + i];
                if (i == j) v += acc[18];
                S.sL[l].k[i * 3 + j] = v;
            }
    } else {
        const CT lam = (CT)S.sLM[p][0], mu = (CT)S.sLM[p][1];
        const CT tr = acc[0] + acc[4] + acc[8];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                CT v = lam * acc[i * 3 + j] + mu * acc[j * 3 + i];
                if (i == j) v += mu * tr;
                S.sL[l].k[i * 3 + j] = v;
            }
    }
}

// Right-hand side of pair p over Gauss points Q0 .. Q0 + QN - 1:
// f += wd N_a f_e.
template <int F, int Q0, int QN, typename Sm, typename CT>
__device__ inline void g_rhs_acc(Sm &S, CT *f, int p, int g0, int tf)
{
    const int a = S.sA[p];
#pragma unroll
    for (int q = Q0; q < Q0 + QN; ++q) {
        const CT wn = S.sWd[g0 + q - Q0] * (CT)S.sN[tf][q][a];
#pragma unroll
        for (int i = 0; i < Sm::B; ++i) f[i] += wn * (CT)S.sF[p][i];
    }
}

// Whole-element strip and right-hand side (tiles of several families).
template <int F, typename Sm>
__device__ inline void g_strip(Sm &S, int p, int b, int l, int g0, int tf)
{
    using CT = typename Sm::CTy;
    CT acc[Sm::ACC];
#pragma unroll
    for (int c = 0; c < Sm::ACC; ++c) acc[c] = 0;
    g_strip_acc<F, 0, Fam<F>::NQ>(S, acc, b, g0, tf, Sm::NHK ? S.sNH[p] : 0);
    g_strip_out(S, acc, p, l);
}

template <int F, typename Sm>
__device__ inline void g_rhs(Sm &S, int p, int g0, int tf)
{
    using CT = typename Sm::CTy;
    CT f[Sm::B];
#pragma unroll
    for (int i = 0; i < Sm::B; ++i) f[i] = 0;
    g_rhs_acc<F, 0, Fam<F>::NQ>(S, f, p, g0, tf);
    // sF[p] and sR[p] share storage; only this thread touches either
#pragma unroll
    for (int i = 0; i < Sm::B; ++i) S.sR[p][i] = (double)f[i];
}

// LDS barrier: waits for this wave's LDS operations only, so global loads
// issued for the next tile stay in flight across it (__syncthreads would
// also wait for every outstanding global access).
__device__ inline void sync_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Inclusive sum over the 64 lanes of the wave (every lane must call it);
// total receives the sum over all lanes.
__device__ inline int wave_scan_incl(int x, int &total)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(x, off, 64);
        if (lane >= off) x += u;
    }
    total = __shfl(x, 63, 64);
    return x;
}

struct TileRec {
    int32_t r0, nr, P0, np, k0, nk, j0, nj;
};

// Per-thread prefetch of one tile: index data (first stage) and what it
// points to (second stage). Thread tid holds lane tid, pair tid, the
// inverse-map offsets of blocks tid and tid + TPB, and row tid.
struct Pre1 {
    int32_t v, e;
    int ok_l, ok_p;
    uint8_t d, a;
    int64_t ip0, ip1, rp;
};
template <int B>
struct Pre2 {
    double x, y, z, E, nu;
    double u[3];
    double f[B];
    int t, nh;
};

__device__ inline TileRec load_rec(const int32_t *tiles, int64_t t)
{
    const int32_t *T = tiles + 8 * t;
    return {T[0], T[1], T[2], T[3], T[4], T[5], T[6], T[7]};
}

template <int TPB>
__device__ inline Pre1 load1(const GatherArgs &A, const TileRec &R, int tid)
{
    Pre1 P = {};
    P.ok_l = tid < R.nj;
    P.ok_p = tid < R.np;
    if (P.ok_l) {
        P.v = A.gnodes[(int64_t)R.j0 + tid];
        P.d = A.desc[(int64_t)R.j0 + tid];
    }
    if (P.ok_p) {
        P.e = A.n2e[(int64_t)R.P0 + tid];
        P.a = A.n2a[(int64_t)R.P0 + tid];
    }
    if (tid <= R.nk) P.ip0 = A.inv_ptr[(int64_t)R.k0 + tid];
    if (tid + TPB <= R.nk) P.ip1 = A.inv_ptr[(int64_t)R.k0 + tid + TPB];
    if (tid <= R.nr) P.rp = A.n2e_ptr[(int64_t)R.r0 + tid];
    return P;
}

template <int B, bool MIX, bool NHK>
__device__ inline Pre2<B> load2(const GatherArgs &A, const Pre1 &P)
{
    Pre2<B> Q = {};
    if (P.ok_l) {
        Q.x = A.x[P.v];
        Q.y = A.y[P.v];
        Q.z = A.z[P.v];
        if (NHK) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Q.u[c] = A.u[3 * (int64_t)P.v + c];
        }
    }
    if (P.ok_p) {
        if (NHK) Q.nh = A.nh_flag[P.e];
        Q.E = A.young ? A.young[P.e] : 1.0;
        if (A.nu) Q.nu = A.nu[P.e];
#pragma unroll
        for (int i = 0; i < B; ++i) Q.f[i] = A.source[(int64_t)P.e * B + i];
        if (MIX) Q.t = A.types[P.e];
    }
    return Q;
}

template <int C, int MODEL, typename CT>
__device__ inline void commit(GatherSmem<C, MODEL, CT> &S, const TileRec &R, const Pre1 &P,
                              const Pre2<GatherSmem<C, MODEL, CT>::B> &Q, int tid)
{
    constexpr int B = GatherSmem<C, MODEL, CT>::B;
    if (P.ok_l) {
        S.sL[tid].x[0] = Q.x;
        S.sL[tid].x[1] = Q.y;
        S.sL[tid].x[2] = Q.z;
        if constexpr (GatherSmem<C, MODEL, CT>::NHK) {
#pragma unroll
            for (int c = 0; c < 3; ++c) S.sL[tid].x[3 + c] = Q.u[c];
        }
        S.sD[tid] = P.d;
    }
    if (P.ok_p) {
        if constexpr (GatherSmem<C, MODEL, CT>::NHK) S.sNH[tid] = Q.nh;
        S.sE[tid] = P.e;
        S.sA[tid] = P.a;
        if constexpr (GatherSmem<C, MODEL, CT>::MIX) S.sT[tid] = Q.t;
#pragma unroll
        for (int i = 0; i < B; ++i) S.sF[tid][i] = Q.f[i];
        if constexpr (MODEL != FEA_POISSON) {
            S.sLM[tid][0] = Q.E * Q.nu / ((1.0 + Q.nu) * (1.0 - 2.0 * Q.nu));
            S.sLM[tid][1] = Q.E / (2.0 * (1.0 + Q.nu));
        }
    }
    if (tid <= R.nk) S.sIP[tid] = (uint16_t)(P.ip0 - R.j0);
    constexpr int TPB = GatherSmem<C, MODEL, CT>::TPB;
    if (tid + TPB <= R.nk) S.sIP[tid + TPB] = (uint16_t)(P.ip1 - R.j0);
    if (tid <= R.nr) S.sRP[tid] = (uint16_t)(P.rp - R.P0);
}

// Chunk CH of a one-family tile: geometry of its Gauss points, then their
// share of every lane's block and every pair's right-hand side.
template <int CH, typename Sm>
__device__ inline void pure_chunk(Sm &S, int32_t *status, const TileRec &R, typename Sm::CTy *acc,
                                  typename Sm::CTy *fr, int tid, int lp, int lb)
{
    constexpr int C = Sm::FAMILY, NN = Sm::NN, QC = Sm::QC, GS = Sm::GS, Q0 = CH * QC;
    for (int g = tid; g < R.np * QC; g += Sm::TPB) {
        const int p = g / QC, qq = g - p * QC;
        g_geometry<C>(S, status, p, p * NN, Q0 + qq, p * GS + qq, 0);
    }
    sync_lds();
    if (tid < R.nj) g_strip_acc<C, Q0, QC>(S, acc, lb, lp * GS, 0, Sm::NHK ? S.sNH[lp] : 0);
    if (tid < R.np) g_rhs_acc<C, Q0, QC>(S, fr, tid, tid * GS, 0);
}

// Waves per SIMD each class is compiled for (a register budget of 512 /
// waves), measured on MI355X: four for tet4 tiles, three for the other
// one-family tiles (their LDS admits three workgroups per CU; a budget of
// four waves spills), two for interface tiles.
constexpr int G_WAVES[5] = {4, 3, 3, 3, 2};
// neo-Hookean kernels hold about twice the accumulators and LDS records
constexpr int G_WAVES_NH[5] = {3, 2, 2, 2, 1};
template <int C, int MODEL>
struct GatherWaves {
    static constexpr int value = MODEL == M_ELASTIC_NH ? G_WAVES_NH[C] : G_WAVES[C];
};

// Persistent workgroups: the tiles of this launch are split into eight
// contiguous chunks, one per XCD (workgroup b runs on XCD b % 8), so that
// tiles sharing nodes share an L2; a workgroup takes every nW-th tile of its
// chunk and prefetches the next tile while it computes the current one.
// BATCHED: the tiles of one launch belong to several meshes; tile t's mesh
// view is meshes[tmesh[t]] (arrays, output offsets, status entry), and the
// launch fields (tiles, outputs, status base, output type) come from L.
template <int C, int MODEL, typename CT, bool BATCHED>
__global__ void __launch_bounds__((GatherSmem<C, MODEL, CT>::TPB))
__attribute__((amdgpu_waves_per_eu(GatherWaves<C, MODEL>::value)))
k_gather(GatherArgs L, const GatherArgs *meshes, const int32_t *tmesh, int64_t ntiles)
{
    using Sm = GatherSmem<C, MODEL, CT>;
    __shared__ Sm S;
    constexpr bool MIX = Sm::MIX;
    constexpr int NN = Sm::NN, NQ = Sm::NQ, B = Sm::B, BB = Sm::BB, GS = Sm::GS, TPB = Sm::TPB;
    const int tid = threadIdx.x;
    const int64_t nW = gridDim.x >> 3, x = blockIdx.x & 7;
    const int64_t c1 = (x + 1) * ntiles / 8;
    int64_t t = x * ntiles / 8 + (blockIdx.x >> 3);
    if (t >= c1) return;

    for (int i = tid; i < Sm::NT * 64; i += TPB) {
        const int tf = i >> 6, q = (i >> 3) & 7, a = i & 7;
        const int ty = MIX ? tf : C;
        S.sN[tf][q][a] = c_ref.N[ty][q][a];
#pragma unroll
        for (int j = 0; j < 3; ++j) S.sDN[tf][q][a][j] = c_ref.dN[ty][q][a][j];
        if (a == 0) S.sW[tf][q] = c_ref.w[ty][q];
    }
    // mesh view of tile t (scalar loads; one mesh when not batched)
    auto mesh_of = [&](int64_t tt) -> int32_t { return BATCHED ? tmesh[tt] : 0; };
    auto M = [&](int32_t m) -> GatherArgs {
        if constexpr (BATCHED) return from_global(reinterpret_cast<const GatherArgsGlobal *>(meshes)[m]);
        else return L;
    };
    TileRec R = load_rec(L.tiles, t);
    int32_t mc = mesh_of(t);
    {
        const Pre1 P = load1<Sm::TPB>(M(mc), R, tid);
        commit<C, MODEL, CT>(S, R, P, load2<B, MIX, Sm::NHK>(M(mc), P), tid);
    }
    int64_t tn = t + nW;
    TileRec Rn = {};
    Pre1 Pn = {};
    int32_t mn = 0;
    if (tn < c1) {
        Rn = load_rec(L.tiles, tn);
        mn = mesh_of(tn);
        Pn = load1<Sm::TPB>(M(mn), Rn, tid);
    }
    sync_lds();

    while (true) {
        // next tile: second-stage loads; the tile after it: first stage
        const bool more = tn < c1;
        Pre2<B> Qn = {};
        if (more) Qn = load2<B, MIX, Sm::NHK>(M(mn), Pn);
        const int64_t tnn = tn + nW;
        TileRec Rnn = {};
        Pre1 Pnn = {};
        int32_t mnn = 0;
        if (tnn < c1) {
            Rnn = load_rec(L.tiles, tnn);
            mnn = mesh_of(tnn);
            Pnn = load1<Sm::TPB>(M(mnn), Rnn, tid);
        }
        int32_t *const st = L.status + M(mc).mesh;

        if constexpr (MIX) {
            // lane and Gauss-point offsets of the pairs, and their places in
            // family-sorted visiting orders (np <= 64: one wave scans)
            if (tid < 64) {
                const bool ok = tid < R.np;
                const int ty = ok ? S.sT[tid] : 0;
                const int n = ok ? nodes_of(ty) : 0, nq = ok ? gauss_of(ty) : 0;
                int tn, tq;
                const int cn = wave_scan_incl(n, tn), cq = wave_scan_incl(nq, tq);
                S.sLane[tid + 1] = cn;
                S.sGeo[tid + 1] = cq;
                if (tid == 0) S.sLane[0] = S.sGeo[0] = 0;
                int bn = 0, bq = 0, sl = 0, sg = 0;
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    int fn, fq;
                    const int xn = ty == f ? n : 0, xq = ty == f ? nq : 0;
                    const int in = wave_scan_incl(xn, fn), iq = wave_scan_incl(xq, fq);
                    if (ty == f) {
                        sl = bn + in - xn;
                        sg = bq + iq - xq;
                    }
                    bn += fn;
                    bq += fq;
                }
                if (ok) {
                    S.sSL[tid] = sl;
                    S.sSG[tid] = sg;
                }
            }
            sync_lds();
            for (int p = tid; p < R.np; p += TPB) {
                for (int l = S.sLane[p]; l < S.sLane[p + 1]; ++l) {
                    S.sLP[l] = (uint8_t)p;
                    S.sLI[S.sSL[p] + l - S.sLane[p]] = (uint8_t)l;
                }
                for (int g = S.sGeo[p]; g < S.sGeo[p + 1]; ++g) {
                    S.sGP[g] = (uint8_t)p;
                    S.sGI[S.sSG[p] + g - S.sGeo[p]] = (uint16_t)g;
                }
            }
            sync_lds();
            const int ng = S.sGeo[R.np];
            // geometry: one thread per (pair, Gauss point), visited family by
            // family so that a wave runs one family's code
            for (int i = tid; i < ng; i += TPB) {
                const int g = S.sGI[i];
                const int p = S.sGP[g], ty = S.sT[p], q = g - S.sGeo[p], x0 = S.sLane[p];
                switch (ty) {
                case 0: g_geometry<0>(S, st, p, x0, q, g, 0); break;
                case 1: g_geometry<1>(S, st, p, x0, q, g, 1); break;
                case 2: g_geometry<2>(S, st, p, x0, q, g, 2); break;
                default: g_geometry<3>(S, st, p, x0, q, g, 3); break;
                }
            }
            sync_lds();
            // strips: one thread per lane (pair, element node), family by
            // family; right-hand side per pair
            for (int i = tid; i < R.nj; i += TPB) {
                const int l = S.sLI[i];
                const int p = S.sLP[l], ty = S.sT[p], b = l - S.sLane[p], g0 = S.sGeo[p];
                switch (ty) {
                case 0: g_strip<0>(S, p, b, l, g0, 0); break;
                case 1: g_strip<1>(S, p, b, l, g0, 1); break;
                case 2: g_strip<2>(S, p, b, l, g0, 2); break;
                default: g_strip<3>(S, p, b, l, g0, 3); break;
                }
            }
            for (int p = tid; p < R.np; p += TPB) {
                const int ty = S.sT[p], g0 = S.sGeo[p];
                switch (ty) {
                case 0: g_rhs<0>(S, p, g0, 0); break;
                case 1: g_rhs<1>(S, p, g0, 1); break;
                case 2: g_rhs<2>(S, p, g0, 2); break;
                default: g_rhs<3>(S, p, g0, 3); break;
                }
            }
        } else {
            // geometry one thread per (pair, Gauss point), strips one thread
            // per lane (pair, element node), right-hand side one per pair;
            // NCH chunks of Gauss points, partial sums in registers
            const int lp = tid / NN, lb = tid - lp * NN;
            CT acc[Sm::ACC], fr[B];
#pragma unroll
            for (int c = 0; c < Sm::ACC; ++c) acc[c] = 0;
#pragma unroll
            for (int i = 0; i < B; ++i) fr[i] = 0;
            pure_chunk<0>(S, st, R, acc, fr, tid, lp, lb);
            if constexpr (Sm::NCH >= 2) {
                sync_lds();  // the chunk's records are no longer read
                pure_chunk<1>(S, st, R, acc, fr, tid, lp, lb);
            }
            if constexpr (Sm::NCH >= 3) {
                sync_lds();
                pure_chunk<2>(S, st, R, acc, fr, tid, lp, lb);
            }
            if constexpr (Sm::NCH >= 4) {
                sync_lds();
                pure_chunk<3>(S, st, R, acc, fr, tid, lp, lb);
            }
            if (tid < R.nj) g_strip_out(S, acc, lp, tid);
            if (tid < R.np) {
#pragma unroll
                for (int i = 0; i < B; ++i) S.sR[tid][i] = (double)fr[i];
            }
        }
        sync_lds();

        // blocks of the tile's rows, one thread per (block, block row): the
        // block's contributions summed in ascending element order
        for (int idx = tid; idx < R.nk * B; idx += TPB) {
            const int k = idx / B, i = idx - k * B;
            double s[B];
#pragma unroll
            for (int c = 0; c < B; ++c) s[c] = 0.0;
            int j = S.sIP[k];
            const int je = S.sIP[k + 1];
            // four contributions' loads in flight; additions in ascending order
            for (; j + 4 <= je; j += 4) {
                const CT *s0 = S.sL[S.sD[j]].k + i * B, *s1 = S.sL[S.sD[j + 1]].k + i * B;
                const CT *s2 = S.sL[S.sD[j + 2]].k + i * B, *s3 = S.sL[S.sD[j + 3]].k + i * B;
                CT v[4][B];
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    v[0][c] = s0[c];
                    v[1][c] = s1[c];
                    v[2][c] = s2[c];
                    v[3][c] = s3[c];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < B; ++c) s[c] += (double)v[u][c];
            }
            for (; j < je; ++j) {
                const CT *src = S.sL[S.sD[j]].k + i * B;
#pragma unroll
                for (int c = 0; c < B; ++c) s[c] += (double)src[c];
            }
            const int64_t o = M(mc).vals_off + ((int64_t)R.k0 + k) * BB + i * B;
#pragma unroll
            for (int c = 0; c < B; ++c) {
                if (L.out_f32) ((float *)L.vals)[o + c] = (float)s[c];
                else ((double *)L.vals)[o + c] = s[c];
            }
        }
        for (int idx = tid; idx < R.nr * B; idx += TPB) {
            const int r = idx / B, c = idx - r * B;
            double s = 0.0;
            for (int p = S.sRP[r]; p < S.sRP[r + 1]; ++p) s += (double)S.sR[p][c];
            const int64_t o = M(mc).rhs_off + ((int64_t)R.r0 + r) * B + c;
            if (L.out_f32) ((float *)L.rhs)[o] = (float)s;
            else ((double *)L.rhs)[o] = s;
        }
        if (!more) break;
        sync_lds();  // the tile's LDS is no longer read
        commit<C, MODEL, CT>(S, Rn, Pn, Qn, tid);
        sync_lds();
        R = Rn;
        Rn = Rnn;
        Pn = Pnn;
        tn = tnn;
        mc = mn;
        mn = mnn;
    }
}

// Per row: incident pairs | family mask << 16, and lanes (sum of the
// elements' node counts) | Gauss points << 16, each saturated at 65535.
__global__ void k_gather_rowinfo(int64_t n_nodes, const int64_t *n2e_ptr, const int32_t *n2e,
                                 const uint8_t *types, uint32_t *info0, uint32_t *info1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const int64_t b = n2e_ptr[i], e = n2e_ptr[i + 1];
    uint32_t mask = 0, lanes = 0, geo = 0;
    for (int64_t p = b; p < e; ++p) {
        const int t = types[n2e[p]];
        mask |= 1u << t;
        lanes += nodes_of(t);
        geo += gauss_of(t);
    }
    const uint32_t pairs = (uint32_t)std::min<int64_t>(e - b, 65535);
    info0[i] = pairs | (mask << 16);
    info1[i] = std::min(lanes, 65535u) | (std::min(geo, 65535u) << 16);
}

// Tile records from the tiles' row ranges (rec[0], rec[1] set by the host).
__global__ void k_gather_records(int64_t ntiles, const int64_t *row_ptr, const int64_t *n2e_ptr,
                                 const int64_t *inv_ptr, int32_t *rec)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int32_t *R = rec + 8 * t;
    const int64_t r0 = R[0], r1 = r0 + R[1];
    const int64_t k0 = row_ptr[r0], k1 = row_ptr[r1];
    R[2] = (int32_t)n2e_ptr[r0];
    R[3] = (int32_t)(n2e_ptr[r1] - n2e_ptr[r0]);
    R[4] = (int32_t)k0;
    R[5] = (int32_t)(k1 - k0);
    R[6] = (int32_t)inv_ptr[k0];
    R[7] = (int32_t)(inv_ptr[k1] - inv_ptr[k0]);
}

// Row i's thread walks its elements in ascending order, as the inverse map
// was filled: it writes the node list of every pair at the pair's place in
// gnodes (the inverse-map position of the row's first slot onward) and, for
// every slot, the tile lane of the contribution at the slot's inverse-map
// position. base[i] is the lane of row i's first pair within its tile.
__global__ void k_gather_maps(int64_t n_nodes, const int64_t *n2e_ptr, const int32_t *n2e,
                              const uint8_t *n2a, const uint8_t *types, const int64_t *conn_ptr,
                              const int32_t *conn, const int64_t *row_ptr, const int64_t *map_ptr,
                              const int32_t *e2nnz, const int64_t *inv_ptr, const uint8_t *base,
                              int32_t *fill, int32_t *gnodes, uint8_t *desc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const int64_t g0 = inv_ptr[row_ptr[i]];
    int off = 0;
    for (int64_t p = n2e_ptr[i]; p < n2e_ptr[i + 1]; ++p) {
        const int32_t e = n2e[p];
        const int a = n2a[p];
        const int nn = nodes_of(types[e]);
        const int64_t cp = conn_ptr[e], m = map_ptr[e] + (int64_t)a * nn;
        for (int b = 0; b < nn; ++b) {
            gnodes[g0 + off + b] = conn[cp + b];
            const int32_t k = e2nnz[m + b];
            desc[inv_ptr[k] + fill[k]] = (uint8_t)(base[i] + off + b);
            fill[k] += 1;
        }
        off += nn;
    }
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { dfree(p); }
};

static int gather_prepare(fea_graph *g, const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                          hipStream_t s)
{
    const int64_t N = g->n_nodes;
    int rc;
    DevBuf info, fill, base;
    if ((rc = dalloc(&info.p, sizeof(uint32_t) * 2 * std::max<int64_t>(N, 1)))) return rc;
    uint32_t *i0 = (uint32_t *)info.p, *i1 = i0 + N;
    if (N) k_gather_rowinfo<<<grid_for(N, 256), 256, 0, s>>>(N, g->n2e_ptr, g->n2e, types, i0, i1);
    FEA_HIP(hipGetLastError());
    std::vector<uint32_t> h0(N), h1(N);
    if (N) {
        FEA_HIP(hipMemcpyAsync(h0.data(), i0, sizeof(uint32_t) * N, hipMemcpyDeviceToHost, s));
        FEA_HIP(hipMemcpyAsync(h1.data(), i1, sizeof(uint32_t) * N, hipMemcpyDeviceToHost, s));
    }
    FEA_HIP(hipStreamSynchronize(s));

    // greedy: consecutive rows of one class while the class's caps hold
    std::vector<int32_t> tiles[5];
    std::vector<uint8_t> hbase(N);
    int cls = -1, rows = 0, pairs = 0, lanes = 0, geo = 0;
    int64_t r0 = 0;
    auto close = [&](int64_t r1) {
        std::vector<int32_t> &v = tiles[cls < 0 ? G_MIXED : cls];
        const int32_t rec[8] = {(int32_t)r0, (int32_t)(r1 - r0), 0, 0, 0, 0, 0, 0};
        v.insert(v.end(), rec, rec + 8);
    };
    for (int64_t i = 0; i < N; ++i) {
        const int rp = (int)(h0[i] & 0xffff), mask = (int)(h0[i] >> 16);
        const int rl = (int)(h1[i] & 0xffff), rg = (int)(h1[i] >> 16);
        int rcl = -1;
        if (mask) {
            rcl = (mask & (mask - 1)) ? G_MIXED : __builtin_ctz(mask);
            if (rcl != G_MIXED && rp > gather_pmax(rcl)) rcl = G_MIXED;
            if (rp > G_PMAX_MIXED || rl > GT || rg > G_GMAX_MIXED)
                return set_error(FEA_ERANGE,
                                 "row gather: node %lld lies in %d elements (%d element nodes, %d Gauss "
                                 "points); the limits are %d, %d and %d",
                                 (long long)i, rp, rl, rg, G_PMAX_MIXED, GT, G_GMAX_MIXED);
        }
        const int c = rcl < 0 ? cls : rcl;
        const bool fits = rows < G_RMAX && (rcl < 0 || cls < 0 || c == cls) &&
                          (c < 0 || (pairs + rp <= gather_pmax(c) && lanes + rl <= gather_tpb(c) &&
                                     geo + rg <= gather_gmax(c)));
        if (rows > 0 && !fits) {
            close(i);
            r0 = i;
            cls = -1;
            rows = pairs = lanes = geo = 0;
        }
        if (rcl >= 0) cls = rcl;
        hbase[i] = (uint8_t)lanes;
        ++rows;
        pairs += rp;
        lanes += rl;
        geo += rg;
    }
    if (rows > 0) close(N);

    std::vector<int32_t> all;
    for (int c = 0; c < 5; ++c) {
        g->gtile_off[c] = (int64_t)all.size() / 8;
        all.insert(all.end(), tiles[c].begin(), tiles[c].end());
    }
    const int64_t ntiles = (int64_t)all.size() / 8;
    g->gtile_off[5] = ntiles;
    dfree(g->gtile);
    dfree(g->gnodes);
    dfree(g->gdesc);
    g->gtile = nullptr;
    g->gnodes = nullptr;
    g->gdesc = nullptr;
    const int64_t ml = std::max<int64_t>(g->map_len, 1);
    if ((rc = dalloc((void **)&g->gtile, sizeof(int32_t) * std::max<int64_t>(8 * ntiles, 1)))) return rc;
    if ((rc = dalloc((void **)&g->gnodes, sizeof(int32_t) * ml))) return rc;
    if ((rc = dalloc((void **)&g->gdesc, ml))) return rc;
    if ((rc = dalloc(&fill.p, sizeof(int32_t) * std::max<int64_t>(g->nnz, 1)))) return rc;
    if ((rc = dalloc(&base.p, std::max<int64_t>(N, 1)))) return rc;
    if (ntiles) {
        FEA_HIP(hipMemcpyAsync(g->gtile, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice, s));
        k_gather_records<<<grid_for(ntiles, 256), 256, 0, s>>>(ntiles, g->row_ptr, g->n2e_ptr, g->inv_ptr,
                                                                g->gtile);
    }
    if (N) FEA_HIP(hipMemcpyAsync(base.p, hbase.data(), N, hipMemcpyHostToDevice, s));
    if (g->nnz) FEA_HIP(hipMemsetAsync(fill.p, 0, sizeof(int32_t) * g->nnz, s));
    if (N)
        k_gather_maps<<<grid_for(N, 256), 256, 0, s>>>(N, g->n2e_ptr, g->n2e, g->n2a, types, conn_ptr, conn,
                                                       g->row_ptr, g->map_ptr, g->e2nnz, g->inv_ptr,
                                                       (const uint8_t *)base.p, (int32_t *)fill.p, g->gnodes,
                                                       g->gdesc);
    FEA_HIP(hipGetLastError());
    FEA_HIP(hipStreamSynchronize(s));
    g->gready = true;
    return FEA_OK;
}

template <int C, int MODEL, typename CT, bool BATCHED>
static int launch_class(const GatherArgs &L, const GatherArgs *meshes, const int32_t *tmesh, int64_t n,
                        hipStream_t s)
{
    constexpr int TPB = GatherSmem<C, MODEL, CT>::TPB;
    // persistent grid: as many workgroups as fit on the device at once, a
    // multiple of the 8 XCDs
    static int per_cu[64] = {0};
    static int cus[64] = {0};
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(FEA_EINVAL, "device index %d unsupported", dev);
    if (!per_cu[dev]) {
        int b = 0, c = 0;
        FEA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_gather<C, MODEL, CT, BATCHED>, TPB, 0));
        FEA_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
        cus[dev] = std::max(c, 8);
        per_cu[dev] = std::max(b, 1);
    }
    int64_t grid = std::min<int64_t>((int64_t)per_cu[dev] * cus[dev], (n + 7) / 8 * 8);
    grid = std::max<int64_t>(grid / 8 * 8, 8);
    k_gather<C, MODEL, CT, BATCHED><<<(unsigned)grid, TPB, 0, s>>>(L, meshes, tmesh, n);
    return FEA_OK;
}

// One launch per tile class; tiles of class c are tiles + 8 * off[c] ..
// (and, batched, their meshes tmesh + off[c] ..). With gev, records an
// event before each class and after the last.
template <int MODEL, typename CT, bool BATCHED>
static int launch_classes(GatherArgs L, const int32_t *tiles, const int64_t *off, const GatherArgs *meshes,
                          const int32_t *tmesh, hipStream_t s, hipEvent_t *gev)
{
    int rc = FEA_OK;
    for (int c = 0; c < 5 && !rc; ++c) {
        if (gev) FEA_HIP(hipEventRecord(gev[c], s));
        const int64_t n = off[c + 1] - off[c];
        if (n <= 0) continue;
        L.tiles = tiles + 8 * off[c];
        const int32_t *tm = BATCHED ? tmesh + off[c] : nullptr;
        switch (c) {
        case 0: rc = launch_class<0, MODEL, CT, BATCHED>(L, meshes, tm, n, s); break;
        case 1: rc = launch_class<1, MODEL, CT, BATCHED>(L, meshes, tm, n, s); break;
        case 2: rc = launch_class<2, MODEL, CT, BATCHED>(L, meshes, tm, n, s); break;
        case 3: rc = launch_class<3, MODEL, CT, BATCHED>(L, meshes, tm, n, s); break;
        default: rc = launch_class<G_MIXED, MODEL, CT, BATCHED>(L, meshes, tm, n, s); break;
        }
    }
    if (!rc && gev) FEA_HIP(hipEventRecord(gev[5], s));
    return rc;
}

template <bool BATCHED>
static int launch_models(int model, int precision, const GatherArgs &L, const int32_t *tiles, const int64_t *off,
                         const GatherArgs *meshes, const int32_t *tmesh, hipStream_t s, hipEvent_t *gev)
{
    if (model == FEA_POISSON)
        return precision == FEA_FP64 ? launch_classes<FEA_POISSON, double, BATCHED>(L, tiles, off, meshes, tmesh, s, gev)
                                     : launch_classes<FEA_POISSON, float, BATCHED>(L, tiles, off, meshes, tmesh, s, gev);
    if (model == FEA_ELASTIC)
        return precision == FEA_FP64 ? launch_classes<FEA_ELASTIC, double, BATCHED>(L, tiles, off, meshes, tmesh, s, gev)
                                     : launch_classes<FEA_ELASTIC, float, BATCHED>(L, tiles, off, meshes, tmesh, s, gev);
    return precision == FEA_FP64 ? launch_classes<M_ELASTIC_NH, double, BATCHED>(L, tiles, off, meshes, tmesh, s, gev)
                                 : launch_classes<M_ELASTIC_NH, float, BATCHED>(L, tiles, off, meshes, tmesh, s, gev);
}

// Mesh view of one mesh and its prepared graph.
static GatherArgs mesh_args(const fea_graph *g, const GatherInput &in)
{
    GatherArgs A = {};
    A.x = in.x;
    A.y = in.y;
    A.z = in.z;
    A.types = in.types;
    A.young = in.young;
    A.nu = in.nu;
    A.source = in.source;
    A.n2e_ptr = g->n2e_ptr;
    A.inv_ptr = g->inv_ptr;
    A.n2e = g->n2e;
    A.n2a = g->n2a;
    A.gnodes = g->gnodes;
    A.desc = g->gdesc;
    A.nh_flag = in.nh_flag;
    A.u = in.u;
    return A;
}

int gather_assemble(fea_graph *g, const GatherInput &in, int model, int precision, bool out_f32,
                    bool timing, hipStream_t s, void *vals, void *rhs)
{
    if (model == FEA_ELASTIC && in.nh_flag) model = M_ELASTIC_NH;
    int rc = ensure_tables();
    if (rc) return rc;
    if (!g->gready && (rc = gather_prepare(g, in.types, in.conn_ptr, in.conn, s))) return rc;
    GatherArgs L = mesh_args(g, in);
    L.status = in.status;
    L.vals = vals;
    L.rhs = rhs;
    L.out_f32 = out_f32 ? 1 : 0;
    g->gtimed = false;
    if (timing) {
        for (hipEvent_t &e : g->gev)
            if (!e) FEA_HIP(hipEventCreate(&e));
        FEA_HIP(hipEventRecord(g->ev[0], s));
    }
    if ((rc = launch_models<false>(model, precision, L, g->gtile, g->gtile_off, nullptr, nullptr, s,
                                   timing ? g->gev : nullptr)))
        return rc;
    FEA_HIP(hipGetLastError());
    g->gtimed = timing;
    if (timing) {
        // one fused kernel per class: no separate block-value phase
        FEA_HIP(hipEventRecord(g->ev[1], s));
        FEA_HIP(hipEventRecord(g->ev[2], s));
        FEA_HIP(hipEventRecord(g->ev[3], s));
    }
    return FEA_OK;
}

struct GatherBatch {
    int n_meshes = 0;
    GatherArgs *d_meshes = nullptr;  // mesh views (outputs as offsets)
    int32_t *d_tiles = nullptr;      // tile records of all meshes, by class
    int32_t *d_tmesh = nullptr;      // mesh of every tile
    int64_t off[6] = {0, 0, 0, 0, 0, 0};
};

void gather_batch_destroy(GatherBatch *gb)
{
    if (!gb) return;
    dfree(gb->d_meshes);
    dfree(gb->d_tiles);
    dfree(gb->d_tmesh);
    delete gb;
}

int gather_batch_build(GatherBatch **out, int n, fea_graph *const *graphs, const GatherInput *in,
                       const int64_t *vals_off, const int64_t *rhs_off, hipStream_t s)
{
    *out = nullptr;
    GatherBatch *gb = new GatherBatch();
    gb->n_meshes = n;
    int rc = FEA_OK;
    std::vector<GatherArgs> views(n);
    for (int m = 0; m < n && !rc; ++m) {
        fea_graph *g = graphs[m];
        if (!g->gready) rc = gather_prepare(g, in[m].types, in[m].conn_ptr, in[m].conn, s);
        views[m] = mesh_args(g, in[m]);
        views[m].vals_off = vals_off[m];
        views[m].rhs_off = rhs_off[m];
        views[m].mesh = m;
    }
    // tiles of class c: those of mesh 0, then mesh 1, ...
    int64_t total = 0;
    for (int c = 0; c < 5 && !rc; ++c) {
        gb->off[c] = total;
        for (int m = 0; m < n; ++m) total += graphs[m]->gtile_off[c + 1] - graphs[m]->gtile_off[c];
    }
    gb->off[5] = total;
    if (!rc && (rc = dalloc((void **)&gb->d_meshes, sizeof(GatherArgs) * std::max(n, 1)))) {}
    if (!rc && (rc = dalloc((void **)&gb->d_tiles, sizeof(int32_t) * 8 * std::max<int64_t>(total, 1)))) {}
    if (!rc && (rc = dalloc((void **)&gb->d_tmesh, sizeof(int32_t) * std::max<int64_t>(total, 1)))) {}
    if (!rc) {
        std::vector<int32_t> tm(total);
        int64_t at = 0;
        for (int c = 0; c < 5 && !rc; ++c)
            for (int m = 0; m < n; ++m) {
                const fea_graph *g = graphs[m];
                const int64_t k = g->gtile_off[c + 1] - g->gtile_off[c];
                if (k <= 0) continue;
                hipError_t e = hipMemcpyAsync(gb->d_tiles + 8 * at, g->gtile + 8 * g->gtile_off[c],
                                              sizeof(int32_t) * 8 * k, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) rc = set_error(FEA_EHIP, "tile copy failed: %s", hipGetErrorString(e));
                std::fill(tm.begin() + at, tm.begin() + at + k, m);
                at += k;
            }
        if (!rc && n) {
            hipError_t e = hipMemcpyAsync(gb->d_meshes, views.data(), sizeof(GatherArgs) * n, hipMemcpyHostToDevice, s);
            if (e == hipSuccess && total)
                e = hipMemcpyAsync(gb->d_tmesh, tm.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = set_error(FEA_EHIP, "batch set-up failed: %s", hipGetErrorString(e));
        }
    }
    if (rc) {
        gather_batch_destroy(gb);
        return rc;
    }
    *out = gb;
    return FEA_OK;
}

int gather_batch_assemble(const GatherBatch *gb, int model, bool nh, int precision, bool out_f32,
                          hipStream_t s, void *vals, void *rhs, int32_t *status)
{
    if (model == FEA_ELASTIC && nh) model = M_ELASTIC_NH;
    int rc = ensure_tables();
    if (rc) return rc;
    GatherArgs L = {};
    L.status = status;
    L.vals = vals;
    L.rhs = rhs;
    L.out_f32 = out_f32 ? 1 : 0;
    if ((rc = launch_models<true>(model, precision, L, gb->d_tiles, gb->off, gb->d_meshes, gb->d_tmesh, s,
                                  nullptr)))
        return rc;
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

}  // namespace fea

using namespace fea;

extern "C" int fea_last_class_timing(const fea_graph *g, float *ms)
{
    clear_error();
    if (!g || !ms) return set_error(FEA_EINVAL, "graph and ms are required");
    if (!g->gtimed) return set_error(FEA_EINVAL, "no timed FEA_ROWGATHER assembly on this graph");
    FEA_HIP(hipEventSynchronize(g->gev[5]));
    for (int c = 0; c < 5; ++c) FEA_HIP(hipEventElapsedTime(&ms[c], g->gev[c], g->gev[c + 1]));
    return FEA_OK;
}
