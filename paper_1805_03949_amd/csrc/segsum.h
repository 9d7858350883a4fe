// Segmented sums over a destination-sorted workspace: the second phase of
// the row-owner scatter (the owner of a block adds every contribution to it,
// the distribution of Section 3.2 applied to block rows) and of its
// upper-triangle form.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fea {

// Segment k of the workspace holds the W-value contributions to output k in
// ascending element order, segments back to back: ptr[k] .. ptr[k+1] (in
// slots of W values). The segments of a workgroup therefore form one
// contiguous range, which the workgroup streams into LDS a chunk at a time
// with coalesced loads of up to 16 bytes (data must be 16-byte aligned, as
// every device allocation is); each thread then adds its (segment,
// component) pairs, one per round, from LDS in ascending order, starting
// from 0, in FP64. The sums are bitwise those of a plain left-to-right loop over the
// segment.
//
// Launch shape per workspace type: bytes per load, rounds (segments per
// thread) and LDS bytes per chunk. Measured on MI355X over the hybrid96
// workspaces: FP64 streams best with 8-byte loads and one segment per
// thread; FP32 segments are half as long, and 16-byte loads with four
// segments per thread amortise the per-workgroup work (about 15% faster than
// one 4-byte load per segment and thread).
template <typename CT>
struct SegCfg {
    static constexpr int LOAD_BYTES = sizeof(CT) == 8 ? 8 : 16;
    static constexpr int ROUNDS = sizeof(CT) == 8 ? 1 : 4;
    static constexpr int CHUNK_BYTES = 16384;
};

template <int W, typename CT, typename OT>
__global__ void __launch_bounds__(256) k_segsum(int64_t n, const int64_t *ptr, const CT *data, OT *out)
{
    constexpr int TPS = 256 / W;                // segments per round
    constexpr int R = SegCfg<CT>::ROUNDS;       // rounds per workgroup
    constexpr int BPW = TPS * R;                // segments per workgroup
    constexpr int VEC = SegCfg<CT>::LOAD_BYTES / (int)sizeof(CT);  // values per load
    constexpr int CAPV = SegCfg<CT>::CHUNK_BYTES / (int)sizeof(CT);  // staged values per chunk
    constexpr int LV = CAPV / (256 * VEC);                    // loads per thread per chunk
    constexpr int CAPS = (CAPV - VEC) / W;      // slots per chunk (room for the alignment shift)
    struct alignas(VEC * sizeof(CT)) Vec {
        CT x[VEC];
    };
    __shared__ Vec sv[CAPV / VEC];
    const CT *svs = sv[0].x;
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * BPW;
    const int64_t mend = m0 + BPW < n ? m0 + BPW : n;
    const int lb = tid / W, c = tid - lb * W;
    int64_t k[R], j0[R], j1[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t m = m0 + lb + r * TPS;
        const bool act = lb < TPS && m < mend;
        k[r] = act ? m : -1;
        j0[r] = act ? ptr[k[r]] : 0;
        j1[r] = act ? ptr[k[r] + 1] : 0;
        acc[r] = 0.0;
    }
    const int64_t s0 = ptr[m0];
    const int64_t s1 = ptr[mend];
    for (int64_t base = s0; base < s1; base += CAPS) {
        const int64_t ns = s1 - base < CAPS ? s1 - base : CAPS;
        const int64_t f0 = base * W, f1 = f0 + ns * W;  // value range of this chunk
        const int64_t a0 = f0 & ~(int64_t)(VEC - 1);      // aligned start
        const int o = (int)(f0 - a0);
        const int nvec = (int)((f1 - a0 + VEC - 1) / VEC);
        Vec v[LV];
#pragma unroll
        for (int q = 0; q < LV; ++q) {
            const int i = tid + q * 256;
            const int64_t g = a0 + (int64_t)i * VEC;
            if (i < nvec && g >= f0 && g + VEC <= f1) {
                v[q] = *reinterpret_cast<const Vec *>(data + g);
            } else {
                // the partial vectors at the two ends of the range
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    v[q].x[e] = (i < nvec && g + e >= f0 && g + e < f1) ? data[g + e] : (CT)0;
            }
        }
        __syncthreads();  // the previous chunk's readers are done
#pragma unroll
        for (int q = 0; q < LV; ++q) {
            const int i = tid + q * 256;
            if (i < nvec) sv[i] = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t lo = j0[r] > base ? j0[r] : base, hi = j1[r] < base + ns ? j1[r] : base + ns;
            for (int64_t j = lo; j < hi; ++j) acc[r] += (double)svs[o + (j - base) * W + c];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (k[r] < 0) continue;
        out[k[r] * W + c] = (OT)acc[r];
    }
}

// The upper-triangle form's block values: output m of the upper-block list
// is block blk[m] (an upper or diagonal block), its tile sums are slots
// uptr[m] .. uptr[m+1] of the workspace (segments of consecutive m are
// adjacent), and the sum is written to block blk[m] and, transposed, to its
// lower partner lp[m] when that is >= 0; lp[m] = -(v + 1) marks the
// diagonal block of row v. With RHSD (3x3 blocks) a diagonal block's
// strictly lower entries (3, 6, 7) carry row v's right-hand side: those
// sums go to rhs[3v .. 3v+2], and entries 1, 2, 5 are written to their
// mirror positions too, so that every diagonal block is symmetric
// bitwise. Every per-output index is read at
// position m, so a workgroup's index loads are contiguous and independent
// of each other, and its workspace range (uptr[m0] .. uptr[m0 + BPW]) is
// known after one load; R rounds of 256 / W outputs per workgroup.
// Measured on MI355X (FP64 / FP32 tile sums, ms): hybrid256 1 round
// 16.55 / 15.15, 2 rounds 17.24-17.43 / 12.20-12.25, 4 rounds - / 12.53;
// hybrid96 1 round 0.92-0.94 / 0.88, 2 rounds 0.95 / 0.70, 4 rounds - /
// 0.71 (with the right-hand side carried in the diagonal tile sums).
// 16-byte FP64 loads, 32 KB chunks with 4-8 rounds (fewer workgroups per
// CU) and an XCD-contiguous workgroup order were all slower.
template <typename CT>
struct SymSegCfg {
    static constexpr int LOAD_BYTES = sizeof(CT) == 8 ? 8 : 16;
    static constexpr int ROUNDS = sizeof(CT) == 8 ? 1 : 2;
    static constexpr int CHUNK_BYTES = 16384;
};

template <int W, typename CT, typename OT, bool RHSD>
__global__ void __launch_bounds__(256) k_segsum_sym(int64_t n, const int32_t *blk, const int32_t *lp,
                                                    const int64_t *uptr, const CT *data, OT *out, OT *rhs)
{
    constexpr int TPS = 256 / W;                                      // outputs per round
    constexpr int R = SymSegCfg<CT>::ROUNDS;                          // rounds per workgroup
    constexpr int BPW = TPS * R;                                      // outputs per workgroup
    constexpr int VEC = SymSegCfg<CT>::LOAD_BYTES / (int)sizeof(CT);  // values per load
    constexpr int CAPV = SymSegCfg<CT>::CHUNK_BYTES / (int)sizeof(CT);
    constexpr int LV = CAPV / (256 * VEC);                            // loads per thread per chunk
    constexpr int CAPS = (CAPV - VEC) / W;                            // slots per chunk
    struct alignas(VEC * sizeof(CT)) Vec {
        CT x[VEC];
    };
    __shared__ Vec sv[CAPV / VEC];
    const CT *svs = sv[0].x;
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * BPW;
    const int64_t mend = m0 + BPW < n ? m0 + BPW : n;
    const int lb = tid / W, c = tid - lb * W;
    const int ct = W == 9 ? (c % 3) * 3 + c / 3 : c;
    int64_t k[R], l[R], j0[R], j1[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t m = m0 + lb + r * TPS;
        const bool act = lb < TPS && m < mend;
        k[r] = act ? (int64_t)blk[m] : -1;
        l[r] = act ? (int64_t)lp[m] : -1;
        j0[r] = act ? uptr[m] : 0;
        j1[r] = act ? uptr[m + 1] : 0;
        acc[r] = 0.0;
    }
    const int64_t s0 = uptr[m0], s1 = uptr[mend];
    for (int64_t base = s0; base < s1; base += CAPS) {
        const int64_t ns = s1 - base < CAPS ? s1 - base : CAPS;
        const int64_t f0 = base * W, f1 = f0 + ns * W;  // value range of this chunk
        const int64_t a0 = f0 & ~(int64_t)(VEC - 1);      // aligned start
        const int o = (int)(f0 - a0);
        const int nvec = (int)((f1 - a0 + VEC - 1) / VEC);
        Vec v[LV];
#pragma unroll
        for (int q = 0; q < LV; ++q) {
            const int i = tid + q * 256;
            const int64_t g = a0 + (int64_t)i * VEC;
            if (i < nvec && g >= f0 && g + VEC <= f1) {
                v[q] = *reinterpret_cast<const Vec *>(data + g);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    v[q].x[e] = (i < nvec && g + e >= f0 && g + e < f1) ? data[g + e] : (CT)0;
            }
        }
        __syncthreads();  // the previous chunk's readers are done
#pragma unroll
        for (int q = 0; q < LV; ++q) {
            const int i = tid + q * 256;
            if (i < nvec) sv[i] = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t lo = j0[r] > base ? j0[r] : base, hi = j1[r] < base + ns ? j1[r] : base + ns;
            for (int64_t j = lo; j < hi; ++j) acc[r] += (double)svs[o + (j - base) * W + c];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (k[r] < 0) continue;
        if (l[r] >= 0) {
            out[k[r] * W + c] = (OT)acc[r];
            out[l[r] * W + ct] = (OT)acc[r];
        } else if (RHSD && (c == 3 || c == 6 || c == 7)) {
            rhs[(-l[r] - 1) * 3 + (c == 3 ? 0 : c == 6 ? 1 : 2)] = (OT)acc[r];
        } else {
            out[k[r] * W + c] = (OT)acc[r];
            if (RHSD && ct != c) out[k[r] * W + ct] = (OT)acc[r];
        }
    }
}

template <int W, typename CT, typename OT>
inline void launch_segsum_sym(int64_t n, const int32_t *blk, const int32_t *lp, const int64_t *uptr,
                              const CT *data, OT *out, OT *rhs, hipStream_t s)
{
    constexpr int BPW = (256 / W) * SymSegCfg<CT>::ROUNDS;
    const unsigned grid = (unsigned)((n + BPW - 1) / BPW);
    k_segsum_sym<W, CT, OT, W == 9><<<grid, 256, 0, s>>>(n, blk, lp, uptr, data, out, rhs);
}

// out[0 .. n) = 0: the right-hand side of rows that no element touches,
// which no diagonal block carries (a kernel rather than a memset, so that
// the sequence can be captured into a graph).
template <typename OT>
__global__ void __launch_bounds__(256) k_zero(int64_t n, OT *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (OT)0;
}

// Launch over n segments (n > 0).
template <int W, typename CT, typename OT>
inline void launch_segsum(int64_t n, const int64_t *ptr, const CT *data, OT *out, hipStream_t s)
{
    constexpr int BPW = (256 / W) * SegCfg<CT>::ROUNDS;
    const unsigned grid = (unsigned)((n + BPW - 1) / BPW);
    k_segsum<W, CT, OT><<<grid, 256, 0, s>>>(n, ptr, data, out);
}

}  // namespace fea
