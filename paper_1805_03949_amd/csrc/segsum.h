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
// slots of W values). The n segments of a workgroup therefore form one
// contiguous range, which the workgroup streams into LDS with coalesced
// loads, a chunk at a time; each thread then adds one (segment, component)
// from LDS in ascending order, starting from 0, in FP64. The sums are
// bitwise those of a plain left-to-right loop over the segment.
//
// SYM: the upper-triangle form. Output m is block blk[m] (an upper or
// diagonal block; the segments of all other blocks are empty, so the
// segments of consecutive m are still adjacent), and the sum is also
// written, transposed, to block lpart[blk[m]] when that is >= 0 (block
// (j, i) of a symmetric matrix is block (i, j) transposed).
template <int W, typename CT, typename OT, bool SYM>
__global__ void __launch_bounds__(256) k_segsum(int64_t n, const int32_t *blk, const int32_t *lpart,
                                                const int64_t *ptr, const CT *data, OT *out)
{
    constexpr int BPW = 256 / W;        // segments per workgroup
    constexpr int LD = 8;               // loads per thread per chunk
    constexpr int CAPS = 256 * LD / W;  // slots per chunk
    __shared__ CT sv[CAPS * W];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * BPW;
    const int64_t mend = m0 + BPW < n ? m0 + BPW : n;
    const int lb = tid / W, c = tid - lb * W;
    const int64_t m = m0 + lb;
    const bool act = lb < BPW && m < mend;
    const int64_t k = act ? (SYM ? (int64_t)blk[m] : m) : 0;
    const int64_t j0 = act ? ptr[k] : 0, j1 = act ? ptr[k + 1] : 0;
    const int64_t s0 = ptr[SYM ? (int64_t)blk[m0] : m0];
    const int64_t s1 = ptr[(SYM ? (int64_t)blk[mend - 1] : mend - 1) + 1];
    double acc = 0.0;
    for (int64_t base = s0; base < s1; base += CAPS) {
        const int ns = (int)(s1 - base < CAPS ? s1 - base : CAPS);
        const int nv = ns * W;
        const CT *src = data + base * W;
        CT r[LD];
#pragma unroll
        for (int q = 0; q < LD; ++q) {
            const int i = tid + q * 256;
            r[q] = i < nv ? src[i] : (CT)0;
        }
        __syncthreads();  // the previous chunk's readers are done
#pragma unroll
        for (int q = 0; q < LD; ++q) {
            const int i = tid + q * 256;
            if (i < nv) sv[i] = r[q];
        }
        __syncthreads();
        const int64_t lo = j0 > base ? j0 : base, hi = j1 < base + ns ? j1 : base + ns;
        for (int64_t j = lo; j < hi; ++j) acc += (double)sv[(j - base) * W + c];
    }
    if (act) {
        out[k * W + c] = (OT)acc;
        if constexpr (SYM) {
            const int64_t l = lpart[k];
            if (l >= 0) out[l * W + (W == 9 ? (c % 3) * 3 + c / 3 : c)] = (OT)acc;
        }
    }
}

// Launch over n segments (n > 0).
template <int W, typename CT, typename OT, bool SYM>
inline void launch_segsum(int64_t n, const int32_t *blk, const int32_t *lpart, const int64_t *ptr,
                          const CT *data, OT *out, hipStream_t s)
{
    constexpr int BPW = 256 / W;
    const unsigned grid = (unsigned)((n + BPW - 1) / BPW);
    k_segsum<W, CT, OT, SYM><<<grid, 256, 0, s>>>(n, blk, lpart, ptr, data, out);
}

}  // namespace fea
