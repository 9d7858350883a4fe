// Graph build: mesh validation, type segmentation, node incidence, block
// sparsity pattern, element-to-nonzero map, inverse map and greedy colouring.
//
// Definitions (paper Section 2.1.1, Algorithm 1; Section 3.2, Algorithm 5):
// a block (i, j) exists when nodes i and j share an element; e2nnz maps the
// element-matrix slot (e, a, b) to the block of (conn[e][a], conn[e][b]);
// the inverse map lists each block's slots in ascending element order;
// elements of one colour share no node.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "fea_internal.h"
#include "host_graph.h"

namespace fea {

// ------------------------------------------------------------ validation
__global__ void k_validate(int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                           const int64_t *conn_ptr, const int32_t *conn, int64_t *bad)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems) return;
    int t = types[e];
    bool ok = t < 4;
    int nn = ok ? nodes_of(t) : 0;
    int64_t b = conn_ptr[e];
    ok = ok && (conn_ptr[e + 1] - b == nn) && b >= 0 && (e > 0 || b == 0);
    if (ok) {
        for (int a = 0; a < nn && ok; ++a) {
            int32_t v = conn[b + a];
            ok = v >= 0 && v < n_nodes;
            for (int c = 0; c < a && ok; ++c) ok = conn[b + c] != v;
        }
    }
    if (!ok) atomicMin((unsigned long long *)bad, (unsigned long long)e);
}

// Fingerprint of a validated mesh's connectivity: the sum over elements,
// modulo 2^64, of a SplitMix64-style mix of the element id, its family and
// its node ids in order (integer addition, so the result does not depend on
// the order the elements are visited in). Graph caches are checked against
// it.
__device__ inline uint64_t fp_mix(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void k_mesh_fingerprint(int64_t n_elems, const uint8_t *types, const int64_t *conn_ptr,
                                   const int32_t *conn, unsigned long long *out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems) return;
    const int t = types[e];
    uint64_t h = fp_mix((uint64_t)e ^ ((uint64_t)t << 56));
    for (int64_t p = conn_ptr[e]; p < conn_ptr[e + 1]; ++p) h = fp_mix(h ^ (uint64_t)(uint32_t)conn[p]);
    atomicAdd(out, (unsigned long long)h);
}

__global__ void k_slot_count(int64_t n_elems, const uint8_t *types, int64_t *cnt)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems) return;
    int nn = nodes_of(types[e]);
    cnt[e] = (int64_t)nn * nn;
}

// ------------------------------------------------------ type segmentation
__global__ void k_type_flags(int64_t n_elems, const uint8_t *types, int t, uint8_t *flag)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n_elems) flag[e] = types[e] == t;
}

__global__ void k_type_place(int64_t n_elems, const uint8_t *types, int t, const int64_t *pos,
                             int64_t base, int32_t *perm)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n_elems && types[e] == t) perm[base + pos[e]] = (int32_t)e;
}

// --------------------------------------------------------- node incidence
__global__ void k_node_count(int64_t conn_len, const int32_t *conn, int32_t *cnt)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < conn_len) atomicAdd(&cnt[conn[p]], 1);
}

__global__ void k_node_fill(int64_t n_elems, const int64_t *conn_ptr, const int32_t *conn,
                            const int64_t *n2e_ptr, int32_t *cursor, int32_t *n2e, uint8_t *n2a)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems) return;
    for (int64_t p = conn_ptr[e]; p < conn_ptr[e + 1]; ++p) {
        int32_t v = conn[p];
        int32_t slot = atomicAdd(&cursor[v], 1);
        n2e[n2e_ptr[v] + slot] = (int32_t)e;
        n2a[n2e_ptr[v] + slot] = (uint8_t)(p - conn_ptr[e]);
    }
}

// Insertion sort of each node's (element, local index) list by element.
__global__ void k_node_sort(int64_t n_nodes, const int64_t *n2e_ptr, int32_t *n2e, uint8_t *n2a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    int64_t b = n2e_ptr[i], e = n2e_ptr[i + 1];
    for (int64_t p = b + 1; p < e; ++p) {
        int32_t ke = n2e[p];
        uint8_t ka = n2a[p];
        int64_t q = p - 1;
        while (q >= b && n2e[q] > ke) {
            n2e[q + 1] = n2e[q];
            n2a[q + 1] = n2a[q];
            --q;
        }
        n2e[q + 1] = ke;
        n2a[q + 1] = ka;
    }
}

// ------------------------------------------------------------- row pattern
// Row i's columns are the distinct nodes of i's incident elements. They are
// produced in ascending order by repeatedly taking the smallest candidate
// above the last one emitted: no per-row buffer, so any row length works.
__device__ inline void row_pattern_serial(int64_t i, const int64_t *n2e_ptr, const int32_t *n2e,
                                          const int64_t *conn_ptr, const int32_t *conn, const int64_t *row_ptr,
                                          int32_t *col, int32_t *deg)
{
    int64_t b = n2e_ptr[i], e = n2e_ptr[i + 1];
    int32_t last = -1;
    int32_t cnt = 0;
    int64_t out = col ? row_ptr[i] : 0;
    for (;;) {
        int32_t best = INT_MAX;
        for (int64_t p = b; p < e; ++p) {
            int32_t el = n2e[p];
            for (int64_t k = conn_ptr[el]; k < conn_ptr[el + 1]; ++k) {
                int32_t v = conn[k];
                if (v > last && v < best) best = v;
            }
        }
        if (best == INT_MAX) break;
        if (col) col[out + cnt] = best;
        ++cnt;
        last = best;
    }
    if (deg) deg[i] = cnt;
}

// One 64-lane wave per row. The row's (element, local node) candidates sit
// on a fixed stride of 8 per incident element (no family has more nodes), so
// candidate f = 8 j + a is node a of the row's j-th element; lane l holds
// candidates l, l + 64, ... in registers (at most 64 elements: 8 each), and
// the wave emits the columns in ascending order by repeated wave-wide
// minimum above the last one emitted. A row with more incident elements
// takes the one-lane loop above.
__global__ void __launch_bounds__(256) k_row_pattern(int64_t n_nodes, const int64_t *n2e_ptr, const int32_t *n2e,
                                                     const int64_t *conn_ptr, const int32_t *conn,
                                                     const int64_t *row_ptr, int32_t *col, int32_t *deg)
{
    constexpr int KMAX = 8;  // candidates per lane: 64 elements of up to 8 nodes
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n_nodes) return;  // the whole wave
    const int64_t b = n2e_ptr[i];
    const int ne = (int)(n2e_ptr[i + 1] - b);
    if (ne > 64) {
        if (lane == 0) row_pattern_serial(i, n2e_ptr, n2e, conn_ptr, conn, row_ptr, col, deg);
        return;
    }
    // lane j < ne: the j-th incident element's first node and node count
    int64_t s = 0;
    int c = 0;
    if (lane < ne) {
        const int32_t el = n2e[b + lane];
        s = conn_ptr[el];
        c = (int)(conn_ptr[el + 1] - s);
    }
    const int K = (ne * 8 + 63) / 64;  // uniform over the wave
    int32_t v[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        v[k] = INT_MAX;
        if (k < K) {
            const int f = lane + 64 * k, j = f >> 3, a = f & 7;
            const int64_t sj = __shfl(s, j);
            const int cj = __shfl(c, j);
            if (j < ne && a < cj) v[k] = conn[sj + a];
        }
    }
    int32_t last = -1, cnt = 0;
    const int64_t out = col ? row_ptr[i] : 0;
    for (;;) {
        int32_t m = INT_MAX;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) m = (v[k] > last && v[k] < m) ? v[k] : m;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const int32_t w = __shfl_xor(m, o);
            m = w < m ? w : m;
        }
        if (m == INT_MAX) break;
        if (col && lane == 0) col[out + cnt] = m;
        ++cnt;
        last = m;
    }
    if (deg && lane == 0) deg[i] = cnt;
}

// e2nnz by binary search of conn[e][b] in row conn[e][a].
__global__ void k_e2nnz(int64_t n_elems, const int64_t *conn_ptr, const int32_t *conn,
                        const int64_t *row_ptr, const int32_t *col, const int64_t *map_ptr,
                        int32_t *e2nnz)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems) return;
    int64_t cb = conn_ptr[e];
    int nn = (int)(conn_ptr[e + 1] - cb);
    int64_t mb = map_ptr[e];
    for (int a = 0; a < nn; ++a) {
        int32_t r = conn[cb + a];
        int64_t rb = row_ptr[r], re = row_ptr[r + 1];
        for (int b = 0; b < nn; ++b) {
            int32_t c = conn[cb + b];
            int64_t lo = rb, hi = re - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (col[mid] < c) lo = mid + 1; else hi = mid;
            }
            e2nnz[mb + a * nn + b] = (int32_t)lo;
        }
    }
}

__global__ void k_inv_count(int64_t map_len, const int32_t *e2nnz, int32_t *cnt)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < map_len) atomicAdd(&cnt[e2nnz[s]], 1);
}

// Row i's thread owns the blocks of row i, so the per-block fill counters
// need no atomics, and walking i's elements in ascending order lists every
// block's slots in ascending element order.
__global__ void k_inv_fill(int64_t n_nodes, const int64_t *n2e_ptr, const int32_t *n2e,
                           const uint8_t *n2a, const int64_t *conn_ptr, const int64_t *map_ptr,
                           const int32_t *e2nnz, const int64_t *inv_ptr, int32_t *fill,
                           int32_t *inv)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    for (int64_t p = n2e_ptr[i]; p < n2e_ptr[i + 1]; ++p) {
        int32_t e = n2e[p];
        int a = n2a[p];
        int nn = (int)(conn_ptr[e + 1] - conn_ptr[e]);
        int64_t base = map_ptr[e] + (int64_t)a * nn;
        for (int b = 0; b < nn; ++b) {
            int64_t s = base + b;
            int32_t k = e2nnz[s];
            inv[inv_ptr[k] + fill[k]] = (int32_t)s;
            fill[k] += 1;
        }
    }
}

// Inverse permutation of the inverse map, and the incidence index of every
// conn position: the places where the element kernel of the row-owner
// variant stores its contributions, so that they lie sorted by destination.
__global__ void k_e2pos(int64_t map_len, const int32_t *inv, int32_t *e2pos)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < map_len) e2pos[inv[j]] = (int32_t)j;
}

__global__ void k_rpos(int64_t n_nodes, const int64_t *n2e_ptr, const int32_t *n2e,
                       const uint8_t *n2a, const int64_t *conn_ptr, int32_t *rpos)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    for (int64_t p = n2e_ptr[i]; p < n2e_ptr[i + 1]; ++p) rpos[conn_ptr[n2e[p]] + n2a[p]] = (int32_t)p;
}

// Row-owner layout in type-sorted order, one thread per position.
struct Bases {
    int64_t seg[5], node[5], slot[5];
};

__global__ void k_position_maps(int64_t n_elems, Bases bs, const int32_t *perm, const int64_t *conn_ptr,
                                const int32_t *conn, const int64_t *map_ptr, const int32_t *e2pos,
                                const int32_t *rpos, int32_t *pnodes, int32_t *pdest, int32_t *prdest)
{
    int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n_elems) return;
    int t = 0;
    while (t < 3 && pos >= bs.seg[t + 1]) ++t;
    const int n = nodes_of(t);
    const int64_t i = pos - bs.seg[t];
    const int32_t e = perm[pos];
    const int64_t c0 = conn_ptr[e], m0 = map_ptr[e];
    int32_t *pn = pnodes + bs.node[t] + i * n, *pr = prdest + bs.node[t] + i * n;
    int32_t *pd = pdest + bs.slot[t] + i * n * n;
    for (int a = 0; a < n; ++a) {
        pn[a] = conn[c0 + a];
        pr[a] = rpos[c0 + a];
    }
    for (int p = 0; p < n * n; ++p) pd[p] = e2pos[m0 + p];
}

struct TmpBuf {
    void *p = nullptr;
    ~TmpBuf() { dfree(p); }
};

// ---------------------------------------------- upper-triangle row-owner
// Block k = (i, j): its transposed partner (j, i) lies in row j (the
// pattern is structurally symmetric); upper blocks (j >= i) are their own.
__global__ void k_sym_partner(int64_t n_nodes, const int64_t *row_ptr, const int32_t *col, int32_t *upart)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const int32_t j = col[k];
        if (j >= i) {
            upart[k] = (int32_t)k;
        } else {
            int64_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < i) lo = mid + 1;
                else hi = mid;
            }
            upart[k] = (int32_t)lo;
        }
    }
}

// Lower partner of every upper block (-1 if none), and the upper blocks
// listed in CSR order (uoff = exclusive count of upper blocks before k).
__global__ void k_sym_lists(int64_t nnz, const int32_t *upart, const int64_t *uoff, int32_t *lpart,
                            int32_t *ublk)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int32_t u = upart[k];
    if (u == k) ublk[uoff[k]] = (int32_t)k;
    else lpart[u] = (int32_t)k;
}

__global__ void k_flag_upper(int64_t nnz, const int32_t *upart, int32_t *flag)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) flag[k] = upart[k] == k ? 1 : 0;
}

struct TileBases {
    int64_t seg[5], node[5], tile[5];
};

// One workgroup per tile: the tile's contributions (lane, transposed?) keyed
// by destination upper block, sorted (bitonic, in LDS) by block then lane.
// Pass 1 (!WRITE) stores the entry and distinct-block counts; pass 2 writes
// the entries and the tile-blocks at the scanned offsets.
template <bool WRITE>
__global__ void __launch_bounds__(256) k_tile_entries(TileBases tb, const int32_t *perm, const int32_t *pnodes,
                                                      const int64_t *map_ptr, const int32_t *e2nnz,
                                                      int32_t *cnt_ent, int32_t *cnt_blk, const int64_t *tent_ptr,
                                                      const int64_t *ttb_ptr, uint16_t *tent, int32_t *tb_blk,
                                                      uint16_t *tb_eend)
{
    constexpr int K = 512;
    constexpr uint64_t NONE = ~0ull;
    __shared__ uint64_t key[K];
    __shared__ int part[256];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    int t = 0;
    while (t < 3 && tile >= tb.tile[t + 1]) ++t;
    const int n = nodes_of(t), pw = n * (n + 1) / 2, epb = 256 / pw;
    const int64_t first = tb.seg[t] + (tile - tb.tile[t]) * epb;
    uint64_t k0 = NONE, k1 = NONE;
    if (tid < epb * pw) {
        const int el = tid / pw;
        int w = tid - el * pw, a = 0;
        while (w >= n - a) {
            w -= n - a;
            ++a;
        }
        const int b = a + w;
        const int64_t p = first + el;
        if (p < tb.seg[t + 1]) {
            const int32_t *pn = pnodes + tb.node[t] + (p - tb.seg[t]) * n;
            const int32_t na = pn[a], nb = pn[b];
            const int64_t m0 = map_ptr[perm[p]];
            const uint64_t kab = (uint64_t)e2nnz[m0 + a * n + b];
            const uint64_t lane = (uint64_t)tid << 1;
            if (a == b || na < nb) {
                k0 = kab << 10 | lane;
            } else if (na > nb) {
                k0 = (uint64_t)e2nnz[m0 + b * n + a] << 10 | lane | 1;
            } else {  // coincident nodes: both blocks land on the diagonal
                k0 = kab << 10 | lane;
                k1 = kab << 10 | lane | 1;
            }
        }
    }
    key[tid] = k0;
    key[tid + 256] = k1;
    __syncthreads();
    for (int size = 2; size <= K; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < K; i += 256) {
                const int j = i ^ stride;
                if (j > i) {
                    const uint64_t x = key[i], y = key[j];
                    if ((x > y) == ((i & size) == 0)) {
                        key[i] = y;
                        key[j] = x;
                    }
                }
            }
            __syncthreads();
        }
    // new-block flags of entries 2 tid and 2 tid + 1, and their scan
    int f[2];
    for (int q = 0; q < 2; ++q) {
        const int i = 2 * tid + q;
        f[q] = key[i] != NONE && (i == 0 || (key[i] >> 10) != (key[i - 1] >> 10));
    }
    part[tid] = f[0] + f[1];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const int nblk = part[255];
    const int nent = __syncthreads_count(key[2 * tid] != NONE) + __syncthreads_count(key[2 * tid + 1] != NONE);
    if constexpr (!WRITE) {
        if (tid == 0) {
            cnt_ent[tile] = nent;
            cnt_blk[tile] = nblk;
        }
    } else {
        const int64_t e0 = tent_ptr[tile], d0 = ttb_ptr[tile];
        int d = part[tid] - f[0] - f[1] - 1;  // tile-block of the entry before 2 tid
        for (int q = 0; q < 2; ++q) {
            const int i = 2 * tid + q;
            if (key[i] == NONE) break;
            d += f[q];
            tent[e0 + i] = (uint16_t)(key[i] & 1023);
            if (i + 1 == nent || (key[i + 1] >> 10) != (key[i] >> 10)) {
                tb_blk[d0 + d] = (int32_t)(key[i] >> 10);
                tb_eend[d0 + d] = (uint16_t)(i + 1);
            }
        }
    }
}

// Per entry m of the upper-block list: its block's lower partner, or
// -(v + 1) for the diagonal block of row v, and the start of its workspace
// segment (uptr[nup] = the workspace length).
__global__ void k_sym_compact(int64_t nup, int64_t nnz, int64_t n_nodes, const int32_t *ublk, const int32_t *lpart,
                              const int64_t *ts_ptr, const int64_t *row_ptr, int32_t *ulp, int64_t *uptr)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m < nup) {
        const int32_t k = ublk[m];
        int32_t l = lpart[k];
        if (l < 0) {
            int64_t lo = 0, hi = n_nodes - 1;  // the row holding block k
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (row_ptr[mid] <= k) lo = mid; else hi = mid - 1;
            }
            l = -(int32_t)lo - 1;
        }
        ulp[m] = l;
        uptr[m] = ts_ptr[k];
    } else if (m == nup) {
        uptr[m] = ts_ptr[nnz];
    }
}

__global__ void k_tb_count(int64_t ntb, const int32_t *tb_blk, int32_t *cnt)
{
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d < ntb) atomicAdd(&cnt[tb_blk[d]], 1);
}

__global__ void k_tb_fill(int64_t ntb, const int32_t *tb_blk, const int64_t *ts_ptr, int32_t *fill, int32_t *lst)
{
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= ntb) return;
    const int32_t k = tb_blk[d];
    lst[ts_ptr[k] + atomicAdd(&fill[k], 1)] = (int32_t)d;
}

// Each block's tile-blocks in ascending tile order (tile-blocks are numbered
// tile by tile), then every tile-block's workspace slot.
__global__ void k_tb_slots(int64_t nnz, const int64_t *ts_ptr, int32_t *lst, int32_t *tb_slot)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int64_t b = ts_ptr[k], e = ts_ptr[k + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        const int32_t v = lst[i];
        int64_t j = i - 1;
        while (j >= b && lst[j] > v) {
            lst[j + 1] = lst[j];
            --j;
        }
        lst[j + 1] = v;
    }
    for (int64_t i = b; i < e; ++i) tb_slot[lst[i]] = (int32_t)i;
}

int sym_prepare(fea_graph *g, hipStream_t s)
{
    constexpr int BS = 256;
    const int64_t N = g->n_nodes, nnz = g->nnz;
    int rc;
    void **bufs[] = {(void **)&g->upart, (void **)&g->ublk,    (void **)&g->lpart,  (void **)&g->tent_ptr,
                     (void **)&g->ttb_ptr, (void **)&g->tent,  (void **)&g->tb_eend, (void **)&g->tb_blk,
                     (void **)&g->tb_slot, (void **)&g->ts_ptr, (void **)&g->ulp, (void **)&g->uptr};
    for (void **b : bufs) {
        dfree(*b);
        *b = nullptr;
    }
    g->nup = 0;
    g->ulen = 0;
    g->nent = 0;
    g->sready = false;
    g->tcready = false;
    // partners and the upper-block list
    TmpBuf flag, uoff, tmp;
    const int64_t nn1 = std::max<int64_t>(nnz, 1);
    if ((rc = dalloc((void **)&g->upart, sizeof(int32_t) * nn1))) return rc;
    if ((rc = dalloc((void **)&g->lpart, sizeof(int32_t) * nn1))) return rc;
    if ((rc = dalloc((void **)&g->ublk, sizeof(int32_t) * nn1))) return rc;
    if ((rc = dalloc(&flag.p, sizeof(int32_t) * nn1))) return rc;
    if ((rc = dalloc(&uoff.p, sizeof(int64_t) * (nnz + 1)))) return rc;
    // the scan scratch serves the tile and block scans below as well
    TileBases tb;
    int64_t nt = 0;
    for (int t = 0; t < 4; ++t) {
        tb.seg[t] = g->seg[t];
        tb.node[t] = g->node_base[t];
        tb.tile[t] = nt;
        const int epb = sym_epb(t);
        nt += (g->seg[t + 1] - g->seg[t] + epb - 1) / epb;
    }
    tb.seg[4] = g->seg[4];
    tb.node[4] = g->node_base[4];
    tb.tile[4] = nt;
    for (int t = 0; t < 5; ++t) g->tile_base[t] = tb.tile[t];
    const int64_t nscan = std::max<int64_t>(std::max<int64_t>(nnz, nt), 1);
    if ((rc = dalloc(&tmp.p, sizeof(int64_t) * (scan_tmp_elems(nscan) + 64)))) return rc;
    if (N) k_sym_partner<<<grid_for(N, BS), BS, 0, s>>>(N, g->row_ptr, g->col, g->upart);
    if (nnz) {
        k_flag_upper<<<grid_for(nnz, BS), BS, 0, s>>>(nnz, g->upart, (int32_t *)flag.p);
        if ((rc = scan_to_ptr_i32((int32_t *)flag.p, nnz, (int64_t *)uoff.p, (int64_t *)tmp.p, s))) return rc;
        FEA_HIP(hipMemsetAsync(g->lpart, 0xff, sizeof(int32_t) * nnz, s));
        k_sym_lists<<<grid_for(nnz, BS), BS, 0, s>>>(nnz, g->upart, (const int64_t *)uoff.p, g->lpart, g->ublk);
        FEA_HIP(hipMemcpyAsync(&g->nup, (int64_t *)uoff.p + nnz, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    FEA_HIP(hipGetLastError());
    // tiles: entry and tile-block counts, offsets, then the entries
    TmpBuf cent, cblk;
    if ((rc = dalloc(&cent.p, sizeof(int32_t) * std::max<int64_t>(nt, 1)))) return rc;
    if ((rc = dalloc(&cblk.p, sizeof(int32_t) * std::max<int64_t>(nt, 1)))) return rc;
    if ((rc = dalloc((void **)&g->tent_ptr, sizeof(int64_t) * (nt + 1)))) return rc;
    if ((rc = dalloc((void **)&g->ttb_ptr, sizeof(int64_t) * (nt + 1)))) return rc;
    int64_t nent = 0, ntb = 0;
    if (nt) {
        k_tile_entries<false><<<(unsigned)nt, 256, 0, s>>>(tb, g->perm, g->pnodes, g->map_ptr, g->e2nnz,
                                                          (int32_t *)cent.p, (int32_t *)cblk.p, nullptr, nullptr,
                                                          nullptr, nullptr, nullptr);
        if ((rc = scan_to_ptr_i32((int32_t *)cent.p, nt, g->tent_ptr, (int64_t *)tmp.p, s))) return rc;
        if ((rc = scan_to_ptr_i32((int32_t *)cblk.p, nt, g->ttb_ptr, (int64_t *)tmp.p, s))) return rc;
        FEA_HIP(hipMemcpyAsync(&nent, g->tent_ptr + nt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        FEA_HIP(hipMemcpyAsync(&ntb, g->ttb_ptr + nt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    } else {
        FEA_HIP(hipMemsetAsync(g->tent_ptr, 0, sizeof(int64_t), s));
        FEA_HIP(hipMemsetAsync(g->ttb_ptr, 0, sizeof(int64_t), s));
    }
    FEA_HIP(hipStreamSynchronize(s));
    if (ntb > INT32_MAX) return set_error(FEA_ERANGE, "%lld tile-blocks exceed the int32 slot range", (long long)ntb);
    // one entry per (element, pair a <= b): the element kernels size their
    // tile buffers by it (an element repeating a node would add entries, and
    // the graph build rejects such elements)
    int64_t lanes = 0;
    for (int t = 0; t < 4; ++t) lanes += (g->seg[t + 1] - g->seg[t]) * (nodes_of(t) * (nodes_of(t) + 1) / 2);
    if (nent != lanes)
        return set_error(FEA_EMESH, "upper-triangle layout: %lld entries for %lld element pairs", (long long)nent,
                         (long long)lanes);
    if ((rc = dalloc((void **)&g->tent, sizeof(uint16_t) * std::max<int64_t>(nent, 1)))) return rc;
    if ((rc = dalloc((void **)&g->tb_eend, sizeof(uint16_t) * std::max<int64_t>(ntb, 1)))) return rc;
    if ((rc = dalloc((void **)&g->tb_blk, sizeof(int32_t) * std::max<int64_t>(ntb, 1)))) return rc;
    if ((rc = dalloc((void **)&g->tb_slot, sizeof(int32_t) * std::max<int64_t>(ntb, 1)))) return rc;
    if ((rc = dalloc((void **)&g->ts_ptr, sizeof(int64_t) * (nnz + 1)))) return rc;
    if (nt)
        k_tile_entries<true><<<(unsigned)nt, 256, 0, s>>>(tb, g->perm, g->pnodes, g->map_ptr, g->e2nnz, nullptr,
                                                         nullptr, g->tent_ptr, g->ttb_ptr, g->tent, g->tb_blk,
                                                         g->tb_eend);
    // workspace segments: per block its tile-blocks, ascending tile
    TmpBuf lst;
    if ((rc = dalloc(&lst.p, sizeof(int32_t) * std::max<int64_t>(ntb, 1)))) return rc;
    if (nnz) {
        FEA_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t) * nnz, s));
        if (ntb) k_tb_count<<<grid_for(ntb, BS), BS, 0, s>>>(ntb, g->tb_blk, (int32_t *)flag.p);
        if ((rc = scan_to_ptr_i32((int32_t *)flag.p, nnz, g->ts_ptr, (int64_t *)tmp.p, s))) return rc;
        FEA_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t) * nnz, s));
        if (ntb) {
            k_tb_fill<<<grid_for(ntb, BS), BS, 0, s>>>(ntb, g->tb_blk, g->ts_ptr, (int32_t *)flag.p,
                                                       (int32_t *)lst.p);
            k_tb_slots<<<grid_for(nnz, BS), BS, 0, s>>>(nnz, g->ts_ptr, (int32_t *)lst.p, g->tb_slot);
        }
    } else {
        FEA_HIP(hipMemsetAsync(g->ts_ptr, 0, sizeof(int64_t), s));
    }
    const int64_t nup = g->nup;
    if ((rc = dalloc((void **)&g->ulp, sizeof(int32_t) * std::max<int64_t>(nup, 1)))) return rc;
    if ((rc = dalloc((void **)&g->uptr, sizeof(int64_t) * (nup + 1)))) return rc;
    k_sym_compact<<<grid_for(nup + 1, BS), BS, 0, s>>>(nup, nnz, N, g->ublk, g->lpart, g->ts_ptr, g->row_ptr, g->ulp,
                                                       g->uptr);
    FEA_HIP(hipGetLastError());
    FEA_HIP(hipStreamSynchronize(s));
    g->ulen = ntb;
    g->nent = nent;
    // every row an element touches has one diagonal block: nnz = 2 nup - rows
    g->sym_empty_rows = N - (2 * nup - nnz);
    g->sready = true;
    return FEA_OK;
}

// Colouring of the upper-triangle tiles, the GPU counterpart of the
// commutative multidependences of Algorithm 7: a tile's nodes are its
// elements' nodes, tiles sharing a node are neighbours, and a tile's
// priority is its neighbour count (nneig). Tiles are coloured greedily
// (first fit) in descending priority, so that the tiles of one colour
// share no node and no block, and each (family, colour) launch lists its
// tiles in descending priority too, so that the most connected tiles are
// dispatched first. Sequential by definition: on the host.
int tile_colour_prepare(fea_graph *g, hipStream_t s)
{
    const int64_t N = g->n_nodes, C = g->conn_len;
    std::vector<int32_t> pn(std::max<int64_t>(C, 1));
    if (C) FEA_HIP(hipMemcpyAsync(pn.data(), g->pnodes, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
    FEA_HIP(hipStreamSynchronize(s));
    const int64_t nt = g->tile_base[4];
    // node ranges of the tiles in pnodes (families and tiles are contiguous)
    std::vector<int64_t> ptr((size_t)nt + 1, 0);
    std::vector<uint8_t> fam((size_t)std::max<int64_t>(nt, 1), 0);
    for (int t = 0; t < 4; ++t) {
        const int n = nodes_of(t), epb = sym_epb(t);
        const int64_t ne = g->seg[t + 1] - g->seg[t];
        for (int64_t i = 0; i < g->tile_base[t + 1] - g->tile_base[t]; ++i) {
            ptr[(size_t)(g->tile_base[t] + i + 1)] = g->node_base[t] + std::min<int64_t>(ne, (i + 1) * epb) * n;
            fam[(size_t)(g->tile_base[t] + i)] = (uint8_t)t;
        }
    }
    std::vector<int32_t> nneig((size_t)std::max<int64_t>(nt, 1), 0);
    host::neighbour_counts(N, nt, ptr.data(), pn.data(), nneig.data());
    const std::vector<int64_t> order = host::priority_order(nt, nneig.data());
    std::vector<int16_t> colour((size_t)std::max<int64_t>(nt, 1), 0);
    const int64_t ncol = host::greedy_first_fit(N, nt, ptr.data(), pn.data(), order.data(), colour.data());
    if (ncol < 0)
        return set_error(FEA_ERANGE, "tile %lld needs more than %d colours", (long long)(-ncol - 1), host::kMaxColours);
    std::vector<int64_t> seg;
    std::vector<int32_t> ctile;
    host::buckets(nt, 4, fam.data(), colour.data(), (int)ncol, order.data(), g->tile_base, seg, ctile);
    dfree(g->ctile);
    g->ctile = nullptr;
    int rc;
    if ((rc = dalloc((void **)&g->ctile, sizeof(int32_t) * std::max<int64_t>(nt, 1)))) return rc;
    if (nt) FEA_HIP(hipMemcpyAsync(g->ctile, ctile.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, s));
    FEA_HIP(hipStreamSynchronize(s));
    g->tc_colours = (int)ncol;
    g->tcseg = std::move(seg);
    g->tc_nneig = std::move(nneig);
    g->tcready = true;
    return FEA_OK;
}

// ------------------------------------------------------------- colouring
// Greedy first-fit in element order (the colouring of Algorithm 5; any
// valid colouring is correct, this one is deterministic). Sequential by
// definition, so it runs on the host over per-node masks of used colours,
// on a thread of its own that starts once the mesh is validated and works
// while the device builds the pattern and the maps.
struct HostColouring {
    std::vector<int64_t> cp;
    std::vector<int32_t> cn;
    std::vector<uint8_t> ty;
    std::vector<int16_t> colour;
    std::vector<int64_t> cseg;
    std::vector<int32_t> cperm;
    int64_t ncol = 0;
    bool nomem = false;
    std::thread th;
    ~HostColouring()
    {
        if (th.joinable()) th.join();
    }
    void run(int64_t N, int64_t E)
    {
        try {
            colour.assign((size_t)std::max<int64_t>(E, 1), 0);
            ncol = host::greedy_first_fit(N, E, cp.data(), cn.data(), nullptr, colour.data());
            // stable buckets by (family, colour) of element ids
            if (ncol >= 0) host::buckets(E, 4, ty.data(), colour.data(), (int)ncol, nullptr, nullptr, cseg, cperm);
        } catch (...) {
            nomem = true;
        }
    }
};

// Copies the (validated) connectivity to the host and starts the colouring.
static int colour_start(fea_graph *g, const int64_t *conn_ptr_d, const int32_t *conn_d, const uint8_t *types_d,
                        hipStream_t s, HostColouring &hc)
{
    const int64_t E = g->n_elems, N = g->n_nodes;
    try {
        hc.cp.resize(E + 1);
        hc.cn.resize(g->conn_len);
        hc.ty.resize(E);
    } catch (...) {
        return set_error(FEA_ENOMEM, "host allocation failed (colouring)");
    }
    FEA_HIP(hipMemcpyAsync(hc.cp.data(), conn_ptr_d, sizeof(int64_t) * (E + 1), hipMemcpyDeviceToHost, s));
    if (g->conn_len)
        FEA_HIP(hipMemcpyAsync(hc.cn.data(), conn_d, sizeof(int32_t) * g->conn_len, hipMemcpyDeviceToHost, s));
    if (E) FEA_HIP(hipMemcpyAsync(hc.ty.data(), types_d, E, hipMemcpyDeviceToHost, s));
    FEA_HIP(hipStreamSynchronize(s));
    try {
        hc.th = std::thread([&hc, N, E] { hc.run(N, E); });
    } catch (...) {
        hc.run(N, E);  // no thread to be had: colour here
    }
    return FEA_OK;
}

// Waits for the colouring and uploads it.
static int colour_finish(fea_graph *g, HostColouring &hc, hipStream_t s)
{
    const int64_t E = g->n_elems;
    if (hc.th.joinable()) hc.th.join();
    if (hc.nomem) return set_error(FEA_ENOMEM, "host allocation failed (colouring)");
    if (hc.ncol < 0)
        return set_error(FEA_ERANGE, "element %lld needs more than %d colours", (long long)(-hc.ncol - 1),
                         host::kMaxColours);
    int rc;
    if ((rc = dalloc((void **)&g->colour, sizeof(int16_t) * std::max<int64_t>(E, 1)))) return rc;
    if ((rc = dalloc((void **)&g->cperm, sizeof(int32_t) * std::max<int64_t>(E, 1)))) return rc;
    if (E) {
        FEA_HIP(hipMemcpyAsync(g->colour, hc.colour.data(), sizeof(int16_t) * E, hipMemcpyHostToDevice, s));
        FEA_HIP(hipMemcpyAsync(g->cperm, hc.cperm.data(), sizeof(int32_t) * E, hipMemcpyHostToDevice, s));
    }
    FEA_HIP(hipStreamSynchronize(s));
    g->n_colours = (int)hc.ncol;
    g->cseg = std::move(hc.cseg);
    return FEA_OK;
}

static void destroy(fea_graph *g)
{
    if (!g) return;
    void *bufs[] = {g->row_ptr, g->col, g->map_ptr, g->e2nnz, g->inv_ptr, g->inv, g->pnodes, g->pdest, g->prdest,
                    g->n2e_ptr, g->n2e, g->n2a, g->perm, g->colour, g->cperm,
                    g->contrib, g->rcontrib, g->acc64, g->gtile, g->gnodes, g->gdesc, g->upart, g->ublk, g->lpart, g->tent_ptr, g->ttb_ptr,
                    g->tent, g->tb_eend, g->tb_blk, g->tb_slot, g->ts_ptr, g->ctile, g->gp_ptr, g->ulp, g->uptr};
    for (void *b : bufs) dfree(b);
    for (hipEvent_t e : g->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : g->gev)
        if (e) (void)hipEventDestroy(e);
    delete g;
}


// Validates a mesh (FEA_EMESH names the first bad element) and returns
// its connectivity fingerprint.
static int mesh_fingerprint(int64_t E, const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                            hipStream_t s, uint64_t *fp)
{
    TmpBuf acc;
    int rc;
    if ((rc = dalloc(&acc.p, sizeof(unsigned long long)))) return rc;
    FEA_HIP(hipMemsetAsync(acc.p, 0, sizeof(unsigned long long), s));
    if (E) k_mesh_fingerprint<<<grid_for(E, 256), 256, 0, s>>>(E, types, conn_ptr, conn, (unsigned long long *)acc.p);
    FEA_HIP(hipGetLastError());
    FEA_HIP(hipMemcpyAsync(fp, acc.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    FEA_HIP(hipStreamSynchronize(s));
    return FEA_OK;
}

static int validate(int64_t N, int64_t E, const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                    hipStream_t s)
{
    TmpBuf bad;
    int rc;
    if ((rc = dalloc(&bad.p, sizeof(int64_t)))) return rc;
    int64_t big = INT64_MAX;
    FEA_HIP(hipMemcpyAsync(bad.p, &big, sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (E) k_validate<<<grid_for(E, 256), 256, 0, s>>>(N, E, types, conn_ptr, conn, (int64_t *)bad.p);
    FEA_HIP(hipGetLastError());
    int64_t first_bad = INT64_MAX;
    FEA_HIP(hipMemcpyAsync(&first_bad, bad.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEA_HIP(hipStreamSynchronize(s));
    if (first_bad != INT64_MAX)
        return set_error(FEA_EMESH, "invalid element %lld (unknown type, wrong node count, node id out "
                         "of range or repeated node)", (long long)first_bad);
    return FEA_OK;
}

static int build(int64_t N, int64_t E, const uint8_t *types, const int64_t *conn_ptr,
                 const int32_t *conn, hipStream_t s, fea_graph *g)
{
    const int BS = 256;
    int rc;
    FEA_HIP(hipGetDevice(&g->device));
    g->n_nodes = N;
    g->n_elems = E;
    if (E > 0)
        FEA_HIP(hipMemcpyAsync(&g->conn_len, conn_ptr + E, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEA_HIP(hipStreamSynchronize(s));

    // validation
    TmpBuf tmp, cnt64, cnt32, flag, fillb;
    if ((rc = validate(N, E, types, conn_ptr, conn, s))) return rc;
    if ((rc = mesh_fingerprint(E, types, conn_ptr, conn, s, &g->mesh_fp))) return rc;
    HostColouring hc;  // joined on every return
    if ((rc = colour_start(g, conn_ptr, conn, types, s, hc))) return rc;

    int64_t scan_n = std::max<int64_t>(std::max<int64_t>(E, N), g->conn_len);
    // slots: map_ptr = prefix sum of n_e^2
    if ((rc = dalloc(&tmp.p, sizeof(int64_t) * (scan_tmp_elems(scan_n) + 64)))) return rc;
    if ((rc = dalloc(&cnt64.p, sizeof(int64_t) * std::max<int64_t>(E, N) + 8))) return rc;
    if ((rc = dalloc((void **)&g->map_ptr, sizeof(int64_t) * (E + 1)))) return rc;
    if (E) k_slot_count<<<grid_for(E, BS), BS, 0, s>>>(E, types, (int64_t *)cnt64.p);
    if ((rc = scan_to_ptr_i64((int64_t *)cnt64.p, E, g->map_ptr, (int64_t *)tmp.p, s))) return rc;
    FEA_HIP(hipMemcpyAsync(&g->map_len, g->map_ptr + E, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEA_HIP(hipStreamSynchronize(s));
    if (g->map_len > INT32_MAX || g->conn_len > INT32_MAX)
        return set_error(FEA_ERANGE, "%lld element-matrix slots / %lld incidences exceed int32 maps",
                         (long long)g->map_len, (long long)g->conn_len);

    // type segmentation (stable partition by family)
    if ((rc = dalloc(&flag.p, std::max<int64_t>(E, 1)))) return rc;
    if ((rc = dalloc((void **)&g->perm, sizeof(int32_t) * std::max<int64_t>(E, 1)))) return rc;
    {
        int64_t base = 0;
        for (int t = 0; t < 4; ++t) {
            g->seg[t] = base;
            if (!E) continue;
            k_type_flags<<<grid_for(E, BS), BS, 0, s>>>(E, types, t, (uint8_t *)flag.p);
            if ((rc = scan_to_ptr_u8((uint8_t *)flag.p, E, (int64_t *)cnt64.p, (int64_t *)tmp.p, s))) return rc;
            k_type_place<<<grid_for(E, BS), BS, 0, s>>>(E, types, t, (int64_t *)cnt64.p, base, g->perm);
            int64_t cnt_t = 0;
            FEA_HIP(hipMemcpyAsync(&cnt_t, (int64_t *)cnt64.p + E, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            FEA_HIP(hipStreamSynchronize(s));
            base += cnt_t;
        }
        g->seg[4] = base;
    }

    // node incidence
    if ((rc = dalloc(&cnt32.p, sizeof(int32_t) * (N + 1)))) return rc;
    if ((rc = dalloc((void **)&g->n2e_ptr, sizeof(int64_t) * (N + 1)))) return rc;
    if ((rc = dalloc((void **)&g->n2e, sizeof(int32_t) * std::max<int64_t>(g->conn_len, 1)))) return rc;
    if ((rc = dalloc((void **)&g->n2a, std::max<int64_t>(g->conn_len, 1)))) return rc;
    FEA_HIP(hipMemsetAsync(cnt32.p, 0, sizeof(int32_t) * (N + 1), s));
    if (g->conn_len) k_node_count<<<grid_for(g->conn_len, BS), BS, 0, s>>>(g->conn_len, conn, (int32_t *)cnt32.p);
    if ((rc = scan_to_ptr_i32((int32_t *)cnt32.p, N, g->n2e_ptr, (int64_t *)tmp.p, s))) return rc;
    FEA_HIP(hipMemsetAsync(cnt32.p, 0, sizeof(int32_t) * (N + 1), s));
    if (E) k_node_fill<<<grid_for(E, BS), BS, 0, s>>>(E, conn_ptr, conn, g->n2e_ptr, (int32_t *)cnt32.p, g->n2e, g->n2a);
    if (N) k_node_sort<<<grid_for(N, BS), BS, 0, s>>>(N, g->n2e_ptr, g->n2e, g->n2a);
    FEA_HIP(hipGetLastError());

    // row pattern: degrees, prefix sum, columns
    if ((rc = dalloc((void **)&g->row_ptr, sizeof(int64_t) * (N + 1)))) return rc;
    if (N) k_row_pattern<<<grid_for(N, 4), 256, 0, s>>>(N, g->n2e_ptr, g->n2e, conn_ptr, conn, nullptr, nullptr, (int32_t *)cnt32.p);
    if ((rc = scan_to_ptr_i32((int32_t *)cnt32.p, N, g->row_ptr, (int64_t *)tmp.p, s))) return rc;
    FEA_HIP(hipMemcpyAsync(&g->nnz, g->row_ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEA_HIP(hipStreamSynchronize(s));
    if (g->nnz > INT32_MAX)
        return set_error(FEA_ERANGE, "%lld nonzero blocks exceed int32 block indices", (long long)g->nnz);
    if ((rc = dalloc((void **)&g->col, sizeof(int32_t) * std::max<int64_t>(g->nnz, 1)))) return rc;
    if (N) k_row_pattern<<<grid_for(N, 4), 256, 0, s>>>(N, g->n2e_ptr, g->n2e, conn_ptr, conn, g->row_ptr, g->col, nullptr);
    FEA_HIP(hipGetLastError());

    // element -> nonzero map
    if ((rc = dalloc((void **)&g->e2nnz, sizeof(int32_t) * std::max<int64_t>(g->map_len, 1)))) return rc;
    if (E) k_e2nnz<<<grid_for(E, BS), BS, 0, s>>>(E, conn_ptr, conn, g->row_ptr, g->col, g->map_ptr, g->e2nnz);

    // inverse map
    if ((rc = dalloc(&fillb.p, sizeof(int32_t) * (g->nnz + 1)))) return rc;
    if ((rc = dalloc((void **)&g->inv_ptr, sizeof(int64_t) * (g->nnz + 1)))) return rc;
    if ((rc = dalloc((void **)&g->inv, sizeof(int32_t) * std::max<int64_t>(g->map_len, 1)))) return rc;
    FEA_HIP(hipMemsetAsync(fillb.p, 0, sizeof(int32_t) * (g->nnz + 1), s));
    if (g->nnz > scan_n) {  // the block-count scan runs over nnz entries
        FEA_HIP(hipStreamSynchronize(s));
        dfree(tmp.p);
        tmp.p = nullptr;
        if ((rc = dalloc(&tmp.p, sizeof(int64_t) * (scan_tmp_elems(g->nnz) + 64)))) return rc;
    }
    if (g->map_len) k_inv_count<<<grid_for(g->map_len, BS), BS, 0, s>>>(g->map_len, g->e2nnz, (int32_t *)fillb.p);
    if ((rc = scan_to_ptr_i32((int32_t *)fillb.p, g->nnz, g->inv_ptr, (int64_t *)tmp.p, s))) return rc;
    FEA_HIP(hipMemsetAsync(fillb.p, 0, sizeof(int32_t) * (g->nnz + 1), s));
    if (N) k_inv_fill<<<grid_for(N, BS), BS, 0, s>>>(N, g->n2e_ptr, g->n2e, g->n2a, conn_ptr, g->map_ptr, g->e2nnz, g->inv_ptr, (int32_t *)fillb.p, g->inv);
    FEA_HIP(hipGetLastError());

    // destination positions for the row-owner workspace, laid out in
    // type-sorted order
    {
        TmpBuf e2pos, rpos;
        if ((rc = dalloc(&e2pos.p, sizeof(int32_t) * std::max<int64_t>(g->map_len, 1)))) return rc;
        if ((rc = dalloc(&rpos.p, sizeof(int32_t) * std::max<int64_t>(g->conn_len, 1)))) return rc;
        if (g->map_len) k_e2pos<<<grid_for(g->map_len, BS), BS, 0, s>>>(g->map_len, g->inv, (int32_t *)e2pos.p);
        if (N) k_rpos<<<grid_for(N, BS), BS, 0, s>>>(N, g->n2e_ptr, g->n2e, g->n2a, conn_ptr, (int32_t *)rpos.p);
        Bases bs;
        for (int t = 0; t <= 4; ++t) bs.seg[t] = g->seg[t];
        bs.node[0] = bs.slot[0] = 0;
        for (int t = 0; t < 4; ++t) {
            const int64_t cnt = g->seg[t + 1] - g->seg[t], n = nodes_of(t);
            bs.node[t + 1] = bs.node[t] + cnt * n;
            bs.slot[t + 1] = bs.slot[t] + cnt * n * n;
        }
        memcpy(g->node_base, bs.node, sizeof(bs.node));
        memcpy(g->slot_base, bs.slot, sizeof(bs.slot));
        if ((rc = dalloc((void **)&g->pnodes, sizeof(int32_t) * std::max<int64_t>(g->conn_len, 1)))) return rc;
        if ((rc = dalloc((void **)&g->prdest, sizeof(int32_t) * std::max<int64_t>(g->conn_len, 1)))) return rc;
        if ((rc = dalloc((void **)&g->pdest, sizeof(int32_t) * std::max<int64_t>(g->map_len, 1)))) return rc;
        if (E) k_position_maps<<<grid_for(E, BS), BS, 0, s>>>(E, bs, g->perm, conn_ptr, conn, g->map_ptr, (int32_t *)e2pos.p, (int32_t *)rpos.p, g->pnodes, g->pdest, g->prdest);
        FEA_HIP(hipGetLastError());
        FEA_HIP(hipStreamSynchronize(s));
    }

    if ((rc = colour_finish(g, hc, s))) return rc;
    return FEA_OK;
}

}  // namespace fea

using namespace fea;

extern "C" int fea_graph_build(int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                               const int64_t *conn_ptr, const int32_t *conn, hipStream_t stream,
                               fea_graph **out)
{
    clear_error();
    if (!out) return set_error(FEA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_nodes < 0 || n_elems < 0) return set_error(FEA_EINVAL, "negative size");
    if (n_elems > 0 && (!types || !conn_ptr || !conn))
        return set_error(FEA_EINVAL, "types, conn_ptr and conn are required");
    if (n_nodes > INT32_MAX || n_elems > INT32_MAX)
        return set_error(FEA_ERANGE, "more than 2^31-1 nodes or elements");
    fea_graph *g = new (std::nothrow) fea_graph();
    if (!g) return set_error(FEA_ENOMEM, "host allocation failed");
    int rc = build(n_nodes, n_elems, types, conn_ptr, conn, stream, g);
    if (rc == FEA_OK) rc = noalloc_setup();
    if (rc != FEA_OK) {
        (void)hipStreamSynchronize(stream);
        destroy(g);
        return rc;
    }
    *out = g;
    return FEA_OK;
}

namespace {

// Graph cache file: header (magic, version, GPU architecture name, sizes,
// mesh fingerprint, family and colour offsets), then the graph's device
// arrays in a fixed order, each preceded by its byte count.
constexpr char kGraphMagic[8] = {'F', 'E', 'A', 'G', 'R', 'A', 'P', 'H'};
constexpr uint32_t kGraphVersion = 1;
constexpr size_t kStage = size_t(64) << 20;  // host staging buffer (bytes)

struct GraphHeader {
    char magic[8];
    uint32_t version;
    int32_t n_colours;
    char arch[64];
    int64_t n_nodes, n_elems, nnz, map_len, conn_len;
    uint64_t mesh_fp;
    int64_t seg[5], node_base[5], slot_base[5];
    int64_t cseg_len;
};

struct HostFile {
    FILE *f = nullptr;
    ~HostFile()
    {
        if (f) fclose(f);
    }
};

struct PinnedBuf {
    void *p = nullptr;
    ~PinnedBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

int device_arch(int dev, char *arch)
{
    hipDeviceProp_t prop;
    FEA_HIP(hipGetDeviceProperties(&prop, dev));
    memset(arch, 0, 64);
    strncpy(arch, prop.gcnArchName, 63);
    return FEA_OK;
}

// The graph's arrays that the cache holds, with their lengths in bytes.
struct GraphArray {
    void **p;
    size_t bytes;
};

std::vector<GraphArray> graph_arrays(fea_graph *g)
{
    const size_t N = (size_t)g->n_nodes, E = (size_t)g->n_elems, nnz = (size_t)g->nnz,
                 ml = (size_t)g->map_len, cl = (size_t)g->conn_len;
    auto one = [](size_t n) { return n ? n : 1; };
    return {{(void **)&g->row_ptr, 8 * (N + 1)},   {(void **)&g->col, 4 * one(nnz)},
            {(void **)&g->map_ptr, 8 * (E + 1)},   {(void **)&g->e2nnz, 4 * one(ml)},
            {(void **)&g->inv_ptr, 8 * (nnz + 1)}, {(void **)&g->inv, 4 * one(ml)},
            {(void **)&g->pnodes, 4 * one(cl)},    {(void **)&g->pdest, 4 * one(ml)},
            {(void **)&g->prdest, 4 * one(cl)},    {(void **)&g->n2e_ptr, 8 * (N + 1)},
            {(void **)&g->n2e, 4 * one(cl)},       {(void **)&g->n2a, one(cl)},
            {(void **)&g->perm, 4 * one(E)},       {(void **)&g->colour, 2 * one(E)},
            {(void **)&g->cperm, 4 * one(E)}};
}

}  // namespace

extern "C" int fea_graph_save(const fea_graph *gc, const char *path)
{
    clear_error();
    if (!gc || !path) return set_error(FEA_EINVAL, "graph and path are required");
    fea_graph *g = const_cast<fea_graph *>(gc);
    GraphHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kGraphMagic, 8);
    h.version = kGraphVersion;
    h.n_colours = g->n_colours;
    int rc = device_arch(g->device, h.arch);
    if (rc) return rc;
    h.n_nodes = g->n_nodes;
    h.n_elems = g->n_elems;
    h.nnz = g->nnz;
    h.map_len = g->map_len;
    h.conn_len = g->conn_len;
    h.mesh_fp = g->mesh_fp;
    memcpy(h.seg, g->seg, sizeof(h.seg));
    memcpy(h.node_base, g->node_base, sizeof(h.node_base));
    memcpy(h.slot_base, g->slot_base, sizeof(h.slot_base));
    h.cseg_len = (int64_t)g->cseg.size();
    HostFile f;
    f.f = fopen(path, "wb");
    if (!f.f) return set_error(FEA_EINVAL, "cannot write %s", path);
    bool ok = fwrite(&h, sizeof(h), 1, f.f) == 1 &&
              (h.cseg_len == 0 || fwrite(g->cseg.data(), 8, (size_t)h.cseg_len, f.f) == (size_t)h.cseg_len);
    PinnedBuf stage;
    FEA_HIP(hipHostMalloc(&stage.p, kStage, hipHostMallocDefault));
    FEA_HIP(hipDeviceSynchronize());
    for (const GraphArray &a : graph_arrays(g)) {
        const uint64_t nb = a.bytes;
        ok = ok && fwrite(&nb, 8, 1, f.f) == 1;
        for (size_t off = 0; ok && off < a.bytes; off += kStage) {
            const size_t n = std::min(kStage, a.bytes - off);
            FEA_HIP(hipMemcpy(stage.p, (char *)*a.p + off, n, hipMemcpyDeviceToHost));
            ok = fwrite(stage.p, 1, n, f.f) == n;
        }
    }
    if (!ok) return set_error(FEA_EINVAL, "short write to %s", path);
    return FEA_OK;
}

extern "C" int fea_graph_load(const char *path, int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                              const int64_t *conn_ptr, const int32_t *conn, hipStream_t stream, fea_graph **out)
{
    clear_error();
    if (!out || !path) return set_error(FEA_EINVAL, "path and out are required");
    *out = nullptr;
    if (n_nodes < 0 || n_elems < 0) return set_error(FEA_EINVAL, "negative size");
    if (n_elems > 0 && (!types || !conn_ptr || !conn))
        return set_error(FEA_EINVAL, "types, conn_ptr and conn are required");
    HostFile f;
    f.f = fopen(path, "rb");
    if (!f.f) return set_error(FEA_EINVAL, "cannot read %s", path);
    GraphHeader h;
    if (fread(&h, sizeof(h), 1, f.f) != 1 || memcmp(h.magic, kGraphMagic, 8) != 0)
        return set_error(FEA_EINVAL, "%s is not a graph cache", path);
    if (h.version != kGraphVersion)
        return set_error(FEA_EINVAL, "%s: graph cache version %u, this library reads %u", path, h.version,
                         kGraphVersion);
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    char arch[64];
    int rc = device_arch(dev, arch);
    if (rc) return rc;
    h.arch[63] = 0;
    if (strcmp(arch, h.arch) != 0)
        return set_error(FEA_EINVAL, "%s was written on %s, this device is %s", path, h.arch, arch);
    if (h.n_nodes != n_nodes || h.n_elems != n_elems)
        return set_error(FEA_EINVAL, "%s holds the graph of a mesh of %lld nodes and %lld elements, not %lld and %lld",
                         path, (long long)h.n_nodes, (long long)h.n_elems, (long long)n_nodes, (long long)n_elems);
    if (h.cseg_len < 0 || h.n_colours < 0 || h.nnz < 0 || h.map_len < 0 || h.conn_len < 0 ||
        h.cseg_len != 4 * ((int64_t)h.n_colours + 1))
        return set_error(FEA_EINVAL, "%s: inconsistent header", path);
    // the mesh must be the one the graph was built for
    if ((rc = validate(n_nodes, n_elems, types, conn_ptr, conn, stream))) return rc;
    uint64_t fp = 0;
    if ((rc = mesh_fingerprint(n_elems, types, conn_ptr, conn, stream, &fp))) return rc;
    if (fp != h.mesh_fp) return set_error(FEA_EINVAL, "%s was built for another mesh (connectivity differs)", path);
    fea_graph *g = new (std::nothrow) fea_graph();
    if (!g) return set_error(FEA_ENOMEM, "host allocation failed");
    FEA_HIP(hipGetDevice(&g->device));
    g->n_nodes = h.n_nodes;
    g->n_elems = h.n_elems;
    g->nnz = h.nnz;
    g->map_len = h.map_len;
    g->conn_len = h.conn_len;
    g->n_colours = h.n_colours;
    g->mesh_fp = h.mesh_fp;
    memcpy(g->seg, h.seg, sizeof(h.seg));
    memcpy(g->node_base, h.node_base, sizeof(h.node_base));
    memcpy(g->slot_base, h.slot_base, sizeof(h.slot_base));
    g->cseg.resize((size_t)h.cseg_len);
    bool ok = h.cseg_len == 0 || fread(g->cseg.data(), 8, (size_t)h.cseg_len, f.f) == (size_t)h.cseg_len;
    PinnedBuf stage;
    if (ok) {
        hipError_t e = hipHostMalloc(&stage.p, kStage, hipHostMallocDefault);
        if (e != hipSuccess) {
            destroy(g);
            return set_error(FEA_ENOMEM, "pinned staging buffer: %s", hipGetErrorString(e));
        }
    }
    for (const GraphArray &a : graph_arrays(g)) {
        if (!ok) break;
        uint64_t nb = 0;
        ok = fread(&nb, 8, 1, f.f) == 1 && nb == a.bytes;
        if (!ok) break;
        if ((rc = dalloc(a.p, a.bytes))) {
            destroy(g);
            return rc;
        }
        for (size_t off = 0; ok && off < a.bytes; off += kStage) {
            const size_t n = std::min(kStage, a.bytes - off);
            ok = fread(stage.p, 1, n, f.f) == n;
            if (ok && hipMemcpy((char *)*a.p + off, stage.p, n, hipMemcpyHostToDevice) != hipSuccess) {
                destroy(g);
                return set_error(FEA_EHIP, "copy of %s to the device failed", path);
            }
        }
    }
    if (!ok) {
        destroy(g);
        return set_error(FEA_EINVAL, "%s is truncated or does not match its header", path);
    }
    if ((rc = noalloc_setup())) {
        destroy(g);
        return rc;
    }
    *out = g;
    return FEA_OK;
}

extern "C" int fea_graph_tile_colouring(const fea_graph *g, int *n_colours, int64_t *bucket_ptr, int32_t *tiles,
                                        int32_t *nneig, hipStream_t stream)
{
    clear_error();
    if (!g) return set_error(FEA_EINVAL, "graph is NULL");
    if (!g->tcready) return set_error(FEA_EINVAL, "the tile colouring has not been built (no FEA_TILECOLOUR call yet)");
    if (n_colours) *n_colours = g->tc_colours;
    if (bucket_ptr) std::copy(g->tcseg.begin(), g->tcseg.end(), bucket_ptr);
    const int64_t nt = g->tile_base[4];
    if (nneig && nt) std::copy(g->tc_nneig.begin(), g->tc_nneig.begin() + nt, nneig);
    if (tiles && nt)
        FEA_HIP(hipMemcpyAsync(tiles, g->ctile, sizeof(int32_t) * nt, hipMemcpyDeviceToDevice, stream));
    return FEA_OK;
}

extern "C" int fea_graph_sizes(const fea_graph *g, int64_t *n_nodes, int64_t *n_elems,
                               int64_t *nnz_blocks, int64_t *map_len, int *n_colours)
{
    clear_error();
    if (!g) return set_error(FEA_EINVAL, "graph is NULL");
    if (n_nodes) *n_nodes = g->n_nodes;
    if (n_elems) *n_elems = g->n_elems;
    if (nnz_blocks) *nnz_blocks = g->nnz;
    if (map_len) *map_len = g->map_len;
    if (n_colours) *n_colours = g->n_colours;
    return FEA_OK;
}

extern "C" int fea_graph_sym_sizes(const fea_graph *g, int64_t *tiles, int64_t *entries, int64_t *tile_blocks,
                                   int64_t *upper_blocks)
{
    clear_error();
    if (!g) return set_error(FEA_EINVAL, "graph is NULL");
    if (!g->sready)
        return set_error(FEA_EINVAL, "the upper-triangle layout is built by the first FEA_ROWSYM assembly");
    if (tiles) *tiles = g->tile_base[4];
    if (entries) *entries = g->nent;
    if (tile_blocks) *tile_blocks = g->ulen;
    if (upper_blocks) *upper_blocks = g->nup;
    return FEA_OK;
}

extern "C" int fea_graph_export(const fea_graph *g, int64_t *row_ptr, int32_t *col,
                                int64_t *map_ptr, int32_t *e2nnz, int64_t *inv_ptr, int32_t *inv,
                                int16_t *colour, int32_t *type_perm, int64_t *type_seg,
                                hipStream_t s)
{
    clear_error();
    if (!g) return set_error(FEA_EINVAL, "graph is NULL");
    const hipMemcpyKind D2D = hipMemcpyDeviceToDevice;
    if (row_ptr) FEA_HIP(hipMemcpyAsync(row_ptr, g->row_ptr, sizeof(int64_t) * (g->n_nodes + 1), D2D, s));
    if (col && g->nnz) FEA_HIP(hipMemcpyAsync(col, g->col, sizeof(int32_t) * g->nnz, D2D, s));
    if (map_ptr) FEA_HIP(hipMemcpyAsync(map_ptr, g->map_ptr, sizeof(int64_t) * (g->n_elems + 1), D2D, s));
    if (e2nnz && g->map_len) FEA_HIP(hipMemcpyAsync(e2nnz, g->e2nnz, sizeof(int32_t) * g->map_len, D2D, s));
    if (inv_ptr) FEA_HIP(hipMemcpyAsync(inv_ptr, g->inv_ptr, sizeof(int64_t) * (g->nnz + 1), D2D, s));
    if (inv && g->map_len) FEA_HIP(hipMemcpyAsync(inv, g->inv, sizeof(int32_t) * g->map_len, D2D, s));
    if (colour && g->n_elems) FEA_HIP(hipMemcpyAsync(colour, g->colour, sizeof(int16_t) * g->n_elems, D2D, s));
    if (type_perm && g->n_elems) FEA_HIP(hipMemcpyAsync(type_perm, g->perm, sizeof(int32_t) * g->n_elems, D2D, s));
    if (type_seg) memcpy(type_seg, g->seg, sizeof(g->seg));
    return FEA_OK;
}

extern "C" void fea_graph_destroy(fea_graph *g)
{
    if (g) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(g->device);
        (void)hipDeviceSynchronize();
        destroy(g);
        (void)hipSetDevice(cur);
    }
}
