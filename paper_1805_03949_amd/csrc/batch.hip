// Batched assembly of many independent meshes in one persistent launch.
//
// The paper distributes the element loop over threads with a dynamic
// schedule and a chunk size (Section 3.2, Algorithms 4 and 5; chunk study
// in Section 5.2) and over ranks with weighted partitions (Section 4.1).
// Here the chunks are work items -- `count` consecutive elements of one
// family of one mesh -- handed out by a device queue (an atomic head over an
// order array) to persistent workgroups. Each workgroup records the shader
// clock around every item it runs; those cycle counts are the measured
// per-item cost (Section 4.1, measured load balance) that the cost model
// learns from. Results are deterministic: each block is summed by the
// row-owner reduction in ascending element order, whatever the queue order.
// The upper-triangle form (FEA_ROWSYM) runs the same items as element
// tiles with their LDS tile sums; item starts are multiples of the family's
// tile size, so its tiles, and its results, are those of the one-mesh
// assembly.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "elem.h"
#include "segsum.h"

namespace fea {

// Per-mesh view used by the persistent kernel.
struct BatchMesh {
    ElemArgs a;      // pointers of the mesh and its graph (elems = perm)
    int64_t seg[5];  // family segments in perm
    int64_t node_base[5], slot_base[5];  // family starts in pnodes/prdest and pdest
    int64_t coff;    // first slot of this mesh in the slot workspace
    int64_t roff;    // first incidence of this mesh in the rhs workspace
    int64_t tile_base[5];  // upper-triangle form: family starts in the tile ranges
    int64_t scoff;         // first tile-block of this mesh in its workspace
};

template <int T, int MODEL, typename CT, int VAR>
__device__ inline void run_item(const ElemArgs &A, int32_t count, ElemSmem<T, MODEL, VAR, CT> &S)
{
    constexpr int EPB = ElemSmem<T, MODEL, VAR, CT>::EPB;
#pragma nounroll
    for (int32_t sub = 0; sub < count; sub += EPB) elem_tile<T, MODEL, VAR, CT>(A, sub, S, opaque_tid());
}

// Persistent kernel of one element family: every workgroup dequeues items
// of family T until that family's queue is empty (each workgroup reaches
// the exit test after every item). One launch per family keeps each
// family's registers and LDS as small as its own element code needs, and
// every item's element arguments are read in place from a prepared
// read-only table (itemargs) as a one-tile kernel reads its kernel
// arguments: arguments assembled in the loop stayed live across the
// element code (98-134 VGPRs instead of 64-82, 4 waves per SIMD).
// The register budget of the linear-elastic upper-triangle instances is
// bounded by the occupancy their LDS allows: inside the item loop the
// scheduler otherwise keeps several Gauss points' gradient products of the
// block contraction live at once (pyr5 and hex8: 131-133 VGPRs and 3 waves
// per SIMD, against 74-90 for the same code in the one-tile kernel).
template <int T, int MODEL, typename CT, int VAR>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, 256),
                               amdgpu_waves_per_eu(persistent_min_waves<T, MODEL, VAR, CT>())))
k_batch(const ElemArgs *__restrict__ itemargs, const int4 *items,
                                               const int32_t *order, int32_t n_items,
                                               int32_t *head, const int32_t *part, uint64_t *cycles,
                                               int32_t *worker, int32_t *cu)
{
    constexpr int B = MODEL == FEA_POISSON ? 1 : 3;
    __shared__ ElemSmem<T, MODEL, VAR, CT> S;
    __shared__ int32_t s_item;
    // static partition: this workgroup runs order[part[w] .. part[w+1])
    int32_t next = part ? part[blockIdx.x] : 0;
    const int32_t last = part ? part[blockIdx.x + 1] : 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t q = part ? next : atomicAdd(head, 1);
            s_item = q < (part ? last : n_items) ? order[q] : -1;
        }
        ++next;
        __syncthreads();
        // the item is the same for the whole workgroup: keep it (and the
        // mesh view it selects) in scalar registers
        const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
        if (it < 0) break;
        const uint64_t t0 = clock64();
        const int32_t count = __builtin_amdgcn_readfirstlane(items[it].w);
        const ElemArgs A = from_global(reinterpret_cast<const ElemArgsGlobal *>(itemargs)[it]);
        run_item<T, MODEL, CT, VAR>(A, count, S);
        __syncthreads();
        if (threadIdx.x == 0) {
            cycles[it] = clock64() - t0;
            worker[it] = blockIdx.x;
            cu[it] = (int32_t)__smid();
        }
    }
}

// Concatenated segment bounds: out[i] = in[i] + off for i in [0, n].
__global__ void k_offset_ptr(const int64_t *in, int64_t n, int64_t off, int64_t *out)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i <= n) out[i] = in[i] + off;
}

// Concatenated block indices: out[i] = in[i] + off for i in [0, n), -1 kept.
__global__ void k_offset_idx(const int32_t *in, int64_t n, int64_t off, int32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = in[i] < 0 ? -1 : (int32_t)(in[i] + off);
}

// Lower partners (>= 0) offset by the mesh's first block, diagonal rows
// (-(v + 1)) by its first node.
__global__ void k_offset_lp(const int32_t *in, int64_t n, int64_t off, int64_t node_off, int32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = in[i] < 0 ? (int32_t)(in[i] - node_off) : (int32_t)(in[i] + off);
}

__global__ void k_batch_begin(int32_t *head, int32_t *status, int n_meshes)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < 4) head[i] = 0;  // one queue head per family
    if (i < n_meshes) status[i] = INT_MAX;
}

__global__ void k_batch_end(int32_t *status, int n_meshes, int32_t *out)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n_meshes) {
        int32_t v = status[i] == INT_MAX ? -1 : status[i];
        if (out) out[i] = v;
    }
}


// Work-item features for the cost model: one workgroup per item.
__device__ inline void block_reduce3(float &a, float &b, float &c, int op_max_b, float *sh)
{
    // sums a and c, and b by max (op_max_b) or sum; fixed tree order
    const int t = threadIdx.x;
    sh[t] = a;
    sh[256 + t] = b;
    sh[512 + t] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            sh[t] += sh[t + off];
            sh[256 + t] = op_max_b ? fmaxf(sh[256 + t], sh[256 + t + off]) : sh[256 + t] + sh[256 + t + off];
            sh[512 + t] += sh[512 + t + off];
        }
        __syncthreads();
    }
    a = sh[0];
    b = sh[256];
    c = sh[512];
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_features(const BatchMesh *meshes, const int4 *items,
                                                  int fp64, float *feats)
{
    __shared__ float sh[768];
    const int4 w = items[blockIdx.x];
    const BatchMesh &M = meshes[w.x];
    const int t = w.y, nn = nodes_of(t);
    const int nq = t == 0 ? 1 : (t == 2 ? 6 : 8);
    float nh = 0.f, nu = 0.f, dsum = 0.f, dmax = 0.f, vol = 0.f;
    float nmin = 3.0e38f, nmax = -1.f;
    for (int j = threadIdx.x; j < w.w; j += 256) {
        const int32_t e = M.a.elems[M.seg[t] + w.z + j];
        if (M.a.nh_flag) nh += M.a.nh_flag[e] ? 1.f : 0.f;
        if (M.a.nu) nu += (float)M.a.nu[e];
        double X[8][3];
        const int64_t c0 = M.a.conn_ptr[e];
        for (int a = 0; a < nn; ++a) {
            const int32_t v = M.a.conn[c0 + a];
            X[a][0] = M.a.x[v];
            X[a][1] = M.a.y[v];
            X[a][2] = M.a.z[v];
            nmin = fminf(nmin, (float)v);
            nmax = fmaxf(nmax, (float)v);
        }
        double dlo = 1e300, dhi = 0.0, ve = 0.0;
        for (int q = 0; q < nq; ++q) {
            double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int a = 0; a < nn; ++a)
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) J[i][k] += X[a][i] * c_ref.dN[t][q][a][k];
            const double d = det3(J);
            dlo = fmin(dlo, d);
            dhi = fmax(dhi, d);
            ve += c_ref.w[t][q] * d;
        }
        const float de = dlo > 0.0 ? (float)(dhi / dlo) : 1.0e6f;
        dsum += de;
        dmax = fmaxf(dmax, de);
        vol += (float)ve;
    }
    block_reduce3(nh, dmax, nu, 1, sh);
    block_reduce3(dsum, nmax, vol, 1, sh);
    // min of node ids through the max of their negation
    float neg = -nmin, zero0 = 0.f, zero1 = 0.f;
    block_reduce3(zero0, neg, zero1, 1, sh);
    nmin = -neg;
    if (threadIdx.x == 0) {
        const float cnt = (float)w.w;
        float *f = feats + (int64_t)blockIdx.x * 12;
        for (int k = 0; k < 4; ++k) f[k] = (k == t) ? 1.f : 0.f;
        f[4] = nh / cnt;
        f[5] = log2f(cnt);
        f[6] = log2f((nmax - nmin + 1.f) / (cnt * nn));
        f[7] = nu / cnt;
        f[8] = logf(dsum / cnt);
        f[9] = logf(dmax);
        f[10] = log10f(fmaxf(vol / cnt, 1e-30f));
        f[11] = fp64 ? 1.f : 0.f;
    }
}

}  // namespace fea

using namespace fea;

struct fea_batch {
    int device = 0;
    int model = FEA_ELASTIC;
    bool has_nh = false;  // some mesh gives neo-Hookean flags
    int n_meshes = 0;
    std::vector<fea_mesh_desc> desc;
    std::vector<fea_graph *> graphs;
    std::vector<int64_t> vals_off, rhs_off, slot_off, inc_off;  // scalars / slots / incidences
    int64_t n_elems = 0, total_blocks = 0, total_slots = 0, total_inc = 0;
    int32_t tile[4] = {75, 34, 24, 14};  // multiples of the upper-triangle tile
    std::vector<int32_t> items;  // 4 per item
    std::vector<int32_t> order;
    // device
    BatchMesh *d_meshes = nullptr;
    int4 *d_items = nullptr;
    int32_t *d_order = nullptr;
    int32_t *d_head = nullptr;
    int32_t *d_status = nullptr;
    int64_t *d_vseg = nullptr, *d_rseg = nullptr;
    uint64_t *d_cycles = nullptr;
    int32_t *d_worker = nullptr, *d_cu = nullptr;
    size_t items_cap = 0;
    void *contrib = nullptr;
    size_t contrib_bytes = 0;
    void *rcontrib = nullptr;
    size_t rcontrib_bytes = 0;
    int workers = 0;       // the largest of the per-family worker counts
    int fworkers[4] = {0, 0, 0, 0};
    int workers_for = -1;  // (model, precision, form) the worker counts were computed for
    // the device queue holds the order grouped by family (stable): family
    // t's items are d_order[foff[t] .. foff[t+1]); its static partition
    // (fworkers[t] + 1 bounds) starts at d_part[poff[t]]
    int64_t foff[5] = {0, 0, 0, 0, 0};
    int64_t poff[5] = {0, 0, 0, 0, 0};
    // static partition of the order over the workers (used when part_for
    // equals the current worker count; -1 = dynamic queue)
    std::vector<double> part_w;  // item weights of the requested partition
    int32_t *d_part = nullptr;
    int part_for = -1;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool timed = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GatherBatch *gbatch = nullptr;  // row-gather form, built on first use
    // upper-triangle form, built on first use: per-mesh views (host copy),
    // the concatenated upper-block list, lower partners and tile-block
    // segment bounds (global block indices and slots)
    std::vector<BatchMesh> hmeshes;
    // per-item element arguments of the persistent kernels, for the form,
    // workspaces and item list they were built for
    ElemArgs *d_itemargs = nullptr;
    size_t itemargs_cap = 0;
    int itemargs_var = -1;
    const void *itemargs_ws[2] = {nullptr, nullptr};
    int64_t items_version = 0, itemargs_version = -1;
    bool sym_ready = false;
    int64_t total_sym_slots = 0, total_nup = 0;
    int32_t *d_sym_ublk = nullptr, *d_sym_lp = nullptr;
    int64_t sym_empty_rows = 0;  // rows of all meshes that no element touches
    int64_t *d_sym_ptr = nullptr;
    // subgrid scale: its own queue heads (one per family) and per-mesh
    // arguments, kept for the outputs and item list they were built for
    int32_t *d_sub_head = nullptr;
    int4 *d_sub_items = nullptr;   // its own work items and family-grouped
    int32_t *d_sub_order = nullptr;  // order (built once: the meshes are fixed)
    int64_t sub_foff[5] = {0, 0, 0, 0, 0};
    void *d_subargs = nullptr;
    size_t subargs_cap = 0;
    const void *subargs_key[2] = {nullptr, nullptr};
};

namespace {

void drop_graph(fea_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void destroy_batch(fea_batch *b)
{
    if (!b) return;
    drop_graph(b);
    gather_batch_destroy(b->gbatch);
    for (fea_graph *g : b->graphs)
        if (g) fea_graph_destroy(g);
    void *bufs[] = {b->d_meshes, b->d_items, b->d_order, b->d_head, b->d_status, b->d_vseg,
                    b->d_rseg, b->d_cycles, b->d_worker, b->d_cu, b->contrib, b->rcontrib,
                    b->d_part, b->d_sym_ublk, b->d_sym_lp, b->d_sym_ptr, b->d_itemargs,
                    b->d_sub_head, b->d_subargs, b->d_sub_items, b->d_sub_order};
    for (void *p : bufs) dfree(p);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

// Uploads the queue order grouped by family (stable: within a family the
// order is kept) and records the family offsets.
int upload_grouped_order(fea_batch *b)
{
    const size_t ni = b->items.size() / 4;
    std::vector<int32_t> g;
    g.reserve(ni);
    b->foff[0] = 0;
    for (int t = 0; t < 4; ++t) {
        for (size_t j = 0; j < ni; ++j)
            if (b->items[4 * (size_t)b->order[j] + 1] == t) g.push_back(b->order[j]);
        b->foff[t + 1] = (int64_t)g.size();
    }
    if (ni) FEA_HIP(hipMemcpy(b->d_order, g.data(), sizeof(int32_t) * ni, hipMemcpyHostToDevice));
    drop_graph(b);
    return FEA_OK;
}

// Elements per item of family t: the requested count rounded up to a
// multiple of the upper-triangle tile, so that items start on tile
// boundaries in both forms.
int64_t item_size(int32_t tile, int t)
{
    const int64_t e = sym_epb(t);
    return (tile + e - 1) / e * e;
}

int build_items(fea_batch *b)
{
    ++b->items_version;
    b->items.clear();
    for (int t = 0; t < 4; ++t)
        for (int m = 0; m < b->n_meshes; ++m) {
            const fea_graph *g = b->graphs[m];
            const int64_t n = g->seg[t + 1] - g->seg[t];
            const int64_t tile = item_size(b->tile[t], t);
            for (int64_t s = 0; s < n; s += tile) {
                b->items.push_back(m);
                b->items.push_back(t);
                b->items.push_back((int32_t)s);
                b->items.push_back((int32_t)std::min<int64_t>(tile, n - s));
            }
        }
    const size_t ni = b->items.size() / 4;
    b->order.resize(ni);
    for (size_t i = 0; i < ni; ++i) b->order[i] = (int32_t)i;
    b->part_for = -1;
    b->part_w.clear();
    if (ni > b->items_cap) {
        void *bufs[] = {b->d_items, b->d_order, b->d_cycles, b->d_worker, b->d_cu};
        for (void *p : bufs) dfree(p);
        b->d_items = nullptr;
        b->d_order = nullptr;
        b->d_cycles = nullptr;
        b->d_worker = b->d_cu = nullptr;
        int rc;
        if ((rc = dalloc((void **)&b->d_items, sizeof(int4) * ni))) return rc;
        if ((rc = dalloc((void **)&b->d_order, sizeof(int32_t) * ni))) return rc;
        if ((rc = dalloc((void **)&b->d_cycles, sizeof(uint64_t) * ni))) return rc;
        if ((rc = dalloc((void **)&b->d_worker, sizeof(int32_t) * ni))) return rc;
        if ((rc = dalloc((void **)&b->d_cu, sizeof(int32_t) * ni))) return rc;
        b->items_cap = ni;
    }
    if (ni) FEA_HIP(hipMemcpy(b->d_items, b->items.data(), sizeof(int4) * ni, hipMemcpyHostToDevice));
    return upload_grouped_order(b);
}

// Splits each family's part of the queue order into that family's worker
// count of contiguous ranges of nearly equal total weight (cut where the
// running sum crosses k * total / workers).
int make_partition(fea_batch *b)
{
    const size_t ni = b->order.size();
    std::vector<int32_t> g;
    g.reserve(ni);
    for (int t = 0; t < 4; ++t)
        for (size_t j = 0; j < ni; ++j)
            if (b->items[4 * (size_t)b->order[j] + 1] == t) g.push_back(b->order[j]);
    std::vector<int32_t> part;
    for (int t = 0; t < 4; ++t) {
        const int W = std::max(1, b->fworkers[t]);
        const int64_t j0 = b->foff[t], n = b->foff[t + 1] - j0;
        b->poff[t] = (int64_t)part.size();
        std::vector<int32_t> pt(W + 1, 0);
        double total = 0.0;
        for (int64_t j = 0; j < n; ++j) total += b->part_w[g[j0 + j]];
        double run = 0.0;
        int k = 1;
        for (int64_t j = 0; j < n && k < W; ++j) {
            const double wj = b->part_w[g[j0 + j]];
            while (k < W && run + 0.5 * wj >= total * k / W) pt[k++] = (int32_t)j;
            run += wj;
        }
        while (k <= W) pt[k++] = (int32_t)n;
        part.insert(part.end(), pt.begin(), pt.end());
    }
    b->poff[4] = (int64_t)part.size();
    dfree(b->d_part);
    b->d_part = nullptr;
    int rc = dalloc((void **)&b->d_part, sizeof(int32_t) * part.size());
    if (rc) return rc;
    FEA_HIP(hipMemcpy(b->d_part, part.data(), sizeof(int32_t) * part.size(), hipMemcpyHostToDevice));
    b->part_for = b->workers_for;
    drop_graph(b);
    return FEA_OK;
}

template <int T, int MODEL, typename CT, int VAR>
int family_workers(int cus, int *w)
{
    int per = 0;
    FEA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<T, MODEL, CT, VAR>, 256, 0));
    *w = std::max(1, cus * std::max(1, per));
    return FEA_OK;
}

template <int MODEL, typename CT, int VAR>
int worker_count(fea_batch *b)
{
    const int key = (MODEL * 2 + (sizeof(CT) == 4)) * 4 + VAR;  // MODEL 0..2
    if (b->workers_for == key) return FEA_OK;
    int cus = 0, rc;
    FEA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    if ((rc = family_workers<0, MODEL, CT, VAR>(cus, &b->fworkers[0]))) return rc;
    if ((rc = family_workers<1, MODEL, CT, VAR>(cus, &b->fworkers[1]))) return rc;
    if ((rc = family_workers<2, MODEL, CT, VAR>(cus, &b->fworkers[2]))) return rc;
    if ((rc = family_workers<3, MODEL, CT, VAR>(cus, &b->fworkers[3]))) return rc;
    b->workers = *std::max_element(b->fworkers, b->fworkers + 4);
    b->workers_for = key;
    if (!b->part_w.empty()) return make_partition(b);
    return FEA_OK;
}

// Upper-triangle layout of every mesh (built once; blocks on the stream),
// the mesh views' tile fields and the concatenated block lists.
int sym_prepare_batch(fea_batch *b, hipStream_t s)
{
    if (b->sym_ready) return FEA_OK;
    int rc;
    const int n = b->n_meshes;
    std::vector<int64_t> soff(n + 1, 0), uoff(n + 1, 0), koff(n + 1, 0), noff(n + 1, 0);
    b->sym_empty_rows = 0;
    for (int m = 0; m < n; ++m) {
        fea_graph *g = b->graphs[m];
        if (!g->sready && (rc = sym_prepare(g, s))) return rc;
        soff[m + 1] = soff[m] + g->ulen;
        uoff[m + 1] = uoff[m] + g->nup;
        koff[m + 1] = koff[m] + g->nnz;
        noff[m + 1] = noff[m] + g->n_nodes;
        b->sym_empty_rows += g->sym_empty_rows;
        BatchMesh &M = b->hmeshes[m];
        M.a.tent_ptr = g->tent_ptr;
        M.a.ttb_ptr = g->ttb_ptr;
        M.a.tent = g->tent;
        M.a.tb_eend = g->tb_eend;
        M.a.tb_slot = g->tb_slot;
        std::copy(g->tile_base, g->tile_base + 5, M.tile_base);
        M.scoff = soff[m];
    }
    dfree(b->d_sym_ublk);
    dfree(b->d_sym_lp);
    dfree(b->d_sym_ptr);
    b->d_sym_ublk = b->d_sym_lp = nullptr;
    b->d_sym_ptr = nullptr;
    if ((rc = dalloc((void **)&b->d_sym_ublk, sizeof(int32_t) * std::max<int64_t>(uoff[n], 1)))) return rc;
    if ((rc = dalloc((void **)&b->d_sym_lp, sizeof(int32_t) * std::max<int64_t>(uoff[n], 1)))) return rc;
    if ((rc = dalloc((void **)&b->d_sym_ptr, sizeof(int64_t) * (uoff[n] + 1)))) return rc;
    if (koff[n] > INT32_MAX || noff[n] > INT32_MAX) return set_error(FEA_ERANGE, "batch has more than 2^31 blocks or nodes");
    int64_t zero = 0;
    FEA_HIP(hipMemcpy(b->d_sym_ptr, &zero, sizeof(int64_t), hipMemcpyHostToDevice));
    // concatenated upper-block lists: block ids and lower partners offset by
    // the mesh's first block, segment bounds by its first workspace slot
    // (mesh m's last bound is mesh m+1's first, written twice with one value)
    for (int m = 0; m < n; ++m) {
        const fea_graph *g = b->graphs[m];
        if (g->nup) {
            k_offset_idx<<<grid_for(g->nup, 256), 256, 0, s>>>(g->ublk, g->nup, koff[m], b->d_sym_ublk + uoff[m]);
            k_offset_lp<<<grid_for(g->nup, 256), 256, 0, s>>>(g->ulp, g->nup, koff[m], noff[m], b->d_sym_lp + uoff[m]);
            k_offset_ptr<<<grid_for(g->nup + 1, 256), 256, 0, s>>>(g->uptr, g->nup, soff[m], b->d_sym_ptr + uoff[m]);
        }
    }
    FEA_HIP(hipGetLastError());
    if (n) FEA_HIP(hipMemcpy(b->d_meshes, b->hmeshes.data(), sizeof(BatchMesh) * n, hipMemcpyHostToDevice));
    FEA_HIP(hipStreamSynchronize(s));
    b->total_sym_slots = soff[n];
    b->total_nup = uoff[n];
    b->sym_ready = true;
    return FEA_OK;
}

// Element arguments of every item (its mesh's view, offset to the item's
// first element, its workspaces and status), rebuilt when the items, the
// form or the workspaces change; waits for the stream (earlier launches may
// still read the table) and blocks on the copy.
template <int MODEL, typename CT, int VAR>
int ensure_itemargs(fea_batch *b, hipStream_t s)
{
    constexpr int B = MODEL == FEA_POISSON ? 1 : 3;
    const int key = (VAR * 2 + (sizeof(CT) == 4)) * 4 + B;
    if (b->itemargs_version == b->items_version && b->itemargs_var == key && b->itemargs_ws[0] == b->contrib &&
        b->itemargs_ws[1] == b->rcontrib)
        return FEA_OK;
    const size_t ni = b->items.size() / 4;
    std::vector<ElemArgs> h(std::max<size_t>(ni, 1));
    for (size_t it = 0; it < ni; ++it) {
        const int m = b->items[4 * it], t = b->items[4 * it + 1], z = b->items[4 * it + 2];
        const BatchMesh &M = b->hmeshes[m];
        ElemArgs A = M.a;
        const int64_t nn = nodes_of(t);
        A.contrib = (CT *)b->contrib + (VAR == V_ROWSYM ? M.scoff : M.coff) * B * B;
        A.rcontrib = (CT *)b->rcontrib + M.roff * B;
        if (VAR == V_ROWSYM) {
            const int64_t tl = M.tile_base[t] + z / sym_epb(t);
            A.tent_ptr = M.a.tent_ptr + tl;
            A.ttb_ptr = M.a.ttb_ptr + tl;
        }
        A.elems = M.a.elems + M.seg[t] + z;
        A.n = b->items[4 * it + 3];
        A.pnodes = M.a.pnodes + M.node_base[t] + (int64_t)z * nn;
        A.prdest = M.a.prdest + M.node_base[t] + (int64_t)z * nn;
        A.pdest = M.a.pdest + M.slot_base[t] + (int64_t)z * nn * nn;
        A.status = b->d_status + m;
        h[it] = A;
    }
    FEA_HIP(hipStreamSynchronize(s));
    if (ni > b->itemargs_cap) {
        dfree(b->d_itemargs);
        b->d_itemargs = nullptr;
        b->itemargs_cap = 0;
        int rc = dalloc((void **)&b->d_itemargs, sizeof(ElemArgs) * ni);
        if (rc) return rc;
        b->itemargs_cap = ni;
    }
    if (ni) FEA_HIP(hipMemcpy(b->d_itemargs, h.data(), sizeof(ElemArgs) * ni, hipMemcpyHostToDevice));
    b->itemargs_version = b->items_version;
    b->itemargs_var = key;
    b->itemargs_ws[0] = b->contrib;
    b->itemargs_ws[1] = b->rcontrib;
    drop_graph(b);
    return FEA_OK;
}

template <int T, int MODEL, typename CT, int VAR>
void launch_family(fea_batch *b, bool part, hipStream_t s)
{
    const int64_t n = b->foff[T + 1] - b->foff[T];
    if (n <= 0) return;
    k_batch<T, MODEL, CT, VAR><<<b->fworkers[T], 256, 0, s>>>(
        b->d_itemargs, b->d_items, b->d_order + b->foff[T], (int32_t)n, b->d_head + T,
        part ? b->d_part + b->poff[T] : nullptr, b->d_cycles, b->d_worker, b->d_cu);
}

template <int MODEL, typename CT, typename OT, int VAR>
int launch_batch(fea_batch *b, const fea_options *o, hipStream_t s, void *vals, void *rhs,
                 int32_t *status)
{
    constexpr int B = MODEL == FEA_POISSON ? 1 : 3;
    constexpr int BB = B * B;
    constexpr bool SYM = VAR == V_ROWSYM;
    int rc;
    if (SYM && (rc = sym_prepare_batch(b, s))) return rc;
    if ((rc = worker_count<MODEL, CT, VAR>(b))) return rc;
    const size_t need_c = sizeof(CT) * (size_t)std::max<int64_t>(SYM ? b->total_sym_slots : b->total_slots, 1) * BB;
    const size_t need_r = sizeof(CT) * (size_t)b->total_inc * B;
    if (b->contrib_bytes < need_c) {
        dfree(b->contrib);
        b->contrib = nullptr;
        b->contrib_bytes = 0;
        if ((rc = dalloc(&b->contrib, need_c))) return rc;
        b->contrib_bytes = need_c;
    }
    if (b->rcontrib_bytes < need_r) {
        dfree(b->rcontrib);
        b->rcontrib = nullptr;
        b->rcontrib_bytes = 0;
        if ((rc = dalloc(&b->rcontrib, need_r))) return rc;
        b->rcontrib_bytes = need_r;
    }
    if ((rc = ensure_itemargs<MODEL, CT, VAR>(b, s))) return rc;
    const int32_t ni = (int32_t)(b->items.size() / 4);
    k_batch_begin<<<grid_for(std::max(b->n_meshes, 1), 256), 256, 0, s>>>(b->d_head, b->d_status, b->n_meshes);
    if (o->timing) FEA_HIP(hipEventRecord(b->ev[0], s));
    if (ni) {
        // one persistent launch per family, each over its part of the queue
        const bool part = b->part_for == b->workers_for;
        launch_family<0, MODEL, CT, VAR>(b, part, s);
        launch_family<1, MODEL, CT, VAR>(b, part, s);
        launch_family<2, MODEL, CT, VAR>(b, part, s);
        launch_family<3, MODEL, CT, VAR>(b, part, s);
    }
    if (o->timing) FEA_HIP(hipEventRecord(b->ev[1], s));
    const int64_t nv = b->total_blocks * BB, nr = b->rhs_off.back();
    // the right-hand side first, while its workspace is still cached (the
    // upper-triangle form with 3x3 blocks carries it in the diagonal
    // blocks' tile sums instead, as one-mesh assembly does)
    constexpr bool RHSD = SYM && B == 3;
    if (RHSD && b->sym_empty_rows && nr) k_zero<OT><<<grid_for(nr, 256), 256, 0, s>>>(nr, (OT *)rhs);
    if (!RHSD && nr) launch_segsum<B, CT, OT>(nr / B, b->d_rseg, (const CT *)b->rcontrib, (OT *)rhs, s);
    if (SYM) {
        if (b->total_nup)
            launch_segsum_sym<BB, CT, OT>(b->total_nup, b->d_sym_ublk, b->d_sym_lp, b->d_sym_ptr,
                                          (const CT *)b->contrib, (OT *)vals, (OT *)rhs, s);
    } else if (nv) {
        launch_segsum<BB, CT, OT>(b->total_blocks, b->d_vseg, (const CT *)b->contrib, (OT *)vals, s);
    }
    k_batch_end<<<grid_for(std::max(b->n_meshes, 1), 256), 256, 0, s>>>(b->d_status, b->n_meshes, status);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

// Row-gather form: the batch's tiles through one persistent launch per
// tile class (no work queue: the tiles of a class are split statically
// over the workgroups, per XCD).
int dispatch_gather(fea_batch *b, const fea_options *o, hipStream_t s, void *vals, void *rhs, int32_t *status)
{
    int rc;
    if (!b->gbatch) {
        std::vector<GatherInput> in(b->n_meshes);
        for (int m = 0; m < b->n_meshes; ++m) {
            const fea_mesh_desc &d = b->desc[m];
            in[m] = {d.x, d.y, d.z, d.types, d.conn_ptr, d.conn, d.young, d.nu, d.source, nullptr,
                     b->model == FEA_ELASTIC ? d.nh_flag : nullptr, d.u};
        }
        if ((rc = gather_batch_build(&b->gbatch, b->n_meshes, b->graphs.data(), in.data(), b->vals_off.data(),
                                     b->rhs_off.data(), s)))
            return rc;
    }
    k_batch_begin<<<grid_for(std::max(b->n_meshes, 1), 256), 256, 0, s>>>(b->d_head, b->d_status, b->n_meshes);
    if (o->timing) FEA_HIP(hipEventRecord(b->ev[0], s));
    if ((rc = gather_batch_assemble(b->gbatch, b->model, b->has_nh, o->precision, o->out_dtype == FEA_F32, s, vals,
                                    rhs, b->d_status)))
        return rc;
    if (o->timing) FEA_HIP(hipEventRecord(b->ev[1], s));
    k_batch_end<<<grid_for(std::max(b->n_meshes, 1), 256), 256, 0, s>>>(b->d_status, b->n_meshes, status);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

template <int VAR>
int dispatch_var(fea_batch *b, const fea_options *o, hipStream_t s, void *vals, void *rhs, int32_t *status)
{
    const bool f32 = o->out_dtype == FEA_F32;
    if (b->model == FEA_POISSON) {
        if (o->precision == FEA_FP64)
            return f32 ? launch_batch<FEA_POISSON, double, float, VAR>(b, o, s, vals, rhs, status)
                       : launch_batch<FEA_POISSON, double, double, VAR>(b, o, s, vals, rhs, status);
        return f32 ? launch_batch<FEA_POISSON, float, float, VAR>(b, o, s, vals, rhs, status)
                   : launch_batch<FEA_POISSON, float, double, VAR>(b, o, s, vals, rhs, status);
    }
    if (b->has_nh) {
        if (o->precision == FEA_FP64)
            return f32 ? launch_batch<M_ELASTIC_NH, double, float, VAR>(b, o, s, vals, rhs, status)
                       : launch_batch<M_ELASTIC_NH, double, double, VAR>(b, o, s, vals, rhs, status);
        return f32 ? launch_batch<M_ELASTIC_NH, float, float, VAR>(b, o, s, vals, rhs, status)
                   : launch_batch<M_ELASTIC_NH, float, double, VAR>(b, o, s, vals, rhs, status);
    }
    if (o->precision == FEA_FP64)
        return f32 ? launch_batch<FEA_ELASTIC, double, float, VAR>(b, o, s, vals, rhs, status)
                   : launch_batch<FEA_ELASTIC, double, double, VAR>(b, o, s, vals, rhs, status);
    return f32 ? launch_batch<FEA_ELASTIC, float, float, VAR>(b, o, s, vals, rhs, status)
               : launch_batch<FEA_ELASTIC, float, double, VAR>(b, o, s, vals, rhs, status);
}

int dispatch(fea_batch *b, const fea_options *o, hipStream_t s, void *vals, void *rhs, int32_t *status)
{
    if (o->variant == FEA_ROWGATHER) return dispatch_gather(b, o, s, vals, rhs, status);
    if (o->variant == FEA_ROWSYM) return dispatch_var<V_ROWSYM>(b, o, s, vals, rhs, status);
    return dispatch_var<V_ROWOWNER>(b, o, s, vals, rhs, status);
}

int check_opts(const fea_batch *b, const fea_options *o)
{
    if (!b || !o) return set_error(FEA_EINVAL, "batch and options are required");
    if (o->variant != FEA_ROWOWNER && o->variant != FEA_ROWGATHER && o->variant != FEA_ROWSYM)
        return set_error(FEA_EINVAL, "batched assembly is row-owner, upper-triangle or row-gather");
    if (o->precision < 0 || o->precision > 1 || o->out_dtype < 0 || o->out_dtype > 1)
        return set_error(FEA_EINVAL, "bad option");
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev != b->device) return set_error(FEA_EINVAL, "batch lives on device %d, current is %d", b->device, dev);
    return FEA_OK;
}

int check_tiles(const int32_t *tile)
{
    for (int t = 0; t < 4; ++t)
        if (tile[t] < 1 || tile[t] > (1 << 20)) return set_error(FEA_EINVAL, "tile[%d] = %d out of range", t, tile[t]);
    return FEA_OK;
}

int build(int n, const fea_mesh_desc *md, int model, const int32_t *tile, hipStream_t s, fea_batch *b)
{
    int rc;
    FEA_HIP(hipGetDevice(&b->device));
    b->model = model;
    b->n_meshes = n;
    b->desc.assign(md, md + n);
    b->graphs.assign(n, nullptr);
    if (tile) {
        if ((rc = check_tiles(tile))) return rc;
        std::copy(tile, tile + 4, b->tile);
    }
    const int B = model == FEA_POISSON ? 1 : 3;
    b->vals_off.assign(1, 0);
    b->rhs_off.assign(1, 0);
    b->slot_off.assign(1, 0);
    b->inc_off.assign(1, 0);
    for (int m = 0; m < n; ++m) {
        const fea_mesh_desc &d = md[m];
        if (d.n_elems > 0 && (!d.x || !d.y || !d.z || !d.source || (model == FEA_ELASTIC && !d.nu) ||
                              (d.nh_flag && !d.u)))
            return set_error(FEA_EINVAL, "mesh %d: NULL array argument", m);
        rc = fea_graph_build(d.n_nodes, d.n_elems, d.types, d.conn_ptr, d.conn, s, &b->graphs[m]);
        if (rc) {
            std::string msg = fea_last_error();
            return set_error(rc, "mesh %d: %s", m, msg.c_str());
        }
        const fea_graph *g = b->graphs[m];
        b->vals_off.push_back(b->vals_off.back() + g->nnz * B * B);
        b->rhs_off.push_back(b->rhs_off.back() + g->n_nodes * B);
        b->slot_off.push_back(b->slot_off.back() + g->map_len);
        b->inc_off.push_back(b->inc_off.back() + g->conn_len);
        b->n_elems += g->n_elems;
        b->total_blocks += g->nnz;
    }
    b->total_slots = b->slot_off.back();
    b->total_inc = b->inc_off.back();
    if (b->total_slots > INT64_MAX / 16) return set_error(FEA_ERANGE, "batch too large");

    // per-mesh kernel views and the concatenated segment bounds
    std::vector<BatchMesh> bm(n);
    for (int m = 0; m < n; ++m) {
        const fea_mesh_desc &d = md[m];
        const fea_graph *g = b->graphs[m];
        ElemArgs a = {};
        a.x = d.x; a.y = d.y; a.z = d.z;
        a.conn_ptr = d.conn_ptr;
        a.conn = d.conn;
        a.elems = g->perm;
        a.map_ptr = g->map_ptr;
        a.e2nnz = g->e2nnz;
        a.pnodes = g->pnodes;
        a.pdest = g->pdest;
        a.prdest = g->prdest;
        a.young = d.young;
        a.nu = d.nu;
        a.nh_flag = model == FEA_ELASTIC ? d.nh_flag : nullptr;
        if (a.nh_flag) b->has_nh = true;
        a.u = d.u;
        a.source = d.source;
        bm[m].a = a;
        std::copy(g->seg, g->seg + 5, bm[m].seg);
        std::copy(g->node_base, g->node_base + 5, bm[m].node_base);
        std::copy(g->slot_base, g->slot_base + 5, bm[m].slot_base);
        bm[m].coff = b->slot_off[m];
        bm[m].roff = b->inc_off[m];
    }
    b->hmeshes = bm;
    if ((rc = dalloc((void **)&b->d_meshes, sizeof(BatchMesh) * std::max(n, 1)))) return rc;
    if (n) FEA_HIP(hipMemcpy(b->d_meshes, bm.data(), sizeof(BatchMesh) * n, hipMemcpyHostToDevice));
    if ((rc = dalloc((void **)&b->d_head, sizeof(int32_t) * 4))) return rc;
    if ((rc = dalloc((void **)&b->d_status, sizeof(int32_t) * std::max(n, 1)))) return rc;
    if ((rc = dalloc((void **)&b->d_vseg, sizeof(int64_t) * (b->total_blocks + 1)))) return rc;
    if ((rc = dalloc((void **)&b->d_rseg, sizeof(int64_t) * (b->rhs_off.back() / B + 1)))) return rc;
    int64_t zero = 0;
    FEA_HIP(hipMemcpy(b->d_vseg, &zero, sizeof(int64_t), hipMemcpyHostToDevice));
    FEA_HIP(hipMemcpy(b->d_rseg, &zero, sizeof(int64_t), hipMemcpyHostToDevice));
    int64_t kb = 0, nb = 0;
    for (int m = 0; m < n; ++m) {
        const fea_graph *g = b->graphs[m];
        if (g->nnz) k_offset_ptr<<<grid_for(g->nnz + 1, 256), 256, 0, s>>>(g->inv_ptr, g->nnz, b->slot_off[m], b->d_vseg + kb);
        if (g->n_nodes) k_offset_ptr<<<grid_for(g->n_nodes + 1, 256), 256, 0, s>>>(g->n2e_ptr, g->n_nodes, b->inc_off[m], b->d_rseg + nb);
        kb += g->nnz;
        nb += g->n_nodes;
    }
    FEA_HIP(hipGetLastError());
    FEA_HIP(hipStreamSynchronize(s));
    for (hipEvent_t &e : b->ev) FEA_HIP(hipEventCreate(&e));
    return build_items(b);
}

}  // namespace


namespace {

// item sizes tried by the autotuner: multiples of the upper-triangle tile
const int kEPB[4] = {sym_epb(0), sym_epb(1), sym_epb(2), sym_epb(3)};
const int kNQ[4] = {1, 8, 6, 8};

int upload_order(fea_batch *b) { return upload_grouped_order(b); }


// median duration (ms) of the persistent kernel over `reps` launches
int time_batch(fea_batch *b, const fea_options *o, int reps, hipStream_t s, void *vals, void *rhs, float *ms)
{
    fea_options t = *o;
    t.timing = 1;
    std::vector<float> v;
    int rc;
    if ((rc = dispatch(b, &t, s, vals, rhs, nullptr))) return rc;  // warm-up
    for (int r = 0; r < reps; ++r) {
        if ((rc = dispatch(b, &t, s, vals, rhs, nullptr))) return rc;
        FEA_HIP(hipEventSynchronize(b->ev[1]));
        float x = 0.f;
        FEA_HIP(hipEventElapsedTime(&x, b->ev[0], b->ev[1]));
        v.push_back(x);
    }
    std::sort(v.begin(), v.end());
    *ms = v[v.size() / 2];
    return FEA_OK;
}

std::string table_key(int model, int precision)
{
    char k[96];
    snprintf(k, sizeof(k), "gfx950 model=%d precision=%d", model, precision);
    return k;
}

}  // namespace

extern "C" int fea_batch_autotune(fea_batch *b, const fea_options *opt, int reps, const char *table_path,
                                  hipStream_t stream, int32_t *tile_out)
{
    clear_error();
    int rc = check_opts(b, opt);
    if (rc) return rc;
    if (opt->variant != FEA_ROWOWNER && opt->variant != FEA_ROWSYM)
        return set_error(FEA_EINVAL, "tiles are tuned for the row-owner and upper-triangle work items");
    if (reps < 1) return set_error(FEA_EINVAL, "reps must be positive");
    if ((rc = ensure_tables())) return rc;
    const size_t esz = opt->out_dtype == FEA_F32 ? 4 : 8;
    void *vals = nullptr, *rhs = nullptr;
    if ((rc = dalloc(&vals, esz * std::max<int64_t>(b->vals_off.back(), 1)))) return rc;
    if ((rc = dalloc(&rhs, esz * std::max<int64_t>(b->rhs_off.back(), 1)))) {
        dfree(vals);
        return rc;
    }
    int32_t best[4];
    std::copy(b->tile, b->tile + 4, best);
    float best_ms = 0.f;
    rc = time_batch(b, opt, reps, stream, vals, rhs, &best_ms);
    const int mult[10] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    for (int sweep = 0; sweep < 2 && !rc; ++sweep)
        for (int t = 0; t < 4 && !rc; ++t) {
            bool present = false;
            for (fea_graph *g : b->graphs) present |= g->seg[t + 1] > g->seg[t];
            if (!present) continue;
            for (int m : mult) {
                int32_t cand[4];
                std::copy(best, best + 4, cand);
                cand[t] = kEPB[t] * m;
                if (cand[t] == best[t]) continue;
                std::copy(cand, cand + 4, b->tile);
                if ((rc = build_items(b))) break;
                float ms = 0.f;
                if ((rc = time_batch(b, opt, reps, stream, vals, rhs, &ms))) break;
                if (ms < 0.99f * best_ms) {  // a gain beyond run-to-run noise
                    best_ms = ms;
                    std::copy(cand, cand + 4, best);
                }
            }
        }
    dfree(vals);
    dfree(rhs);
    if (rc) return rc;
    std::copy(best, best + 4, b->tile);
    if ((rc = build_items(b))) return rc;
    if (tile_out) std::copy(best, best + 4, tile_out);
    if (table_path) {
        std::vector<std::string> lines;
        const std::string key = table_key(b->model, opt->precision);
        if (FILE *f = fopen(table_path, "r")) {
            char buf[512];
            while (fgets(buf, sizeof(buf), f)) {
                std::string l(buf);
                if (l.compare(0, key.size(), key) != 0) lines.push_back(l);
            }
            fclose(f);
        }
        char entry[256];
        snprintf(entry, sizeof(entry), "%s tiles=%d,%d,%d,%d ms=%.4f\n", key.c_str(), best[0], best[1],
                 best[2], best[3], best_ms);
        lines.push_back(entry);
        FILE *f = fopen(table_path, "w");
        if (!f) return set_error(FEA_EINVAL, "cannot write %s", table_path);
        for (const std::string &l : lines) fputs(l.c_str(), f);
        fclose(f);
    }
    return FEA_OK;
}

extern "C" int fea_tile_table_load(const char *table_path, int model, int precision, int32_t *tile_out)
{
    clear_error();
    if (!table_path || !tile_out) return set_error(FEA_EINVAL, "path and tile_out are required");
    FILE *f = fopen(table_path, "r");
    if (!f) return set_error(FEA_EINVAL, "cannot read %s", table_path);
    const std::string key = table_key(model, precision);
    char buf[512];
    int found = 0;
    while (fgets(buf, sizeof(buf), f)) {
        if (strncmp(buf, key.c_str(), key.size()) != 0) continue;
        const char *p = strstr(buf, "tiles=");
        if (p && sscanf(p, "tiles=%d,%d,%d,%d", &tile_out[0], &tile_out[1], &tile_out[2], &tile_out[3]) == 4)
            found = 1;
    }
    fclose(f);
    if (!found) return set_error(FEA_EINVAL, "no entry for %s in %s", key.c_str(), table_path);
    return check_tiles(tile_out);
}

extern "C" int fea_batch_order(fea_batch *b, int schedule, const float *pred, hipStream_t stream)
{
    clear_error();
    if (!b) return set_error(FEA_EINVAL, "batch is NULL");
    const size_t ni = b->items.size() / 4;
    std::vector<double> w(ni, 0.0);
    if (schedule == FEA_TYPE_SORTED) {
        b->part_for = -1;
        b->part_w.clear();
        for (size_t i = 0; i < ni; ++i) b->order[i] = (int32_t)i;
        return upload_order(b);
    } else if (schedule == FEA_GP_WEIGHT) {
        for (size_t i = 0; i < ni; ++i) w[i] = (double)b->items[4 * i + 3] * kNQ[b->items[4 * i + 1]];
    } else if (schedule == FEA_LEARNED || schedule == FEA_LEARNED_CLASSES) {
        if (!pred && ni) return set_error(FEA_EINVAL, "pred is required for the learned schedule");
        std::vector<float> p(ni);
        if (ni) FEA_HIP(hipMemcpyAsync(p.data(), pred, sizeof(float) * ni, hipMemcpyDeviceToHost, stream));
        FEA_HIP(hipStreamSynchronize(stream));
        for (size_t i = 0; i < ni; ++i) {
            if (!std::isfinite(p[i])) return set_error(FEA_EINVAL, "pred[%zu] is not finite", i);
            w[i] = p[i];
        }
        if (schedule == FEA_LEARNED_CLASSES) {
            // cost classes a factor of two wide, centred on the family's
            // lower-median prediction: items of near-equal predicted cost
            // share a class and keep the type-sorted order among themselves
            for (int t = 0; t < 4; ++t) {
                std::vector<double> ft;
                for (size_t i = 0; i < ni; ++i)
                    if (b->items[4 * i + 1] == t) ft.push_back(w[i]);
                if (ft.empty()) continue;
                const size_t mid = (ft.size() - 1) / 2;
                std::nth_element(ft.begin(), ft.begin() + mid, ft.end());
                const double med = ft[mid];
                for (size_t i = 0; i < ni; ++i)
                    if (b->items[4 * i + 1] == t) w[i] = floor((w[i] - med) / M_LN2 + 0.5);
            }
        }
    } else {
        return set_error(FEA_EINVAL, "unknown schedule %d", schedule);
    }
    // the arguments are valid: back to the dynamic queue, in the new order
    b->part_for = -1;
    b->part_w.clear();
    // longest processing time first; ties keep the item order
    for (size_t i = 0; i < ni; ++i) b->order[i] = (int32_t)i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t x, int32_t y) { return w[x] > w[y]; });
    return upload_order(b);
}


extern "C" int fea_batch_partition(fea_batch *b, int weights, const float *pred, hipStream_t stream)
{
    clear_error();
    if (!b) return set_error(FEA_EINVAL, "batch is NULL");
    const size_t ni = b->items.size() / 4;
    std::vector<double> w(ni, 0.0);
    if (weights == FEA_TYPE_SORTED) {
        for (size_t i = 0; i < ni; ++i) w[i] = (double)b->items[4 * i + 3];
    } else if (weights == FEA_GP_WEIGHT) {
        for (size_t i = 0; i < ni; ++i) w[i] = (double)b->items[4 * i + 3] * kNQ[b->items[4 * i + 1]];
    } else if (weights == FEA_LEARNED) {
        if (!pred && ni) return set_error(FEA_EINVAL, "pred is required for learned weights");
        std::vector<float> p(ni);
        if (ni) FEA_HIP(hipMemcpyAsync(p.data(), pred, sizeof(float) * ni, hipMemcpyDeviceToHost, stream));
        FEA_HIP(hipStreamSynchronize(stream));
        for (size_t i = 0; i < ni; ++i) {
            if (!std::isfinite(p[i])) return set_error(FEA_EINVAL, "pred[%zu] is not finite", i);
            w[i] = exp((double)p[i]);
        }
    } else {
        return set_error(FEA_EINVAL, "unknown weights %d", weights);
    }
    // items keep the type-sorted order (neighbouring elements stay together)
    for (size_t i = 0; i < ni; ++i) b->order[i] = (int32_t)i;
    int rc = upload_order(b);
    if (rc) return rc;
    b->part_w = std::move(w);
    b->part_for = -1;
    if (b->workers_for >= 0) return make_partition(b);
    return FEA_OK;  // computed at the first launch, once the worker count is known
}

extern "C" int fea_batch_features(const fea_batch *b, int fp64_geometry, float *feats, hipStream_t stream)
{
    clear_error();
    if (!b || !feats) return set_error(FEA_EINVAL, "batch and feats are required");
    int rc = ensure_tables();
    if (rc) return rc;
    const int32_t ni = (int32_t)(b->items.size() / 4);
    if (ni) k_features<<<ni, 256, 0, stream>>>(b->d_meshes, b->d_items, fp64_geometry ? 1 : 0, feats);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

extern "C" int fea_batch_build(int n_meshes, const fea_mesh_desc *meshes, int model, const int32_t *tile,
                               hipStream_t stream, fea_batch **out)
{
    clear_error();
    if (!out) return set_error(FEA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_meshes < 0 || (n_meshes > 0 && !meshes)) return set_error(FEA_EINVAL, "bad mesh list");
    if (model != FEA_POISSON && model != FEA_ELASTIC) return set_error(FEA_EINVAL, "unknown model %d", model);
    fea_batch *b = new (std::nothrow) fea_batch();
    if (!b) return set_error(FEA_ENOMEM, "host allocation failed");
    int rc = ensure_tables();
    if (!rc) rc = build(n_meshes, meshes, model, tile, stream, b);
    if (rc) {
        std::string msg = fea_last_error();
        (void)hipStreamSynchronize(stream);
        destroy_batch(b);
        return set_error(rc, "%s", msg.c_str());
    }
    *out = b;
    return FEA_OK;
}

extern "C" int fea_batch_sizes(const fea_batch *b, int64_t *vals_len, int64_t *rhs_len, int64_t *n_items,
                               int64_t *n_elems)
{
    clear_error();
    if (!b) return set_error(FEA_EINVAL, "batch is NULL");
    if (vals_len) *vals_len = b->vals_off.back();
    if (rhs_len) *rhs_len = b->rhs_off.back();
    if (n_items) *n_items = (int64_t)(b->items.size() / 4);
    if (n_elems) *n_elems = b->n_elems;
    return FEA_OK;
}

extern "C" int fea_batch_offsets(const fea_batch *b, int64_t *vals_off, int64_t *rhs_off)
{
    clear_error();
    if (!b) return set_error(FEA_EINVAL, "batch is NULL");
    if (vals_off) std::copy(b->vals_off.begin(), b->vals_off.end(), vals_off);
    if (rhs_off) std::copy(b->rhs_off.begin(), b->rhs_off.end(), rhs_off);
    return FEA_OK;
}

extern "C" int fea_batch_items(const fea_batch *b, int32_t *items)
{
    clear_error();
    if (!b || !items) return set_error(FEA_EINVAL, "batch and items are required");
    std::copy(b->items.begin(), b->items.end(), items);
    return FEA_OK;
}

extern "C" int fea_batch_set_tiles(fea_batch *b, const int32_t *tile)
{
    clear_error();
    if (!b || !tile) return set_error(FEA_EINVAL, "batch and tile are required");
    int rc = check_tiles(tile);
    if (rc) return rc;
    std::copy(tile, tile + 4, b->tile);
    return build_items(b);
}

extern "C" int fea_batch_get_order(const fea_batch *b, int32_t *order)
{
    clear_error();
    if (!b || !order) return set_error(FEA_EINVAL, "batch and order are required");
    std::copy(b->order.begin(), b->order.end(), order);
    return FEA_OK;
}

extern "C" int fea_batch_set_order(fea_batch *b, const int32_t *order)
{
    clear_error();
    if (!b || !order) return set_error(FEA_EINVAL, "batch and order are required");
    const size_t ni = b->items.size() / 4;
    std::vector<char> seen(ni, 0);
    for (size_t j = 0; j < ni; ++j) {
        if (order[j] < 0 || (size_t)order[j] >= ni || seen[order[j]])
            return set_error(FEA_EINVAL, "order is not a permutation of the %zu items", ni);
        seen[order[j]] = 1;
    }
    b->order.assign(order, order + ni);
    b->part_for = -1;
    b->part_w.clear();
    return upload_grouped_order(b);
}

extern "C" int fea_batch_assemble(fea_batch *b, const fea_options *opt, hipStream_t stream, void *vals,
                                  void *rhs, int32_t *status)
{
    clear_error();
    int rc = check_opts(b, opt);
    if (rc) return rc;
    if ((b->vals_off.back() && !vals) || (b->rhs_off.back() && !rhs))
        return set_error(FEA_EINVAL, "NULL output argument");
    if ((rc = ensure_tables())) return rc;
    b->timed = false;
    if ((rc = dispatch(b, opt, stream, vals, rhs, status))) return rc;
    b->timed = opt->timing != 0;
    return FEA_OK;
}

extern "C" int fea_batch_capture(fea_batch *b, const fea_options *opt, hipStream_t stream, void *vals,
                                 void *rhs, int32_t *status)
{
    clear_error();
    int rc = check_opts(b, opt);
    if (rc) return rc;
    if ((b->vals_off.back() && !vals) || (b->rhs_off.back() && !rhs))
        return set_error(FEA_EINVAL, "NULL output argument");
    if ((rc = ensure_tables())) return rc;
    fea_options o = *opt;
    o.timing = 0;
    // size the workspaces and the worker count outside the capture
    if ((rc = dispatch(b, &o, stream, vals, rhs, status))) return rc;
    FEA_HIP(hipStreamSynchronize(stream));
    drop_graph(b);
    FEA_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    rc = dispatch(b, &o, stream, vals, rhs, status);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return set_error(FEA_EHIP, "stream capture failed: %s", hipGetErrorString(e));
    b->graph = graph;
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return set_error(FEA_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    return FEA_OK;
}

extern "C" int fea_batch_replay(fea_batch *b, int n, hipStream_t stream)
{
    clear_error();
    if (!b || !b->exec) return set_error(FEA_EINVAL, "no captured graph");
    for (int i = 0; i < n; ++i) FEA_HIP(hipGraphLaunch(b->exec, stream));
    return FEA_OK;
}

extern "C" int fea_batch_cycles(const fea_batch *b, uint64_t *cycles, int32_t *worker, int32_t *cu,
                                hipStream_t s)
{
    clear_error();
    if (!b) return set_error(FEA_EINVAL, "batch is NULL");
    const size_t ni = b->items.size() / 4;
    if (!ni) return FEA_OK;
    if (cycles) FEA_HIP(hipMemcpyAsync(cycles, b->d_cycles, sizeof(uint64_t) * ni, hipMemcpyDeviceToDevice, s));
    if (worker) FEA_HIP(hipMemcpyAsync(worker, b->d_worker, sizeof(int32_t) * ni, hipMemcpyDeviceToDevice, s));
    if (cu) FEA_HIP(hipMemcpyAsync(cu, b->d_cu, sizeof(int32_t) * ni, hipMemcpyDeviceToDevice, s));
    return FEA_OK;
}

extern "C" int fea_batch_last_ms(const fea_batch *b, float *ms)
{
    clear_error();
    if (!b || !ms) return set_error(FEA_EINVAL, "batch and ms are required");
    if (!b->timed) return set_error(FEA_EINVAL, "no timed batched assembly");
    FEA_HIP(hipEventSynchronize(b->ev[1]));
    FEA_HIP(hipEventElapsedTime(ms, b->ev[0], b->ev[1]));
    return FEA_OK;
}

extern "C" int fea_batch_workers(const fea_batch *b, int *workers)
{
    clear_error();
    if (!b || !workers) return set_error(FEA_EINVAL, "batch and workers are required");
    *workers = b->workers;
    return FEA_OK;
}

extern "C" void fea_batch_destroy(fea_batch *b)
{
    if (b) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(b->device);
        (void)hipDeviceSynchronize();
        destroy_batch(b);
        (void)hipSetDevice(cur);
    }
}

int fea::batch_view(fea_batch *b, BatchView *v)
{
    int rc;
    if (!b->d_sub_head && (rc = dalloc((void **)&b->d_sub_head, sizeof(int32_t) * 4))) return rc;
    v->device = b->device;
    v->model = b->model;
    v->n_meshes = b->n_meshes;
    v->desc = b->desc.data();
    v->graphs = b->graphs.data();
    v->items = b->d_sub_items;
    v->order = b->d_sub_order;
    for (int t = 0; t < 5; ++t) v->foff[t] = b->sub_foff[t];
    v->head = b->d_sub_head;
    v->items_owner = &b->d_sub_items;
    v->order_owner = &b->d_sub_order;
    v->foff_owner = b->sub_foff;
    v->args = &b->d_subargs;
    v->args_cap = &b->subargs_cap;
    v->args_key = b->subargs_key;
    return FEA_OK;
}
