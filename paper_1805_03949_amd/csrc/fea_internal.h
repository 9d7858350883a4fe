// Internal declarations of the gfx950 assembly library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fea.h"

namespace fea {

// Nodes per family: tet4, pyr5, pen6, hex8.
__host__ __device__ constexpr inline int nodes_of(int t) { return 4 + t + (t == 3); }
// Elements per tile of the upper-triangle form: one lane per local pair
// a <= b, 256 lanes per workgroup.
__host__ __device__ constexpr inline int sym_epb(int t) { return 256 / (nodes_of(t) * (nodes_of(t) + 1) / 2); }

// Records a message for fea_last_error() and returns `code`.
int set_error(int code, const char *fmt, ...);
void clear_error();

#define FEA_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::fea::set_error(FEA_EHIP, "%s failed: %s (%s:%d)", #call,          \
                                    hipGetErrorString(e_), __FILE__, __LINE__);        \
    } while (0)

// Device allocation that records an error message on failure.
int dalloc(void **p, size_t bytes);
void dfree(void *p);

// ptr[0] = 0, ptr[i+1] = in[0] + ... + in[i] for i < n (int64 result).
// `tmp` must hold scan_tmp_elems(n) int64 values.
int64_t scan_tmp_elems(int64_t n);
int scan_to_ptr_u8(const uint8_t *in, int64_t n, int64_t *ptr, int64_t *tmp, hipStream_t s);
int scan_to_ptr_i32(const int32_t *in, int64_t n, int64_t *ptr, int64_t *tmp, hipStream_t s);
int scan_to_ptr_i64(const int64_t *in, int64_t n, int64_t *ptr, int64_t *tmp, hipStream_t s);

// Grid size for a 1-D launch of n threads in blocks of `bs`.
inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct GatherInput {
    const double *x, *y, *z;
    const uint8_t *types;
    const int64_t *conn_ptr;
    const int32_t *conn;
    const double *young, *nu;
    const double *source;
    int32_t *status;
    const uint8_t *nh_flag;  // NULL, or neo-Hookean tangent where set
    const double *u;
};

// What the subgrid scale needs of a batch (fea_batch is private to the
// batch code): its meshes and graphs, its own work items and
// family-grouped order (sized for the subgrid scale's element groups, kept
// in the batch), queue heads of its own and a cache slot for per-mesh
// arguments (valid for the key recorded with it).
struct BatchView {
    int device, model, n_meshes;
    const fea_mesh_desc *desc;
    fea_graph *const *graphs;
    const int4 *items;
    const int32_t *order;
    int64_t foff[5];
    int32_t *head;
    // where the subgrid scale's own items live (built on its first call)
    int4 **items_owner;
    int32_t **order_owner;
    int64_t *foff_owner;
    void **args;
    size_t *args_cap;
    const void **args_key;
};
int batch_view(fea_batch *b, BatchView *v);

}  // namespace fea

// The graph object behind the opaque fea_graph handle.
struct fea_graph {
    int device = 0;
    int64_t n_nodes = 0, n_elems = 0, nnz = 0, map_len = 0, conn_len = 0;
    uint64_t mesh_fp = 0;  // connectivity fingerprint of the mesh it was built for
    int n_colours = 0;
    // block pattern, element-to-nonzero map and its inverse
    int64_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    int64_t *map_ptr = nullptr;
    int32_t *e2nnz = nullptr;
    int64_t *inv_ptr = nullptr;
    int32_t *inv = nullptr;
    // Row-owner layout, in type-sorted element order (position p = index in
    // perm): node ids pnodes, destination of every slot pdest (its index in
    // the inverse map, so the workspace lies sorted by destination block) and
    // of every right-hand-side entry prdest (its incidence index). Family t
    // starts at node_base[t] (pnodes, prdest) and slot_base[t] (pdest).
    int32_t *pnodes = nullptr;
    int32_t *pdest = nullptr;
    int32_t *prdest = nullptr;
    int64_t node_base[5] = {0, 0, 0, 0, 0};
    int64_t slot_base[5] = {0, 0, 0, 0, 0};
    // node -> incident elements (ascending element id) and local index
    int64_t *n2e_ptr = nullptr;
    int32_t *n2e = nullptr;
    uint8_t *n2a = nullptr;
    // elements stably sorted by family; seg[t]..seg[t+1] in perm (host copy)
    int32_t *perm = nullptr;
    int64_t seg[5] = {0, 0, 0, 0, 0};
    // greedy colouring and (family, colour) buckets, cseg host copy:
    // bucket (t, c) = cperm[cseg[t*(n_colours+1)+c] .. cseg[t*(n_colours+1)+c+1])
    int16_t *colour = nullptr;
    int32_t *cperm = nullptr;
    std::vector<int64_t> cseg;
    // Row-gather layout (built by the first FEA_ROWGATHER assembly). Tiles
    // of consecutive rows, listed by class (rows of pure tet4, pyr5, pen6,
    // hex8, then rows touching several families), class c at gtile_off[c] ..
    // gtile_off[c+1]; each tile record holds r0, rows, first pair, pairs,
    // first block, blocks, first inverse-map entry, entries (8 x int32). The
    // (row, element) pairs of a tile are its rows' incidence entries; lane l
    // of a tile is node l of the concatenated node lists of its pairs, whose
    // node ids are gnodes[j0 + l]; gdesc[j] is the tile lane of inverse-map
    // entry j's contribution.
    int32_t *gtile = nullptr;
    int64_t gtile_off[6] = {0, 0, 0, 0, 0, 0};
    int32_t *gnodes = nullptr;
    uint8_t *gdesc = nullptr;
    bool gready = false;
    // events around the five class kernels of the last timed row-gather
    // assembly (gev[c] before class c, gev[5] after the last)
    hipEvent_t gev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool gtimed = false;
    // Upper-triangle layout (built by the first FEA_ROWSYM assembly).
    // upart[k] = block k itself if col >= row, else the block at the
    // transposed position; ublk = the nup upper (and diagonal) blocks in CSR
    // order; lpart[k] = lower partner of upper block k (-1 for diagonal and
    // lower blocks).
    int32_t *upart = nullptr;
    int32_t *ublk = nullptr;
    int32_t *lpart = nullptr;
    int64_t nup = 0;
    // the same per entry m of the upper-block list: lower partner of ublk[m]
    // (ulp; -(v + 1) for the diagonal block of row v) and its workspace segment uptr[m] ..
    // uptr[m+1] (segments of consecutive entries are adjacent)
    int32_t *ulp = nullptr;
    int64_t *uptr = nullptr;
    int64_t sym_empty_rows = 0;  // rows no element touches (no diagonal block)
    // Element tiles: family t's elements in type-sorted order, EPB_t =
    // 256 / (n(n+1)/2) consecutive ones per tile, tiles tile_base[t] ..
    // tile_base[t+1]. Lane l = el * n(n+1)/2 + w of a tile is the w-th local
    // pair a <= b of its el-th element. Tile τ's entries tent[tent_ptr[τ] ..
    // tent_ptr[τ+1]) (lane << 1 | transposed) are sorted by destination
    // upper block, then lane; its distinct blocks are tile-blocks ttb_ptr[τ]
    // .. ttb_ptr[τ+1], tile-block d holding entries up to tb_eend[d]
    // (exclusive, within the tile), block id tb_blk[d] and workspace slot
    // tb_slot[d]. The workspace lies sorted by block, then tile: block k's
    // tile sums are ts_ptr[k] .. ts_ptr[k+1]; ulen = tile-blocks.
    int64_t tile_base[5] = {0, 0, 0, 0, 0};
    int64_t *tent_ptr = nullptr;
    int64_t *ttb_ptr = nullptr;
    uint16_t *tent = nullptr;
    uint16_t *tb_eend = nullptr;
    int32_t *tb_blk = nullptr;
    int32_t *tb_slot = nullptr;
    int64_t *ts_ptr = nullptr;
    int64_t ulen = 0, nent = 0;
    // Tile colouring (built by the first FEA_TILECOLOUR assembly): greedy
    // first-fit over the tiles in descending neighbour count, no two tiles
    // of a colour sharing a node; bucket (t, c) = family t's tiles of
    // colour c, ctile[tcseg[t*(tc_colours+1)+c] .. tcseg[t*(tc_colours+1)+c+1])
    // (family-local tile indices in descending neighbour count, ties by
    // index; tcseg is a host copy).
    int32_t *ctile = nullptr;
    std::vector<int64_t> tcseg;
    std::vector<int32_t> tc_nneig;  // neighbour count of every tile (global tile index)
    int tc_colours = 0;
    bool tcready = false;
    bool sready = false;
    // Gauss-point offsets in element order (built by the first subgrid-scale
    // call or query): element e's points are gp_ptr[e] .. gp_ptr[e+1]
    int64_t *gp_ptr = nullptr;
    int64_t n_gp = 0;
    bool gpready = false;
    // lazily allocated workspaces of the scatter variants
    void *contrib = nullptr;
    size_t contrib_bytes = 0;
    void *rcontrib = nullptr;
    size_t rcontrib_bytes = 0;
    double *acc64 = nullptr;
    size_t acc64_bytes = 0;
    // events of the last timed fea_assemble: begin, element kernels done,
    // block-value scatter kernel done, end
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
};

namespace fea {
// Fused owner-computes assembly (FEA_ROWGATHER), in gather.hip. Builds the
// row tiles on first use (blocks on the stream). model: FEA_POISSON or
// FEA_ELASTIC (with in.nh_flag: the neo-Hookean tangent where flagged);
// precision: enum fea_precision.
int gather_assemble(fea_graph *g, const GatherInput &in, int model, int precision, bool out_f32,
                    bool timing, hipStream_t s, void *vals, void *rhs);
}  // namespace fea

namespace fea {
// Row-gather form of a batch (gather.hip): the tiles of every mesh in one
// list per class, with each tile's mesh. Built once per batch from its
// graphs (preparing each graph's tiles; blocks on the stream).
struct GatherBatch;
int gather_batch_build(GatherBatch **out, int n, fea_graph *const *graphs, const GatherInput *in,
                       const int64_t *vals_off, const int64_t *rhs_off, hipStream_t s);
// Enqueues the batch's class kernels: mesh m's values at vals + vals_off[m]
// and status entry status[m] (set by atomic minimum; initialised by the caller).
int gather_batch_assemble(const GatherBatch *gb, int model, bool nh, int precision, bool out_f32,
                          hipStream_t s, void *vals, void *rhs, int32_t *status);
void gather_batch_destroy(GatherBatch *gb);
}  // namespace fea

namespace fea {
// Set-up of fea_assemble_noalloc on the current device (assemble.hip):
// uploads the reference tables and looks up the device address of its
// scratch array, once per device. Called by the graph build.
int noalloc_setup();
}  // namespace fea

namespace fea {
// Builds the upper-triangle row-owner layout of a graph (graph.hip; blocks
// on the stream).
int sym_prepare(fea_graph *g, hipStream_t s);
// Colours the upper-triangle tiles (graph.hip; needs sym_prepare; blocks
// on the stream).
int tile_colour_prepare(fea_graph *g, hipStream_t s);
}  // namespace fea
