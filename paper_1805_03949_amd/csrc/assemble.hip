// Element quadrature and scatter kernels (paper Section 2.1.1, Algorithm 1;
// race treatments of Section 3.2: Algorithm 4 ATOMIC, Algorithm 5 colouring).
// The element device code lives in elem.h.
#include <climits>
#include <cstring>
#include <mutex>

#include "elem.h"
#include "segsum.h"

namespace fea {

template <int T, int MODEL, int VAR, typename CT>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, 256),
                               amdgpu_waves_per_eu(one_tile_min_waves<T, MODEL, VAR, CT>()))) k_element(ElemArgs A)
{
    __shared__ ElemSmem<T, MODEL, VAR, CT> S;
    constexpr int EPB = ElemSmem<T, MODEL, VAR, CT>::EPB;
    const int64_t b = xcd_tile(blockIdx.x, gridDim.x);
    elem_tile<T, MODEL, VAR, CT>(A, (VAR == V_TILECOL ? (int64_t)A.tiles[b] : b) * EPB, S);
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
    constexpr int EPB = ElemSmem<T, MODEL, VAR, CT>::EPB;
    if (a.n <= 0) return;
    if (VAR == V_TILECOL) {
        if (a.ntiles > 0) k_element<T, MODEL, VAR, CT><<<(unsigned)a.ntiles, 256, 0, s>>>(a);
        return;
    }
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

// Row-owner workspaces supplied by the caller of run() instead of the
// graph's own (allocated on first use): contrib holds map_len blocks and
// rcontrib conn_len right-hand-side entries in the compute type.
struct Workspace {
    void *contrib = nullptr;
    void *rcontrib = nullptr;
};

template <int MODEL, typename CT>
static int run(fea_graph *g, ElemArgs a, const fea_options *o, hipStream_t s, void *vals, void *rhs,
               const Workspace &ws = Workspace())
{
    constexpr int B = MODEL == FEA_POISSON ? 1 : 3;
    constexpr int BB = B * B;
    const int64_t nv = g->nnz * BB, nr = g->n_nodes * B;
    const bool f32 = o->out_dtype == FEA_F32;
    int rc;
    if (o->variant == FEA_ROWSYM) {
        // 3x3 blocks: the right-hand side rides in the diagonal blocks' tile
        // sums (no workspace of its own); 1x1: its own workspace and sums
        constexpr bool RHSD = B == 3;
        if (!g->sready && (rc = sym_prepare(g, s))) return rc;
        if ((rc = ensure_ws(&g->contrib, &g->contrib_bytes, sizeof(CT) * (size_t)std::max<int64_t>(g->ulen, 1) * BB))) return rc;
        if (!RHSD && (rc = ensure_ws(&g->rcontrib, &g->rcontrib_bytes, sizeof(CT) * (size_t)g->conn_len * B))) return rc;
        a.contrib = g->contrib;
        a.rcontrib = RHSD ? nullptr : g->rcontrib;
        a.tent = g->tent;
        a.tb_eend = g->tb_eend;
        a.tb_slot = g->tb_slot;
        mark(g, 0, o, s);
        for (int t = 0; t < 4; ++t) {
            a.elems = g->perm + g->seg[t];
            a.n = g->seg[t + 1] - g->seg[t];
            a.pnodes = g->pnodes + g->node_base[t];
            a.prdest = g->prdest + g->node_base[t];
            a.tent_ptr = g->tent_ptr + g->tile_base[t];
            a.ttb_ptr = g->ttb_ptr + g->tile_base[t];
            launch_type<MODEL, V_ROWSYM, CT>(t, a, s);
        }
        // 1x1: the right-hand side first, while its workspace (just written)
        // is still in the caches; then the block values (3x3: with the
        // right-hand side, rows that no element touches set to zero first)
        if (f32) {
            if (RHSD && g->sym_empty_rows && nr) k_zero<float><<<grid_for(nr, 256), 256, 0, s>>>(nr, (float *)rhs);
            if (!RHSD && nr) launch_segsum<B, CT, float>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (float *)rhs, s);
            mark(g, 1, o, s);
            if (g->nup)
                launch_segsum_sym<BB, CT, float>(g->nup, g->ublk, g->ulp, g->uptr, (const CT *)g->contrib, (float *)vals,
                                                 (float *)rhs, s);
        } else {
            if (RHSD && g->sym_empty_rows && nr) k_zero<double><<<grid_for(nr, 256), 256, 0, s>>>(nr, (double *)rhs);
            if (!RHSD && nr) launch_segsum<B, CT, double>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (double *)rhs, s);
            mark(g, 1, o, s);
            if (g->nup)
                launch_segsum_sym<BB, CT, double>(g->nup, g->ublk, g->ulp, g->uptr, (const CT *)g->contrib,
                                                  (double *)vals, (double *)rhs, s);
        }
        mark(g, 2, o, s);
        mark(g, 3, o, s);
        FEA_HIP(hipGetLastError());
        return FEA_OK;
    }
    if (o->variant == FEA_TILECOLOUR) {
        if (!g->sready && (rc = sym_prepare(g, s))) return rc;
        if (!g->tcready && (rc = tile_colour_prepare(g, s))) return rc;
        if ((rc = ensure_ws(&g->rcontrib, &g->rcontrib_bytes, sizeof(CT) * (size_t)g->conn_len * B))) return rc;
        double *tv = (double *)vals;
        if (f32) {
            if ((rc = ensure_ws((void **)&g->acc64, &g->acc64_bytes, sizeof(double) * (size_t)std::max<int64_t>(nv, 1)))) return rc;
            tv = g->acc64;
        }
        a.rcontrib = g->rcontrib;
        a.vals = tv;
        a.tent = g->tent;
        a.tb_eend = g->tb_eend;
        a.tb_blk = g->tb_blk;
        a.lpart = g->lpart;
        mark(g, 0, o, s);
        if (nv) k_fill_f64<<<grid_for(nv, 256), 256, 0, s>>>(tv, nv, 0.0);
        const int nc = g->tc_colours;
        for (int c = 0; c < nc; ++c)
            for (int t = 0; t < 4; ++t) {
                const int64_t b = g->tcseg[(size_t)t * (nc + 1) + c], e = g->tcseg[(size_t)t * (nc + 1) + c + 1];
                a.elems = g->perm + g->seg[t];
                a.n = g->seg[t + 1] - g->seg[t];
                a.pnodes = g->pnodes + g->node_base[t];
                a.prdest = g->prdest + g->node_base[t];
                a.tent_ptr = g->tent_ptr + g->tile_base[t];
                a.ttb_ptr = g->ttb_ptr + g->tile_base[t];
                a.tiles = g->ctile + b;
                a.ntiles = e - b;
                launch_type<MODEL, V_TILECOL, CT>(t, a, s);
            }
        mark(g, 1, o, s);
        if (f32 && nv) k_to_f32<<<grid_for(nv, 256), 256, 0, s>>>(tv, (float *)vals, nv);
        mark(g, 2, o, s);
        if (nr) {
            if (f32)
                launch_segsum<B, CT, float>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (float *)rhs, s);
            else
                launch_segsum<B, CT, double>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (double *)rhs, s);
        }
        mark(g, 3, o, s);
        FEA_HIP(hipGetLastError());
        return FEA_OK;
    }
    if (o->variant == FEA_ROWOWNER) {
        if (ws.contrib) {
            a.contrib = ws.contrib;
            a.rcontrib = ws.rcontrib;
        } else {
            if ((rc = ensure_ws(&g->contrib, &g->contrib_bytes, sizeof(CT) * (size_t)g->map_len * BB))) return rc;
            if ((rc = ensure_ws(&g->rcontrib, &g->rcontrib_bytes, sizeof(CT) * (size_t)g->conn_len * B))) return rc;
            a.contrib = g->contrib;
            a.rcontrib = g->rcontrib;
        }
        mark(g, 0, o, s);
        for (int t = 0; t < 4; ++t) {
            a.elems = g->perm + g->seg[t];
            a.n = g->seg[t + 1] - g->seg[t];
            a.pnodes = g->pnodes + g->node_base[t];
            a.prdest = g->prdest + g->node_base[t];
            a.pdest = g->pdest + g->slot_base[t];
            launch_type<MODEL, V_ROWOWNER, CT>(t, a, s);
        }
        // the right-hand side first (its workspace is still cached)
        if (f32) {
            if (nr) launch_segsum<B, CT, float>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (float *)rhs, s);
            mark(g, 1, o, s);
            if (nv) launch_segsum<BB, CT, float>(g->nnz, g->inv_ptr, (const CT *)g->contrib, (float *)vals, s);
        } else {
            if (nr) launch_segsum<B, CT, double>(g->n_nodes, g->n2e_ptr, (const CT *)g->rcontrib, (double *)rhs, s);
            mark(g, 1, o, s);
            if (nv) launch_segsum<BB, CT, double>(g->nnz, g->inv_ptr, (const CT *)g->contrib, (double *)vals, s);
        }
        mark(g, 2, o, s);
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

namespace fea {

// Argument checks shared by fea_assemble and fea_assemble_noalloc.
static int check_assemble(const fea_graph *g, const double *x, const double *y, const double *z,
                          const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                          const fea_material *mat, const double *source, const fea_options *o, void *vals,
                          void *rhs)
{
    if (!g || !mat) return set_error(FEA_EINVAL, "graph and material are required");
    if (o->precision < 0 || o->precision > 1 || o->variant < 0 || o->variant > 5 ||
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
    if (mat->residual) {
        if (mat->model != FEA_ELASTIC || (g->n_elems > 0 && !mat->u))
            return set_error(FEA_EINVAL, "the residual needs the elastic model and u");
        if (o->precision != FEA_FP64 || o->variant == FEA_ROWGATHER)
            return set_error(FEA_EINVAL, "the residual is assembled in FP64 by the element-tile forms only");
    }
    if ((g->nnz > 0 && !vals) || (g->n_nodes > 0 && !rhs))
        return set_error(FEA_EINVAL, "NULL output argument");
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev != g->device) return set_error(FEA_EINVAL, "graph lives on device %d, current is %d", g->device, dev);
    return FEA_OK;
}

// The assembly proper (after check_assemble): status is a device int32
// (required), ws an optional row-owner workspace.
static int assemble_impl(fea_graph *g, const double *x, const double *y, const double *z, const uint8_t *types,
                         const int64_t *conn_ptr, const int32_t *conn, const fea_material *mat,
                         const double *source, const fea_options *o, hipStream_t stream, void *vals, void *rhs,
                         int32_t *st, const Workspace &ws)
{
    int rc;
    k_status_init<<<1, 1, 0, stream>>>(st);

    ElemArgs a = {};
    a.x = x; a.y = y; a.z = z;
    a.conn_ptr = conn_ptr;
    a.conn = conn;
    a.map_ptr = g->map_ptr;
    a.e2nnz = g->e2nnz;
    a.young = mat->young;
    a.nu = mat->nu;
    a.nh_flag = mat->model == FEA_ELASTIC ? mat->nh_flag : nullptr;
    a.u = mat->u;
    a.source = source;
    a.status = st;

    if (g->n_elems > 0 && o->variant == FEA_ROWGATHER) {
        GatherInput in = {x, y, z, types, conn_ptr, conn, mat->young, mat->nu, source, st, a.nh_flag, mat->u};
        if ((rc = gather_assemble(g, in, mat->model, o->precision, o->out_dtype == FEA_F32, o->timing != 0,
                                  stream, vals, rhs)))
            return rc;
    } else if (g->n_elems > 0) {
        if (mat->model == FEA_POISSON)
            rc = o->precision == FEA_FP64 ? run<FEA_POISSON, double>(g, a, o, stream, vals, rhs, ws)
                                          : run<FEA_POISSON, float>(g, a, o, stream, vals, rhs, ws);
        else if (mat->residual)
            rc = run<M_ELASTIC_RES, double>(g, a, o, stream, vals, rhs, ws);
        else if (!a.nh_flag)
            rc = o->precision == FEA_FP64 ? run<FEA_ELASTIC, double>(g, a, o, stream, vals, rhs, ws)
                                          : run<FEA_ELASTIC, float>(g, a, o, stream, vals, rhs, ws);
        else
            rc = o->precision == FEA_FP64 ? run<M_ELASTIC_NH, double>(g, a, o, stream, vals, rhs, ws)
                                          : run<M_ELASTIC_NH, float>(g, a, o, stream, vals, rhs, ws);
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

// Scratch of the allocation-free entry point: one array per device, set up
// once per device (reference tables uploaded, the array's device address
// looked up) by the graph build on that device, or else by the entry
// point's first call there. Layout: the status word, then the slot
// workspace, then the right-hand-side workspace, each 256-byte aligned.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr size_t kScratchHead = 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void *g_scratch[64] = {nullptr};
static std::mutex g_scratch_mtx;

static inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

int noalloc_setup()
{
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(FEA_EINVAL, "device index %d unsupported", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    if (g_scratch[dev]) return FEA_OK;
    int rc = ensure_tables();
    if (rc) return rc;
    void *ptr = nullptr;
    FEA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return set_error(FEA_EHIP, "scratch array has no device address");
    g_scratch[dev] = ptr;
    return FEA_OK;
}

}  // namespace fea

extern "C" int fea_assemble(const fea_graph *gc, const double *x, const double *y, const double *z,
                            const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                            const fea_material *mat, const double *source, const fea_options *opt,
                            hipStream_t stream, void *vals, void *rhs, int32_t *status)
{
    clear_error();
    fea_graph *g = const_cast<fea_graph *>(gc);
    fea_options dflt = {0, 0, 0, 0};
    const fea_options *o = opt ? opt : &dflt;
    int rc = check_assemble(g, x, y, z, types, conn_ptr, conn, mat, source, o, vals, rhs);
    if (rc) return rc;
    if ((rc = ensure_tables())) return rc;
    if (o->timing) {
        for (hipEvent_t &e : g->ev)
            if (!e) FEA_HIP(hipEventCreate(&e));
    }
    g->timed = false;
    g->gtimed = false;
    int32_t *st = status;
    if (!st) {
        static thread_local int32_t *own[64] = {nullptr};
        const int dev = g->device;
        if (!own[dev] && (rc = dalloc((void **)&own[dev], sizeof(int32_t)))) return rc;
        st = own[dev];
    }
    return assemble_impl(g, x, y, z, types, conn_ptr, conn, mat, source, o, stream, vals, rhs, st, Workspace());
}

extern "C" int fea_assemble_noalloc(const fea_graph *gc, const double *x, const double *y, const double *z,
                                    const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                                    const fea_material *mat, const double *source, const fea_options *opt,
                                    hipStream_t stream, void *vals, void *rhs, int32_t *status)
{
    clear_error();
    fea_graph *g = const_cast<fea_graph *>(gc);
    fea_options dflt = {0, 0, 0, 0};
    const fea_options *o = opt ? opt : &dflt;
    int rc = check_assemble(g, x, y, z, types, conn_ptr, conn, mat, source, o, vals, rhs);
    if (rc) return rc;
    if (o->variant != FEA_ROWOWNER)
        return set_error(FEA_EINVAL, "fea_assemble_noalloc runs the row-owner variant only (variant %d)", o->variant);
    if (o->timing) return set_error(FEA_EINVAL, "fea_assemble_noalloc records no timing");
    const size_t cs = o->precision == FEA_FP64 ? sizeof(double) : sizeof(float);
    const size_t B = mat->model == FEA_POISSON ? 1 : 3;
    const size_t need_c = align256(cs * (size_t)g->map_len * B * B);
    const size_t need_r = align256(cs * (size_t)g->conn_len * B);
    if (kScratchHead + need_c + need_r > kScratchBytes)
        return set_error(FEA_ERANGE, "fea_assemble_noalloc: the workspace needs %zu bytes, more than its %zu-byte "
                                     "scratch", kScratchHead + need_c + need_r, kScratchBytes);
    if ((rc = noalloc_setup())) return rc;
    unsigned char *base = (unsigned char *)g_scratch[g->device];
    Workspace ws;
    ws.contrib = base + kScratchHead;
    ws.rcontrib = base + kScratchHead + need_c;
    g->timed = false;
    g->gtimed = false;
    int32_t *st = status ? status : (int32_t *)base;
    return assemble_impl(g, x, y, z, types, conn_ptr, conn, mat, source, o, stream, vals, rhs, st, ws);
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
