/*
 * fea.h -- C ABI of the MI355X (gfx950) finite-element assembly library.
 *
 * The library implements the element loop of the paper's Algorithm 1
 * (Section 2.1.1): for every element, the element matrix A^e and
 * right-hand side b^e are computed by Gauss quadrature and added into a
 * global block-sparse matrix A and vector b. The race on shared rows that
 * the paper's Section 3.2 treats with OpenMP ATOMIC (Algorithm 4) or element
 * colouring (Algorithm 5) is treated here by selectable scatter variants.
 *
 * Conventions shared by every entry point
 *   - Element families (types[e]): 0 = tet4, 1 = pyr5, 2 = pen6, 3 = hex8,
 *     with 4, 5, 6, 8 nodes; node order and reference elements as in the
 *     library documentation (hex8 nodes (-1,-1,-1),(1,-1,-1),(1,1,-1),
 *     (-1,1,-1) then the same at zeta = +1; pen6 triangle (0,0),(1,0),(0,1)
 *     at t = -1 then t = +1; tet4 (0,0,0),(1,0,0),(0,1,0),(0,0,1); pyr5 base
 *     counter-clockwise seen from the apex, then the apex).
 *   - Connectivity: conn_ptr[n_elems+1] (int64, conn_ptr[0] = 0) and
 *     conn[conn_ptr[n_elems]] (int32 node ids, zero-based).
 *   - Block sparsity: rows and columns are nodes; row i lists every node
 *     sharing an element with i, diagonal included, columns strictly
 *     ascending. Poisson uses 1x1 blocks (CSR), elasticity 3x3 blocks (BSR,
 *     block row-major: vals[9k + 3i + j], dof = 3*node + i).
 *   - e2nnz[map_ptr[e] + a*n_e + b] = block index of (conn[e][a], conn[e][b]);
 *     map_ptr is the prefix sum of n_e^2. The inverse map lists, for block k,
 *     the slots inv[inv_ptr[k] .. inv_ptr[k+1]) in ascending element order.
 *   - Pointers named "device" must point to device memory of the current
 *     HIP device; the caller keeps ownership. All work is enqueued on the
 *     given stream; functions return after enqueueing unless stated.
 *   - Return values: FEA_OK (0) or a negative FEA_E* code; fea_last_error()
 *     then returns a message for the calling thread.
 */
#ifndef FEA_H
#define FEA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEA_OK 0
#define FEA_EINVAL (-1) /* bad argument (NULL where required, bad option)   */
#define FEA_EMESH (-2)  /* bad mesh: unknown type, node id out of range,
                           repeated node in an element, wrong conn_ptr span  */
#define FEA_ENOMEM (-3) /* device or host allocation failed                 */
#define FEA_EHIP (-4)   /* a HIP runtime call failed                         */
#define FEA_ERANGE (-5) /* a size exceeds the library's index limits         */

enum fea_precision { FEA_FP64 = 0, FEA_MIXED = 1 };
/* Scatter variants (Section 3.2 of the paper treats the same race):
 *   ROWOWNER  element kernel writes each block contribution to its own slot
 *             in a workspace; a second kernel sums every block's
 *             contributions in ascending element order (deterministic,
 *             bitwise reproducible, independent of execution order);
 *   ATOMIC    element kernel adds into A and b with hardware atomics
 *             (the GPU counterpart of Algorithm 4);
 *   COLOUR    one launch per colour of a greedy element colouring, plain
 *             read-add-write (Algorithm 5); deterministic;
 *   ROWGATHER fused owner-computes: each row's owner recomputes the element
 *             rows that touch it and sums them in ascending element order
 *             (deterministic, no workspace, no atomics);
 *   ROWSYM    row-owner on the upper triangle: every element matrix here is
 *             symmetric (K_ba = K_ab^T), so each element computes its
 *             n(n+1)/2 blocks a <= b and stores each one, or its transpose,
 *             as the contribution to an upper block (i <= j); a lower block
 *             (j, i) is written as the transpose of the ordered sum of block
 *             (i, j), and each element's diagonal blocks are made
 *             symmetric by copying their upper entries (with 3x3 blocks,
 *             when the block values are written: the strictly lower
 *             entries of an element's diagonal block carry that node's
 *             right-hand side through the tile sums instead, so b needs no
 *             workspace or reduction of its own and equals the other
 *             forms' up to the rounding of that grouping). About 40% less
 *             element work and workspace traffic; deterministic, and A
 *             equals its transpose bitwise. Also runs batched
 *             (fea_batch_assemble);
 *   TILECOLOUR the GPU counterpart of commutative multidependences
 *             (Algorithm 7): the ROWSYM element tiles, greedily coloured in
 *             descending neighbour count so that no two tiles of a colour
 *             share a node (built by the first such call, on the host;
 *             fea_graph_tile_colouring exports it); one launch per
 *             (colour, family), its tiles in descending neighbour count,
 *             each tile adding its LDS tile sums and their transposes
 *             straight into FP64 block values (no block workspace, no
 *             atomics); right-hand side as ROWOWNER; deterministic.
 *             Single-mesh assembly only. */
enum fea_variant { FEA_ROWOWNER = 0, FEA_ATOMIC = 1, FEA_COLOUR = 2, FEA_ROWGATHER = 3, FEA_ROWSYM = 4,
                   FEA_TILECOLOUR = 5 };
enum fea_dtype { FEA_F64 = 0, FEA_F32 = 1 };
enum fea_model { FEA_POISSON = 0, FEA_ELASTIC = 1 };
enum fea_schedule { FEA_TYPE_SORTED = 0, FEA_LEARNED = 1, FEA_GP_WEIGHT = 2, FEA_LEARNED_CLASSES = 3 };

/* Options. A zero-initialised struct is FP64, row-owner, f64 output. */
typedef struct fea_options {
    int precision; /* enum fea_precision */
    int variant;   /* enum fea_variant */
    int out_dtype; /* enum fea_dtype: element type of vals and rhs */
    int timing;    /* nonzero: record HIP events around the phases of this
                      call on its stream (read with fea_last_timing) */
} fea_options;

/* Material and model. Per-element arrays are device pointers of length
 * n_elems; u is a device array of 3*n_nodes displacements (node-major). */
typedef struct fea_material {
    int model;              /* enum fea_model */
    const double *young;    /* Young's modulus per element; NULL = 1.0      */
    const double *nu;       /* Poisson ratio per element (elasticity)       */
    const uint8_t *nh_flag; /* NULL, or 1 = neo-Hookean tangent at u        */
    const double *u;        /* required when nh_flag is given or residual   */
    int residual;           /* nonzero: rhs is the Newton residual
                               b = f_ext - f_int(u) (Section 2.2), f_int the
                               neo-Hookean internal force sum_q w detJ P
                               grad N_a where nh_flag is set, the linear-
                               elastic one (sum_q w detJ sigma grad N_a =
                               K^e u^e) elsewhere; FEA_ELASTIC, FP64 and
                               the element-tile scatter forms only (not
                               FEA_ROWGATHER): FEA_EINVAL otherwise */
} fea_material;

typedef struct fea_graph fea_graph;

/*
 * Builds the block sparsity pattern, the element-to-nonzero map, the
 * inverse map, the node-to-element incidence, the type segmentation
 * (elements stably sorted by family) and a greedy element colouring from
 * the connectivity (device pointers). The graph keeps its own device
 * buffers until fea_graph_destroy. Blocks on `stream` (it must learn the
 * number of nonzeros). Errors: FEA_EINVAL, FEA_EMESH (the message names the
 * first bad element), FEA_ERANGE (more than 2^31-1 nonzero blocks or
 * slots), FEA_ENOMEM, FEA_EHIP. Nodes in no element get empty rows.
 */
int fea_graph_build(int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                    const int64_t *conn_ptr, const int32_t *conn, hipStream_t stream,
                    fea_graph **out);

/* Graph cache (a checkpoint of the graph, so that a later run can skip
 * fea_graph_build): fea_graph_save writes the graph's pattern, maps,
 * incidence, type segmentation and colouring to `path` (binary: a header
 * with a magic string, format version, the GPU architecture name, the
 * sizes and a fingerprint of the mesh's connectivity, then the arrays);
 * the layouts built on first use by FEA_ROWSYM, FEA_TILECOLOUR and
 * FEA_ROWGATHER are not saved (the first such call builds them again).
 * Synchronises the device. fea_graph_load reads such a file for the mesh
 * given (device arrays as fea_graph_build, which it validates the same
 * way) on `stream`, into a new graph equal to the one saved, for callers
 * that assemble the same mesh in several processes. Errors: FEA_EINVAL
 * (cannot open or write the file, not a graph cache, another format
 * version, written on another GPU architecture, mesh sizes or connectivity
 * fingerprint differ from the saved graph's, file truncated), FEA_EMESH
 * (invalid mesh), FEA_ENOMEM, FEA_EHIP. */
int fea_graph_save(const fea_graph *g, const char *path);
int fea_graph_load(const char *path, int64_t n_nodes, int64_t n_elems, const uint8_t *types,
                   const int64_t *conn_ptr, const int32_t *conn, hipStream_t stream, fea_graph **out);

/* Sizes: nodes (block rows), elements, nonzero blocks, slots (sum n_e^2),
 * colours. Any output pointer may be NULL. */
int fea_graph_sizes(const fea_graph *g, int64_t *n_nodes, int64_t *n_elems,
                    int64_t *nnz_blocks, int64_t *map_len, int *n_colours);

/* Sizes of the upper-triangle (FEA_ROWSYM) layout, built by the first
 * FEA_ROWSYM assembly on the graph: element tiles (per family, 256 / (n(n+1)/2)
 * consecutive elements of the type-sorted order), tile entries (one per
 * (element, local pair a <= b), two where nodes a and b coincide), tile-blocks
 * (distinct (tile, upper block) pairs = workspace slots, each 3x3 or 1x1) and
 * upper blocks (col >= row). Any output pointer may be NULL. FEA_EINVAL if the
 * layout has not been built yet. */
int fea_graph_sym_sizes(const fea_graph *g, int64_t *tiles, int64_t *entries, int64_t *tile_blocks,
                        int64_t *upper_blocks);

/* The tile colouring of FEA_TILECOLOUR (built by the first such call; the
 * counterpart of Algorithm 7's commutative multidependences with priority
 * by neighbour count, Section 3.2): tiles sharing a node are neighbours,
 * nneig is a tile's neighbour count, tiles are coloured greedily (first fit)
 * in descending nneig, ties by tile index. *n_colours = C; bucket_ptr (HOST
 * int64[4 * (C + 1)]): family t's colour-c tiles are
 * tiles[bucket_ptr[t*(C+1)+c] .. bucket_ptr[t*(C+1)+c+1]) (the end of
 * family t's last colour is the start of family t+1's first); tiles (DEVICE
 * int32[n_tiles], enqueued on `stream`): family-local tile indices in launch
 * order, descending nneig within a bucket; nneig (HOST int32[n_tiles]):
 * the neighbour count of every tile, families in order (tile
 * fea_graph_sym_sizes order). Any output may be NULL. FEA_EINVAL if the
 * colouring has not been built. */
int fea_graph_tile_colouring(const fea_graph *g, int *n_colours, int64_t *bucket_ptr, int32_t *tiles,
                             int32_t *nneig, hipStream_t stream);

/* Copies graph arrays into caller-owned DEVICE buffers (any may be NULL):
 * row_ptr[n_nodes+1], col[nnz], map_ptr[n_elems+1], e2nnz[map_len],
 * inv_ptr[nnz+1], inv[map_len], colour[n_elems], type_perm[n_elems]
 * (element ids sorted stably by type) and type_seg[5] (HOST array: segment
 * offsets of the four families in type_perm). Enqueued on `stream`. */
int fea_graph_export(const fea_graph *g, int64_t *row_ptr, int32_t *col, int64_t *map_ptr,
                     int32_t *e2nnz, int64_t *inv_ptr, int32_t *inv, int16_t *colour,
                     int32_t *type_perm, int64_t *type_seg, hipStream_t stream);

void fea_graph_destroy(fea_graph *g);

/*
 * Assembles A (vals, nnz*b*b) and b (rhs, n_nodes*b), b = 1 for Poisson and
 * 3 for elasticity, overwriting both (caller-owned device buffers of the
 * element type opt->out_dtype). x, y, z: device FP64 node coordinates;
 * types/conn_ptr/conn: the device arrays the graph was built from; source:
 * device FP64 per-element constant source, b values per element.
 * status (device int32, may be NULL) receives the smallest element id whose
 * Jacobian determinant (or deformation-gradient determinant) is not
 * positive at a Gauss point, or -1. Enqueued on `stream`; the first call
 * with a given variant may allocate a workspace held by the graph.
 * FEA_ROWGATHER: the first call on a graph builds the row tiles and blocks
 * on `stream`; a
 * node may lie in at most 64 elements (and its elements may hold at most
 * 256 nodes and 384 Gauss points in total), else FEA_ERANGE naming the node.
 * Errors: FEA_EINVAL (NULL pointer, bad option), FEA_ERANGE, FEA_ENOMEM,
 * FEA_EHIP.
 */
int fea_assemble(const fea_graph *g, const double *x, const double *y, const double *z,
                 const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                 const fea_material *mat, const double *source, const fea_options *opt,
                 hipStream_t stream, void *vals, void *rhs, int32_t *status);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * FEA_ROWOWNER assembly of fea_assemble, with the same kernels and a
 * bitwise equal result, that calls no hipMalloc, hipFree or allocating
 * library routine. Its slot and right-hand-side workspaces live in one
 * static device array of 256 MiB held by every GPU the library runs on
 * until the process ends (set up by fea_graph_build on that device).
 * Arguments as fea_assemble; opt->variant must be FEA_ROWOWNER and
 * opt->timing 0 (else FEA_EINVAL). The workspaces need
 * sizeof(compute type) * (map_len * b * b + n_conn * b) bytes (each part
 * rounded up to 256, plus 256), b = 1 (Poisson) or 3; larger meshes get
 * FEA_ERANGE before anything is enqueued. status may be NULL (the scratch
 * then holds it). Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams, other threads) race: order them.
 */
int fea_assemble_noalloc(const fea_graph *g, const double *x, const double *y, const double *z,
                         const uint8_t *types, const int64_t *conn_ptr, const int32_t *conn,
                         const fea_material *mat, const double *source, const fea_options *opt,
                         hipStream_t stream, void *vals, void *rhs, int32_t *status);

/* Phase durations of the graph's last fea_assemble call made with
 * opt->timing set, in milliseconds, measured with HIP events on that call's
 * stream: ms[0] element kernels (with the fused scatter for ATOMIC, COLOUR
 * and TILECOLOUR, and all of ROWGATHER; for ROWOWNER, and ROWSYM with 1x1
 * blocks, also the right-hand-side reduction, which runs first), ms[1] the
 * one kernel that forms the matrix values after them (ROWOWNER/ROWSYM: the
 * segmented reduction of the block values, for ROWSYM with 3x3 blocks also
 * of the right-hand side; ATOMIC/COLOUR/TILECOLOUR with FP32 output:
 * the conversion; otherwise empty), ms[2] the whole call including
 * zero-fill and the right-hand side. Waits for the events. FEA_EINVAL if no
 * timed call was made. */
int fea_last_timing(const fea_graph *g, float *ms);

/* Durations (ms, HIP events on the call's stream) of the five kernels of
 * the graph's last timed FEA_ROWGATHER assembly, one per row-tile class:
 * ms[0..3] rows whose elements are all tet4, pyr5, pen6, hex8, ms[4] rows
 * on family interfaces (0 for a class with no rows). Waits for the events.
 * FEA_EINVAL if the last timed assembly was not FEA_ROWGATHER. */
int fea_last_class_timing(const fea_graph *g, float *ms);

/* ------------------------------------------------------------------ *
 * Subgrid scale: an element loop with nothing assembled.              *
 * ------------------------------------------------------------------ */

/* Gauss-point layout of a graph's elements (the first call builds it on
 * `stream` and blocks on it once): *n_points (may be NULL) = total Gauss
 * points (tet4 1, pyr5 8, pen6 6, hex8 8 per element); gp_ptr (caller-owned
 * DEVICE buffer of n_elems+1 int64, may be NULL) receives the offsets in
 * element order, element e's points at gp_ptr[e] .. gp_ptr[e+1], enqueued on
 * `stream`. Errors: FEA_EINVAL, FEA_ENOMEM, FEA_EHIP. */
int fea_graph_gauss_points(const fea_graph *g, int64_t *n_points, int64_t *gp_ptr, hipStream_t stream);

/*
 * Subgrid scale (Section 2.1.3: the subscale is obtained element by element
 * from the strong residual at the Gauss points and a diagonal stabilisation
 * matrix, in a loop over the elements that forms no system). For the linear
 * models, at every Gauss point q of every element e, in FP64:
 *   out[(gp_ptr[e] + q)*b + c] = tau_e (f_e,c + L(u_h)_c(x_q)),
 * L = Laplacian (FEA_POISSON, b = 1) or div sigma = mu Lap u +
 * (lam + mu) grad div u (FEA_ELASTIC, b = 3, lam and mu from young and nu
 * per element); u_h interpolates the nodal field u; tau_e = V_e^(2/3) / (4k)
 * with V_e = sum_q w_q detJ_q and k = 1 (Poisson) or mu_e (elasticity).
 * x, y, z: device FP64 node coordinates; u: device FP64 nodal field, b
 * values per node (node-major); source: device FP64, b values per element;
 * out: caller-owned device FP64 buffer of n_points*b values (gp_ptr and
 * n_points from fea_graph_gauss_points), overwritten. mat->nh_flag must be
 * NULL (FEA_EINVAL); mat->u and mat->residual are not used. status (device
 * int32, may be NULL) receives the smallest element id with detJ <= 0 at a
 * Gauss point (that element's outputs are then unspecified), or -1.
 * Enqueued on `stream` (the first call on a graph builds the Gauss-point
 * layout and blocks once). Errors: FEA_EINVAL, FEA_ENOMEM, FEA_EHIP.
 */
int fea_subscale(const fea_graph *g, const double *x, const double *y, const double *z,
                 const fea_material *mat, const double *u, const double *source, hipStream_t stream,
                 double *out, int32_t *status);

/* ------------------------------------------------------------------ *
 * Batched assembly: many independent meshes in one persistent launch. *
 * ------------------------------------------------------------------ */

/* One mesh of a batch. All pointers are device pointers owned by the
 * caller and must stay valid while the batch is used; fields as in
 * fea_assemble (source: b values per element; nh_flag/u may be NULL). */
typedef struct fea_mesh_desc {
    int64_t n_nodes, n_elems;
    const uint8_t *types;
    const int64_t *conn_ptr;
    const int32_t *conn;
    const double *x, *y, *z;
    const double *young, *nu;
    const uint8_t *nh_flag;
    const double *u;
    const double *source;
} fea_mesh_desc;

typedef struct fea_batch fea_batch;

/*
 * Builds a graph per mesh and the work items of one persistent launch. A
 * work item is `count` consecutive elements of one family of one mesh, in
 * that mesh's type-sorted element order; tile[f] (elements per item for
 * family f = tet4, pyr5, pen6, hex8; NULL = defaults 75, 34, 24, 14) sets
 * the item sizes, each rounded up to a multiple of the family's
 * upper-triangle tile (25, 17, 12, 7 elements), so that items start on
 * tile boundaries in every form.
 * The paper's dynamic schedule with a chunk size (Section 5.2, chunk study)
 * is the analogue: items are chunks handed out by a device work queue.
 * The queue order starts type-sorted (family, mesh, first element).
 * Outputs of all meshes are concatenated: mesh m's values start at
 * vals_off[m] and its right-hand side at rhs_off[m] (fea_batch_offsets).
 * model: enum fea_model, common to all meshes. Blocks on `stream`.
 * Errors as fea_graph_build (the message names the mesh), FEA_EINVAL.
 */
int fea_batch_build(int n_meshes, const fea_mesh_desc *meshes, int model, const int32_t *tile,
                    hipStream_t stream, fea_batch **out);

/* Totals: value and right-hand-side lengths (scalars), work items, elements. */
int fea_batch_sizes(const fea_batch *b, int64_t *vals_len, int64_t *rhs_len, int64_t *n_items,
                    int64_t *n_elems);

/* HOST arrays of n_meshes+1 scalar offsets into vals and rhs. */
int fea_batch_offsets(const fea_batch *b, int64_t *vals_off, int64_t *rhs_off);

/* HOST array of n_items x 4 int32: mesh, family, first element, count. */
int fea_batch_items(const fea_batch *b, int32_t *items);

/* Replaces the work items with new per-family tile sizes (resets the
 * queue order to type-sorted and drops a captured graph). */
int fea_batch_set_tiles(fea_batch *b, const int32_t *tile);

/* Sets the queue order: HOST permutation of 0..n_items-1, item order[j] is
 * dequeued j-th among the items of its family (each family has its own
 * persistent launch and queue, in family order). Returns to the dynamic
 * queue and drops a captured graph. FEA_EINVAL if not a permutation. */
int fea_batch_set_order(fea_batch *b, const int32_t *order);

/* The current queue order (HOST int32[n_items]): the permutation set by
 * fea_batch_set_order or fea_batch_order (identity after fea_batch_build,
 * fea_batch_set_tiles and fea_batch_partition). */
int fea_batch_get_order(const fea_batch *b, int32_t *order);

/*
 * One batched assembly on `stream`: reset the queue heads, one persistent
 * kernel per element family, each dequeuing that family's items in queue
 * order (row-owner slot contributions, FP64 or mixed per opt->precision),
 * then the block-value and right-hand-side reductions over all meshes.
 * vals/rhs: device buffers of the lengths from fea_batch_sizes, element
 * type opt->out_dtype, overwritten. status: device int32[n_meshes] (may be
 * NULL), per mesh the smallest rejected element id or -1. opt->variant:
 * FEA_ROWOWNER as above; FEA_ROWSYM: the same items run as element tiles
 * with their LDS tile sums (upper-triangle form, as in fea_assemble; the
 * first such call builds every mesh's tile layout, blocking on `stream`),
 * then the upper-triangle block values over all meshes, bitwise equal to
 * one-mesh FEA_ROWSYM assemblies; or FEA_ROWGATHER: the row tiles of all meshes in
 * one persistent launch per tile class, written straight into vals/rhs
 * (the first such call prepares every mesh's tiles and blocks on `stream`;
 * no work queue, no cycle records, tiles and queue order do not apply).
 * With opt->timing, fea_batch_last_ms reads the persistent kernels'
 * duration.
 */
int fea_batch_assemble(fea_batch *b, const fea_options *opt, hipStream_t stream, void *vals,
                       void *rhs, int32_t *status);

/* Captures the sequence of fea_batch_assemble into a HIP graph (stream
 * capture on `stream`, which must not be the legacy default stream) and
 * keeps the executable graph in the batch; fea_batch_replay launches it
 * `n` times on `stream`. The captured graph contains kernels only. */
int fea_batch_capture(fea_batch *b, const fea_options *opt, hipStream_t stream, void *vals,
                      void *rhs, int32_t *status);
int fea_batch_replay(fea_batch *b, int n, hipStream_t stream);

/* Per-item records of the last persistent launch, copied into DEVICE
 * buffers of n_items entries (any may be NULL): shader-clock cycles from
 * the item's dequeue to its completion, the workgroup that ran it and the
 * compute unit (hardware id). */
int fea_batch_cycles(const fea_batch *b, uint64_t *cycles, int32_t *worker, int32_t *cu,
                     hipStream_t stream);

/* Duration in ms of the persistent kernel of the last timed assemble. */
int fea_batch_last_ms(const fea_batch *b, float *ms);

/* Number of persistent workgroups (workers) the batch launches. */
int fea_batch_workers(const fea_batch *b, int *workers);

void fea_batch_destroy(fea_batch *b);

/* Gauss-point offsets of a batch's meshes in the concatenated subgrid-scale
 * output: offsets (HOST array of n_meshes+1, may be NULL) receives the
 * first Gauss point of every mesh and the total. The first call builds each
 * mesh's Gauss-point layout on `stream` and blocks. Errors: FEA_EINVAL,
 * FEA_ENOMEM, FEA_EHIP. */
int fea_batch_gauss_points(fea_batch *b, int64_t *offsets, hipStream_t stream);

/*
 * Batched subgrid scale (Section 2.1.3, as fea_subscale, FEA_ELASTIC): work
 * items of its own (runs of four element groups of one family of one mesh:
 * 1024 tet4, 128 pyr5, 168 pen6 or 128 hex8 elements; built by the first
 * call, independent of the assembly's tile sizes) dequeued by persistent
 * workgroups, one launch and queue per element family, with each mesh's
 * coordinates, material, source and displacement u (its fea_mesh_desc) as
 * the field; nothing is assembled. Mesh m's Gauss point
 * q of element e is row offsets[m] + gp_ptr_m[e] + q of out (device FP64,
 * 3 values per Gauss point, offsets from fea_batch_gauss_points),
 * overwritten; the values equal fea_subscale's for that mesh. status
 * (device int32[n_meshes], required unless the batch has no mesh) receives
 * per mesh the smallest element
 * id with detJ <= 0, or -1. Enqueued on `stream`; the first call, and a
 * call with other output or status pointers, builds a small argument table
 * and blocks on `stream` first. Meshes with neo-Hookean
 * flags, a missing u, nu, source or coordinate array, or a batch of
 * another model: FEA_EINVAL.
 */
int fea_batch_subscale(fea_batch *b, hipStream_t stream, double *out, int32_t *status);

/*
 * Tile autotuner: chooses the elements per work item of each family by
 * timing the batch's persistent kernel (the GPU counterpart of the paper's
 * chunk-size study, Section 5.2). Coordinate descent from the batch's
 * current tiles: for each family in turn the candidates
 * EPB*{1,2,3,4,6,8,12,16,24,32} are tried with the other tiles fixed (EPB =
 * the upper-triangle tile: 25 tet4, 17 pyr5, 12 pen6, 7 hex8), two sweeps,
 * each candidate timed as the median of `reps` launches of opt->variant
 * (FEA_ROWOWNER or FEA_ROWSYM) and taken only if at least 1% faster than
 * the best so far (smaller gains are within run-to-run noise). The best tiles
 * are applied to the batch, returned in tile_out
 * (HOST int32[4]) and, if table_path is not NULL, stored in that text file
 * under the key (gfx950, model, precision). Allocates temporary outputs.
 */
int fea_batch_autotune(fea_batch *b, const fea_options *opt, int reps, const char *table_path,
                       hipStream_t stream, int32_t *tile_out);

/* Reads the tiles stored for (gfx950, model, precision) from a table file
 * written by fea_batch_autotune. FEA_EINVAL if the file has no such entry. */
int fea_tile_table_load(const char *table_path, int model, int precision, int32_t *tile_out);

/*
 * Queue order of a batch (enum fea_schedule):
 *   FEA_TYPE_SORTED  items by (family, mesh, first element): the static
 *                    fallback;
 *   FEA_GP_WEIGHT    largest first by (Gauss points x elements), the paper's
 *                    a-priori element weight (Section 4.1);
 *   FEA_LEARNED      largest first by pred[item] (device float[n_items],
 *                    e.g. fea_cost_predict output), ties by item index;
 *   FEA_LEARNED_CLASSES  largest cost class first, the items of a class in
 *                    type-sorted order: with pred a predicted log-cost, an
 *                    item's class is round((pred[item] - med) / ln 2), med
 *                    the lower median of pred over its family's items (in
 *                    double precision; round = floor(x + 0.5)). Exact
 *                    longest-first order scatters items of near-equal cost
 *                    across the mesh, and with them the nodes and cache
 *                    lines that neighbouring items share; classes a factor
 *                    of two wide still start the expensive items first.
 * Drops a captured graph. Waits on `stream` to read pred. FEA_EINVAL if
 * pred is NULL or holds a value that is not finite (learned schedules).
 */
int fea_batch_order(fea_batch *b, int schedule, const float *pred, hipStream_t stream);

/*
 * Static partition instead of the dynamic queue: the items, in type-sorted
 * order (neighbouring elements stay together), are split, family by
 * family, into one contiguous range per persistent workgroup of that
 * family's launch with nearly equal total weight, and every workgroup runs
 * its own range without touching the queue head.
 * The counterpart of the paper's weighted partitions (Section 4.1):
 * weights = FEA_TYPE_SORTED: element count (non-weighted); FEA_GP_WEIGHT:
 * Gauss points x elements; FEA_LEARNED: exp(pred[item]) with pred a
 * predicted log-cost (device float[n_items]). fea_batch_order returns to
 * the dynamic queue. Drops a captured graph.
 */
int fea_batch_partition(fea_batch *b, int weights, const float *pred, hipStream_t stream);

/*
 * Cost-model features of every work item (device float[n_items x 12]),
 * per item: family one-hot (4), fraction of neo-Hookean elements,
 * log2(element count), log2 of the node-id span per element node
 * (a locality proxy), mean Poisson ratio, log of the mean and of the
 * largest element distortion max_q detJ / min_q detJ, log10 of the mean
 * element volume, and `fp64_geometry` (1 when the geometry runs in FP64).
 */
int fea_batch_features(const fea_batch *b, int fp64_geometry, float *feats, hipStream_t stream);

/* ------------------------------------------------------------------ *
 * Learned cost model: a 12 -> 64 -> 64 -> 1 ReLU perceptron (FP32)      *
 * predicting log(cycles) of a work item. The paper finds that element   *
 * cost cannot be known a priori and that Gauss-point weights balance    *
 * poorly (abstract; Section 4.1); this model learns the weight from the *
 * cycle counts the batched assembly records.                           *
 * Parameters: W1[64][12], b1[64], W2[64][64], b2[64], W3[64], b3 (5,057). *
 * Inputs are standardised with a per-feature mean and scale.           *
 * ------------------------------------------------------------------ */
typedef struct fea_cost fea_cost;

#define FEA_COST_FEATURES 12
#define FEA_COST_PARAMS 5057

/* He-normal weights (seeded, counter-based generator), zero biases,
 * mean 0 / scale 1, Adam state zero. */
int fea_cost_create(uint64_t seed, fea_cost **out);
void fea_cost_destroy(fea_cost *c);

/* HOST copies of the parameters (float[5057]) and of the input
 * standardisation (float[12] each). */
int fea_cost_get_params(const fea_cost *c, float *params);
int fea_cost_set_params(fea_cost *c, const float *params);
int fea_cost_set_norm(fea_cost *c, const float *mean, const float *scale);

/* Sets the standardisation from device features (float[n x 12]): mean and
 * population standard deviation per feature (scale 1 where it is 0). */
int fea_cost_fit_norm(fea_cost *c, const float *feats, int64_t n, hipStream_t stream);

/* pred[i] = model(feats[i]) for i < n (device arrays). */
int fea_cost_predict(const fea_cost *c, const float *feats, int64_t n, float *pred,
                     hipStream_t stream);

/* Mean squared error against target (device float[n]) and its gradient
 * (device float[5057], parameter order), reduced in a fixed order. */
int fea_cost_grad(const fea_cost *c, const float *feats, const float *target, int64_t n,
                  float *grad, float *loss, hipStream_t stream);

/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, step
 * size lr); loss_hist (device float[steps], may be NULL) receives the loss
 * before each step. */
int fea_cost_train(fea_cost *c, const float *feats, const float *target, int64_t n, int steps,
                   float lr, float *loss_hist, hipStream_t stream);

/* target[i] = log(cycles[i]) (device arrays). */
int fea_cost_log_cycles(const uint64_t *cycles, int64_t n, float *target, hipStream_t stream);

/* Binary checkpoint: magic, version, "gfx950", standardisation, parameters,
 * Adam moments and step count. */
int fea_cost_save(const fea_cost *c, const char *path);
int fea_cost_load(fea_cost *c, const char *path);

/* Message for the last error on the calling thread ("" if none). */
const char *fea_last_error(void);

/* Library version string. */
const char *fea_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FEA_H */
