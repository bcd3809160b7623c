/*
 * msc.h -- C-ABI of libmsc.so: path-compression Morse-Smale segmentation and
 * connected components on AMD Instinct MI355X (gfx950).
 *
 * Method: Will, Lukasczyk, Tierny, Garth, "Distributed Path Compression for
 * Piecewise Linear Morse-Smale Segmentations and Connected Components",
 * arXiv 2409.03771.
 *
 * General rules for every entry point:
 *  - Buffers named "device" are device pointers on the context's GPU, owned
 *    by the caller; the library never frees or keeps them past the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is enqueued on it.  msc_segment,
 *    msc_segment_batched, cc_label_grid and cc_label_grid_batched return
 *    with their work only enqueued (the host waits only when a workspace has
 *    to grow, or when more than four segmentation calls of one context are
 *    still running: the oldest is waited for); their
 *    outputs are complete once `stream` has completed, and conditions that
 *    the device detects (a NaN in a field) are reported afterwards by
 *    msc_last_status and the stats calls.  Calls documented as synchronising
 *    read counts back and return when their work is done.  Calls on one
 *    context are ordered in call order even across streams (a call on
 *    another stream waits for the previous call's work on the device).
 *  - Outputs must not alias inputs or each other.
 *  - Return value: MSC_OK (0) or one of the MSC_E* codes below; nothing is
 *    thrown across the ABI.  On an error the contents of the outputs are
 *    unspecified.  msc_strerror() names a code.
 *  - A context is not thread-safe: one host thread at a time per context.
 *
 * Grids: dims = {X, Y, Z}, every entry >= 1.  Vertex (x, y, z) has id
 * x + X*y + X*Y*z and arrays are stored in id order (x fastest).  The grid is
 * triangulated by the Freudenthal (Kuhn) subdivision: vertex v is adjacent to
 * v + (dx,dy,dz) for the 14 non-zero offsets with entries all in {0,1} or all
 * in {0,-1}, when that vertex lies inside the grid.  Degenerate grids (Z = 1,
 * or Y = Z = 1) are the 2-D and 1-D restrictions of the same rule.
 */
#ifndef MSC_H
#define MSC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define MSC_API __attribute__((visibility("default")))
#else
#define MSC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MSC_OK = 0,
  MSC_EINVAL = 1,  /* bad dims, NULL required pointer, bad argument       */
  MSC_ERANGE = 2,  /* vertex count does not fit the id type of an output  */
  MSC_ENAN = 3,    /* NaN in the scalar field: there is no total order    */
  MSC_ENOMEM = 4,  /* device workspace could not be allocated             */
  MSC_EBUDGET = 5, /* request larger than a queue's memory budget         */
  MSC_EHIP = 6,    /* a HIP runtime call failed                           */
  MSC_ECANCELED = 7,/* request cancelled before it ran                     */
  MSC_EBUSY = 8    /* ticket not finished (msc_poll)                      */
};

/* Kinds of work: segmentation of a float32 field, CC of a grid mask. */
enum { MSC_REQ_SEGMENT = 1, MSC_REQ_CC_GRID = 2 };

/*
 * Host-side fault injection, for tests of the error paths (failure
 * detection): after `after` more checks of the given kind succeed, the next
 * one fails, once.  MSC_INJECT_ENOMEM fails a device or pinned host
 * allocation of the library (nothing is allocated; the call reports
 * MSC_ENOMEM); MSC_INJECT_EHIP makes a checked HIP runtime call report
 * failure after it has run (the call reports MSC_EHIP; work it already
 * enqueued runs normally).  after < 0 disarms.  Process-wide, thread-safe;
 * no device is touched.  Errors: MSC_EINVAL (unknown kind).
 */
enum { MSC_INJECT_ENOMEM = 1, MSC_INJECT_EHIP = 2 };
MSC_API int msc_debug_inject(int what, int after);

typedef struct msc_ctx msc_ctx;

/* Static string for an error code (never NULL). */
MSC_API const char *msc_strerror(int code);

/* Create a context on HIP device `device`.  The context owns a growable
 * device workspace (allocated lazily).  *out is NULL on failure. */
MSC_API int msc_create(msc_ctx **out, int device);

/* Release the context and its workspace.  Synchronises the device first.
 * NULL is ignored. */
MSC_API void msc_destroy(msc_ctx *ctx);

/*
 * Caller-owned workspace.  msc_set_workspace makes the context carve every
 * call's per-call scratch from `ptr` (device memory of the context's GPU,
 * 256-byte aligned, `bytes` long) instead of memory it allocates: a call
 * whose scratch does not fit returns MSC_ENOMEM and allocates nothing for
 * it.  msc_segment, msc_segment_batched, cc_label_grid and
 * cc_label_grid_batched need nothing else; the virtual-rank calls and
 * msc_segment_csr also keep buffers of their own that the library
 * allocates.  ptr == NULL returns to a library-owned workspace.  Waits for the context's earlier work (the old
 * workspace may still be in use); the memory must stay valid, and unused by
 * anything else while the context's work runs, until it is replaced or the
 * context is destroyed.
 *  Errors: MSC_EINVAL (ctx NULL, ptr misaligned, bytes < 4096 with ptr set),
 *  MSC_EHIP.
 *
 * msc_workspace_size: the scratch bytes one call needs, with the context's
 * current tile shape: kind MSC_REQ_SEGMENT for msc_segment_batched over
 * `n` msc_field descriptors, MSC_REQ_CC_GRID for cc_label_grid_batched over
 * `n` msc_mask descriptors (n = 1: msc_segment / cc_label_grid).  Only the
 * descriptors' dims and which outputs are NULL are read.
 *  Errors: MSC_EINVAL, MSC_ERANGE (the call itself would fail with it).
 */
MSC_API int msc_set_workspace(msc_ctx *ctx, void *ptr, size_t bytes);
MSC_API int msc_workspace_size(const msc_ctx *ctx, int kind, int n,
                               const void *descs, size_t *bytes);

/*
 * Morse-Smale segmentation of a float32 scalar field on a grid.
 *
 * Paper: the input is a PL scalar field on a simplicial complex (background,
 * "Scalar Fields"); vertices are totally ordered by (value, global id), the
 * simulation-of-simplicity order of the preprocessing section.  Each vertex
 * points to the largest vertex of its closed neighbourhood (Alg. 1,
 * initialisation) and pointer jumping compresses every path onto its
 * extremum (Alg. 1, main loop); the same is done downwards, and vertices
 * whose two extrema agree form one Morse-Smale cell (methods, "Ascending and
 * Descending Segmentation").
 *
 *  field  device, float32[N], N = X*Y*Z, read only.  No value may be NaN.
 *         Values are compared as IEEE floats (-0.0 == +0.0, so the id
 *         decides); they are never converted.
 *  dims   host, int64[3] = {X, Y, Z}.
 *  asc    device, int32[N] or NULL: id of the maximum reached by steepest
 *         ascent from each vertex (the paper's "descending manifold").
 *  desc   device, int32[N] or NULL: id of the minimum reached by steepest
 *         descent (the paper's "ascending manifold").
 *  ms     device, int32[N] or NULL: Morse-Smale cell id = smallest vertex id
 *         u with asc[u] == asc[v] and desc[u] == desc[v].
 *  Asynchronous on `stream`.  Workspace (device, held by the context):
 *  about 9.5 bytes per vertex with 32x16x16 tiles, plus a cell table of
 *  which at most 2 * N slots of 12 bytes are reserved and only the part the
 *  extremum counts call for is used; msc_workspace_size gives the exact
 *  figure.  Labels passed as NULL are neither written nor kept.
 *  Errors returned: MSC_EINVAL (dims < 1, field NULL, all outputs NULL),
 *          MSC_ERANGE (N > INT32_MAX), MSC_ENOMEM, MSC_EHIP.
 *  Reported by msc_last_status after the work has run: MSC_ENAN (outputs
 *  undefined), MSC_EHIP (a broken internal invariant).
 */
MSC_API int msc_segment(msc_ctx *ctx, const float *field, const int64_t dims[3],
                int32_t *asc, int32_t *desc, int32_t *ms, void *stream);

/*
 * The paper's distributed scheme (Alg. 1 and 2) with `ranks` virtual ranks
 * on one device, for comparison with the single-domain path: the z-extent
 * is split into `ranks` slabs of planes [r*Z/ranks, (r+1)*Z/ranks); each
 * slab is segmented as a field of its own together with one ghost plane on
 * each side that has a neighbour, the ghost vertices being fixed points
 * (Alg. 1's ghost rule); the exchange then gives every ghost vertex its
 * owner's result, compresses that ghost graph and relabels every vertex
 * whose slab result is a ghost (Alg. 2); cells are paired over the final
 * labels.  Outputs, layout and errors as msc_segment, and bit-identical to
 * it; MSC_EINVAL also for ranks < 1 or ranks > Z.  msc_last_stats reports
 * the final extremum and cell counts.
 */
MSC_API int msc_segment_ranks(msc_ctx *ctx, const float *field,
                              const int64_t dims[3], int ranks, int32_t *asc,
                              int32_t *desc, int32_t *ms, void *stream);

/*
 * msc_segment on a general simplicial complex given by the adjacency of its
 * vertices (the problem statement's K; a grid is one case): steepest
 * ascent / descent over the closed neighbourhood {v} u row(v) in the
 * (value, id) order, path compression onto the extrema, cells as for the
 * grid.
 *
 *  n        number of vertices (0 is a no-op, whatever the pointers; at
 *           most INT32_MAX).
 *  row_ptr  device, int64[n+1], row_ptr[0] = 0, non-decreasing.
 *  col_idx  device, int32[row_ptr[n]] (may be NULL when row_ptr[n] is 0;
 *           rows are only read inside [0, row_ptr[n])): the neighbours of v are
 *           col_idx[row_ptr[v] .. row_ptr[v+1]).  For the paper's
 *           semantics the rows are the symmetric 1-skeleton adjacency; the
 *           call uses each row as given (an edge listed in one row only is
 *           seen from that vertex only).  Entries equal to v are harmless.
 *  field    device, float32[n], values in vertex-id order.
 *  asc, desc, ms  as msc_segment (device int32[n], any may be NULL, not
 *           all); asc and desc are computed in place of the caller's
 *           buffers when given, in library scratch otherwise.
 *  Errors: MSC_EINVAL (NULL arguments, n < 0, a column index outside
 *          [0, n): outputs undefined), MSC_ERANGE, MSC_ENAN, MSC_ENOMEM,
 *          MSC_EHIP.  msc_last_stats reports extremum and cell counts.
 */
MSC_API int msc_segment_csr(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
                            const int32_t *col_idx, const float *field,
                            int32_t *asc, int32_t *desc, int32_t *ms,
                            void *stream);

/*
 * Segmentation of a batch of fields of independent shapes in one set of
 * launches: every pass of msc_segment runs once over the tiles of all
 * fields, so per-call launch and synchronisation costs are paid once per
 * batch.  Each field's outputs are bit-identical to its own msc_segment call.
 *
 *  fields   host array of `nfields` descriptors; each is checked as the
 *           arguments of msc_segment (same errors); outputs of different
 *           fields must not overlap.
 *  Per-field counters of the call: msc_last_field_stats(ctx, i, out).
 */
typedef struct msc_field {
  const float *field;   /* device float32[X*Y*Z]                   */
  int64_t dims[3];      /* X, Y, Z                                 */
  int32_t *asc;         /* device int32[N] or NULL                 */
  int32_t *desc;        /* device int32[N] or NULL                 */
  int32_t *ms;          /* device int32[N] or NULL                 */
} msc_field;

MSC_API int msc_segment_batched(msc_ctx *ctx, int nfields,
                                const msc_field *fields, void *stream);

/*
 * Autotuner: runs the batch once per compiled tile shape (one untimed run,
 * then the best of two runs timed with HIP events on `stream`), selects the
 * fastest shape for this context and reports every time.  The outputs hold
 * the batch's results afterwards.  Blocks until the runs have finished.
 */
typedef struct msc_tune {
  int best;             /* index into msc_tile_shapes              */
  int tile[3];          /* the chosen shape                        */
  int n_shapes;         /* shapes timed (entries of ms)            */
  float ms[8];          /* best time per shape, milliseconds       */
} msc_tune;

MSC_API int msc_autotune(msc_ctx *ctx, int nfields, const msc_field *fields,
                         void *stream, msc_tune *out);

/*
 * Tile shape of the segmentation's fused LDS pass (a tuning knob; results
 * do not depend on it).  msc_tile_shapes writes up to `max` compiled shapes
 * as {tx, ty, tz} triples to `out` (host int[3*max]) and returns their
 * number; the first is the default.  msc_set_tile selects one for this
 * context (MSC_EINVAL if it is not compiled in).  The environment variable
 * MSC_TILE="TXxTYxTZ" sets the initial choice of new contexts.
 */
MSC_API int msc_tile_shapes(int *out, int max);
MSC_API int msc_set_tile(msc_ctx *ctx, int tx, int ty, int tz);

/*
 * First capacity (slots) of the table of (ascending, descending) label pairs
 * that gives the MS labels (a tuning knob; results do not depend on it).
 * 0, the default, sizes it from the extremum counts.  A pass whose pairs do
 * not fit runs again on a table four times larger, up to a capacity that
 * always suffices (twice the smaller of the vertex count and the product of
 * the extremum counts), so a small value costs time, never correctness.
 * Values are rounded up to a power of two of at least 1024.  MSC_EINVAL for
 * a NULL context or a value above 2^32.
 */
MSC_API int msc_set_table_capacity(msc_ctx *ctx, uint64_t first_capacity);

/* Counters of the last successful msc_segment on this context. */
typedef struct msc_stats {
  int64_t n_vertices;
  int64_t n_maxima;      /* distinct ascent roots                     */
  int64_t n_minima;      /* distinct descent roots                    */
  int64_t n_cells;       /* distinct (asc, desc) pairs                */
  int64_t n_exits;       /* tile exits (halo targets), both directions */
  int32_t jump_rounds;   /* longest exit-graph chain one exit followed */
  int32_t tile_x, tile_y, tile_z; /* tile of the fused local pass     */
  int64_t exit_steps;    /* exit-graph links followed in total        */
  int32_t status;        /* outcome on the device (MSC_OK, MSC_ENAN)  */
  int32_t reserved;
} msc_stats;

/* Counters of the last segmentation call (they wait for its work). */
MSC_API int msc_last_stats(const msc_ctx *ctx, msc_stats *out);

/*
 * Outcome of the last asynchronous call on this context, as the device
 * found it: waits until the call's work has run, then sets *status to
 * MSC_OK, MSC_ENAN (a field held a NaN; in a batch, the fields whose
 * msc_last_field_stats status is MSC_ENAN) or MSC_EHIP.  Returns MSC_EINVAL
 * for NULL arguments or MSC_EHIP if the wait fails.
 */
MSC_API int msc_last_status(msc_ctx *ctx, int *status);

/* Counters of field `index` of the last segmentation call (a single
 * msc_segment is a batch of one); `status` is that field's outcome, so a
 * NaN in one field of a batch does not invalidate the others. */
MSC_API int msc_last_field_stats(const msc_ctx *ctx, int index,
                                 msc_stats *out);

/*
 * Graph-captured batched segmentation, for fields segmented again and again
 * with the same buffers and shapes (a time series, a serving loop with
 * fixed slots).  msc_graph_create runs one msc_segment_batched call over
 * `fields`, ordered after the work already on `stream`, and returns when it
 * has run (the outputs hold its result), having captured the same call
 * into a HIP graph; msc_graph_launch replays
 * it on `stream` with one launch call, reading the fields' current
 * contents and rewriting the same outputs.  The graph owns its workspace,
 * counters and copy of the descriptors, so replays share no memory with
 * `ctx` or with other graphs; `ctx` only gives the device and tile shape.
 * Replays of one graph must not overlap (issue them on one stream, or
 * order them).  The fields and outputs must stay allocated until
 * msc_graph_destroy; the descriptor array is read during msc_graph_create
 * only.
 *  msc_graph_field_stats: waits for the last replay and reports field
 *  `index`'s counts and status (MSC_ENAN for a NaN in that field).
 *  Errors: as msc_segment_batched; MSC_EINVAL for a replay-less stats call.
 */
typedef struct msc_graph msc_graph;
MSC_API int msc_graph_create(msc_ctx *ctx, int nfields, const msc_field *fields,
                             void *stream, msc_graph **out);
MSC_API int msc_graph_launch(msc_graph *g, void *stream);
MSC_API int msc_graph_field_stats(msc_graph *g, int index, msc_stats *out);
MSC_API void msc_graph_destroy(msc_graph *g);

/*
 * Per-kernel timing (the library's own trace).  While enabled, every kernel
 * launch of the calls on this context is bracketed by HIP events recorded on
 * the call's stream, and its elapsed time is added to a per-kernel record
 * together with the kernel's algorithmic HBM bytes (the bytes the algorithm
 * must move: inputs read once, outputs written once, pointer gathers counted
 * once per access).  Recording adds two event records per launch.
 *
 *  msc_profile: enable != 0 clears the records and starts recording;
 *               enable == 0 stops recording (records are kept).
 *  msc_profile_read: copies up to `max` records to `out` (host array) and
 *               sets *count to the number of records available.
 */
typedef struct msc_phase {
  char name[32];
  int64_t launches;
  double total_ms;
  double bytes;
} msc_phase;

MSC_API int msc_profile(msc_ctx *ctx, int enable);
MSC_API int msc_profile_read(const msc_ctx *ctx, msc_phase *out, int max,
                             int *count);

/*
 * Connected components of the feature mask on a grid (Alg. 3, implicit
 * thresholding): the graph is the Freudenthal grid restricted to vertices
 * with mask != 0.
 *
 *  mask    device, uint8[N], read only; nonzero = feature.
 *  dims    host, int64[3].
 *  labels  device, int64[N]: smallest vertex id of the vertex's component,
 *          -1 for vertices outside the mask (Alg. 3 gives them a negative
 *          label; the paper names a component by its largest id, this
 *          library by its smallest).
 *  Errors: MSC_EINVAL, MSC_ENOMEM, MSC_EHIP.
 */
MSC_API int cc_label_grid(msc_ctx *ctx, const uint8_t *mask, const int64_t dims[3],
                  int64_t *labels, void *stream);

/*
 * cc_label_grid over several masks of independent shapes in shared
 * launches (up to 32 masks per launch): each mask is labelled on its own,
 * with ids local to it, bit-identical to a cc_label_grid call per mask.
 * Asynchronous like cc_label_grid; the masks' outputs must not overlap.
 *
 *  masks   host array of `nmasks` descriptors (read during the call only);
 *          each holds a device mask, its dims and its device labels.
 *  Errors: MSC_EINVAL (NULL pointers, dims < 1, nmasks < 0), MSC_ERANGE,
 *  MSC_ENOMEM, MSC_EHIP.  nmasks == 0 does nothing.
 */
typedef struct msc_mask {
  const uint8_t *mask;  /* device, uint8[N]                */
  int64_t dims[3];      /* X, Y, Z                         */
  int64_t *labels;      /* device, int64[N]                */
} msc_mask;

MSC_API int cc_label_grid_batched(msc_ctx *ctx, int nmasks,
                                  const msc_mask *masks, void *stream);

/*
 * cc_label_grid through the paper's distributed scheme with `ranks` virtual
 * ranks on one device (Alg. 3 followed by the communication phase it
 * shares with the MS segmentation): the z-extent is split into slabs of
 * planes [r*Z/ranks, (r+1)*Z/ranks), each slab is labelled as a grid of its
 * own, and the exchange across every slab boundary joins the labels of the
 * two ends of each Freudenthal edge that crosses it (both in the mask; the
 * smaller label wins), after which every vertex takes its merged label.
 * Outputs, layout and errors as cc_label_grid, and bit-identical to it;
 * MSC_EINVAL also for ranks < 1 or ranks > Z.
 */
MSC_API int cc_label_grid_ranks(msc_ctx *ctx, const uint8_t *mask,
                                const int64_t dims[3], int ranks,
                                int64_t *labels, void *stream);

/*
 * cc_label_grid for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * labels, with no context and no allocation of any kind.  The tile-local
 * roots live in a static device array of 2^27 16-bit entries (256 MiB on
 * each GPU the library runs on, held until the process ends), taken on the
 * call's first use on a device.  The roots are stored by whole 32x16x16
 * tiles, so a call may cover at most 2^14 tiles: ceil(X/32) * ceil(Y/16) *
 * ceil(Z/16) <= 16384 (512^3 vertices, or fewer when the sides are not
 * multiples of the tile).
 *
 *  Runs on the current HIP device; mask, dims, labels and stream as
 *  cc_label_grid.
 *  Every call on one GPU shares that GPU's array: calls whose work overlaps
 *  on the device (two streams, or two host threads) race; calls on one
 *  stream are ordered and safe.
 *  Errors: MSC_EINVAL (NULL pointers, dims < 1), MSC_ERANGE (more than 2^14
 *  tiles), MSC_EHIP.
 */
MSC_API int cc_label_grid_noalloc(const uint8_t *mask, const int64_t dims[3],
                                  int64_t *labels, void *stream);

/*
 * Critical points by the connected components of each vertex's lower and
 * upper link (background, "Critical Points"): the link of v in the
 * Freudenthal triangulation restricted to the vertices below / above v in
 * the (value, id) order.  0 lower components: minimum; 0 upper: maximum;
 * one of each: regular; more: a saddle (two or more lower components: a
 * 1-saddle, upper: a 2-saddle; more than two, or both: degenerate).
 *
 *  field  device, float32[N] as msc_segment (N <= INT32_MAX).
 *  code   device, uint8[N]: lower components | upper components << 4.
 *  Errors: MSC_EINVAL, MSC_ERANGE, MSC_ENAN, MSC_EHIP.
 */
MSC_API int msc_critical_points(msc_ctx *ctx, const float *field,
                                const int64_t dims[3], uint8_t *code,
                                void *stream);

/*
 * The extremum graph that the segmentations provide (the paper's outlook:
 * the input of a merge tree computation): for every vertex whose upper link
 * has two or more components, one edge per component to the maximum that
 * steepest ascent reaches from the component's highest vertex; likewise
 * through the lower link to minima.
 *
 *  asc, desc  device, int32[N]: the maps msc_segment wrote for this field.
 *  edges      device, int32[capacity][3] = (vertex, extremum, +1 for a
 *             maximum / -1 for a minimum), or NULL; written only when
 *             capacity >= the edge count, by increasing vertex, a vertex's
 *             ascending edges first, its components by increasing id of
 *             their highest / lowest vertex.
 *  count      host, receives the edge count.
 *  Synchronises the stream.  Errors: MSC_EINVAL, MSC_ERANGE, MSC_ENAN,
 *  MSC_ENOMEM, MSC_EHIP.
 */
MSC_API int msc_extremum_graph(msc_ctx *ctx, const float *field,
                               const int64_t dims[3], const int32_t *asc,
                               const int32_t *desc, int32_t *edges,
                               int64_t capacity, int64_t *count, void *stream);

/*
 * CSR adjacency of the 1-skeleton of a tetrahedral complex given by its
 * tetrahedra (the mesh of the explicit pipeline, where extracted geometry
 * is triangulated before its components are labelled, and the input of
 * msc_segment_csr and cc_label_csr): u is a neighbour of v when some
 * tetrahedron holds both and u != v.
 *
 *  n         number of vertices (0 gives row_ptr = {0}).
 *  ntets     number of tetrahedra (workspace: 48 bytes each).
 *  tets      device, int32[ntets][4] vertex ids (repeats allowed).
 *  row_ptr   device, int64[n+1], always written.
 *  col_idx   device, int32[capacity], or NULL: written (rows in increasing
 *            order, no duplicates, symmetric) only when capacity >= the
 *            entry count; otherwise call again with a larger buffer.
 *  nnz       host, receives the entry count row_ptr[n].
 *  Synchronises the stream (the entry count is read back).  Errors:
 *  MSC_EINVAL (NULL arguments, negative sizes, a vertex id outside
 *  [0, n): outputs undefined), MSC_ERANGE, MSC_ENOMEM, MSC_EHIP.
 */
MSC_API int msc_csr_from_tets(msc_ctx *ctx, int64_t n, int64_t ntets,
                              const int32_t *tets, int64_t *row_ptr,
                              int32_t *col_idx, int64_t capacity,
                              int64_t *nnz, void *stream);

/*
 * Connected components of an explicit graph in CSR form (the paper's
 * "explicit" CC on extracted geometry).
 *
 *  n        number of vertices (>= 0; 0 is a no-op).
 *  row_ptr  device, int64[n+1], row_ptr[0] = 0, non-decreasing.
 *  col_idx  device, int32[row_ptr[n]], each in [0, n).  Edges are used in
 *           both directions, so listing an edge once suffices; duplicates
 *           and self-loops are allowed.
 *  mask     device, uint8[n] or NULL (NULL = every vertex is a feature).
 *  labels   device, int64[n]: smallest id of the component, -1 outside mask.
 *  Errors: MSC_EINVAL (NULL pointers, n < 0, n > INT32_MAX), MSC_ENOMEM,
 *          MSC_EHIP.  Out-of-range col_idx entries are reported as
 *          MSC_EINVAL after the call's kernels have checked them.
 */
MSC_API int cc_label_csr(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
                 const int32_t *col_idx, const uint8_t *mask, int64_t *labels,
                 void *stream);

/*
 * Path compression of a pointer forest in place (Alg. 1 main loop; the
 * synchronous form is pointer doubling as tabulated in Fig. 2).
 *
 *  d        device, int64[n]: d[v] in [0, n); the pointers must form a forest
 *           whose roots point to themselves (no longer cycles).
 *  rounds   >= 1: number of rounds to run; 0 = until every vertex points to a
 *           root.
 *  synchronous  nonzero: each round computes d'[v] = d[d[v]] from the
 *           previous round's array (double buffered, as in the worked
 *           example); zero: rounds update d in place (the paper's production
 *           form), which converges at least as fast.
 *  Errors: MSC_EINVAL (d NULL, n < 0, rounds < 0), MSC_ENOMEM, MSC_EHIP.
 */
MSC_API int msc_pointer_jump(msc_ctx *ctx, int64_t *d, int64_t n, int rounds,
                     int synchronous, void *stream);

/*
 * Serving: a request queue with continuous batching.
 *
 * A queue takes `hbm_budget` bytes of device memory at creation and splits
 * it: a workspace for segmentation launches (a quarter of the budget, at
 * most 8 GiB), one for mask-CC launches (a sixteenth, at most 1 GiB), and an
 * arena for request-resident buffers (each request's input and outputs).
 * Requests are admitted in arrival order within their kind while the arena
 * holds their buffers and their kind has fewer than 8 requests staged ahead
 * of its launches (copies issued further ahead would share the host link
 * with the ones a launch waits for); a request of one kind never waits for
 * the other kind's window.  Admitted inputs are copied to the device on a
 * copy stream.  Each kind has its own stream: staged requests that arrive
 * while launches run join the next launch of their kind (one batched call of
 * at most `max_batch` requests and, unless a single request is larger, at
 * most 2^26 vertices, since a launch's requests all complete together), at
 * most two launches per kind are in flight, and the two kinds overlap on the
 * device.  The workspaces are never reallocated while the queue serves.
 * Results stay on the device until msc_release; a finished request that is
 * never released keeps its arena space, so the requests behind it wait.
 * Every call is thread-safe.  A request that fails (e.g. NaN in its field)
 * fails alone: the other requests of its launch keep their results.
 *
 *  msc_queue_create: `device` is the HIP device index, `hbm_budget` at least
 *  1 MiB, `max_batch` >= 1 (1 = one request per launch).  MSC_EINVAL,
 *  MSC_ENOMEM (allocation failed), MSC_EHIP.  Starts five host threads;
 *  msc_queue_destroy joins them after the running launches end and frees
 *  everything, including unreleased results.
 *  msc_request.host_input: the input, read until the request is staged:
 *  host memory (page-locked memory makes the copy asynchronous) or device
 *  memory of the queue's device; float32[N] for MSC_REQ_SEGMENT, uint8
 *  mask[N] for MSC_REQ_CC_GRID.  It is copied into the queue's arena on the
 *  queue's own streams, which are not ordered after any stream of the
 *  caller: an input in device memory must be complete (its producer
 *  synchronised) before msc_submit.
 *  msc_submit: MSC_EBUDGET if the request's buffers exceed the arena or its
 *  launch scratch exceeds its kind's workspace, MSC_EINVAL / MSC_ERANGE as
 *  msc_segment.  *ticket names the request.
 *  msc_poll: *status = MSC_EBUSY while queued or running, MSC_ECANCELED, or
 *  the request's own result code.
 *  msc_wait: blocks until the request is finished; returns its result code.
 *  msc_get_result: device pointers of the outputs (valid until msc_release) and
 *  host steady-clock times (ns) of submission, launch start and completion.
 *  msc_cancel: removes a request that is still waiting for admission
 *  (MSC_EBUSY once admitted).
 *  msc_release: frees a finished or cancelled request's device memory.
 *  msc_queue_info: budget; arena_size and arena_used (request buffers);
 *  workspace_reserved (the two workspaces); request counts by state;
 *  launches issued; workspace_grows (0 while serving: the workspaces are
 *  fixed) and host_waits (times a worker's host thread waited for the device
 *  before enqueuing a launch).
 */
typedef struct msc_queue msc_queue;

typedef struct msc_request {
  int kind;                /* MSC_REQ_SEGMENT or MSC_REQ_CC_GRID      */
  int64_t dims[3];         /* X, Y, Z                                 */
  const void *host_input;  /* float32 field or uint8 mask (host or device) */
} msc_request;

typedef struct msc_result {
  int kind;
  int status;              /* the request's result code               */
  int64_t n;               /* vertices                                */
  int32_t *asc, *desc, *ms;/* device outputs of a segmentation        */
  int64_t *labels;         /* device output of a mask CC              */
  int64_t t_submit_ns, t_start_ns, t_done_ns;
  int batch_size;          /* requests in the launch that ran it      */
} msc_result;

typedef struct msc_queue_stats {
  size_t budget, arena_used, workspace_reserved;
  int64_t pending, running, finished;
  size_t arena_size;
  int64_t launches, workspace_grows, host_waits;
} msc_queue_stats;

MSC_API int msc_queue_create(int device, size_t hbm_budget, int max_batch,
                             msc_queue **out);
MSC_API void msc_queue_destroy(msc_queue *q);
MSC_API int msc_submit(msc_queue *q, const msc_request *req,
                       uint64_t *ticket);
MSC_API int msc_poll(msc_queue *q, uint64_t ticket, int *status);
MSC_API int msc_wait(msc_queue *q, uint64_t ticket);
MSC_API int msc_get_result(msc_queue *q, uint64_t ticket, msc_result *out);
/* Copies output `which` (0 asc, 1 desc, 2 ms of a segmentation; 3 labels of
 * a CC) of a finished request to `dst` (host or device memory, at least
 * n * 4 bytes, n * 8 for labels).  Blocks until the copy is done. */
MSC_API int msc_copy_result(msc_queue *q, uint64_t ticket, int which,
                            void *dst);
MSC_API int msc_cancel(msc_queue *q, uint64_t ticket);
MSC_API int msc_release(msc_queue *q, uint64_t ticket);
MSC_API int msc_queue_info(msc_queue *q, msc_queue_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* MSC_H */
