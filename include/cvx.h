/*
 * libcvx: per-pixel ray casting of volumetric canvases stored as arrays of
 * deep octrees, with front-to-back RGBA compositing, on one MI355X (gfx950).
 *
 * Source of the operations (CanvoX, Kim et al., arXiv:1704.02724):
 *  - canvas = uniform array of R^3 octree roots, each refinable to a large
 *    depth (Sec. 4);
 *  - pointer-free linear pools indexed by cell id; a refined cell always has
 *    8 consecutive children and only parent and first child are stored
 *    (Sec. 4.1.1, "Tree Graph G_p"); three outer-face neighbours per cell are
 *    derived from that tree on the GPU (Sec. 4.1.1 "Neighbor Graph G_3" and
 *    Sec. 4.1.2);
 *  - rays start from an eye kept in full precision (Sec. 6.1), are traversed
 *    in cell-local coordinates from face to face using the neighbour graph and
 *    accumulate colour until full opacity or canvas exit (Sec. 6.2-6.3).
 *
 * Conventions
 *  - Child octant numbering: x | y<<1 | z<<2 (the sibling across the x face of
 *    child 0 is child 1).
 *  - Canvas positions are measured in root-edge units: q = (p - origin) /
 *    root_edge, so the canvas is [0, R]^3 and a depth-d cell has edge 2^-d.
 *  - Pixel (x, y), row 0 at the top, unit direction in FP64:
 *      u = (2(x+1/2)/W - 1) tan_half_fov_x,  v = (1 - 2(y+1/2)/H) tan_half_fov_y,
 *      d = normalize(fwd + u right + v up).
 *  - Compositing: emission-absorption through piecewise-constant leaves.  A
 *    leaf holds colour c and kappa = optical depth across one leaf edge; a
 *    segment of length l leaf edges does T' = T exp(-kappa l),
 *    C += (T - T') c, T = T'.  Output RGBA = (C, 1 - T), premultiplied,
 *    black background.  alpha_stop >= 1 disables early termination;
 *    otherwise a ray stops after the segment where 1 - T >= alpha_stop.
 *
 * Errors: every entry point returns CVX_OK (0) or a negative CVX_ERR_* code;
 * no C++ exception crosses this boundary.  A failed call leaves previously
 * uploaded pools unchanged.  A context is bound to one HIP device and one
 * stream and is not thread-safe.
 */
#ifndef CVX_H
#define CVX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CVX_OK 0
#define CVX_ERR_INVALID_ARG (-1)
#define CVX_ERR_BAD_POOL (-2)
#define CVX_ERR_OOM (-3)
#define CVX_ERR_HIP (-4)
#define CVX_ERR_NOT_FOUND (-5)

#define CVX_LEAF_RGBA8_F16 0u /* {u8 r,g,b,a; u16 kappa (IEEE half); u16 pad}, 8 bytes */
#define CVX_LEAF_F64 1u       /* {double r,g,b,kappa}, 32 bytes */

#define CVX_VARIANT_FP32_REBASED 0u /* FP32 cell-local traversal, FP64 rebase */
#define CVX_VARIANT_FP64_PLAIN 1u   /* FP64 canvas-global traversal and compositing */
#define CVX_VARIANT_FP32_NAIVE 2u   /* FP32 canvas-global traversal (drifts at depth) */
#define CVX_VARIANT_FP32_CELL_LOCAL 3u /* the paper's uncertified FP32 cell-local traversal
                                          (Sec. 6.2), for the precision experiment */
#define CVX_VARIANT_FP16_CELL_LOCAL 4u /* the same traversal in IEEE half precision (the
                                          closing remark of Sec. 6.3), for the experiment */

#define CVX_MAX_CANVASES 64
#define CVX_MAX_DEPTH 30
#define CVX_MAX_VIEWS 4096

/* Per-ray flag bits reported by trace mode. */
#define CVX_RAYFLAG_STEP_CAP 1u    /* watchdog: traversal stopped at max steps */
#define CVX_RAYFLAG_FP64_EXIT 2u   /* an exit decision needed the FP64 fallback */
#define CVX_RAYFLAG_BAD_LINK 4u    /* a neighbour link was null inside the canvas */

typedef struct cvx_ctx cvx_ctx;

/* Canvas description.  The canvas covers origin + [0, R*root_edge]^3. */
typedef struct {
  double origin[3];
  double root_edge;     /* > 0 */
  uint32_t R;           /* roots per axis, 1..64 */
  uint32_t max_depth;   /* deepest level present, <= CVX_MAX_DEPTH; R * 2^max_depth <= 2^30 */
  uint32_t leaf_format; /* CVX_LEAF_* */
  uint32_t reserved;    /* must be 0 */
} cvx_canvas_desc;

/* Tree node (Sec. 4.1.1 G_p).  child: bit 31 set -> leaf, low 31 bits index
 * the leaf array; otherwise the first of 8 consecutive children, a multiple
 * of 8.  parent: index of the parent, 0xffffffff for roots.  Roots are nodes
 * [0, R^3) in x-fastest order; slots [R^3, roundup8(R^3)) are padding and are
 * ignored.  Nodes not reachable from the roots are ignored. */
typedef struct {
  uint32_t child;
  uint32_t parent;
} cvx_node;

typedef struct {
  uint8_t r, g, b, a; /* colour byte/255 (linear); a is not read by the renderer */
  uint16_t kappa_f16; /* optical depth across one leaf edge, IEEE half, >= 0, finite */
  uint16_t pad;
} cvx_leaf_rgba8_f16;

typedef struct {
  double r, g, b, kappa; /* kappa >= 0, finite */
} cvx_leaf_f64;

/* One pinhole view.  right, up, fwd: orthonormal (|dot| and |norm-1| below
 * 1e-9).  Its W*H pixels are written to out[(out_offset_px + y*W + x)]. */
typedef struct {
  int32_t canvas_id;
  uint32_t W, H;
  float alpha_stop; /* in (0, 1]; >= 1 disables early termination */
  double eye[3];
  double right[3], up[3], fwd[3];
  double tan_half_fov_x, tan_half_fov_y; /* > 0 */
  uint64_t out_offset_px;
} cvx_view;

/* Trace mode: only the listed rays are traced and, for each, the visited
 * leaves (node ids of the uploaded pool, in front-to-back order), their local
 * segment lengths l and the final RGBA are written.  All pointers are device
 * pointers owned by the caller.  Every visited leaf is recorded, also when
 * its length rounds to 0 in the variant's precision. */
typedef struct {
  uint64_t n;              /* number of rays */
  const uint64_t* ray_ids; /* (view index << 32) | (y*W + x) */
  uint32_t max_leaves;     /* capacity per ray of leaf_ids / local_len */
  uint32_t reserved;
  uint32_t* leaf_ids;      /* n * max_leaves */
  float* local_len;        /* n * max_leaves, may be NULL */
  double* local_len64;     /* n * max_leaves, may be NULL */
  uint32_t* n_leaves;      /* n: total segments (may exceed max_leaves) */
  uint32_t* flags;         /* n: CVX_RAYFLAG_* */
  float* rgba;             /* 4n */
  double* end_point;       /* 3n, may be NULL: exit point of the last leaf as the variant
                              computed it, canvas units (root edge 1, canvas corner 0) */
} cvx_trace;

/* Render options.  Zero means "default" for every tuning field. */
typedef struct {
  uint32_t variant;     /* CVX_VARIANT_* */
  uint32_t tile_w;      /* pixel tile width; tile_w * tile_h must be 64 (one wavefront) */
  uint32_t tile_h;
  uint32_t workgroups;  /* persistent grid size */
  uint32_t wg_size;     /* threads per workgroup: 64, 128 or 256 */
  uint32_t use_graph;   /* 1: capture the launch in a HIP graph and replay it */
  uint32_t out_f64;     /* FP64_PLAIN only: out is double RGBA instead of float */
  uint32_t top_lookup;  /* 0: ray starts are located through the pool's top-level table;
                           1: they descend from the root array (same result).  This table,
                           read through the L2, stands in for top tree levels staged in
                           LDS (there is no LDS-depth option): the LDS holds each lane's
                           FP64 ray slot, which lets the render kernel keep 8 wavefronts
                           per SIMD, and only ray starts read the top levels */
  uint32_t single_queue; /* 0: the tiles are split into 8 contiguous ranges, one per XCD
                            (workgroup i starts on range i mod 8, then helps the others);
                            1: one queue over all tiles (same result) */
  uint32_t per_ray_start; /* 0: when a view's eye lies inside the canvas (off every cell
                            plane), its rays share the leaf holding the eye, located once
                            per view; 1: every ray locates its own first leaf (same result) */
  uint32_t wide_offsets; /* 0: pools of at most 2^28 nodes are read with 32-bit byte offsets
                            from the pool base, larger ones with 64-bit addresses; 1: every
                            pool is read with 64-bit addresses, the code that pools above
                            2^28 nodes always take (same result; for checking that code on
                            any pool) */
  uint32_t rays_per_wave; /* FP32_REBASED renders (not trace or stats): rays one wavefront
                            takes per work item, a multiple of 64 up to 1024 (0 = 64).  64:
                            one tile, one ray per lane, the wavefront ends the item with its
                            longest ray.  Above 64: up to rays_per_wave / 64 consecutive
                            tiles of one view, and lanes whose ray ended take the item's next
                            rays (assigned by a wavefront ballot) once refill_min lanes wait
                            (Sec. 6.2: a ray stops at full opacity or at the canvas exit;
                            refilling keeps the other lanes busy).  Same result. */
  uint32_t refill_min;  /* lanes that must wait before they are refilled, 1..64 (0 = 32) */
  uint32_t chord_pieces; /* FP32_REBASED only, 1 (0 = 1), 2, 4 or 8: the canvas chord [t0, t1]
                            of every ray of a view that runs to the canvas exit (alpha_stop
                            >= 1) is cut at t0 + (t1 - t0) (67 j + 1) / (67 chord_pieces)
                            (not at dyadic fractions, so that no cut lies on a cell plane by
                            construction) into pieces traced
                            as separate work items, each compositing its leaves (the leaf
                            holding a cut contributes the part on each side to each piece)
                            into a colour and transmittance, merged front to back per pixel
                            by the associative over operator (C1 + T1 C2, T1 T2) (Sec. 6.2
                            composites front to back; the operator is that compositing
                            regrouped).  Several short work items per ray shorten the end of
                            a launch that holds few rays per lane.  Images agree with the
                            whole chord's within the FP32 length precision of the traversal
                            (the pieces rebase at their cuts; not bit for bit).  With trace,
                            the buffers hold n * chord_pieces rows, ray-major, (ray, piece)
                            each, rgba = (the piece's premultiplied colour, its
                            transmittance); rows past a view's piece count are empty.  Not
                            with rays_per_wave > 64, with trace and stats together, or in
                            cvx_render_noalloc (merging needs a buffer the context
                            allocates); stats renders run whole chords. */
  const void* cast_events; /* optional, eager launches only (use_graph = 0): a pointer to two
                            hipEvent_t created by the caller, recorded on the context stream
                            right before and right after the cast kernel, so that the
                            kernel's own duration can be read (the call also stages the
                            views and locates shared first leaves before it) */
  const cvx_trace* trace; /* non-NULL: trace mode (views' out_offset_px unused) */
  uint64_t* stats;      /* optional device array of CVX_STAT_COUNT u64 counters (added to) */
} cvx_render_opts;

#define CVX_STAT_RAYS 0        /* rays traced */
#define CVX_STAT_LEAVES 1      /* visited leaves (segments composited) */
#define CVX_STAT_OUTER 2       /* transitions through an outer face (neighbour link read) */
#define CVX_STAT_DESCENT 3     /* tree levels descended (first leaf depth + depth increases) */
#define CVX_STAT_FP64_EXIT 4   /* exit decisions taken by the FP64 fallback */
#define CVX_STAT_REBASE 5      /* FP64 rebases of the cell-local point */
#define CVX_STAT_STEPS 6       /* traversal loop iterations, summed over rays */
#define CVX_STAT_SLOTS 7       /* lane slots: per 64-ray tile, 64 x its longest ray's iterations */
#define CVX_STAT_COUNT 8

/* Create a context on HIP device `hip_device` that enqueues on `hip_stream`
 * (a hipStream_t, borrowed; NULL = the null stream).  The context owns the
 * GPU-side pools of the canvases uploaded to it (the GPU memory layout of
 * Sec. 4.1.2).  Device memory is allocated per uploaded pool and per render
 * configuration.  Returns CVX_ERR_INVALID_ARG for a NULL ctx or a device
 * index out of range, CVX_ERR_HIP if the runtime fails, CVX_ERR_OOM if the
 * host allocation fails; *ctx is NULL on failure. */
int cvx_create(cvx_ctx** ctx, int hip_device, void* hip_stream);

/* Upload a canvas pool (Sec. 4.1.1-4.1.2): host arrays are read during the
 * call only.  The pool is validated (indices in range, children groups
 * 8-aligned, each node reached once, parents consistent, depth <= max_depth,
 * leaf indices < n_leaves, finite non-negative kappa), re-laid out on the
 * device into 16-byte node records plus a node-indexed payload array, and
 * the three outer-face neighbour links per node are built on the GPU level
 * by level.  A top-level table (for every cell of depth L <= 6, at most 2^18
 * cells, the node of depth <= L covering it) is built on the GPU too; ray
 * starts use it to skip the first L levels of their descent.  Replaces any pool under canvas_id only on success.  Returns
 * CVX_ERR_BAD_POOL for an invalid pool, CVX_ERR_OOM when the device lacks
 * room (checked before any allocation). Synchronous. */
int cvx_upload_pool(cvx_ctx* ctx, int canvas_id, const cvx_canvas_desc* desc,
                    const cvx_node* nodes, uint64_t n_nodes, const void* leaves,
                    uint64_t n_leaves);

/* Render n_views views into out_dev (a device buffer of at least
 * max(out_offset_px + W*H) RGBA pixels, float unless opts->out_f64): one ray
 * per pixel from the full-precision eye (Sec. 6.1), traversed leaf to leaf
 * through the neighbour graph and composited front to back until the stop
 * opacity or the canvas exit (Sec. 6.2).  Asynchronous on the context
 * stream; the caller synchronises.  The views array is copied before return.
 * Every pixel is computed by one lane in a fixed order, so the output does
 * not depend on scheduling or tuning.  Returns CVX_ERR_INVALID_ARG for bad
 * options or views (nothing is launched), CVX_ERR_HIP if a launch fails. */
int cvx_render(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
               const cvx_render_opts* opts);

/* Allocation-free rendering, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same as cvx_render with the same arguments and the same
 * result, except that the per-call view table and work-queue header live in
 * a fixed device array of the library (one per GPU, held until the process
 * ends) instead of memory the context allocates: the call makes no
 * hipMalloc, hipFree or other allocation.  n_views is limited to
 * CVX_NOALLOC_MAX_VIEWS (CVX_ERR_INVALID_ARG beyond it, nothing launched) and
 * opts->use_graph must be 0 (instantiating a graph allocates).  Every call on
 * one GPU shares that GPU's array, whatever the context: calls that overlap
 * on one GPU (from two streams or two contexts) race and are not allowed;
 * calls on one context's stream are ordered and safe. */
#define CVX_NOALLOC_MAX_VIEWS 256
int cvx_render_noalloc(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
                       const cvx_render_opts* opts);

/* One candidate launch shape timed by cvx_autotune. */
typedef struct {
  uint32_t tile_w, tile_h; /* pixel tile, tile_w * tile_h = 64 */
  uint32_t wg_size;        /* threads per workgroup */
  uint32_t workgroups;     /* persistent grid size */
  float ms;                /* mean time of one render, milliseconds */
  uint32_t top_lookup;     /* as in cvx_render_opts */
  uint32_t single_queue;   /* as in cvx_render_opts */
  uint32_t rays_per_wave;  /* as in cvx_render_opts (64: no refill) */
  uint32_t refill_min;     /* as in cvx_render_opts (0 when rays_per_wave is 64) */
  uint32_t chord_pieces;   /* as in cvx_render_opts (1: whole chords) */
} cvx_tune_result;

/* Autotuner of the batch scheduler's launch shape: renders `views` exactly as
 * cvx_render would with base's variant and use_graph, once per candidate
 * tile shape (8x8, 16x4, 4x16, 32x2), workgroup size (64, 128, 256),
 * persistent grid (16, 28, 32, 64 wavefronts per CU), top-level lookup
 * (on, off) and work queues (per XCD, single), one untimed warm-up
 * then `reps` renders timed with HIP events on the context stream.  For
 * FP32_REBASED the fastest of those shapes is then timed with lane refill,
 * rays_per_wave 128 and 256 with refill_min 16, 32 and 48, and with
 * chord_pieces 2, 4 and 8, which are candidates like the others (the split
 * renders agree with the others within the FP32 length precision, not bit
 * for bit).  Writes
 * base with the fastest shape filled in to *best and, when results is not
 * NULL, up to max_results timed candidates in the order tried (the count
 * tried goes to *n_results when not NULL).  out_dev receives the renders
 * (identical for every candidate but the chord-piece ones, which agree
 * within the FP32 length precision).  base->trace and base->stats must be
 * NULL; reps in [1, 1000].  Synchronous; an error from a candidate's render
 * is returned as is. */
int cvx_autotune(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
                 const cvx_render_opts* base, uint32_t reps, cvx_render_opts* best,
                 cvx_tune_result* results, uint32_t max_results, uint32_t* n_results);

/* Pool edits (Sec. 5.1-5.3: a stroke paints leaves, refines leaves down to
 * the brush resolution and coarsens groups that became uniform; Sec. 4.1.2:
 * the GPU pools and the neighbour graph G_3 are brought up to date after
 * every change). */
#define CVX_EDIT_PAINT 0u   /* node: a leaf; its payload becomes payloads[first_payload] */
#define CVX_EDIT_REFINE 1u  /* node: a leaf of depth < desc.max_depth; it gets 8 leaf children
                               (octant order x | y<<1 | z<<2) with payloads
                               [first_payload, first_payload + 8) */
#define CVX_EDIT_COARSEN 2u /* node: refined, its 8 children all leaves; it becomes a leaf with
                               payload payloads[first_payload]; the children's group is freed */

typedef struct {
  uint32_t op;            /* CVX_EDIT_* */
  uint32_t node;          /* node id in the current pool */
  uint64_t first_payload; /* index into the payloads array */
} cvx_edit;

/* Apply n_edits edits to the pool under canvas_id, in order (an edit sees
 * the pool the earlier ones produced).  payloads is a host array of
 * n_payloads leaf records in the pool's leaf format, read during the call.
 * A refined leaf's children take the most recently freed group of 8 node
 * ids, else 8 new ids at the end of the pool (which grows; node ids of
 * existing nodes never change).  If first_child_out is not NULL, it receives
 * per edit the first child id of a REFINE and CVX_NONE_ID otherwise.  Every
 * edit is checked first (node state, depth limit, payload index and kappa);
 * on any error nothing changes.  The records, payloads, the outer-face
 * links (rebuilt on the GPU below the cells the edits refined or coarsened
 * and their same-depth face neighbours) and the top-level table are updated
 * before the call returns.  A brush stroke still in progress on the canvas
 * (cvx_stroke_begin) is ended first: its remaining splits are dropped and the
 * leaves keep their immediate paint.  Synchronous. */
#define CVX_NONE_ID 0xffffffffu
int cvx_edit_pool(cvx_ctx* ctx, int canvas_id, const cvx_edit* edits, uint32_t n_edits,
                  const void* payloads, uint64_t n_payloads, uint32_t* first_child_out);

/* Number of node ids of the pool under canvas_id (including freed groups). */
int cvx_pool_nodes(cvx_ctx* ctx, int canvas_id, uint64_t* n_nodes);

/* Diagnostic copy of device node records [first, first + count) into the host
 * array out (4 uint32 per node): x = first child, or 1 | depth << 1 for a
 * leaf, or 0xffffffff for an id not in the tree; then the outer-face
 * neighbours on the x, y, z axes (0xffffffff for none).  Synchronous;
 * CVX_ERR_INVALID_ARG if the range passes the pool's node count. */
int cvx_read_records(cvx_ctx* ctx, int canvas_id, uint64_t first, uint64_t count, uint32_t* out);

/* Diagnostic copy of device leaf payloads [first, first + count) (indexed by
 * node id, in the pool's leaf format; unspecified for ids that are not
 * leaves) into the host array out.  Synchronous; CVX_ERR_INVALID_ARG if the
 * range passes the pool's node count. */
int cvx_read_payloads(cvx_ctx* ctx, int canvas_id, uint64_t first, uint64_t count, void* out);

/* Brush strokes (Sec. 5.1-5.3).  A stroke is a list of spherical stamps
 * (x, y, z, r in world units, as the canvas descriptor) with one brush colour,
 * one opacity density per brush radius and one brush radius.  Its effect on
 * a leaf: a leaf the stamps overlap (its closed box lies at a distance < r
 * from a stamp centre) is split into 8 children while its edge exceeds
 * radius / k_refine and it is above desc.max_depth (Sec. 5.2; children keep
 * the colour and take half the optical depth per edge); a leaf that is not
 * split and whose centre lies in a stamp (distance <= r) takes the stroke
 * once: kb = sigma * edge / radius, m = kb / (kb + kappa) (0 if both are 0),
 * colour = m * rgb + (1 - m) * colour, kappa = kb + kappa (Sec. 5.1, density
 * as the alpha term).  RGBA8_F16 leaves are decoded (byte / 255, half kappa),
 * mixed in FP64 and encoded again (bytes and A = 255 (1 - exp(-kappa)) rounded
 * to nearest even, kappa to half through float).  As in Sec. 5.3 the splits
 * are deferred: cvx_stroke_begin paints the stroke into the leaves that exist
 * and records the leaves that still need a split; each cvx_stroke_step splits
 * them by one level and paints the new children.  When *pending reaches 0 the
 * canvas is the one the stroke would give applied at once (then, with
 * coarsen = 1, coarsened as stated below: *pending also counts the cells
 * waiting for a merge). */
typedef struct {
  double rgb[3];   /* brush colour, each in [0, 1] */
  double sigma;    /* opacity density per brush radius, finite, >= 0 */
  double radius;   /* brush radius in world units, finite, > 0 */
  double k_refine; /* leaves are split while their edge exceeds radius / k_refine; > 0 */
  uint32_t coarsen; /* 1: after the splits, coarsen without loss, one level per step: a
                       refined cell the stamps overlap whose 8 children are leaves with
                       identical payloads becomes one leaf of twice the optical depth
                       per edge, until none is left; 0: no coarsening */
  uint32_t reserved;
} cvx_stroke;

#define CVX_MAX_STAMPS 65536u

/* Start a stroke on the pool under canvas_id: stamps is a host array of
 * n_stamps (1..CVX_MAX_STAMPS) x 4 doubles, each r finite and >= 0, read
 * during the call.  A stroke still in progress on the canvas is completed
 * first.  *pending receives the number of leaves waiting for a split.
 * Synchronous; on an argument error nothing changes (a device error during
 * the walk can leave the stroke painted into part of the leaves). */
int cvx_stroke_begin(cvx_ctx* ctx, int canvas_id, const cvx_stroke* stroke, const double* stamps,
                     uint32_t n_stamps, uint64_t* pending);

/* One deferred level of the stroke in progress: every waiting leaf is split
 * (through the same machinery as cvx_edit_pool, with children that take the
 * leaf's payload from before the stroke), the stroke is painted into the
 * children, and *pending receives the number of children that still need a
 * split; once none is left, a coarsening stroke merges every waiting cell
 * instead (cvx_edit_pool COARSEN) and *pending receives the number of cells
 * that can merge next.  With no stroke in progress it returns CVX_OK and *pending = 0.
 * Synchronous.  On an error the stroke is dropped: if the splits fail (e.g.
 * CVX_ERR_OOM while the pool grows) the pool is left as after the previous
 * step; a device error after them leaves the splits in place, their children
 * possibly not yet painted. */
int cvx_stroke_step(cvx_ctx* ctx, int canvas_id, uint64_t* pending);

/* Release the GPU pool (Sec. 4.1.2) under canvas_id after the context's
 * stream has drained (CVX_ERR_NOT_FOUND if none, CVX_ERR_INVALID_ARG for an
 * id out of range). */
int cvx_free_pool(cvx_ctx* ctx, int canvas_id);

/* Release everything owned by the context, the GPU pools of Sec. 4.1.2
 * included (waits for its stream first).  NULL is ignored. */
void cvx_destroy(cvx_ctx* ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char* cvx_last_error(cvx_ctx* ctx);

/* Static name of a status code. */
const char* cvx_status_str(int status);

/* Host-only validation of a pool, the same checks cvx_upload_pool makes.
 * Writes a message into msg (may be NULL). Touches no GPU. */
int cvx_validate_pool(const cvx_canvas_desc* desc, const cvx_node* nodes, uint64_t n_nodes,
                      const void* leaves, uint64_t n_leaves, char* msg, size_t msg_len);

/* Host-only validation of views against the given canvas descriptions
 * (canvases[i] may be NULL for an absent canvas).  Touches no GPU. */
int cvx_validate_views(const cvx_view* views, int n_views,
                       const cvx_canvas_desc* const* canvases, int n_canvases, char* msg,
                       size_t msg_len);

/* Device bytes held by the pool under canvas_id. */
int cvx_pool_bytes(cvx_ctx* ctx, int canvas_id, uint64_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* CVX_H */
