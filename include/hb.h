/*
 * hb.h -- C ABI of the MI355X (gfx950) edge-bundling hot path.
 *
 * The library runs the per-iteration loop of 3D-density-histogram edge bundling
 * (Moura, arXiv 1504.02687, Section 3 and Fig. 1) on one GPU:
 *
 *   resample every edge polyline into equally spaced points   (Section 2.1, Section 3)
 *   splat the points into one integer histogram per edge group (Section 3.1 Eq. 1, 3.2 Eq. 3)
 *   smooth each histogram with P box passes via integral sums  (Section 3.1)
 *   mix the smoothed maps through the interaction matrix M     (Section 3.2 Eq. 3-4)
 *   move interior points along the normalised density gradient with step halving
 *                                                              (Section 3.3 Eq. 5)
 *   Laplacian-smooth every polyline                            (Section 3.3)
 *
 * Conventions for every call:
 *   - Return value: HB_OK (0) or a negative hb_status. Calls never abort. The text of the
 *     last error of a context is returned by hb_last_error(ctx).
 *   - A HIP failure is sticky: after HB_EDEVICE the context only accepts hb_destroy.
 *   - Inputs are owned by the caller and are not retained: the library copies them. By
 *     default pointers are host pointers and the call returns after the copy; with
 *     HB_DEVICE_PTRS they are device pointers on the context's device, read in stream
 *     order on the context's stream before the call returns.
 *   - Outputs go to caller-allocated buffers (host, or device with HB_DEVICE_PTRS). A
 *     buffer that is too small gives HB_EINVAL; query sizes with hb_get_num_points.
 *   - Coordinates of points are pixel units of the grid: pixel (u, v) covers
 *     [u, u+1) x [v, v+1). Node coordinates are in user units and are mapped from the
 *     bounding box bbox = [x0, y0, x1, y1] to [0, W] x [0, H].
 *   - Polylines are stored in CSR form: offsets[E+1] (int64, offsets[0] = 0) and
 *     xy[N][2] (float32, x then y). Every polyline has at least two points; its first and
 *     last points are the edge's end points and never move.
 *   - Maps are [B][H][W] row-major.
 *   - One context per host thread; calls on one context must not overlap.
 *   - Failure injection for tests: while the environment variable HB_TEST_FAIL_ALLOC is
 *     set, every device allocation of the library fails and the call returns HB_ENOMEM.
 */
#ifndef HB_H
#define HB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hb_ctx hb_ctx;
typedef int32_t hb_status;

enum {
    HB_OK = 0,
    HB_EINVAL = -1,     /* bad argument, size or index */
    HB_ENOMEM = -2,     /* device allocation failed */
    HB_EDEVICE = -3,    /* HIP error (sticky) */
    HB_ESTATE = -4,     /* call order: e.g. hb_run before graph, groups and parameters */
    HB_EOVERFLOW = -5,  /* integer range of the histogram or the box sums would be exceeded,
                           or one edge would get 2^31 samples or more */
    HB_EINTERNAL = -6   /* an internal consistency check of the device code failed */
};

/* flags of the data-movement calls */
enum { HB_DEVICE_PTRS = 1u };

/* flags of hb_run */
enum {
    HB_RUN_SAMPLES_GIVEN = 1u,     /* the first iteration takes the current polylines as its
                                      sample points (no resampling in that iteration) */
    HB_RUN_RECORD_DECISIONS = 2u,  /* keep the accepted halving index of every sample point of
                                      the last iteration (hb_get_decisions) */
    HB_RUN_ASYNC = 4u,             /* return without waiting; errors surface at hb_sync */
    HB_RUN_GRAPH = 8u              /* capture the n_iters iterations as one hipGraph and replay
                                      it on later runs with the same layout (graph count, sizes,
                                      n_iters and flags) */
};

/* which point set hb_get_num_points / hb_get_points read */
enum {
    HB_POINTS_STATE = 0,    /* the current polylines (after the last Laplacian smoothing) */
    HB_POINTS_SAMPLES = 1   /* the sample points of the last iteration (after resampling) */
};

/* map kinds of hb_get_map */
enum {
    HB_MAP_HIST = 0,        /* int32 [H][W]: histogram of group b (Eq. 1) */
    HB_MAP_BOX = 1,         /* int64 [H][W]: box pass k (1..P) of group b, un-normalised sums */
    HB_MAP_DENSITY = 2,     /* float32 [H][W]: layer l of the density stack (Eq. 3) */
    HB_MAP_GRAD = 3         /* float32 [H][W][2]: central-difference gradient of layer l */
};

/* splat modes (hb_params.splat_mode) */
enum { HB_SPLAT_POINTS = 0, HB_SPLAT_STRIP = 1 };
/* resampling modes (hb_params.resample_mode) */
enum { HB_RESAMPLE_UNIFORM = 0, HB_RESAMPLE_INSERT_DELETE = 1 };
/* when the directed push is applied (hb_params.directed_mode) */
enum { HB_DIRECTED_ONCE = 0, HB_DIRECTED_EVERY_ITER = 1 };

#define HB_MAX_GROUPS 64
#define HB_MAX_PASSES 8
#define HB_MAX_GRID 8192
#define HB_MAX_HALVINGS 30
#define HB_MAX_EDGE_WEIGHT 1048575   /* 2^20 - 1 */

/*
 * Parameters of the method. Section numbers refer to the paper.
 */
typedef struct hb_params {
    uint32_t struct_size;       /* sizeof(hb_params), for ABI versioning */
    int32_t grid_w, grid_h;     /* histogram size W x H (Section 5: dominant side 800) */
    float bbox[4];              /* node-coordinate box [x0, y0, x1, y1] mapped to [0,W]x[0,H] */
    float delta_px;             /* sampling step between resampled points (Section 2.1) */
    int32_t box_passes;         /* P repeated box filters (Section 3.1: 3) */
    int32_t n_radii;            /* length of radius_per_iter (>= 1) */
    const int32_t *radius_per_iter; /* box radius r_i per iteration; the last value repeats.
                                       Copied by hb_set_params. */
    float h_max_px;             /* first step h_max; <= 0 selects 2 sigma(r_0) with
                                   sigma(r)^2 = P r (r+1) / 3 (Section 3.3, Fig. 2) */
    float lambda;               /* bandwidth decay h_i = lambda^i h_max (Section 2.1: 0.5..0.9) */
    float eps;                  /* epsilon of Eq. 5 (density units per pixel) */
    int32_t max_halvings;       /* K: step halvings tried before a point stays (Section 3.3),
                                   in [0, HB_MAX_HALVINGS]; -1: the original fixed step of
                                   Section 2 (every interior point moves by h, no density
                                   test), the baseline Section 3.3 compares against */
    float smooth_weight;        /* Laplacian weight s in y = (1-s) x + s (x- + x+)/2 */
    int32_t smooth_passes;      /* Jacobi passes of the Laplacian smoothing (1) */
    const float *pass_weights;  /* a[P]: density = sum_k a_k * pass_k / (2r+1)^(2k);
                                   NULL selects the last pass only. Copied. */
    float capacity_factor;      /* point-buffer capacity relative to the first sample count
                                   (>= 1.1; grown automatically when exceeded) */
    float directed_offset_px;   /* directed graphs (Section 3, the pipeline of Fig. 1): right
                                   after resampling and before the histogram, each sample
                                   except the two end points is moved by this signed distance
                                   (px) along the left normal (-t_y, t_x) of the polyline
                                   segment it was interpolated on, t the unit direction of that
                                   segment from source towards target (a zero-length segment
                                   moves nothing); 0 (default) disables it. When the push is
                                   applied is set by directed_mode. |value| <= max(W, H) / 16
                                   (the paper uses 0.1 % to 0.5 % of the drawing). Not applied
                                   to samples given with HB_RUN_SAMPLES_GIVEN; not
                                   differentiated (hb_forward_ckpt requires 0). */
    int32_t splat_mode;         /* what the histogram H of Eq. 1 counts. HB_SPLAT_POINTS
                                   (default): every sample point adds the edge weight to the
                                   pixel it falls in. HB_SPLAT_STRIP: the polyline is drawn as a
                                   line strip through the pixels of its samples, as the paper's
                                   implementation draws edges with Bresenham's algorithm
                                   (Section 4): segment (x_j, x_j+1) draws the n = max(|du|,
                                   |dv|) pixels (u0 + round(t du / n), v0 + round(t dv / n)),
                                   t = 0..n-1, halves rounded up, the last sample its own pixel;
                                   every drawn pixel adds the edge weight. The strip needs an
                                   entry buffer of (ceil(delta_px + 2 |directed_offset_px|) + 2)
                                   x 4 bytes per point of capacity; given polylines
                                   (HB_RUN_SAMPLES_GIVEN) with much longer segments can exceed it
                                   (HB_EOVERFLOW). Not differentiated (hb_forward_ckpt requires
                                   HB_SPLAT_POINTS). */
    int32_t resample_mode;      /* how each iteration resamples the polylines (Section 3, the
                                   pipeline). HB_RESAMPLE_UNIFORM (default): n = max(1,
                                   ceil(L / delta_px)) + 1 points at equal arclength.
                                   HB_RESAMPLE_INSERT_DELETE: points are removed where they are
                                   too close and created where they are too far apart: an
                                   interior point closer than delta_min_px to its predecessor
                                   in the polyline is removed, and the gap g between consecutive
                                   kept points is cut into max(1, ceil(g / delta_px)) equal parts
                                   (FP64). Needs directed_offset_px = 0; not differentiated. */
    float delta_min_px;         /* removal spacing of HB_RESAMPLE_INSERT_DELETE; 0 (default):
                                   delta_px / 2; else in (0, delta_px) */
    int32_t n_sigmas;           /* 0 (default): the box radius of every pass is radius_per_iter.
                                   > 0: length of sigma_per_iter, which then replaces the radius
                                   list: iteration i smooths with a real sigma_i (the last value
                                   repeats) by P boxes of two odd widths w_l and w_l + 2 chosen
                                   by Kovesi's rule (ideal width w = sqrt(12 sigma^2 / P + 1),
                                   w_l the largest odd integer <= w, m = round((12 sigma^2 -
                                   P w_l^2 - 4 P w_l - 3 P) / (-4 w_l - 4)) passes of w_l first);
                                   pass k is normalised by prod_{q<=k} (2 r_q + 1)^2 and h_max
                                   defaults to 2 sigma_0. Every width must fit the grid. Not
                                   differentiated (hb_forward_ckpt requires 0). */
    const float *sigma_per_iter; /* sigma_i in pixels (finite, > 0); copied by hb_set_params */
    int32_t directed_mode;      /* HB_DIRECTED_ONCE (default): the push follows the first
                                   sampling only, i.e. the resampling of iteration 0 of the
                                   schedule, as the pipeline of Section 3 pushes once and then
                                   loops from the resampling, which keeps the offset (it
                                   interpolates along the pushed polyline). HB_DIRECTED_EVERY_ITER:
                                   the push follows the resampling of every iteration, so the
                                   offset is renewed against the bundling each time. */
} hb_params;

/* Fill p with the paper's defaults for a W x H grid: bbox [0,0,1,1], delta 1 px, P = 3,
 * radius W/32 for every iteration, h_max = 2 sigma(r_0), lambda 0.9, eps 1e-6, K = 8,
 * s = 0.5, one smoothing pass, last-pass density, capacity factor 2. Host only. */
void hb_default_params(hb_params *p, int32_t grid_w, int32_t grid_h);

/* Check p without a context or a device (the same checks hb_set_params makes). */
hb_status hb_validate_params(const hb_params *p);

/* Create a context on HIP device `device`. hip_stream is a hipStream_t on that device or
 * NULL (the context creates its own stream of default priority). */
hb_status hb_create(hb_ctx **out, int32_t device, void *hip_stream);

/* Free every device buffer of ctx; NULL is accepted. Waits for the context's stream. */
void hb_destroy(hb_ctx *ctx);

/* Set the parameters (Section 3; see hb_params). May be called between runs. */
hb_status hb_set_params(hb_ctx *ctx, const hb_params *p);

/* Set the graph G = {N, E} (Section 3.1): node positions node_xy[n_nodes][2] in user
 * coordinates, edges (src[e], dst[e]) with integer weights 1 <= weight[e] <=
 * HB_MAX_EDGE_WEIGHT (NULL: all 1); a sample of edge e adds weight[e] to its pixel.
 * Resets the polylines to the straight segments and the iteration counter to 0.
 * Requires hb_set_params first (the grid and the bounding box). */
hb_status hb_set_graph(hb_ctx *ctx, int32_t n_nodes, const float *node_xy, int64_t n_edges,
                       const int32_t *src, const int32_t *dst, const int32_t *weight,
                       uint32_t flags);

/* Orientation bins of the edges (Section 5): the angle of the direction (dx, dy) from the
 * first to the last point of each current polyline (source to target; the end points never
 * move), in grid (pixel) coordinates measured from +x towards +y, discretised into 4 slices of
 * 90 degrees centred on 0, 90, 180 and 270 degrees: slice k holds the angles in
 * [90k - 45, 90k + 45), so an angle of exactly 45, 135, 225 or 315 degrees goes to the slice
 * above it; an edge whose end points coincide is in slice 0. Writes E int32 values in [0, 4)
 * to group (host memory, or device memory with HB_DEVICE_PTRS; caller-owned, E = the edge
 * count of hb_set_graph), ready for hb_set_groups with B = 4. Synchronous. Requires
 * hb_set_graph (HB_ESTATE otherwise); NULL group with E > 0 gives HB_EINVAL. */
hb_status hb_orientation_groups(hb_ctx *ctx, int32_t *group, uint32_t flags);

/* ---- grouping (Section 5): bins found by k-means on an edge property with the Euclidean
 * distance; the number of bins B chosen between 4 and 16 by the lowest Davies-Bouldin index,
 * k-means being run from many random initialisations for every B. */

/* edge properties of hb_edge_features (grid / pixel units, from the end points) */
enum {
    HB_FEAT_ORIGIN = 0,              /* (x_s, y_s): 2 floats per edge */
    HB_FEAT_DESTINATION = 1,         /* (x_t, y_t): 2 floats per edge */
    HB_FEAT_ORIGIN_DESTINATION = 2,  /* (x_s, y_s, x_t, y_t): 4 floats per edge */
    HB_FEAT_LENGTH = 3               /* |x_t - x_s| (FP64, rounded): 1 float per edge */
};
#define HB_KMEANS_MAX_K 64
#define HB_KMEANS_MAX_DIM 8

/* Write the property `kind` of every edge, E x dim floats row-major (dim 2, 2, 4 or 1), to out
 * (host memory, or device memory with HB_DEVICE_PTRS; caller-owned). cap_floats < E dim gives
 * HB_EINVAL. Requires hb_set_graph. Synchronous. */
hb_status hb_edge_features(hb_ctx *ctx, int32_t kind, float *out, int64_t cap_floats, uint32_t flags);

/* Lloyd's k-means of the n points X[n][dim] (float32 row-major; dim in [1, HB_KMEANS_MAX_DIM],
 * k in [1, HB_KMEANS_MAX_K], n >= k): each round assigns every point to its nearest centre
 * (squared Euclidean distance summed over the coordinates in order in FP64, ties to the lower
 * index), then moves every centre with points to their mean (a centre without points stays);
 * it stops when no label changes, or after max_iters rounds (then the labels are those of the
 * last round and the centres their means). centers[k][dim] (host, FP64) holds the starting
 * centres on entry and the final ones on return; labels[n] (int32) receives the clusters;
 * *inertia the sum of squared distances to the assigned centres, *rounds the rounds made
 * (either may be NULL). X and labels are host memory, or device memory with HB_DEVICE_PTRS.
 * Uses the context's device and stream (hb_set_graph not needed). Synchronous. */
hb_status hb_kmeans(hb_ctx *ctx, const float *X, int64_t n, int32_t dim, int32_t k, double *centers,
                    int32_t max_iters, int32_t *labels, double *inertia, int32_t *rounds,
                    uint32_t flags);

/* Davies-Bouldin index of the labelling labels[n] in [0, k) of X[n][dim]: with s_i the mean
 * distance of the points of cluster i to its centroid and d_ij the distance between centroids,
 * the mean over the non-empty clusters of max over j != i of (s_i + s_j) / d_ij (coincident
 * centroids count 0; fewer than two clusters give 0). Memory as in hb_kmeans. */
hb_status hb_davies_bouldin(hb_ctx *ctx, const float *X, int64_t n, int32_t dim, int32_t k,
                            const int32_t *labels, double *db, uint32_t flags);

/* hb_davies_bouldin for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same index, with X and
 * labels required in device memory of the context's device (no HB_DEVICE_PTRS flag: device
 * pointers are the only form) and db in host memory. The call allocates nothing: its work
 * memory is a fixed array of about 1.2 MB per GPU held by the library until the process ends
 * (the partial sums of chunks of 16384 points, added chunk by chunk in a fixed order, so the
 * result can differ from hb_davies_bouldin's in the last bits). k (dim + 1) + 2 <= 578, which
 * every k <= HB_KMEANS_MAX_K, dim <= HB_KMEANS_MAX_DIM meets. All calls on one GPU share that
 * array: calls that overlap on one GPU (from several contexts or threads) race. HB_ESTATE
 * while an asynchronous run of the context is pending; labels outside [0, k) give HB_EINVAL.
 * Synchronous on the context's stream. */
hb_status hb_davies_bouldin_noalloc(hb_ctx *ctx, const float *X, int64_t n, int32_t dim,
                                    int32_t k, const int32_t *labels, double *db);

/* The choice of B (Section 5): for every B in [kmin, kmax] (1 <= kmin <= kmax <=
 * HB_KMEANS_MAX_K, n >= kmax), `restarts` k-means runs of at most max_iters rounds, run r
 * starting from the B distinct points whose indices are the values t = 0, 1, ... of the
 * counter-based SplitMix64 stream value(seed, B, r, t) = mix(seed + 0x9E3779B97F4A7C15
 * (1 + t + 4096 (r + 1024 B))) taken modulo n (repeats skipped; mix is SplitMix64's output
 * function); the run of lowest inertia is kept (the first on a tie) and db[B - kmin] receives
 * its Davies-Bouldin index. *n_groups gets the B of the lowest index (the smallest on a tie)
 * and labels[n] its clusters. X and labels as in hb_kmeans; db is host memory. */
hb_status hb_choose_groups(hb_ctx *ctx, const float *X, int64_t n, int32_t dim, int32_t kmin,
                           int32_t kmax, int32_t restarts, uint64_t seed, int32_t max_iters,
                           int32_t *labels, int32_t *n_groups, double *db, uint32_t flags);

/* Set the edge groups b_e in [0, B) and the B x B interaction matrix M (Section 3.2 Eq. 3):
 * M[l * B + b] is the weight of bin b on layer l. B in [1, 64]. */
hb_status hb_set_groups(hb_ctx *ctx, int32_t n_groups, const int32_t *group, const float *M,
                        uint32_t flags);

/* Run n_iters iterations of the loop above, continuing the iteration counter (which sets
 * the radius r_i and the step h_i). Stream ordered; waits at the end unless HB_RUN_ASYNC. */
hb_status hb_run(hb_ctx *ctx, int32_t n_iters, uint32_t flags);

/* Wait for the context's stream and report deferred errors of an asynchronous run. */
hb_status hb_sync(hb_ctx *ctx);

/* Number of points of the state or of the last sample set (HB_POINTS_*). */
hb_status hb_get_num_points(hb_ctx *ctx, int32_t which, int64_t *n_points);

/* Copy offsets[E+1] and xy[N][2] of the state or of the last samples. cap_points is the
 * capacity of xy in points. */
hb_status hb_get_points(hb_ctx *ctx, int32_t which, int64_t *offsets, float *xy,
                        int64_t cap_points, uint32_t flags);

/* Replace the polylines (resume from saved points, or inject test inputs). Every edge
 * needs at least two points. The iteration counter is not changed. */
hb_status hb_set_points(hb_ctx *ctx, const int64_t *offsets, const float *xy,
                        int64_t n_points, uint32_t flags);

/* Copy one map of the last iteration: kind HB_MAP_*, group (or layer) index, pass (1..P,
 * for HB_MAP_BOX only). bytes is the size of out. */
hb_status hb_get_map(hb_ctx *ctx, int32_t kind, int32_t group, int32_t pass, void *out,
                     int64_t bytes, uint32_t flags);

/* Accepted halving index j (step h / 2^j) of every sample point of the last iteration run
 * with HB_RUN_RECORD_DECISIONS: -1 no move, -2 end point. */
hb_status hb_get_decisions(hb_ctx *ctx, int8_t *jacc, int64_t cap_points, uint32_t flags);

/* Sample-point counts N_i of the iterations of the last hb_run (host array of n_iters). */
hb_status hb_get_iter_counts(hb_ctx *ctx, int64_t *counts, int32_t cap);

/* Total polyline length of the state ("ink"), summed in FP64. */
hb_status hb_get_ink(hb_ctx *ctx, double *ink);

/* Iteration counter (the index i of the next iteration). */
hb_status hb_get_iteration(hb_ctx *ctx, int32_t *iter);
hb_status hb_set_iteration(hb_ctx *ctx, int32_t iter);

/* Message of the last error of ctx (ctx NULL: of the calling thread). */
const char *hb_last_error(const hb_ctx *ctx);

/* Library version string. */
const char *hb_version(void);

/*
 * Batched form: many independent graphs (each in its own context, all on one device) advance
 * together. Every stage of an iteration is one kernel launch for the whole batch, over a
 * device table of per-graph descriptors; graphs may differ in edge count, group count, grid
 * size and schedule. Launches go to the stream of ctxs[0] (the streams of the other contexts
 * are drained first). flags: HB_RUN_ASYNC, HB_RUN_GRAPH, HB_RUN_RECORD_DECISIONS (each
 * context keeps the decisions of its last iteration). A context whose point buffers
 * overflow is grown and finished on its own stream. Errors name the first failing context in
 * hb_last_error(ctxs[0]).
 */
hb_status hb_batch_run(hb_ctx *const *ctxs, int32_t n, int32_t n_iters, uint32_t flags);

/* Choose the launch shapes of a batch by timing n_iters iterations of each candidate from the
 * current polylines and restoring them afterwards, one shape at a time (each stage keeps the
 * best of the stages before it): the work chunks per trip of the resampling and advection
 * kernels (1, 2 or 4 each), the rows per thread of the column box pass (64, 128, 256), the
 * tile-count sets of the splat, i.e. how many privatised copies of the per-tile counters
 * the edge blocks spread their atomics over (4, 16, 64; fewer when the counters of all sets
 * would pass 2^18), and the entries per tile-histogram work item (2^14 .. 2^17). Every
 * choice gives the same results bit for bit. The choice is stored in every context and,
 * when choice is not NULL, written to choice[5] = {resample chunks, advect chunks, column
 * rows, sets, log2 item entries}. */
hb_status hb_autotune(hb_ctx *const *ctxs, int32_t n, int32_t n_iters, int32_t *choice);

/* Set / read the kernel variants directly (chunks 1, 2 or 4). */
hb_status hb_set_tuning(hb_ctx *ctx, int32_t resample_chunks, int32_t advect_chunks);
hb_status hb_get_tuning(hb_ctx *ctx, int32_t *resample_chunks, int32_t *advect_chunks);

/* Set / read the map-stage launch shapes directly: rows per thread of the column box pass (a
 * power of two in [16, 1024]), the most tile-count sets of the splat (a power of two in
 * [1, 64]) and log2 of the entries per tile-histogram work item (in [12, 20]). Results do
 * not depend on them. Setting them discards the checkpoints of hb_forward_ckpt. */
hb_status hb_set_tiling(hb_ctx *ctx, int32_t col_rows, int32_t sets_max, int32_t item_entries_log2);
hb_status hb_get_tiling(hb_ctx *ctx, int32_t *col_rows, int32_t *sets_max, int32_t *item_entries_log2);

/*
 * Differentiable form. With the discrete choices of a forward run held fixed (sample counts
 * and interpolation segments of every resampling, the histograms -- so the integer box sums
 * are constants -- and the accepted halving of every point), T iterations of Section 3 are a
 * piecewise smooth function of the polylines that entered them, of the interaction matrix M
 * (Eq. 3-4) and of the pass weights a of the density. hb_backward applies the transpose of
 * its Jacobian to the gradient of a loss of the final polylines: one the caller supplies,
 * or by default L = total length of the final polylines ("ink").
 *
 * hb_forward_ckpt runs n_iters iterations like hb_run from the context's current iteration
 * (hb_set_iteration) and keeps, for every iteration, the polylines entering it (with their
 * lengths and next sample counts) on the device; it needs B <= 16. *generation (may be NULL)
 * receives a number that identifies these checkpoints: it grows with every call on the
 * context. Any later call that changes the polylines, the parameters, the groups or the
 * iteration counter discards the checkpoints. flags: none (0).
 */
hb_status hb_forward_ckpt(hb_ctx *ctx, int32_t n_iters, uint32_t flags, int64_t *generation);

/* After hb_forward_ckpt. generation: the value hb_forward_ckpt returned (HB_ESTATE when the
 * context's checkpoints are not those any more), or -1 for the current checkpoints.
 * dL_dxy_T[n_points_T][2] (may be NULL): gradient of the caller's loss with respect to the
 * final polylines (the state of hb_get_points, in its layout); n_points_T must equal their
 * point count (HB_EINVAL otherwise). NULL selects the ink loss. loss (may be NULL) receives
 * the ink of the final polylines. Outputs: dL_dM[B*B] (row-major, may be NULL); dL_da[P] (may
 * be NULL); dL_dxy0[N0][2] (may be NULL) = gradient with respect to the points of the
 * polylines that entered the checkpointed run (N0 of them, same layout as hb_get_points;
 * cap_points is the capacity of dL_dxy0 in points). Each iteration is recomputed from its
 * checkpoint; all reductions run in a fixed order (bit-reproducible). The checkpoints stay,
 * so several losses can be differentiated in turn. flags: HB_DEVICE_PTRS for dL_dxy_T and
 * dL_dxy0 (device memory of the context's device, read and written in stream order). */
hb_status hb_backward(hb_ctx *ctx, int64_t generation, const float *dL_dxy_T, int64_t n_points_T,
                      double *loss, float *dL_dM, float *dL_da, float *dL_dxy0,
                      int64_t cap_points, uint32_t flags);

/* Polylines that entered checkpointed iteration t (0 = the start of the run). */
hb_status hb_get_ckpt_points(hb_ctx *ctx, int32_t t, int64_t *offsets, float *xy,
                             int64_t cap_points, uint32_t flags);

/* Sample offsets [E+1] and accepted halving index of every sample [N_t] of checkpointed
 * iteration t (the discrete choices the adjoint holds fixed; same codes as
 * hb_get_decisions). cap_points is the capacity of jacc in samples. */
hb_status hb_get_ckpt_decisions(hb_ctx *ctx, int32_t t, int64_t *offsets, int8_t *jacc,
                                int64_t cap_points, uint32_t flags);

/* Stages of one iteration, for hb_get_stage_times. */
enum {
    HB_STAGE_SCAN = 0,            /* sample-count scan -> offsets */
    HB_STAGE_CLEAR = 1,           /* histogram clear */
    HB_STAGE_RESAMPLE_SPLAT = 2,  /* resampling + samples per histogram tile (or counting
                                     the given samples) */
    HB_STAGE_BOX = 3,             /* one box pass (row + column kernels) */
    HB_STAGE_DENSITY_GRAD = 4,    /* density stack + gradient */
    HB_STAGE_ADVECT_SMOOTH = 5,   /* advection + Laplacian smoothing + next counts */
    HB_STAGE_BIN = 6,             /* splatting: samples binned by tile, tile histograms in LDS */
    HB_NUM_STAGES = 7
};

/* Enable (1) or disable (0) per-stage timing with HIP events on the context's stream.
 * While enabled, every stage launch of hb_run is bracketed by two events. */
hb_status hb_set_profiling(hb_ctx *ctx, int32_t enable);

/* Accumulated stage times (milliseconds) and launch counts since profiling was enabled or
 * last reset; ms and launches are arrays of n_stages (<= HB_NUM_STAGES). reset != 0 clears
 * the accumulators after reading. */
hb_status hb_get_stage_times(hb_ctx *ctx, double *ms, int64_t *launches, int32_t n_stages,
                             int32_t reset);

/* ---- rendering (Section 3.4): the density map sets the width of the drawn bundles. */

/* Width of every point of the current polylines (the state of hb_get_points, in its order)
 * from the density of the edge's own layer at the point. The maps are rebuilt from the
 * polylines taken as samples (splat of the current splat_mode, the box radii of iteration
 * `iter` >= 0, the densities of Eq. 3; no resampling or advection), so the context's maps
 * then hold these (hb_get_map). Per point: dens = the bilinear density of its edge's layer at
 * the point (taps as in the advection; negative values count 0) and
 * width = w_min + (w_max - w_min) f(dens) / f(max dens), f(x) = x (log_scale 0) or
 * log(1 + x) (log_scale 1), in FP32; all points get w_min when the largest density is 0. w_min and
 * w_max finite with 0 <= w_min <= w_max. dens (may be NULL) and widths receive n_state floats
 * each: host memory, or device memory with HB_DEVICE_PTRS; caller-owned; cap_points < n_state
 * gives HB_EINVAL. A histogram bin or splat-entry overflow gives HB_EOVERFLOW. Synchronous. */
hb_status hb_point_widths(hb_ctx *ctx, int32_t iter, float w_min, float w_max, int32_t log_scale,
                          float *dens, float *widths, int64_t cap_points, uint32_t flags);

#ifdef __cplusplus
}
#endif

#endif /* HB_H */
