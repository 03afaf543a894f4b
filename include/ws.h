/*
 * ws.h -- C ABI of the MI355X (gfx950) watershed / waterfall library.
 *
 * Implements the hot path of "Parallel Watershed Partitioning: GPU-Based
 * Hierarchical Image Segmentation" (arXiv 2410.08946): gradient pre-processing,
 * the watershed transform of Alg. 1 (Steps I-IV) and repeated waterfall levels
 * (Section 4, Alg. 4 Step V and the hierarchical loop of Alg. 5).
 *
 * General conventions (every entry point):
 *   - Images are C-contiguous with x fastest: pixel p = x + nx*(y + ny*z)
 *     (the row-major pixel order Step I requires, Section 3.1). nz == 1 is a
 *     2D image; ny == nz == 1 a 1D row (only the +-x neighbours exist).
 *   - Pointers named img/grad/labels/out/mag/nregions are DEVICE pointers on
 *     the context's device, allocated and owned by the caller. The library
 *     never frees them and keeps no reference to them after the work it
 *     enqueued has completed.
 *   - `stream` is a hipStream_t (NULL = the default stream). Calls validate
 *     their arguments synchronously, then enqueue work on `stream` and return.
 *     Some calls wait on `stream` internally to read a convergence counter
 *     (documented per call). Results are ready once `stream` has completed.
 *   - Return value: WS_OK or a negative ws_status. On WS_EINVAL nothing was
 *     written and nothing was launched. ws_last_error() gives a message.
 *   - Calls on one context are not thread-safe; use one context per thread.
 *   - Maximum size: nx*ny*nz < 2^31 (labels are int32 pixel indices).
 */
#ifndef WS_H
#define WS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum ws_status {
    WS_OK = 0,
    WS_EINVAL = -1,       /* bad argument: nothing written, nothing launched */
    WS_ENOMEM = -2,       /* device workspace allocation failed */
    WS_EDEVICE = -3,      /* a HIP runtime call failed */
    WS_ENOCONV = -4,      /* the Step II sweep cap was reached before convergence */
    WS_EUNSUPPORTED = -5  /* valid request the library does not implement */
};

/* Grey-value types of a quantised gradient image. */
enum ws_dtype {
    WS_U8 = 1,   /* uint8_t,  values 0..255   */
    WS_U16 = 2   /* uint16_t, values 0..65535 */
};

typedef struct ws_ctx ws_ctx;

/*
 * Create a context bound to HIP device `device`. The context owns all device
 * scratch memory (grow-only; freed by ws_destroy).
 *   scratch_budget_bytes  upper bound on the device scratch the context may
 *          hold at once (0 = no bound). A call whose scratch would exceed it
 *          returns WS_ENOMEM; every call except ws_rag sizes all its scratch
 *          before launching anything, so nothing was launched then (ws_rag
 *          sizes its sort buffers after counting the edges on the device).
 *          The caller's own buffers (images, labels) do not count.
 * Returns WS_EINVAL for a bad device index or NULL ctx, WS_EDEVICE if the
 * device cannot be used.
 */
int ws_create(ws_ctx **ctx, int device, size_t scratch_budget_bytes);

/* Free the context and its device scratch memory. NULL is ignored. The
 * caller must make sure no work of this context is still running. */
void ws_destroy(ws_ctx *ctx);

/* Message of the last failed call on this context ("" if none). With a NULL
 * context: the message of the last argument error seen with no context. */
const char *ws_last_error(const ws_ctx *ctx);

/* Wait for `stream`; returns WS_EDEVICE if the device reported an error. */
int ws_sync(ws_ctx *ctx, void *stream);

/*
 * Device bytes one watershed + waterfall job of this size needs: the job's own
 * buffers (gradient, NL label layers) plus the context scratch it uses
 * (distances and border records of the watershed; for NL >= 2 the dense
 * region tables and the per-tile edge slabs of the waterfall, whose size
 * grows with conn). Pure host arithmetic; 0 on invalid sizes, dtype, NL or a
 * conn that does not match the dimensionality.
 */
size_t ws_footprint_bytes(int64_t nx, int64_t ny, int64_t nz, int conn, int dtype, int NL);

/*
 * Gradient magnitude pre-processing (Introduction: smooth, then gradient
 * magnitude; Fig. "PRUF pipeline" caption: both optional before Step I).
 *   img    float32[N] input image.
 *   sigma  Gaussian blur sigma; <= 0 skips the blur. The blur is separable,
 *          radius floor(4*sigma + 0.5) (at most 64), weights exp(-k^2/2s^2)
 *          normalised, borders mirrored half-sample-symmetrically.
 *   dtype  WS_U8 or WS_U16: quantisation to 0..Q (Q = 255 or 65535) as
 *          rint(mag * Q / max(mag)) (ties to even), all zero if max is 0.
 *   grad   uint8_t[N] or uint16_t[N] output (device).
 *   mag    optional float32[N] output of the unquantised magnitude.
 * The magnitude is the unnormalised Sobel magnitude: per axis the taps
 * [-1, 0, 1] along it and [1, 2, 1] along every other axis (2D: 3x3, 3D:
 * 3x3x3), borders replicated. Arithmetic in float32; summation order per
 * pixel is fixed, so results do not depend on launch configuration.
 * Fully asynchronous (the maximum stays on the device).
 */
int ws_gradient(ws_ctx *ctx, const float *img, int64_t nx, int64_t ny, int64_t nz, float sigma,
                int dtype, void *grad, float *mag_or_null, void *stream);

/*
 * Watershed transform (Alg. 1, Steps I-IV) of an integer gradient image.
 *   grad    uint8_t[N] / uint16_t[N] grey values (read only).
 *   conn    4 or 8 when nz == 1; 6 or 26 when nz > 1 (von Neumann / Moore
 *           neighbourhoods of Section 3.1; out-of-image pixels are not
 *           neighbours).
 *   labels  int32[N] output: every pixel's catchment basin, named by the
 *           smallest linear pixel index in that basin (canonical label).
 * Arrows follow Eq. (1) (largest index among the lowest neighbours).
 * Non-minimal plateau pixels point to the equal neighbour one geodesic step
 * closer to the plateau's lower border, the smallest index among several
 * (the fair split of Sections 3.3-3.4). Minimal plateaux form one basin each
 * (Step IV). The result is a pure function of (grad, dims, conn).
 * Waits on `stream` a few times to read the Step II convergence counter.
 * Returns WS_ENOCONV if the sweep cap set with ws_set_option was reached.
 */
int ws_watershed(ws_ctx *ctx, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz,
                 int conn, int32_t *labels, void *stream);

/*
 * ws_watershed for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, result and options as ws_watershed under the tile
 * schedule, but its scratch (distances, tile stamps, counters, border
 * records) lives in a fixed device area of WS_NOALLOC_SCRATCH_MIB MiB that
 * the library holds on every device it runs on until the process ends; the
 * call allocates nothing (no hipMalloc, hipFree or allocating library call),
 * and it is never captured into a launch graph.
 *   Limit: the image's scratch (4 bytes per pixel plus 20 bytes per tile plus
 *   4 bytes per tile border cell) must fit the area: WS_EINVAL (nothing
 *   launched) otherwise. At the default tile shapes that holds up to about
 *   30 Mpx in 2D and 22 Mvoxel in 3D (4096 x 4096 and 256^3 fit).
 *   Every call on one device shares that device's area and leaves its
 *   contents behind (each call clears what it reads before use): calls that
 *   overlap in time on one device, from any context or stream, race.
 *   WS_EUNSUPPORTED for options "schedule" = 1 or "step4" = 1.
 * Waits on `stream` like ws_watershed.
 */
#define WS_NOALLOC_SCRATCH_MIB 128
int ws_watershed_noalloc(ws_ctx *ctx, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz,
                         int conn, int32_t *labels, void *stream);

/*
 * Hierarchical waterfall (Section 4 / Alg. 5 layer loop): NL layers.
 *   labels     int32[N] canonical watershed labels (layer 0); may alias out.
 *   grad       the grey values the watershed was computed from (read only).
 *   NL         number of layers >= 1, layer 0 included.
 *   out        int32[NL*N] output, layer k at out + k*N, canonical labels.
 *   nregions   optional int64[NL] device output: region count per layer.
 * Layer k joins every region of layer k-1 with the region across its lowest
 * boundary pass: key(R) = min over pixel pairs (p in R, q in N(p) outside R)
 * of (max(I(p), I(q)), label(q)) compared lexicographically (Alg. 4 Step V
 * height; ties broken by the smaller neighbouring label). Joined groups take
 * their smallest label. Layers are nested and counts at least halve while
 * more than one region remains. Fully asynchronous.
 */
int ws_waterfall(ws_ctx *ctx, const int32_t *labels, const void *grad, int dtype, int64_t nx,
                 int64_t ny, int64_t nz, int conn, int NL, int32_t *out, int64_t *nregions_or_null,
                 void *stream);

/*
 * One image of a batched call (ws_batch).
 *   grad      grey values (device, u8/u16 as the batch's dtype), read only.
 *   nx,ny,nz  its size (same rules as ws_watershed).
 *   conn      its connectivity: 4 or 8 when nz == 1, 6 or 26 when nz > 1
 *             (Section 3.1 neighbourhoods); items of one batch may differ.
 *   out       int32[NL*N] (device): layer k at out + k*N, canonical labels
 *             local to the image (smallest pixel index of the image).
 *   nregions  optional int64[NL] (device): region count per layer.
 */
typedef struct {
    const void *grad;
    int64_t nx, ny, nz;
    int32_t conn;
    int32_t *out;
    int64_t *nregions;
} ws_item;

/*
 * Reconstruction waterfall, the paper's literal procedure (Alg. 4 Steps V-VI
 * followed by the watershed again, as in the Alg. 5 layer loop): layer 0 is
 * `labels`; for every later layer each region R of the previous layer gets
 * newmin(R) = min over pixel pairs (p in R, q in N(p) outside R) of
 * max(I(p), I(q)) (65535 for a region without boundary), the image is raised
 * to I(p) = max(I(p), newmin(region of p)), and layer k is the watershed
 * (canonical labels) of the raised image. The raised image starts from `grad`
 * and is kept by the context as uint16; `grad` is not written.
 *   labels, grad, dtype, sizes, conn, NL, out, nregions: as for ws_waterfall.
 * Unlike ws_waterfall the layers need not be nested (a region can be split).
 * Waits on `stream` like ws_watershed (once per layer after the first).
 * Returns WS_ENOCONV if a watershed reached the sweep cap.
 */
int ws_waterfall_recon(ws_ctx *ctx, const int32_t *labels, const void *grad, int dtype, int64_t nx,
                       int64_t ny, int64_t nz, int conn, int NL, int32_t *out,
                       int64_t *nregions_or_null, void *stream);

/*
 * Region adjacency graph of one labelling (the graph the waterfall's layers
 * are built on, Section 4): every pair of regions a < b (canonical labels)
 * that share a boundary, with h = min over pixel pairs (p in a, q in N(p) in
 * b) of max(I(p), I(q)), the pair's lowest pass.
 *   labels    int32[N] canonical labels (the watershed's, or any layer of
 *             ws_waterfall / ws_waterfall_recon); read only.
 *   grad, dtype, sizes, conn: as for ws_waterfall.
 *   capacity  entries the three edge buffers hold (may be 0).
 *   edge_a, edge_b, edge_h  int32[capacity] device outputs: the edges sorted
 *             by (a, b); the first min(count, capacity) are written.
 *   n_edges   int64 device output (may be NULL): the number of edges (count).
 * Waits on `stream` once (to size its sort buffers). A call with capacity 0
 * returns the count only, so a caller can size the buffers and call again.
 */
int ws_rag(ws_ctx *ctx, const int32_t *labels, const void *grad, int dtype, int64_t nx, int64_t ny,
           int64_t nz, int conn, int64_t capacity, int32_t *edge_a, int32_t *edge_b, int32_t *edge_h,
           int64_t *n_edges, void *stream);

/*
 * Watershed + NL-layer waterfall of many images of uneven sizes, 2D and 3D
 * mixed, in one set of launches: images are grouped by connectivity, every
 * tile kernel covers the tiles of one group's images through a tile -> image
 * table, and the Step II convergence loop and the region-level waterfall
 * passes are shared by all images. The result of every image is
 * bit-identical to ws_watershed followed by ws_waterfall on it alone.
 *   items    host array of n_items >= 1 items (each with its own conn); the
 *            total pixel count must be below 2^31.
 *   dtype    grey type of every item.
 * Waits on `stream` a few times (Step II convergence, and to reuse the
 * pinned staging of the previous call's tables). Same errors as ws_watershed;
 * WS_EINVAL names the first offending item.
 */
int ws_batch(ws_ctx *ctx, const ws_item *items, int n_items, int dtype, int NL, void *stream);

/*
 * Step-level outputs of the watershed for verification (Alg. 1, Steps I-II;
 * balanced encoding of Section 3.4).
 *   bal    int32[N]: -d for a non-minimal plateau pixel resolved at geodesic
 *          distance d >= 1 from its plateau's lower border; otherwise the
 *          Step I state (0 lower neighbour, 1 local minimum, 2/3 minimal
 *          plateau pixel with / without an equal neighbour after it).
 *   arrow  int32[N]: the pointer L after Step II (Eq. (1) target for states 0
 *          and 2, itself for states 1 and 3, the chosen equal neighbour for a
 *          resolved plateau pixel).
 * Same waiting behaviour and errors as ws_watershed.
 */
int ws_watershed_stages(ws_ctx *ctx, const void *grad, int dtype, int64_t nx, int64_t ny,
                        int64_t nz, int conn, int32_t *bal, int32_t *arrow, void *stream);

/*
 * Options. None of them changes any result, only time.
 *   "schedule"     0 = tile schedule (default): LDS tiles, fused Steps
 *                  III-IV inside tiles, global union-find across them.
 *                  1 = per-pixel synchronous schedule of Section 3.3: one
 *                  thread per pixel, one launch per Step II sweep, per Step
 *                  III synchronisation and per Step IV pass, Step II decisions
 *                  taken from the previous sweep's states. Applies to
 *                  ws_watershed and ws_watershed_stages; ws_batch,
 *                  ws_waterfall_recon and ws_rag always use the tile schedule.
 *                  Step II needs as many sweeps as the longest geodesic
 *                  distance in a non-minimal plateau (one counter read-back
 *                  per "sweep_batch" sweeps).
 *   "step3"        0 = per-pixel Find (APRUF, Section 3.2), 1 = RR pointer
 *                  jumps per synchronisation (PRUF, Alg. 1 Step III).
 *   "step4"        0 = union-find over adjacent minimal-plateau pixels
 *                  (PRUF / APRUF, Alg. 1 Step IV); 1 = the label exchange
 *                  passes of PRW (Alg. 2), repeated until a pass changes
 *                  nothing. 1 needs schedule = 1: ws_watershed returns
 *                  WS_EUNSUPPORTED for it under the tile schedule.
 *   "rr"           reduction rate for step3 = 1 (default 6, Section 5).
 *   "sweep_batch"  Step II sweeps launched per convergence read (default 4).
 *   "max_sweeps"   cap on Step II sweeps; reaching it returns WS_ENOCONV
 *                  (default 2^31-1).
 *   "timing"       1 = record a HIP event pair around every kernel launch.
 *   "graph"        1 = ws_gradient, ws_watershed, ws_waterfall and ws_batch
 *                  replay launch graphs: a call is captured
 *                  (hipStreamBeginCapture on a stream of the context) the
 *                  second time the same arguments (pointers, sizes, options)
 *                  are seen, and its instantiated graph is launched on
 *                  `stream` for every later identical call. Buffers are read
 *                  when the graph runs, so their contents may change between
 *                  calls. A captured ws_watershed / ws_batch launches a fixed
 *                  number of Step II sweeps (each returns at once after a sweep
 *                  that changed nothing): one more than the previous direct
 *                  run of the same arguments needed, plus one; the call then
 *                  waits once for `stream` and reads the last sweep's counter,
 *                  and if that sweep still changed distances it runs again
 *                  directly (result unchanged) and the next identical call is
 *                  captured anew. ws_batch's captured graph reads a device copy
 *                  of its image tables that it owns. With "step3" = 1 the
 *                  watershed is never captured. Any scratch reallocation drops
 *                  the graphs. Ignored while "timing" is on. Default 0.
 *   "tile2d", "tile3d"  watershed tile shape of 2D / 3D images (shape ids):
 *                  2D 2 = 64x32 (default), 12 = 128x16, 22 = 32x32,
 *                  32 = 64x64; 3D 3 = 32x8x8 (default), 13 = 16x16x8,
 *                  23 = 32x16x8, 33 = 16x16x16 (x fastest). Tiles of 64x64,
 *                  32x16x8 and 16x16x16 keep up to 512 unresolved plateau
 *                  pixels in their Step II list, the others 256. Block size
 *                  changes only time (Section 5, parameters paragraph).
 *   "reserve_pixels"  allocate now the scratch (device buffers, batch tables
 *                  and the pinned staging) of calls covering up to this many
 *                  pixels, so later calls do not allocate (allocation waits
 *                  for the whole device): any 2D/3D mix, conn 4/6/8, NL <= 8,
 *                  up to 1024 images per ws_batch call, each image either
 *                  smaller than one tile or with sides of at least about 300
 *                  (2D) / 100 (3D) pixels (thinner images need more partial
 *                  tiles and may still grow the scratch); out[5] of
 *                  ws_get_stats counts the allocations. May return WS_ENOMEM.
 * Returns WS_EINVAL for an unknown name or out-of-range value.
 */
int ws_set_option(ws_ctx *ctx, const char *name, int64_t value);

/*
 * Counters of the last ws_watershed call: out[0] Step II sweeps launched
 * (including the initial tile pass), out[1] sweeps that changed a tile
 * border, out[2] Step III synchronisations (step3 = 1), out[3] tiles;
 * out[4] the launch graphs replayed by this context so far ("graph" option);
 * out[5] the device and pinned host allocations this context has made;
 * out[6] Step IV passes that changed a label (step4 = 1). Under schedule = 1,
 * out[0] counts the Step I pass and the sweeps, out[3] is 0.
 * Returns the number of counters written (<= n).
 */
int ws_get_stats(const ws_ctx *ctx, int64_t *out, int n);

/*
 * Per-kernel timings recorded while the "timing" option was on, summed by
 * kernel name since the last ws_timing_reset. Waits for all recorded events.
 * Writes up to `cap` entries (name copied into names + i*name_len), returns
 * the number of kernel names recorded, or a negative ws_status.
 */
int ws_timing_read(ws_ctx *ctx, char *names, int name_len, double *total_ms, int64_t *launches, int cap);
int ws_timing_reset(ws_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* WS_H */
