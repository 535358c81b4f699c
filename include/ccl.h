/*
 * ccl.h -- C ABI of libccl, union-find connected-components labeling of 2D
 * binary images on AMD Instinct MI355X (gfx950).
 *
 * Method: the three phases of Chen et al., "An Optimized Union-Find
 * Algorithm for Connected Components Labeling Using GPUs" (arXiv 1708.08180):
 *   1. local union-find merge with coarse (row-run) labeling inside each tile
 *      (Sec. II-A, Kernel 1),
 *   2. boundary analysis that runs union-find only on tile-edge cells
 *      (Sec. II-B, Kernel 2, Eqs. (1)-(2)),
 *   3. link: every pixel is resolved to the root of its tree (Sec. II-C).
 *
 * Output contract (every entry point): labels[y*W + x] = 0 for a background
 * pixel (value 0); for a foreground pixel (any nonzero value) it is 1 plus
 * the smallest raster index y'*W + x' over the pixel's connected component.
 * The merge always links the larger index under the smaller (Sec. II-A-3),
 * so the root of every component is its smallest index; the +1 keeps 0 free
 * for background.  Raster indices use the width W, never the row pitch.
 * The labeling is unique, so results are bit-exact and deterministic.
 *
 * Linking: libccl.so does not link a HIP runtime itself; it binds to the
 * libamdhip64 the host process provides (link the program with -lamdhip64,
 * or load the runtime with RTLD_GLOBAL before loading libccl.so).  Device
 * pointers and streams passed in must come from that same runtime.
 *
 * Conventions
 *   - Pointers named img/labels/workspace are DEVICE pointers (hipMalloc or
 *     equivalent) unless stated; descriptor arrays are HOST pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously; the caller synchronizes.
 *   - Every entry point validates all arguments before enqueuing anything
 *     and returns a ccl_status.  No exception crosses the ABI.
 *   - img and labels must not overlap: an entry point whose image (or
 *     volume) bytes and label bytes intersect returns CCL_ERR_INVALID_ARG.
 *     The caller owns all buffers it passes; the library never frees them.
 *   - The contents of `labels` on entry are ignored; the buffer is fully
 *     overwritten.  It also serves as the union-find forest while the call
 *     runs, so it must not be read until the work on `stream` completes.
 */
#ifndef CCL_H_
#define CCL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ccl_status {
    CCL_OK = 0,
    CCL_ERR_INVALID_ARG = 1,  /* null pointer, H or W <= 0, pitch < W, n < 0, bad option */
    CCL_ERR_UNSUPPORTED = 2,  /* connectivity not in {4, 8}, unsupported tile config */
    CCL_ERR_TOO_LARGE = 3,    /* H*W > 2^32 - 1: a label would overflow uint32 */
    CCL_ERR_HIP = 4,          /* a HIP runtime call or launch failed; see ccl_last_hip_error */
    CCL_ERR_OUT_OF_MEMORY = 5,/* a workspace allocation failed */
    CCL_ERR_CAPACITY = 6,     /* a batch exceeds the context's fixed capacity */
    CCL_ERR_WORKSPACE = 7     /* a caller-supplied workspace is too small */
} ccl_status;

/* Tile configuration of the three kernels.  A tile is 64 pixels wide (one
 * 64-lane wavefront spans a tile row) and tile_h rows tall; each workgroup
 * runs `waves` wavefronts, each owning tile_h / waves consecutive rows.
 * Supported pairs: tile_h in {16, 32, 64, 128}; waves in {1, 2, 4, 8, 16} with
 * tile_h / waves >= 2 and tile_h / waves <= 64 (the binary local merge gives every wavefront whole
 * two-row bands).  A zeroed struct or a NULL pointer selects the default. */
typedef struct ccl_config {
    int32_t tile_h;
    int32_t waves;
} ccl_config;

/* Human-readable name of a status code (static storage; never NULL). */
const char *ccl_status_string(int status);

/* hipError_t of the most recent CCL_ERR_HIP on the calling thread (0 if none). */
int ccl_last_hip_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int ccl_version(void);

/*
 * ccl_label_2d -- label one 2D binary image (Secs. II-A to II-C).
 *
 * img     device pointer to H rows of `pitch` bytes; pixel (y, x) is
 *         img[y*pitch + x]; nonzero = foreground.
 * H, W    image height and width in pixels, both >= 1, H*W <= 2^32 - 1.
 * pitch   row stride of img in bytes, pitch >= W.
 * connectivity  4 (edge neighbours, the paper's Kernel 1) or 8 (edge and
 *         corner neighbours).
 * labels  device pointer to a dense H*W uint32 array (row stride W),
 *         written as described at the top of this file.
 * stream  hipStream_t (void*), NULL for the null stream.
 *
 * Scratch: a per-(device, stream) workspace (about 1.5 bytes per pixel for
 * the default tiles) is allocated on first use and grown when a larger
 * image arrives on the same stream.  Both are stream-ordered allocations on
 * that stream (hipMallocAsync / hipFreeAsync): the old buffer is freed
 * after the work already enqueued on the stream, and the host does not
 * wait.  ccl_shutdown releases it.  Calls on the same stream, from any
 * thread, are ordered by the stream; calls on different streams use
 * different workspaces.  Callers that must not allocate at all pass their
 * own workspace to ccl_label_2d_ex.
 * Returns CCL_OK or an error; on error nothing has been enqueued (except
 * CCL_ERR_HIP from a failed launch).
 */
int ccl_label_2d(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                 int32_t connectivity, uint32_t *labels, void *stream);

/* Bytes of workspace ccl_label_2d_ex needs for an H x W image with tile
 * configuration cfg.  cfg NULL or zeroed: the library's choice, which the
 * tuning table may make per connectivity; the size then covers both
 * connectivities.  Writes *bytes; returns a status. */
int ccl_workspace_size(int32_t H, int32_t W, const ccl_config *cfg, size_t *bytes);

/*
 * ccl_label_2d_ex -- as ccl_label_2d, with an explicit tile configuration
 * and an optional caller-owned workspace.
 *
 * workspace, workspace_bytes  device buffer of at least
 *         ccl_workspace_size(H, W, cfg) bytes, 256-byte aligned, not in
 *         use by any other call until this call's work on `stream` has
 *         completed.  NULL selects the library's per-stream workspace.
 *         Too small: CCL_ERR_WORKSPACE.
 * cfg     tile configuration, NULL or zeroed = default.  Unsupported
 *         pairs return CCL_ERR_UNSUPPORTED.
 */
int ccl_label_2d_ex(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                    int32_t connectivity, uint32_t *labels, void *workspace,
                    size_t workspace_bytes, const ccl_config *cfg, void *stream);

/*
 * ccl_label_2d_noalloc -- ccl_label_2d for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, output, kernels and
 * default tile configuration as ccl_label_2d; the tile workspace is a fixed
 * array of CCL_NOALLOC_SCRATCH_BYTES in device memory, one per device, held
 * from the library's load until the process ends.  The call allocates and
 * frees nothing (its first call on a device looks the array's address up).
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: calls whose work overlaps on one device (different
 * streams, or host threads racing on unordered streams) race on it and give
 * wrong labels; calls ordered on one stream are safe.
 * Errors: as ccl_label_2d, plus CCL_ERR_WORKSPACE, before anything is
 * enqueued, when the image needs more workspace than the array holds
 * (ccl_workspace_size(H, W, NULL) > CCL_NOALLOC_SCRATCH_BYTES; a 4096 x 4096
 * image fits).
 */
#define CCL_NOALLOC_SCRATCH_BYTES (32u << 20)
int ccl_label_2d_noalloc(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                         int32_t connectivity, uint32_t *labels, void *stream);

/*
 * ccl_label_2d_timed -- ccl_label_2d with a HIP event recorded before,
 * between and after the three phases on `stream`; blocks until the work is
 * done and writes the elapsed milliseconds of phase 1 (local merge), phase 2
 * (boundary analysis) and phase 3 (link) to phase_ms[0..2] (host array of 3
 * floats).  Same labels and errors as ccl_label_2d_ex (library workspace).
 * Meant for measurement; the events add a few microseconds per call.
 */
int ccl_label_2d_timed(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                       int32_t connectivity, uint32_t *labels, const ccl_config *cfg,
                       void *stream, float *phase_ms);

/*
 * ccl_label_2d_equal -- equal-value labeling: every pixel, of any value and
 * background included, joins the 4- or 8-neighbours whose image value equals
 * its own (the literal "same property" test of Kernels 1 and 2, Sec. II-A/B,
 * applied to every value class).
 * Output: labels[y*W+x] = 1 + the smallest raster index y'*W+x' of the
 * pixel's equal-valued component (never 0).  Arguments, layout, ownership,
 * stream and workspace behaviour as in ccl_label_2d; cfg NULL or zeroed =
 * default.  Compiled tile configurations: (16,4), (32,2), (32,8), (64,4),
 * (64,8); any other cfg gives CCL_ERR_UNSUPPORTED.  The workspace is about
 * 2 bytes per pixel larger than the binary one (up to 64 runs per row).
 */
int ccl_label_2d_equal(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                       int32_t connectivity, uint32_t *labels, const ccl_config *cfg,
                       void *stream);

/* ------------------------------------------------------------ statistics
 *
 * Per-component statistics of a canonical labeling (the output of
 * ccl_label_2d or ccl_label_2d_equal): the size and location of every
 * component, the quantities the paper's introduction lists as the uses of
 * the labels. */

/* One component: label = 1 + smallest raster index of the component; area
 * = pixel count; inclusive bounding box; sums of the pixels' column (x) and
 * row (y) indices, so the centroid is (sum_x / area, sum_y / area). */
typedef struct ccl_component {
    uint32_t label, area;
    uint32_t x_min, y_min, x_max, y_max;
    uint64_t sum_x, sum_y;
} ccl_component;

/*
 * ccl_component_stats -- statistics of every component of `labels`.
 * labels    DEVICE, H x W u32, row stride W: a canonical labeling (0 =
 *           background; a component's pixels all hold 1 + the raster index
 *           of its first pixel).  Not modified.
 * out       DEVICE array of `capacity` records, caller-owned; record k is
 *           the component with the k-th smallest label.  Only the first
 *           `capacity` components are written (capacity 0: count only).
 * n_out     DEVICE pointer to one u32: the number of components (all of
 *           them, also beyond capacity).
 * stream    hipStream_t; asynchronous like ccl_label_2d, and uses the same
 *           per-stream workspace (about 0.2 bytes per pixel).
 * Errors: CCL_ERR_INVALID_ARG (null pointers, H or W <= 0, capacity < 0),
 * CCL_ERR_TOO_LARGE (H*W > 2^32-1), CCL_ERR_OUT_OF_MEMORY, CCL_ERR_HIP.
 * Behaviour on a labeling that is not canonical is undefined.
 */
int ccl_component_stats(const uint32_t *labels, int32_t H, int32_t W, ccl_component *out,
                        int64_t capacity, uint32_t *n_out, void *stream);

/*
 * ccl_label_2d_stats -- ccl_label_2d and ccl_component_stats in one call:
 * the link phase (Sec. II-C) also accumulates each component's area,
 * bounding box and coordinate sums while it holds every pixel's final root,
 * so the labels are not read back.
 * img, H, W, pitch, connectivity, labels   as for ccl_label_2d (binary).
 * out, capacity, n_out   as for ccl_component_stats: record k is the
 *           component with the k-th smallest label; the first `capacity`
 *           records are written (capacity 0: count only); *n_out = the
 *           number of components.
 * stream    hipStream_t; asynchronous.  Uses the per-stream workspace of
 *           ccl_label_2d plus about 0.3 bytes per pixel and 16 bytes per
 *           possible tile-local component (at most one per 2 x 2 pixels
 *           under 8-connectivity, one per 2 pixels under 4-connectivity).
 * cfg       tile configuration, or NULL / {0, 0}: the tuning table's for
 *           (H, W, connectivity), with tiles of more than 64 rows replaced
 *           by (64, 4).  Tiles of more than 64 rows are not compiled for
 *           this entry point (CCL_ERR_UNSUPPORTED).
 * Errors: as ccl_label_2d; CCL_ERR_INVALID_ARG also for a null n_out,
 * capacity < 0, or capacity > 0 with a null out.
 */
int ccl_label_2d_stats(const uint8_t *img, int32_t H, int32_t W, int64_t pitch, int32_t connectivity,
                       uint32_t *labels, ccl_component *out, int64_t capacity, uint32_t *n_out,
                       const ccl_config *cfg, void *stream);

/*
 * ccl_label_3d -- label a binary volume (the method on a 3D grid).
 * vol     DEVICE, D slices of H rows of W voxels: voxel (z, y, x) at
 *         vol[z * pitch_z + y * pitch_y + x]; nonzero = foreground.
 *         pitch_y >= W, pitch_z >= H * pitch_y (bytes).
 * connectivity  6 (face neighbours), 18 (faces and edges) or 26 (faces,
 *         edges and corners).
 * labels  DEVICE, dense D x H x W u32 (strides H*W and W), caller-owned;
 *         labels[(z*H + y)*W + x] = 0 for background, else 1 + the smallest
 *         raster index z'*H*W + y'*W + x' of the voxel's component.
 *         Overwritten; also used as the union-find forest while the call
 *         runs.  No workspace.
 * Errors: CCL_ERR_INVALID_ARG (null pointers, sizes <= 0, pitches too
 * small), CCL_ERR_UNSUPPORTED (connectivity), CCL_ERR_TOO_LARGE
 * (D*H*W > 2^32-1), CCL_ERR_HIP.
 */
int ccl_label_3d(const uint8_t *vol, int32_t D, int32_t H, int32_t W, int64_t pitch_y,
                 int64_t pitch_z, int32_t connectivity, uint32_t *labels, void *stream);

/* ------------------------------------------------------------------ batch
 *
 * A context labels many images of different sizes in one call (the batched
 * form): each phase is one launch over the tiles (edge segments) of all
 * images, numbered consecutively, with grids sized for the call; the three
 * launches can be replayed from a hipGraph whose kernel nodes are updated
 * with each call's grids and arguments.  Results are bit-identical to
 * ccl_label_2d on each image.
 */
typedef struct ccl_ctx ccl_ctx;

/* One image of a batch.  img and labels are device pointers with the same
 * meaning and layout as in ccl_label_2d. */
typedef struct ccl_image_desc {
    const uint8_t *img;
    uint32_t *labels;
    int32_t H, W;
    int64_t pitch;
} ccl_image_desc;

/* Fixed capacity of a context.
 * max_images  most images per call (>= 1).
 * max_pixels  most pixels per call, summed over images (>= 1); the tile
 *             workspace is sized for it with room for partial tiles.
 * cfg         tile configuration for every call ({0,0} = the library's
 *             choice per connectivity for one image of max_pixels pixels,
 *             since a call's grid covers the tiles of all its images; it
 *             can then be retuned with ccl_ctx_autotune).
 * use_graph   nonzero: build one three-node hipGraph per connectivity and
 *             replay it; when a call's grids or arguments differ from the
 *             previous call's, the nodes are updated first (after waiting
 *             for the context's previous call to finish on the device). */
typedef struct ccl_ctx_opts {
    int32_t max_images;
    int64_t max_pixels;
    ccl_config cfg;
    int32_t use_graph;
} ccl_ctx_opts;

/* Create a context on the current device; allocates its device buffers and
 * a pinned staging area once.  *out receives the handle. */
int ccl_ctx_create(ccl_ctx **out, const ccl_ctx_opts *opts);

/* Wait for the context's last call on the device and free everything it
 * owns. */
int ccl_ctx_destroy(ccl_ctx *ctx);

/*
 * ccl_label_batch -- label n images in one call (same output contract as
 * ccl_label_2d for every image).
 * descs  HOST array of n descriptors; copied into the context (the call
 *        returns before the GPU work finishes; the array may be reused
 *        immediately).
 * n      1 <= n <= max_images; 0 is a no-op.
 * Errors: CCL_ERR_INVALID_ARG for a bad descriptor (index not reported),
 * CCL_ERR_UNSUPPORTED for connectivity, CCL_ERR_CAPACITY when n or the
 * total tile count exceeds the context.  One context must not be used by
 * two host threads at once, and its calls must be ordered on the device:
 * the kernels of a call read the context's device buffers until they
 * finish and the next call overwrites them, so use one stream per context
 * (or order the streams yourself).  The staging area is reused only after
 * the previous call's copy has completed.  The call blocks only for those
 * two waits (staging reuse, graph update); back-to-back calls on the same
 * batch shape never block.
 */
int ccl_label_batch(ccl_ctx *ctx, const ccl_image_desc *descs, int32_t n, int32_t connectivity,
                    void *stream);

/* Tile configuration the context uses for `connectivity` (4 or 8): the one
 * it was created with, or the autotuner's choice.  Writes *out. */
int ccl_ctx_config(const ccl_ctx *ctx, int32_t connectivity, ccl_config *out);

/*
 * ccl_ctx_autotune -- choose the context's tile configuration for one
 * connectivity by timing the batch `descs` (n images, as in
 * ccl_label_batch) under every compiled configuration that fits the
 * context, `reps` calls each after one warm-up call on `stream`, and keep
 * the fastest for the context's later calls with that connectivity.  The
 * images' labels are overwritten (the last call leaves valid labels).
 * Blocks until the timing is done.  *best / *best_ms (either may be NULL)
 * receive the winner and its mean milliseconds per call.  A context
 * created with an explicit cfg keeps it: CCL_ERR_UNSUPPORTED.  Other
 * errors as ccl_label_batch; on error the previous configuration stays.
 * The workspace of a context created without a cfg is sized at creation
 * for every configuration (the largest need over tile heights), so tuning
 * never allocates.
 */
int ccl_ctx_autotune(ccl_ctx *ctx, const ccl_image_desc *descs, int32_t n, int32_t connectivity,
                     int32_t reps, void *stream, ccl_config *best, float *best_ms);

/* ----------------------------------------------------------------- serve
 *
 * A request loop for frames that arrive over time (the served form).  Frames
 * are device-resident images; the server owns the label buffers: a pool of
 * slots of max_frame_pixels labels each, as many as fit in hbm_budget bytes.
 * A scheduler thread admits submitted frames in arrival order while a slot
 * is free, and hands the admitted frames to every idle worker as one batch
 * (each worker has its own HIP stream, batch context and graph), so
 * frames that arrive while other batches run are admitted and start on the
 * next free worker while those batches are still on the device.  Labels and
 * their contract are exactly those of ccl_label_2d for every frame.
 * plain = 1 selects the per-frame baseline: one worker, one ccl_label_2d
 * call per frame, same admission and bookkeeping.
 */
typedef struct ccl_server ccl_server;

typedef struct ccl_server_opts {
    int32_t n_workers;         /* >= 1 device streams the batches overlap on */
    int32_t max_batch;         /* most frames per batch (1 in plain mode) */
    int64_t max_frame_pixels;  /* largest H*W a frame may have (slot size) */
    int64_t max_batch_pixels;  /* most pixels per batch (>= max_frame_pixels) */
    int64_t hbm_budget;        /* bytes of label slots (>= one slot) */
    int32_t connectivity;      /* 4 or 8, for every frame */
    ccl_config cfg;            /* tile configuration, {0,0} = library choice */
    int32_t use_graph;         /* workers replay their batch graphs */
    int32_t plain;             /* per-frame baseline (n_workers = max_batch = 1) */
} ccl_server_opts;

/* One finished frame.  labels points into the server's slot `slot` and
 * stays valid until ccl_server_release(slot).  Times are host steady-clock
 * nanoseconds: submission, slot granted, batch launched, completion seen
 * (t_done_ns = -1 when the frame's launch failed). */
typedef struct ccl_frame_result {
    uint64_t tag;
    uint32_t *labels;
    int32_t slot;
    int64_t t_submit_ns, t_admit_ns, t_launch_ns, t_done_ns;
} ccl_frame_result;

/* Create a server on the current device and start its scheduler thread. */
int ccl_server_create(ccl_server **out, const ccl_server_opts *opts);

/* Number of label slots the HBM budget bought. */
int ccl_server_slots(const ccl_server *s, int32_t *n_slots);

/* Enqueue one frame (device image, H x W, row pitch in bytes); returns at
 * once.  `tag` is returned with the result.  The image must stay unchanged
 * until the frame completes.  CCL_ERR_CAPACITY if H*W > max_frame_pixels. */
int ccl_server_submit(ccl_server *s, const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                      uint64_t tag);

/* Move up to `max` finished frames into out[] (completion order); *n_out
 * receives the count.  Returns the first error the loop met, else CCL_OK. */
int ccl_server_poll(ccl_server *s, ccl_frame_result *out, int32_t max, int32_t *n_out);

/* Give a finished frame's label slot back for admission.  Only a slot that
 * an admitted frame holds may be released, once: a slot outside
 * [0, n_slots) or one that is not held gives CCL_ERR_INVALID_ARG and
 * changes nothing. */
int ccl_server_release(ccl_server *s, int32_t slot);

/* Frames submitted and not yet finished. */
int ccl_server_pending(ccl_server *s, int64_t *in_flight);

/* Stop admitting, drop frames still waiting for a slot, wait for every
 * admitted frame to finish, and free everything. */
int ccl_server_destroy(ccl_server *s);

/* ---------------------------------------------------------------- tuning
 *
 * The tile configuration of ccl_label_2d is taken from a process-wide table
 * keyed by (size class = floor(log2(H*W)), connectivity); entries come from
 * ccl_autotune or ccl_tuning_load, misses use the built-in default:
 * tile_h 32 with 4 wavefronts below 2^22 pixels, tile_h 64 with 4 from
 * there up.  Equal-value labeling, which is not compiled for (32,4), takes
 * (32,8) below 2^22 pixels instead. */

/* Time every supported tile configuration on the given image (device
 * buffers as in ccl_label_2d; `labels` is overwritten), `reps` calls each,
 * and record the fastest for the image's size class and connectivity.
 * Writes the winner to *best and its mean milliseconds per call to
 * *best_ms (either may be NULL).  Blocks. */
int ccl_autotune(const uint8_t *img, int32_t H, int32_t W, int64_t pitch, int32_t connectivity,
                 uint32_t *labels, int32_t reps, void *stream, ccl_config *best, float *best_ms);

/* Look up the configuration ccl_label_2d would use for H x W. */
int ccl_tuning_get(int32_t H, int32_t W, int32_t connectivity, ccl_config *out);

/* Save / load the tuning table as JSON lines
 * {"class": c, "conn": k, "tile_h": t, "waves": w, "ms": m}.
 * Loading merges into the table; CCL_ERR_INVALID_ARG on a bad file. */
int ccl_tuning_save(const char *path);
int ccl_tuning_load(const char *path);

/* Drop every table entry (defaults apply again). */
void ccl_tuning_clear(void);

/* Release every workspace the library allocated (all devices) after
 * synchronizing the devices that own them.  Later calls allocate again. */
void ccl_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* CCL_H_ */
