// Batched form: a context with fixed capacity labels many images per call.
//
// Per call the host writes one descriptor per image (tile and edge-segment
// bases from prefix sums) into a pinned staging area, copies it to the
// device on the caller's stream, and replays (or launches) the three batch
// kernels.  Everything the kernels touch lives in buffers allocated once at
// context creation, so the captured hipGraph stays valid for every call.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "ccl.h"
#include "ccl_internal.h"

using namespace ccl;

struct ccl_ctx {
    int dev = 0;
    int th = 0, nw = 0;
    int32_t max_images = 0;
    uint64_t max_tiles = 0, max_segs = 0;
    size_t desc_bytes = 0;       // header + max_images descriptors
    char *d_desc = nullptr;      // device copy of header + descriptors
    char *h_staging = nullptr;   // pinned host staging of the same layout
    void *d_ws = nullptr;
    BatchWs ws{};
    uint32_t *d_queue = nullptr;
    hipEvent_t staged = nullptr;  // recorded after each staging copy
    bool staged_pending = false;
    int use_graph = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // connectivity 4, 8
    bool warmed[2] = {false, false};
};

namespace {

void free_ctx(ccl_ctx *c) {
    if (!c) return;
    for (auto &g : c->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->staged) (void)hipEventDestroy(c->staged);
    if (c->d_desc) (void)hipFree(c->d_desc);
    if (c->d_ws) (void)hipFree(c->d_ws);
    if (c->d_queue) (void)hipFree(c->d_queue);
    if (c->h_staging) (void)hipHostFree(c->h_staging);
    delete c;
}

}  // namespace

extern "C" {

int ccl_ctx_create(ccl_ctx **out, const ccl_ctx_opts *opts) {
    if (!out || !opts) return CCL_ERR_INVALID_ARG;
    *out = nullptr;
    if (opts->max_images < 1 || opts->max_pixels < 1) return CCL_ERR_INVALID_ARG;
    ccl_ctx *c = new (std::nothrow) ccl_ctx();
    if (!c) return CCL_ERR_OUT_OF_MEMORY;
    hipError_t e = hipGetDevice(&c->dev);
    if (e != hipSuccess) {
        delete c;
        return fail_hip(e);
    }
    // default tiles: the choice for an average image, seen as a 1-row image of
    // that many pixels (only the pixel count selects the size class)
    const int64_t avg = opts->max_pixels / opts->max_images;
    const int avg_w = (int)(avg < 1 ? 1 : (avg > 0x7fffffff ? 0x7fffffff : avg));
    int rc = resolve_config(1, avg_w, 8, &opts->cfg, &c->th, &c->nw);
    if (rc != CCL_OK) {
        delete c;
        return rc;
    }
    c->max_images = opts->max_images;
    c->use_graph = opts->use_graph;
    // twice the full-tile count plus two tiles per image: room for the partial
    // tile rows and columns of ordinary image shapes (very thin images may
    // still exceed it and get CCL_ERR_CAPACITY)
    const uint64_t full = (uint64_t)((opts->max_pixels + (int64_t)kTileW * c->th - 1) /
                                     ((int64_t)kTileW * c->th));
    c->max_tiles = 2u * full + 2u * (uint64_t)opts->max_images + 64u;
    if (c->max_tiles > 0xFFFFFFF0ull) {
        delete c;
        return CCL_ERR_TOO_LARGE;
    }
    c->max_segs = 2 * c->max_tiles;
    c->desc_bytes = sizeof(BatchHeader) + (size_t)c->max_images * sizeof(BatchImage);

    const size_t T = (size_t)c->max_tiles;
    const size_t mb = align_up(T * 4 * sizeof(uint64_t), 256);
    const size_t rb = align_up(T * (size_t)roots_per_tile(c->th) * sizeof(uint32_t), 256);
    const size_t rmb = align_up(T * (size_t)c->th * sizeof(uint64_t), 256);
    const size_t sb = align_up(T * (size_t)c->th * kSlotsPerRow * sizeof(uint16_t), 256);
    if ((e = hipMalloc(&c->d_ws, mb + rb + rmb + sb)) != hipSuccess ||
        (e = hipMalloc(&c->d_desc, c->desc_bytes)) != hipSuccess ||
        (e = hipMalloc(&c->d_queue, 256)) != hipSuccess ||
        (e = hipHostMalloc(&c->h_staging, c->desc_bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMemset(c->d_queue, 0, 256)) != hipSuccess) {
        (void)hipGetLastError();
        free_ctx(c);
        return e == hipErrorOutOfMemory ? CCL_ERR_OUT_OF_MEMORY : fail_hip(e);
    }
    char *base = (char *)c->d_ws;
    c->ws.masks = (uint64_t *)base;
    c->ws.roots = (uint32_t *)(base + mb);
    c->ws.rowmask = (uint64_t *)(base + mb + rb);
    c->ws.slots = (uint16_t *)(base + mb + rb + rmb);
    *out = c;
    return CCL_OK;
}

int ccl_ctx_destroy(ccl_ctx *ctx) {
    if (!ctx) return CCL_ERR_INVALID_ARG;
    if (ctx->staged_pending) (void)hipEventSynchronize(ctx->staged);
    free_ctx(ctx);
    return CCL_OK;
}

int ccl_label_batch(ccl_ctx *ctx, const ccl_image_desc *descs, int32_t n, int32_t connectivity,
                    void *stream) {
    if (!ctx) return CCL_ERR_INVALID_ARG;
    if (n < 0) return CCL_ERR_INVALID_ARG;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    if (n == 0) return CCL_OK;
    if (!descs) return CCL_ERR_INVALID_ARG;
    if (n > ctx->max_images) return CCL_ERR_CAPACITY;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e);
    if (dev != ctx->dev) return CCL_ERR_INVALID_ARG;

    // validate everything and total the tiles before touching the staging area
    uint64_t tiles = 0, segs = 0;
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc &d = descs[i];
        const int rc = validate_image(d.img, d.H, d.W, d.pitch, d.labels);
        if (rc != CCL_OK) return rc;
        const uint64_t tx = (uint64_t)((d.W + kTileW - 1) / kTileW);
        const uint64_t ty = (uint64_t)((d.H + ctx->th - 1) / ctx->th);
        tiles += tx * ty;
        segs += tx * (ty - 1) + (tx - 1) * ty;
    }
    if (tiles > ctx->max_tiles || segs > ctx->max_segs) return CCL_ERR_CAPACITY;

    hipStream_t s = (hipStream_t)stream;
    if (ctx->staged_pending) {
        e = hipEventSynchronize(ctx->staged);  // the previous copy still reads the staging area
        if (e != hipSuccess) return fail_hip(e);
        ctx->staged_pending = false;
    }
    BatchHeader *hh = (BatchHeader *)ctx->h_staging;
    BatchImage *hd = (BatchImage *)(ctx->h_staging + sizeof(BatchHeader));
    uint32_t tb = 0, sb = 0;
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc &d = descs[i];
        BatchImage &b = hd[i];
        b.img = d.img;
        b.labels = d.labels;
        b.pitch = d.pitch;
        b.H = d.H;
        b.W = d.W;
        b.tilesX = (d.W + kTileW - 1) / kTileW;
        b.tilesY = (d.H + ctx->th - 1) / ctx->th;
        b.n = (uint32_t)((uint64_t)d.H * (uint64_t)d.W);
        b.aligned16 = (((uintptr_t)d.img & 15u) == 0 && (d.pitch & 15) == 0) ? 1 : 0;
        b.tile_base = tb;
        b.seg_base = sb;
        b.nH = (uint32_t)b.tilesX * (uint32_t)(b.tilesY - 1);
        b.nV = (uint32_t)(b.tilesX - 1) * (uint32_t)b.tilesY;
        tb += (uint32_t)b.tilesX * (uint32_t)b.tilesY;
        sb += b.nH + b.nV;
    }
    hh->n_images = (uint32_t)n;
    hh->total_tiles = tb;
    hh->total_segs = sb;
    hh->pad = 0;
    const size_t bytes = sizeof(BatchHeader) + (size_t)n * sizeof(BatchImage);
    e = hipMemcpyAsync(ctx->d_desc, ctx->h_staging, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e);
    e = hipEventRecord(ctx->staged, s);
    if (e != hipSuccess) return fail_hip(e);
    ctx->staged_pending = true;

    const BatchHeader *dh = (const BatchHeader *)ctx->d_desc;
    const BatchImage *dd = (const BatchImage *)(ctx->d_desc + sizeof(BatchHeader));
    const int gi = connectivity == 8 ? 1 : 0;
    if (ctx->use_graph && s != nullptr && ctx->warmed[gi]) {
        if (!ctx->graph[gi]) {
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return fail_hip(e);
            const hipError_t le = launch_batch(dh, dd, ctx->ws, ctx->d_queue, ctx->th, ctx->nw,
                                               connectivity, s);
            e = hipStreamEndCapture(s, &g);
            if (le != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail_hip(le);
            }
            if (e != hipSuccess) return fail_hip(e);
            e = hipGraphInstantiate(&ctx->graph[gi], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                ctx->graph[gi] = nullptr;
                return fail_hip(e);
            }
        }
        e = hipGraphLaunch(ctx->graph[gi], s);
        if (e != hipSuccess) return fail_hip(e);
        return CCL_OK;
    }
    // direct launches (also the first call per connectivity, which sizes the
    // persistent grids outside any capture)
    e = launch_batch(dh, dd, ctx->ws, ctx->d_queue, ctx->th, ctx->nw, connectivity, s);
    if (e != hipSuccess) return fail_hip(e);
    ctx->warmed[gi] = true;
    return CCL_OK;
}

}  // extern "C"
