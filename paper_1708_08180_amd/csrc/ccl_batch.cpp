// Batched form: a context with fixed capacity labels many images per call.
//
// Per call the host writes one descriptor per image plus the images' first
// global tiles (prefix sums) into a pinned staging area, copies
// them to the device on the caller's stream, and runs the three batch
// kernels with grids sized for that call: directly, or by replaying a
// three-node hipGraph whose kernel nodes get the call's grid and arguments.
// Every buffer the kernels touch is allocated once at context creation.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "ccl.h"
#include "ccl_internal.h"

using namespace ccl;

namespace {

struct GraphSet {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node[3] = {nullptr, nullptr, nullptr};
    BatchArgs args{};
    unsigned grid[3] = {0, 0, 0};
};

}  // namespace

struct ccl_ctx {
    int dev = 0;
    int th[2] = {0, 0}, nw[2] = {0, 0};  // tile configuration per connectivity (4, 8)
    bool fixed_cfg = false;              // created with an explicit configuration
    int32_t max_images = 0;
    int64_t max_pixels = 0;
    size_t desc_bytes = 0;       // descriptors + tile bases + coarse bases
    char *d_desc = nullptr;      // device copy of that area
    char *h_staging = nullptr;   // pinned host staging of the same layout
    void *d_ws = nullptr;
    size_t ws_bytes = 0;         // covers every configuration the context may use
    BatchKernels kern[2]{};      // connectivity 4, 8
    hipEvent_t staged = nullptr;    // recorded after each staging copy
    hipEvent_t launched = nullptr;  // recorded after each call's kernels
    bool staged_pending = false, launched_pending = false;
    int use_graph = 0;
    GraphSet gs[2];
};

namespace {

// Offsets of the three arrays for n images (64-byte aligned): descriptors,
// tile bases, and every 64th tile base.
void desc_layout(int32_t n, size_t *off_tb, size_t *off_cb, size_t *bytes) {
    *off_tb = align_up((size_t)n * sizeof(BatchImage), 64);
    *off_cb = *off_tb + align_up((size_t)n * sizeof(uint32_t), 64);
    *bytes = *off_cb + (size_t)((n + 63) / 64) * sizeof(uint32_t);
}

void drop_graph(GraphSet &g);

void free_ctx(ccl_ctx *c) {
    if (!c) return;
    for (GraphSet &g : c->gs) drop_graph(g);
    if (c->staged) (void)hipEventDestroy(c->staged);
    if (c->launched) (void)hipEventDestroy(c->launched);
    if (c->d_desc) (void)hipFree(c->d_desc);
    if (c->d_ws) (void)hipFree(c->d_ws);
    if (c->h_staging) (void)hipHostFree(c->h_staging);
    delete c;
}

// Tiles a context keeps room for with tile height th: twice the full-tile
// count of max_pixels plus two tiles per image (the partial tile rows and
// columns of ordinary image shapes; very thin images may still exceed it
// and get CCL_ERR_CAPACITY).
uint64_t max_tiles(const ccl_ctx *c, int th) {
    const uint64_t full = (uint64_t)((c->max_pixels + (int64_t)kTileW * th - 1) / ((int64_t)kTileW * th));
    return 2u * full + 2u * (uint64_t)c->max_images + 64u;
}

// Workspace of a context with tile height th: per-tile arrays of
// max_tiles(th) tiles (masks, edge roots, row data, records, tile image).
struct CtxLayout {
    size_t mb, rb, rmb, sb, ib, total;
};
CtxLayout ctx_layout(const ccl_ctx *c, int th) {
    const size_t T = (size_t)max_tiles(c, th);
    CtxLayout l;
    l.mb = align_up(T * (size_t)mask_words(th) * sizeof(uint64_t), 256);
    l.rb = align_up(T * (size_t)roots_per_tile(th) * sizeof(uint32_t), 256);
    l.rmb = align_up(T * (size_t)rowmask_words(th) * sizeof(uint64_t), 256);
    l.sb = align_up(T * (size_t)th * kSlotsPerRow * sizeof(uint16_t), 256);
    l.ib = align_up(T * sizeof(uint32_t), 256);
    l.total = l.mb + l.rb + l.rmb + l.sb + l.ib;
    return l;
}

BatchWs ctx_ws(const ccl_ctx *c, int th) {
    const CtxLayout l = ctx_layout(c, th);
    char *base = (char *)c->d_ws;
    BatchWs w;
    w.masks = (uint64_t *)base;
    w.roots = (uint32_t *)(base + l.mb);
    w.rowmask = (uint64_t *)(base + l.mb + l.rb);
    w.slots = (uint16_t *)(base + l.mb + l.rb + l.rmb);
    w.tile_img = (uint32_t *)(base + l.mb + l.rb + l.rmb + l.sb);
    return w;
}

// Every tile configuration the context may be switched to.
constexpr int kCfgTh[] = {16, 32, 64, 128};
constexpr int kCfgNw[] = {1, 2, 4, 8, 16};

void drop_graph(GraphSet &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = GraphSet{};
}

// Use (th, nw) for connectivity slot gi from the next call on.
int set_config(ccl_ctx *c, int gi, int th, int nw) {
    BatchKernels k;
    if (!batch_kernels(th, nw, gi ? 8 : 4, &k)) return CCL_ERR_UNSUPPORTED;
    if (ctx_layout(c, th).total > c->ws_bytes) return CCL_ERR_UNSUPPORTED;
    if (c->th[gi] == th && c->nw[gi] == nw) return CCL_OK;
    // a graph launch of the old kernels may still be queued
    if (c->launched_pending) {
        const hipError_t e = hipEventSynchronize(c->launched);
        if (e != hipSuccess) return fail_hip(e);
        c->launched_pending = false;
    }
    drop_graph(c->gs[gi]);
    c->kern[gi] = k;
    c->th[gi] = th;
    c->nw[gi] = nw;
    return CCL_OK;
}

void node_params(const BatchKernels &k, int j, unsigned grid, void **args, hipKernelNodeParams *p) {
    std::memset(p, 0, sizeof(*p));
    p->func = (void *)(j == 0 ? k.k1 : j == 1 ? k.k2 : k.k3);
    p->gridDim = dim3(grid);
    p->blockDim = dim3(j == 0 ? k.block1 : j == 1 ? k.block2 : k.block3);
    p->sharedMemBytes = 0;
    p->kernelParams = args;
    p->extra = nullptr;
}

// Build and instantiate the graph K1 -> K2 -> K3 with the given arguments.
hipError_t build_graph(GraphSet &g, const BatchKernels &k, const BatchArgs &a,
                       const unsigned grid[3]) {
    BatchArgs copy = a;
    void *args[] = {&copy};
    hipError_t e = hipGraphCreate(&g.graph, 0);
    for (int j = 0; j < 3 && e == hipSuccess; ++j) {
        hipKernelNodeParams p;
        node_params(k, j, grid[j], args, &p);
        e = hipGraphAddKernelNode(&g.node[j], g.graph, j ? &g.node[j - 1] : nullptr, j ? 1 : 0, &p);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g = GraphSet{};
        return e;
    }
    g.args = a;
    for (int j = 0; j < 3; ++j) g.grid[j] = grid[j];
    return hipSuccess;
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
    c->max_images = opts->max_images;
    c->max_pixels = opts->max_pixels;
    c->use_graph = opts->use_graph;
    c->fixed_cfg = opts->cfg.tile_h != 0 || opts->cfg.waves != 0;
    // default tiles per connectivity: one call covers the tiles of all its
    // images, so the grid is sized like one image of max_pixels pixels (seen
    // as one row: only the pixel count selects the size class)
    const int px_w = (int)(opts->max_pixels > 0x7fffffff ? 0x7fffffff : opts->max_pixels);
    for (int gi = 0; gi < 2; ++gi) {
        const int rc = resolve_config(1, px_w, gi ? 8 : 4, &opts->cfg, &c->th[gi], &c->nw[gi]);
        if (rc != CCL_OK) {
            delete c;
            return rc;
        }
        if (!batch_kernels(c->th[gi], c->nw[gi], gi ? 8 : 4, &c->kern[gi])) {
            delete c;
            return CCL_ERR_UNSUPPORTED;
        }
    }
    // the workspace covers the configurations the context may use: its
    // fixed one, or every one the autotuner may pick
    c->ws_bytes = 0;
    for (int th : kCfgTh) {
        if (c->fixed_cfg && th != c->th[0]) continue;
        if (max_tiles(c, th) > 0xFFFFFFF0ull) {
            delete c;
            return CCL_ERR_TOO_LARGE;
        }
        // one workgroup per tile: the grid's thread count must fit in 32 bits
        if (max_tiles(c, th) * 1024u > 0xFFFFFFFFull) {
            delete c;
            return CCL_ERR_TOO_LARGE;
        }
        const size_t b = ctx_layout(c, th).total;
        c->ws_bytes = b > c->ws_bytes ? b : c->ws_bytes;
    }
    {
        size_t tb, sb;
        desc_layout(c->max_images, &tb, &sb, &c->desc_bytes);
    }
    if ((e = hipMalloc(&c->d_ws, c->ws_bytes)) != hipSuccess ||
        (e = hipMalloc(&c->d_desc, c->desc_bytes)) != hipSuccess ||
        (e = hipHostMalloc(&c->h_staging, c->desc_bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->launched, hipEventDisableTiming)) != hipSuccess) {
        (void)hipGetLastError();
        free_ctx(c);
        return e == hipErrorOutOfMemory ? CCL_ERR_OUT_OF_MEMORY : fail_hip(e);
    }
    *out = c;
    return CCL_OK;
}

int ccl_ctx_destroy(ccl_ctx *ctx) {
    if (!ctx) return CCL_ERR_INVALID_ARG;
    if (ctx->staged_pending) (void)hipEventSynchronize(ctx->staged);
    if (ctx->launched_pending) (void)hipEventSynchronize(ctx->launched);
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

    const int gi = connectivity == 8 ? 1 : 0;
    const int th = ctx->th[gi];
    // validate everything and total the tiles before touching the staging area
    uint64_t tiles = 0;
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc &d = descs[i];
        const int rc = validate_image(d.img, d.H, d.W, d.pitch, d.labels);
        if (rc != CCL_OK) return rc;
        const uint64_t tx = (uint64_t)((d.W + kTileW - 1) / kTileW);
        const uint64_t ty = (uint64_t)((d.H + th - 1) / th);
        tiles += tx * ty;
    }
    if (tiles > max_tiles(ctx, th)) return CCL_ERR_CAPACITY;

    hipStream_t s = (hipStream_t)stream;
    if (ctx->staged_pending) {
        e = hipEventSynchronize(ctx->staged);  // the previous copy still reads the staging area
        if (e != hipSuccess) return fail_hip(e);
        ctx->staged_pending = false;
    }
    size_t off_tb, off_cb, bytes;
    desc_layout(n, &off_tb, &off_cb, &bytes);
    BatchImage *hd = (BatchImage *)ctx->h_staging;
    uint32_t *htb = (uint32_t *)(ctx->h_staging + off_tb);
    uint32_t *hcb = (uint32_t *)(ctx->h_staging + off_cb);
    uint32_t tb = 0;
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc &d = descs[i];
        BatchImage &b = hd[i];
        b.img = d.img;
        b.labels = d.labels;
        b.pitch = d.pitch;
        b.H = d.H;
        b.W = d.W;
        b.tilesX = (d.W + kTileW - 1) / kTileW;
        b.tilesY = (d.H + th - 1) / th;
        b.n = (uint32_t)((uint64_t)d.H * (uint64_t)d.W);
        b.aligned16 = (((uintptr_t)d.img & 15u) == 0 && (d.pitch & 15) == 0) ? 1 : 0;
        b.tile_base = tb;
        b.pad = 0;
        htb[i] = tb;
        if ((i & 63) == 0) hcb[i >> 6] = tb;
        tb += (uint32_t)b.tilesX * (uint32_t)b.tilesY;
    }
    e = hipMemcpyAsync(ctx->d_desc, ctx->h_staging, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e);
    e = hipEventRecord(ctx->staged, s);
    if (e != hipSuccess) return fail_hip(e);
    ctx->staged_pending = true;

    BatchArgs a{};
    a.descs = (const BatchImage *)ctx->d_desc;
    a.tile_base = (const uint32_t *)(ctx->d_desc + off_tb);
    a.coarse = (const uint32_t *)(ctx->d_desc + off_cb);
    a.w = ctx_ws(ctx, th);
    a.n = (uint32_t)n;
    a.tiles = tb;
    const BatchKernels &k = ctx->kern[gi];
    const unsigned grid[3] = {tb, (tb + k.tiles_per_group2 - 1) / k.tiles_per_group2, tb};
    if (ctx->use_graph) {
        GraphSet &g = ctx->gs[gi];
        if (!g.exec) {
            e = build_graph(g, k, a, grid);
            if (e != hipSuccess) return fail_hip(e);
        } else if (std::memcmp(&g.args, &a, sizeof(a)) != 0 || g.grid[0] != grid[0] ||
                   g.grid[1] != grid[1] || g.grid[2] != grid[2]) {
            // an earlier launch of this graph may not have read its arguments yet
            if (ctx->launched_pending) {
                e = hipEventSynchronize(ctx->launched);
                if (e != hipSuccess) return fail_hip(e);
                ctx->launched_pending = false;
            }
            BatchArgs copy = a;
            void *args[] = {&copy};
            for (int j = 0; j < 3; ++j) {
                hipKernelNodeParams p;
                node_params(k, j, grid[j], args, &p);
                e = hipGraphExecKernelNodeSetParams(g.exec, g.node[j], &p);
                if (e != hipSuccess) return fail_hip(e);
            }
            g.args = a;
            for (int j = 0; j < 3; ++j) g.grid[j] = grid[j];
        }
        e = hipGraphLaunch(g.exec, s);
        if (e != hipSuccess) return fail_hip(e);
    } else {
        void *args[] = {&a};
        const unsigned blk[3] = {k.block1, k.block2, k.block3};
        const void *fn[3] = {k.k1, k.k2, k.k3};
        for (int j = 0; j < 3; ++j) {
            e = hipLaunchKernel(fn[j], dim3(grid[j]), dim3(blk[j]), args, 0, s);
            if (e != hipSuccess) return fail_hip(e);
        }
    }
    e = hipEventRecord(ctx->launched, s);
    if (e != hipSuccess) return fail_hip(e);
    ctx->launched_pending = true;
    return CCL_OK;
}

int ccl_ctx_config(const ccl_ctx *ctx, int32_t connectivity, ccl_config *out) {
    if (!ctx || !out) return CCL_ERR_INVALID_ARG;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    const int gi = connectivity == 8 ? 1 : 0;
    out->tile_h = ctx->th[gi];
    out->waves = ctx->nw[gi];
    return CCL_OK;
}

int ccl_ctx_autotune(ccl_ctx *ctx, const ccl_image_desc *descs, int32_t n, int32_t connectivity,
                     int32_t reps, void *stream, ccl_config *best, float *best_ms) {
    if (!ctx || !descs || n < 1 || reps < 1) return CCL_ERR_INVALID_ARG;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    if (ctx->fixed_cfg) return CCL_ERR_UNSUPPORTED;
    const int gi = connectivity == 8 ? 1 : 0;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        return fail_hip(e);
    }
    const int th0 = ctx->th[gi], nw0 = ctx->nw[gi];
    int bt = th0, bn = nw0, rc = CCL_OK;
    float bms = -1.0f;
    for (int th : kCfgTh) {
        for (int nw : kCfgNw) {
            if (!config_supported(th, nw)) continue;
            rc = set_config(ctx, gi, th, nw);
            if (rc == CCL_ERR_UNSUPPORTED) {  // not compiled, or the images need more tiles
                rc = CCL_OK;
                continue;
            }
            if (rc != CCL_OK) break;
            rc = ccl_label_batch(ctx, descs, n, connectivity, stream);  // warm-up (and capacity check)
            if (rc == CCL_ERR_CAPACITY) {
                rc = CCL_OK;
                continue;
            }
            if (rc != CCL_OK) break;
            if ((e = hipEventRecord(ev[0], s)) != hipSuccess) {
                rc = fail_hip(e);
                break;
            }
            for (int r = 0; r < reps && rc == CCL_OK; ++r) rc = ccl_label_batch(ctx, descs, n, connectivity, stream);
            if (rc != CCL_OK) break;
            float ms = 0.0f;
            if ((e = hipEventRecord(ev[1], s)) != hipSuccess || (e = hipEventSynchronize(ev[1])) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) {
                rc = fail_hip(e);
                break;
            }
            ms /= (float)reps;
            if (bms < 0.0f || ms < bms) {
                bms = ms;
                bt = th;
                bn = nw;
            }
        }
        if (rc != CCL_OK) break;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    const int rc2 = set_config(ctx, gi, rc == CCL_OK ? bt : th0, rc == CCL_OK ? bn : nw0);
    if (rc != CCL_OK) return rc;
    if (rc2 != CCL_OK) return rc2;
    if (bms < 0.0f) return CCL_ERR_CAPACITY;
    if (best) {
        best->tile_h = bt;
        best->waves = bn;
    }
    if (best_ms) *best_ms = bms;
    return CCL_OK;
}

}  // extern "C"
