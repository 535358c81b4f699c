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
    int th = 0, nw = 0;
    int32_t max_images = 0;
    uint64_t max_tiles = 0;
    size_t desc_bytes = 0;       // descriptors + tile bases + coarse bases
    char *d_desc = nullptr;      // device copy of that area
    char *h_staging = nullptr;   // pinned host staging of the same layout
    void *d_ws = nullptr;
    BatchWs ws{};
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

void free_ctx(ccl_ctx *c) {
    if (!c) return;
    for (GraphSet &g : c->gs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (c->staged) (void)hipEventDestroy(c->staged);
    if (c->launched) (void)hipEventDestroy(c->launched);
    if (c->d_desc) (void)hipFree(c->d_desc);
    if (c->d_ws) (void)hipFree(c->d_ws);
    if (c->h_staging) (void)hipHostFree(c->h_staging);
    delete c;
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
    // default tiles: one call covers the tiles of all its images, so the
    // grid is sized like one image of max_pixels pixels (seen as one row:
    // only the pixel count selects the size class)
    const int64_t px = opts->max_pixels;
    const int px_w = (int)(px > 0x7fffffff ? 0x7fffffff : px);
    int rc = resolve_config(1, px_w, 8, &opts->cfg, &c->th, &c->nw);
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
    if (!batch_kernels(c->th, c->nw, 4, &c->kern[0]) || !batch_kernels(c->th, c->nw, 8, &c->kern[1])) {
        delete c;
        return CCL_ERR_UNSUPPORTED;
    }
    // one workgroup per tile: the grid's thread count must fit in 32 bits
    if (c->max_tiles * (uint64_t)c->kern[1].block1 > 0xFFFFFFFFull) {
        delete c;
        return CCL_ERR_TOO_LARGE;
    }
    {
        size_t tb, sb;
        desc_layout(c->max_images, &tb, &sb, &c->desc_bytes);
    }

    const size_t T = (size_t)c->max_tiles;
    const size_t mb = align_up(T * (size_t)mask_words(c->th) * sizeof(uint64_t), 256);
    const size_t rb = align_up(T * (size_t)roots_per_tile(c->th) * sizeof(uint32_t), 256);
    const size_t rmb = align_up(T * (size_t)rowmask_words(c->th) * sizeof(uint64_t), 256);
    const size_t sb = align_up(T * (size_t)c->th * kSlotsPerRow * sizeof(uint16_t), 256);
    const size_t ib = align_up(T * sizeof(uint32_t), 256);
    if ((e = hipMalloc(&c->d_ws, mb + rb + rmb + sb + ib)) != hipSuccess ||
        (e = hipMalloc(&c->d_desc, c->desc_bytes)) != hipSuccess ||
        (e = hipHostMalloc(&c->h_staging, c->desc_bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->launched, hipEventDisableTiming)) != hipSuccess) {
        (void)hipGetLastError();
        free_ctx(c);
        return e == hipErrorOutOfMemory ? CCL_ERR_OUT_OF_MEMORY : fail_hip(e);
    }
    char *base = (char *)c->d_ws;
    c->ws.masks = (uint64_t *)base;
    c->ws.roots = (uint32_t *)(base + mb);
    c->ws.rowmask = (uint64_t *)(base + mb + rb);
    c->ws.slots = (uint16_t *)(base + mb + rb + rmb);
    c->ws.tile_img = (uint32_t *)(base + mb + rb + rmb + sb);
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

    // validate everything and total the tiles before touching the staging area
    uint64_t tiles = 0;
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc &d = descs[i];
        const int rc = validate_image(d.img, d.H, d.W, d.pitch, d.labels);
        if (rc != CCL_OK) return rc;
        const uint64_t tx = (uint64_t)((d.W + kTileW - 1) / kTileW);
        const uint64_t ty = (uint64_t)((d.H + ctx->th - 1) / ctx->th);
        tiles += tx * ty;
    }
    if (tiles > ctx->max_tiles) return CCL_ERR_CAPACITY;

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
        b.tilesY = (d.H + ctx->th - 1) / ctx->th;
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
    a.w = ctx->ws;
    a.n = (uint32_t)n;
    a.tiles = tb;
    const int gi = connectivity == 8 ? 1 : 0;
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

}  // extern "C"
