// C ABI of libccl: argument validation, tile-configuration choice, the
// per-stream workspace cache and the single-image entry points.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "ccl.h"
#include "ccl_internal.h"

namespace ccl {

static thread_local int g_last_hip_error = 0;

int fail_hip(hipError_t e) {
    g_last_hip_error = (int)e;
    return CCL_ERR_HIP;
}

namespace {

struct WsEntry {
    void *ptr = nullptr;
    size_t bytes = 0;
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, WsEntry> g_ws;

}  // namespace

// Workspace owned by the library for (current device, stream); grown on
// demand.  The buffers are stream-ordered allocations on that stream: the
// old buffer of a growth is freed in stream order, after the work already
// enqueued on the stream that reads it, without blocking the host.  `held`
// receives the cache lock; the caller keeps it until its kernels are
// enqueued, so no other thread can replace the buffer in between.
int stream_workspace(hipStream_t s, size_t need, void **out, std::unique_lock<std::mutex> *held) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e);
    std::unique_lock<std::mutex> lk(g_ws_mu);
    WsEntry &w = g_ws[std::make_pair(dev, s)];
    if (w.bytes < need) {
        if (w.ptr) {
            e = hipFreeAsync(w.ptr, s);
            if (e != hipSuccess) return fail_hip(e);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t bytes = need + need / 4;  // headroom so slowly growing sizes do not reallocate
        e = hipMallocAsync(&w.ptr, bytes, s);
        if (e != hipSuccess) {
            w.ptr = nullptr;
            (void)hipGetLastError();
            return CCL_ERR_OUT_OF_MEMORY;
        }
        w.bytes = bytes;
    }
    *out = w.ptr;
    *held = std::move(lk);
    return CCL_OK;
}

void release_stream_workspace(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find(std::make_pair(dev, s));
    if (it == g_ws.end()) return;
    if (it->second.ptr) (void)hipFreeAsync(it->second.ptr, s);
    g_ws.erase(it);
}

void release_stream_workspaces() {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto &kv : g_ws) {
        if (!kv.second.ptr) continue;
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(kv.first.first);
        // the owning stream may no longer exist: wait for the device, then
        // free in the order of the null stream
        (void)hipDeviceSynchronize();
        (void)hipFreeAsync(kv.second.ptr, nullptr);
        (void)hipDeviceSynchronize();
        (void)hipSetDevice(prev);
    }
    g_ws.clear();
}

int validate_image_only(const void *img, int32_t H, int32_t W, int64_t pitch) {
    if (!img) return CCL_ERR_INVALID_ARG;
    if (H <= 0 || W <= 0 || pitch < (int64_t)W) return CCL_ERR_INVALID_ARG;
    if ((uint64_t)H * (uint64_t)W > 0xFFFFFFFFull) return CCL_ERR_TOO_LARGE;
    return CCL_OK;
}

bool byte_ranges_overlap(const void *a, unsigned __int128 na, const void *b, unsigned __int128 nb) {
    const unsigned __int128 pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

int validate_image(const void *img, int32_t H, int32_t W, int64_t pitch, const void *labels) {
    const int rc = validate_image_only(img, H, W, pitch);
    if (rc != CCL_OK) return rc;
    if (!labels) return CCL_ERR_INVALID_ARG;
    // the image's bytes (its last row ends at W) against the labels' u32s
    const unsigned __int128 img_bytes = (unsigned __int128)(H - 1) * (uint64_t)pitch + (uint64_t)W;
    const unsigned __int128 lab_bytes = (unsigned __int128)H * (uint64_t)W * 4u;
    if (byte_ranges_overlap(img, img_bytes, labels, lab_bytes)) return CCL_ERR_INVALID_ARG;
    return CCL_OK;
}

int resolve_config(int H, int W, int conn, const ccl_config *cfg, int *th, int *nw) {
    if (cfg && (cfg->tile_h != 0 || cfg->waves != 0)) {
        if (!config_supported(cfg->tile_h, cfg->waves)) return CCL_ERR_UNSUPPORTED;
        *th = cfg->tile_h;
        *nw = cfg->waves;
        return CCL_OK;
    }
    default_config(H, W, conn, th, nw);
    return CCL_OK;
}

ImgView make_view(const uint8_t *img, int32_t H, int32_t W, int64_t pitch, uint32_t *labels,
                  void *ws, int th, bool equal) {
    const WsLayout l = ws_layout(H, W, th, equal);
    ImgView v;
    v.img = img;
    v.labels = labels;
    v.masks = (uint64_t *)ws;
    char *base = (char *)ws;
    v.roots = (uint32_t *)(base + l.mask_bytes);
    v.rowmask = (uint64_t *)(base + l.mask_bytes + l.root_bytes);
    v.slots = (uint16_t *)(base + l.mask_bytes + l.root_bytes + l.rowmask_bytes);
    v.pitch = pitch;
    v.H = H;
    v.W = W;
    v.tilesX = (W + kTileW - 1) / kTileW;
    v.tilesY = (H + th - 1) / th;
    v.n = (uint32_t)((uint64_t)H * (uint64_t)W);
    v.aligned16 = (((uintptr_t)img & 15u) == 0 && (pitch & 15) == 0) ? 1 : 0;
    return v;
}

}  // namespace ccl

using namespace ccl;

extern "C" {

const char *ccl_status_string(int status) {
    switch (status) {
        case CCL_OK: return "CCL_OK";
        case CCL_ERR_INVALID_ARG: return "CCL_ERR_INVALID_ARG: invalid argument";
        case CCL_ERR_UNSUPPORTED: return "CCL_ERR_UNSUPPORTED: unsupported connectivity or configuration";
        case CCL_ERR_TOO_LARGE: return "CCL_ERR_TOO_LARGE: H*W exceeds 2^32-1";
        case CCL_ERR_HIP: return "CCL_ERR_HIP: HIP runtime error";
        case CCL_ERR_OUT_OF_MEMORY: return "CCL_ERR_OUT_OF_MEMORY: workspace allocation failed";
        case CCL_ERR_CAPACITY: return "CCL_ERR_CAPACITY: batch exceeds context capacity";
        case CCL_ERR_WORKSPACE: return "CCL_ERR_WORKSPACE: workspace too small";
        default: return "unknown ccl status";
    }
}

int ccl_last_hip_error(void) { return g_last_hip_error; }

int ccl_version(void) { return 10000; }

int ccl_workspace_size(int32_t H, int32_t W, const ccl_config *cfg, size_t *bytes) {
    if (!bytes || H <= 0 || W <= 0) return CCL_ERR_INVALID_ARG;
    if ((uint64_t)H * (uint64_t)W > 0xFFFFFFFFull) return CCL_ERR_TOO_LARGE;
    // without a configuration the tuning table may hold a different tile
    // height per connectivity: the size covers both
    size_t most = 0;
    for (int conn = 4; conn <= 8; conn += 4) {
        int th = 0, nw = 0;
        const int rc = resolve_config(H, W, conn, cfg, &th, &nw);
        if (rc != CCL_OK) return rc;
        const size_t b = ws_layout(H, W, th).total;
        most = b > most ? b : most;
    }
    *bytes = most;
    return CCL_OK;
}

int ccl_label_2d_ex(const uint8_t *img, int32_t H, int32_t W, int64_t pitch, int32_t connectivity,
                    uint32_t *labels, void *workspace, size_t workspace_bytes,
                    const ccl_config *cfg, void *stream) {
    int rc = validate_image(img, H, W, pitch, labels);
    if (rc != CCL_OK) return rc;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    int th = 0, nw = 0;
    rc = resolve_config(H, W, connectivity, cfg, &th, &nw);
    if (rc != CCL_OK) return rc;
    const size_t need = ws_layout(H, W, th).total;
    hipStream_t s = (hipStream_t)stream;
    void *ws = workspace;
    std::unique_lock<std::mutex> held;
    if (ws) {
        if (workspace_bytes < need) return CCL_ERR_WORKSPACE;
        if (((uintptr_t)ws & 255u) != 0) return CCL_ERR_INVALID_ARG;
    } else {
        rc = stream_workspace(s, need, &ws, &held);
        if (rc != CCL_OK) return rc;
    }
    const ImgView v = make_view(img, H, W, pitch, labels, ws, th);
    const hipError_t e = launch_plain(v, th, nw, connectivity, s);
    if (e != hipSuccess) return fail_hip(e);
    return CCL_OK;
}

int ccl_label_2d(const uint8_t *img, int32_t H, int32_t W, int64_t pitch, int32_t connectivity,
                 uint32_t *labels, void *stream) {
    return ccl_label_2d_ex(img, H, W, pitch, connectivity, labels, nullptr, 0, nullptr, stream);
}

int ccl_label_2d_timed(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                       int32_t connectivity, uint32_t *labels, const ccl_config *cfg,
                       void *stream, float *phase_ms) {
    if (!phase_ms) return CCL_ERR_INVALID_ARG;
    int rc = validate_image(img, H, W, pitch, labels);
    if (rc != CCL_OK) return rc;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    int th = 0, nw = 0;
    rc = resolve_config(H, W, connectivity, cfg, &th, &nw);
    if (rc != CCL_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    std::unique_lock<std::mutex> held;
    rc = stream_workspace(s, ws_layout(H, W, th).total, &ws, &held);
    if (rc != CCL_OK) return rc;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    if (e == hipSuccess) {
        const ImgView v = make_view(img, H, W, pitch, labels, ws, th);
        e = launch_plain(v, th, nw, connectivity, s, ev);
    }
    held.unlock();
    if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventElapsedTime(&phase_ms[i], ev[i], ev[i + 1]);
    for (int i = 0; i < 4; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return fail_hip(e);
    return CCL_OK;
}

int ccl_label_2d_equal(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                       int32_t connectivity, uint32_t *labels, const ccl_config *cfg,
                       void *stream) {
    int rc = validate_image(img, H, W, pitch, labels);
    if (rc != CCL_OK) return rc;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    int th = 0, nw = 0;
    if (cfg && (cfg->tile_h != 0 || cfg->waves != 0)) {
        if (!config_supported_equal(cfg->tile_h, cfg->waves)) return CCL_ERR_UNSUPPORTED;
        th = cfg->tile_h;
        nw = cfg->waves;
    } else {
        default_config(H, W, connectivity, &th, &nw);
        if (!config_supported_equal(th, nw)) {
            // a tuning-table entry this mode is not compiled for: size rule
            th = (int64_t)H * W < ((int64_t)1 << 22) ? 32 : 64;
            nw = th == 32 ? 8 : 4;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    std::unique_lock<std::mutex> held;
    rc = stream_workspace(s, ws_layout(H, W, th, true).total, &ws, &held);
    if (rc != CCL_OK) return rc;
    const ImgView v = make_view(img, H, W, pitch, labels, ws, th, true);
    const hipError_t e = launch_plain(v, th, nw, connectivity, s, nullptr, true);
    if (e != hipSuccess) return fail_hip(e);
    return CCL_OK;
}

void ccl_shutdown(void) { release_stream_workspaces(); }

}  // extern "C"
