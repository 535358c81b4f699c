// Tile-configuration choice: a process-wide table keyed by
// (size class = floor(log2(H*W)), connectivity), filled by the autotuner or
// loaded from a JSON-lines file; misses fall back to a built-in default.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "ccl.h"
#include "ccl_internal.h"

namespace ccl {

namespace {

struct Entry {
    int th, nw;
    float ms;
};

std::mutex g_mu;
std::map<std::pair<int, int>, Entry> g_table;

int size_class(int H, int W) {
    const uint64_t px = (uint64_t)(H > 0 ? H : 1) * (uint64_t)(W > 0 ? W : 1);
    int c = 0;
    while ((px >> (c + 1)) != 0) ++c;
    return c;
}

}  // namespace

void default_config(int H, int W, int conn, int *th, int *nw) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(std::make_pair(size_class(H, W), conn));
        if (it != g_table.end()) {
            *th = it->second.th;
            *nw = it->second.nw;
            return;
        }
    }
    // built-in choice (measured on MI355X over 320x240 .. 8192^2, noise and
    // smoothed masks, both connectivities): 32-row tiles while the grid is
    // small, 64-row tiles from about 4 Mpixels up, 4 wavefronts each
    if ((int64_t)H * W < ((int64_t)1 << 22)) {
        *th = 32;
        *nw = 4;
    } else {
        *th = 64;
        *nw = 4;
    }
}

}  // namespace ccl

using namespace ccl;

extern "C" {

int ccl_tuning_get(int32_t H, int32_t W, int32_t connectivity, ccl_config *out) {
    if (!out || H <= 0 || W <= 0) return CCL_ERR_INVALID_ARG;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    int th = 0, nw = 0;
    default_config(H, W, connectivity, &th, &nw);
    out->tile_h = th;
    out->waves = nw;
    return CCL_OK;
}

int ccl_autotune(const uint8_t *img, int32_t H, int32_t W, int64_t pitch, int32_t connectivity,
                 uint32_t *labels, int32_t reps, void *stream, ccl_config *best, float *best_ms) {
    int rc = validate_image(img, H, W, pitch, labels);
    if (rc != CCL_OK) return rc;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    if (reps < 1) return CCL_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return fail_hip(e);
    }
    static const int kTh[] = {16, 32, 64, 128};
    static const int kNw[] = {1, 2, 4, 8, 16};
    float bestv = 1e30f;
    ccl_config bc = {0, 0};
    for (int th : kTh) {
        for (int nw : kNw) {
            if (!config_supported(th, nw)) continue;
            ccl_config cfg = {th, nw};
            // one untimed call (allocates the workspace, warms caches)
            rc = ccl_label_2d_ex(img, H, W, pitch, connectivity, labels, nullptr, 0, &cfg, stream);
            if (rc != CCL_OK) break;
            (void)hipEventRecord(a, s);
            for (int r = 0; r < reps && rc == CCL_OK; ++r)
                rc = ccl_label_2d_ex(img, H, W, pitch, connectivity, labels, nullptr, 0, &cfg, stream);
            (void)hipEventRecord(b, s);
            if (rc != CCL_OK) break;
            e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess) {
                rc = fail_hip(e);
                break;
            }
            ms /= (float)reps;
            if (ms < bestv) {
                bestv = ms;
                bc = cfg;
            }
        }
        if (rc != CCL_OK) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != CCL_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[std::make_pair(size_class(H, W), (int)connectivity)] = Entry{bc.tile_h, bc.waves, bestv};
    }
    if (best) *best = bc;
    if (best_ms) *best_ms = bestv;
    return CCL_OK;
}

int ccl_tuning_save(const char *path) {
    if (!path) return CCL_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return CCL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : g_table)
        std::fprintf(f, "{\"class\": %d, \"conn\": %d, \"tile_h\": %d, \"waves\": %d, \"ms\": %.6f}\n",
                     kv.first.first, kv.first.second, kv.second.th, kv.second.nw, kv.second.ms);
    std::fclose(f);
    return CCL_OK;
}

int ccl_tuning_load(const char *path) {
    if (!path) return CCL_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return CCL_ERR_INVALID_ARG;
    char line[512];
    std::map<std::pair<int, int>, Entry> add;
    int rc = CCL_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '\n' || line[0] == '\0') continue;
        int c = 0, k = 0, th = 0, nw = 0;
        float ms = 0.f;
        if (std::sscanf(line, " {\"class\": %d, \"conn\": %d, \"tile_h\": %d, \"waves\": %d, \"ms\": %f}",
                        &c, &k, &th, &nw, &ms) != 5 ||
            (k != 4 && k != 8) || !config_supported(th, nw) || c < 0 || c > 63) {
            rc = CCL_ERR_INVALID_ARG;
            break;
        }
        add[std::make_pair(c, k)] = Entry{th, nw, ms};
    }
    std::fclose(f);
    if (rc != CCL_OK) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : add) g_table[kv.first] = kv.second;
    return CCL_OK;
}

void ccl_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

}  // extern "C"
