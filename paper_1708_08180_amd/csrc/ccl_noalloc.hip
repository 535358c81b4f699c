// Single-image labeling for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the same three kernels as ccl_label_2d_ex, with the tile
// workspace taken from a fixed array in device memory instead of the
// library's per-stream cache or a caller buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ccl.h"
#include "ccl_internal.h"

namespace ccl {
namespace {

// The workspace of every call on a device.  Each device that runs the
// library holds its own copy of this array until the process ends.
static __device__ __align__(256) unsigned char scratch[CCL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` on each device (set once)

// Device address of the array on the current device.  The array's name in
// host code is only a stand-in for the symbol, so the address is looked up
// once per device, with that device current, and kept.
int scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e);
    if (dev < 0 || dev >= kMaxDevices) return CCL_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e);
        if (!p) return fail_hip(hipErrorInvalidSymbol);
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return CCL_OK;
}

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" int ccl_label_2d_noalloc(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                                    int32_t connectivity, uint32_t *labels, void *stream) {
    int rc = validate_image(img, H, W, pitch, labels);
    if (rc != CCL_OK) return rc;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    int th = 0, nw = 0;
    rc = resolve_config(H, W, connectivity, nullptr, &th, &nw);
    if (rc != CCL_OK) return rc;
    // rejected before any HIP call: the image needs more workspace than the
    // fixed array holds
    if (ws_layout(H, W, th).total > (size_t)CCL_NOALLOC_SCRATCH_BYTES) return CCL_ERR_WORKSPACE;
    void *ws = nullptr;
    rc = scratch_ptr(&ws);
    if (rc != CCL_OK) return rc;
    // every workspace word the later phases read is written by the local
    // merge of the same call, so nothing is cleared here
    const ImgView v = make_view(img, H, W, pitch, labels, ws, th);
    const hipError_t e = launch_plain(v, th, nw, connectivity, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e);
    return CCL_OK;
}
