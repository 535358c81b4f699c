// Host-side interface between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>

#include "ccl.h"
#include "ccl_device.h"

namespace ccl {

// True when (tile_h, waves) names a compiled kernel configuration.
bool config_supported(int th, int nw);

// The three batch kernels of one configuration.  Each takes one BatchArgs
// by value.  Grids: local merge and link one workgroup (block1 / block3
// threads) per tile; boundary analysis one workgroup (block2 threads) per
// tiles_per_group2 tiles.
struct BatchKernels {
    const void *k1, *k2, *k3;
    unsigned block1, block2, block3;
    unsigned tiles_per_group2;
};
bool batch_kernels(int th, int nw, int conn, BatchKernels *out);

// True when (tile_h, waves) is compiled for equal-value labeling.
bool config_supported_equal(int th, int nw);

// Enqueue the three phases for one image on `s`.  With ev != nullptr,
// ev[0..3] are recorded before phase 1, between the phases and after phase 3.
// equal: label every equal-value class instead of the nonzero foreground.
hipError_t launch_plain(const ImgView &v, int th, int nw, int conn, hipStream_t s,
                        hipEvent_t *ev = nullptr, bool equal = false);

// The local merge and the boundary analysis of binary labeling for one
// image on `s`, without the link.
hipError_t launch_merge(const ImgView &v, int th, int nw, int conn, hipStream_t s);

// Workspace layout for one image: edge masks, edge-cell roots, row masks
// (row foreground and edge-root masks), run slots.
struct WsLayout {
    size_t tiles;
    size_t mask_bytes;
    size_t root_bytes;
    size_t rowmask_bytes;
    size_t slot_bytes;
    size_t total;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline WsLayout ws_layout(int H, int W, int th, bool equal = false) {
    WsLayout l;
    const size_t tx = ((size_t)W + kTileW - 1) / kTileW;
    const size_t ty = ((size_t)H + th - 1) / th;
    l.tiles = tx * ty;
    l.mask_bytes = align_up(l.tiles * (size_t)mask_words(th) * sizeof(uint64_t), 256);
    l.root_bytes = align_up(l.tiles * (size_t)roots_per_tile(th) * sizeof(uint32_t), 256);
    l.rowmask_bytes = align_up(l.tiles * (size_t)rowmask_words(th) * sizeof(uint64_t), 256);
    const size_t spr = equal ? (size_t)slots_per_row<true>() : (size_t)slots_per_row<false>();
    l.slot_bytes = align_up(l.tiles * (size_t)th * spr * sizeof(uint16_t), 256);
    l.total = l.mask_bytes + l.root_bytes + l.rowmask_bytes + l.slot_bytes;
    return l;
}

// Shared by the entry points.
int fail_hip(hipError_t e);
// The library's workspace for (current device, stream), at least `need`
// bytes (grown on demand, in stream order).  *held receives the cache lock,
// to be kept until the kernels that use the buffer are enqueued.
int stream_workspace(hipStream_t s, size_t need, void **out, std::unique_lock<std::mutex> *held);
// Frees the cached workspace of (current device, s), in stream order on s.
void release_stream_workspace(hipStream_t s);
// Image arguments: a non-null image of H x W >= 1 bytes per row pitch >= W
// and H * W <= 2^32 - 1.
int validate_image_only(const void *img, int32_t H, int32_t W, int64_t pitch);
// The same, and a non-null label buffer of H * W u32 whose bytes do not
// overlap the image's.
int validate_image(const void *img, int32_t H, int32_t W, int64_t pitch, const void *labels);
// True when [a, a + na) and [b, b + nb) share a byte.
bool byte_ranges_overlap(const void *a, unsigned __int128 na, const void *b, unsigned __int128 nb);
int resolve_config(int H, int W, int conn, const ccl_config *cfg, int *th, int *nw);
void default_config(int H, int W, int conn, int *th, int *nw);
// The kernels' view of one image whose workspace (ws_layout(H, W, th,
// equal).total bytes, 256-byte aligned) starts at ws.
ImgView make_view(const uint8_t *img, int32_t H, int32_t W, int64_t pitch, uint32_t *labels,
                  void *ws, int th, bool equal = false);

}  // namespace ccl
