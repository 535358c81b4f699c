// Host-side interface between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ccl_device.h"

namespace ccl {

// True when (tile_h, waves) names a compiled kernel configuration.
bool config_supported(int th, int nw);

// Enqueue the three phases for one image on `s`.  With ev != nullptr,
// ev[0..3] are recorded before phase 1, between the phases and after phase 3.
hipError_t launch_plain(const ImgView &v, int th, int nw, int conn, hipStream_t s,
                        hipEvent_t *ev = nullptr);

// Workspace layout for one image: edge masks, edge-cell roots, row masks, run slots.
struct WsLayout {
    size_t tiles;
    size_t mask_bytes;
    size_t root_bytes;
    size_t rowmask_bytes;
    size_t slot_bytes;
    size_t total;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline WsLayout ws_layout(int H, int W, int th) {
    WsLayout l;
    const size_t tx = ((size_t)W + kTileW - 1) / kTileW;
    const size_t ty = ((size_t)H + th - 1) / th;
    l.tiles = tx * ty;
    l.mask_bytes = align_up(l.tiles * 4 * sizeof(uint64_t), 256);
    l.root_bytes = align_up(l.tiles * (size_t)roots_per_tile(th) * sizeof(uint32_t), 256);
    l.rowmask_bytes = align_up(l.tiles * (size_t)th * sizeof(uint64_t), 256);
    l.slot_bytes = align_up(l.tiles * (size_t)th * kSlotsPerRow * sizeof(uint16_t), 256);
    l.total = l.mask_bytes + l.root_bytes + l.rowmask_bytes + l.slot_bytes;
    return l;
}

}  // namespace ccl
