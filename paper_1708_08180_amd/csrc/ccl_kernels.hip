// The three labeling kernels for one image (gfx950) and their launchers.
//
//   k1_local_merge     Sec. II-A (Kernel 1): tile-local merge with coarse
//                      labeling; writes the tile's edge masks and edge-cell
//                      roots to the workspace and seeds labels[root] = root+1
//                      for roots whose component touches a shared tile edge.
//   k2_boundary        Sec. II-B (Kernel 2): union-find on tile-edge cells
//                      only, one wavefront per tile edge; the only kernel
//                      with global atomics.
//   k3_link            Sec. II-C: re-derives each tile's local roots in LDS
//                      from the image, resolves each edge-touching local root
//                      once in the global forest and writes the dense output
//                      labels (1 + root, 0 for background).
#include "ccl_device.h"
#include "ccl_internal.h"

namespace ccl {

// Consecutive workgroup ids are spread round-robin over the 8 XCDs; remap
// them so that each XCD works on one contiguous run of tiles and
// horizontally adjacent tiles (which share image cache lines) meet in the
// same L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nb) {
    constexpr uint32_t X = 8;
    const uint32_t q = nb / X, r = nb % X;
    const uint32_t xcd = bid % X, i = bid / X;
    return xcd * q + (xcd < r ? xcd : r) + i;
}

template <int TH, int NW, bool CONN8>
__global__ void __launch_bounds__(NW * 64) k1_local_merge(ImgView v) {
    constexpr int RPW = TH / NW;
    __shared__ TileLds<TH, NW> sh;
    TileRegs<RPW> rg;
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (uint32_t)v.tilesX), ty = (int)(t / (uint32_t)v.tilesX);
    tile_local<TH, NW, CONN8>(v, tx, ty, sh, rg);

    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    // seed the global forest with the edge-touching roots
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        const uint32_t l = (uint32_t)(r * kTileW + lane);
        if (!is_run_start(rg.m[k], lane)) continue;
        const uint32_t pv = lds_ld(&sh.par[l]);
        if ((pv & kIdx) == l && (pv & kFlag)) {
            const uint32_t g = global_index(v, tx, ty, TH, l);
            v.labels[g] = g + 1u;
        }
    }
    // edge masks and edge-cell roots for the boundary analysis
    if (wave == 0) {
        uint64_t *mk = v.masks + (size_t)t * 4;
        uint32_t *rt = v.roots + (size_t)t * roots_per_tile(TH);
        const uint64_t mTop = lds_ld(&sh.msk[0]);
        const uint64_t mBot = lds_ld(&sh.msk[TH - 1]);
        const bool hasUp = ty > 0, hasDown = ty + 1 < v.tilesY;
        const bool hasLeft = tx > 0, hasRight = tx + 1 < v.tilesX;
        if (hasUp && bit(mTop, lane)) {
            const uint32_t rt0 = lds_ld(&sh.par[run_start(mTop, lane)]) & kIdx;
            rt[roots_top(TH) + lane] = global_index(v, tx, ty, TH, rt0);
        }
        if (hasDown && bit(mBot, lane)) {
            const uint32_t s = (uint32_t)((TH - 1) * kTileW + run_start(mBot, lane));
            rt[roots_bottom(TH) + lane] = global_index(v, tx, ty, TH, lds_ld(&sh.par[s]) & kIdx);
        }
        const uint64_t mr = lane < TH ? lds_ld(&sh.msk[lane]) : 0ull;
        const bool lb = (mr & 1ull) != 0, rb = (mr >> 63) != 0;
        const uint64_t mLeft = __ballot(lb), mRight = __ballot(rb);
        if (hasLeft && lb) {
            const uint32_t s = (uint32_t)(lane * kTileW);
            rt[roots_left(TH) + lane] = global_index(v, tx, ty, TH, lds_ld(&sh.par[s]) & kIdx);
        }
        if (hasRight && rb) {
            const uint32_t s = (uint32_t)(lane * kTileW + run_start(mr, 63));
            rt[roots_right(TH) + lane] = global_index(v, tx, ty, TH, lds_ld(&sh.par[s]) & kIdx);
        }
        if (lane == 0) {
            mk[kMaskTop] = mTop;
            mk[kMaskBottom] = mBot;
            mk[kMaskLeft] = mLeft;
            mk[kMaskRight] = mRight;
        }
    }
}

// One wavefront per tile edge.  Edge segments [0, nH) are the horizontal
// edges (tile (tx, ty) against the tile above, ty >= 1), segments
// [nH, nH + nV) the vertical edges (tile (tx, ty) against the tile on its
// left, tx >= 1).  Horizontal edges also take the diagonal pairs that cross
// a tile corner; vertical edges take only pairs inside one tile row, so every
// adjacent foreground pair that crosses tiles is examined by exactly one edge.
template <int TH, bool CONN8>
__global__ void __launch_bounds__(256) k2_boundary(ImgView v, uint32_t nH, uint32_t nV) {
    const uint32_t seg = blockIdx.x * 4u + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (seg >= nH + nV) return;
    constexpr int RT = roots_per_tile(TH);
    const uint32_t TX = (uint32_t)v.tilesX;
    if (seg < nH) {
        const uint32_t tx = seg % TX, ty = seg / TX + 1u;
        const uint32_t tl = ty * TX + tx, tu = tl - TX;
        const uint64_t d = v.masks[(size_t)tl * 4 + kMaskTop];
        if (!bit(d, lane)) return;
        const uint64_t u = v.masks[(size_t)tu * 4 + kMaskBottom];
        const bool hasL = tx > 0, hasR = tx + 1u < TX;
        const bool cL = lane > 0 ? bit(u, lane - 1)
                                 : (hasL && (v.masks[(size_t)(tu - 1) * 4 + kMaskBottom] >> 63));
        const bool cM = bit(u, lane);
        const bool cR = lane < 63 ? bit(u, lane + 1)
                                  : (hasR && (v.masks[(size_t)(tu + 1) * 4 + kMaskBottom] & 1ull));
        const bool start = !(lane > 0 && bit(d, lane - 1));
        const Plan p = plan_pairs<CONN8>(start, cL, cM, cR, lane > 0 && cL && cM,
                                         lane < 63 && cM && cR);
        if (!(p.l || p.m || p.r)) return;
        const uint32_t *ru = v.roots + (size_t)tu * RT + roots_bottom(TH);
        const uint32_t a = v.roots[(size_t)tl * RT + roots_top(TH) + lane];
        if (p.l) g_union(v.labels, v.n, a, lane > 0 ? ru[lane - 1] : ru[-RT + 63]);
        if (p.m) g_union(v.labels, v.n, a, ru[lane]);
        if (p.r) g_union(v.labels, v.n, a, lane < 63 ? ru[lane + 1] : ru[RT]);
    } else {
        const uint32_t s = seg - nH;
        const uint32_t tx = s % (TX - 1u) + 1u, ty = s / (TX - 1u);
        const uint32_t tr = ty * TX + tx, tlft = tr - 1u;
        if (lane >= TH) return;
        const uint64_t d = v.masks[(size_t)tr * 4 + kMaskLeft];
        if (!bit(d, lane)) return;
        const uint64_t u = v.masks[(size_t)tlft * 4 + kMaskRight];
        const bool cL = lane > 0 && bit(u, lane - 1);
        const bool cM = bit(u, lane);
        const bool cR = lane + 1 < TH && bit(u, lane + 1);
        const bool start = !(lane > 0 && bit(d, lane - 1));
        const Plan p = plan_pairs<CONN8>(start, cL, cM, cR, cL && cM, cM && cR);
        if (!(p.l || p.m || p.r)) return;
        const uint32_t *ru = v.roots + (size_t)tlft * RT + roots_right(TH);
        const uint32_t a = v.roots[(size_t)tr * RT + roots_left(TH) + lane];
        if (p.l) g_union(v.labels, v.n, a, ru[lane - 1]);
        if (p.m) g_union(v.labels, v.n, a, ru[lane]);
        if (p.r) g_union(v.labels, v.n, a, ru[lane + 1]);
    }
}

template <int TH, int NW, bool CONN8>
__global__ void __launch_bounds__(NW * 64) k3_link(ImgView v) {
    constexpr int RPW = TH / NW;
    __shared__ TileLds<TH, NW> sh;
    TileRegs<RPW> rg;
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (uint32_t)v.tilesX), ty = (int)(t / (uint32_t)v.tilesX);
    tile_local<TH, NW, CONN8>(v, tx, ty, sh, rg);

    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    // resolve every local root once: edge-touching roots through the global
    // forest, the others are already final
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        const uint32_t l = (uint32_t)(r * kTileW + lane);
        if (!is_run_start(rg.m[k], lane)) continue;
        const uint32_t pv = lds_ld(&sh.par[l]);
        if ((pv & kIdx) != l) continue;
        const uint32_t g = global_index(v, tx, ty, TH, l);
        const uint32_t fin = (pv & kFlag) ? g_find_final(v.labels, g) : g;
        lds_st(&sh.par[l], fin);
    }
    __syncthreads();
    const int x = tx * kTileW + lane;
    if (x >= v.W) return;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int y = ty * TH + wave * RPW + k;
        if (y >= v.H) break;
        const uint32_t out = bit(rg.m[k], lane) ? lds_ld(&sh.par[rg.root[k]]) + 1u : 0u;
        v.labels[(size_t)y * (size_t)v.W + (size_t)x] = out;
    }
}

// ---------------------------------------------------------------- launchers

template <int TH, int NW, bool CONN8>
static hipError_t launch_plain_t(const ImgView &v, hipStream_t stream, hipEvent_t *ev) {
    const uint32_t tiles = (uint32_t)v.tilesX * (uint32_t)v.tilesY;
    const uint32_t nH = (uint32_t)v.tilesX * (uint32_t)(v.tilesY - 1);
    const uint32_t nV = (uint32_t)(v.tilesX - 1) * (uint32_t)v.tilesY;
    if (ev) (void)hipEventRecord(ev[0], stream);
    hipLaunchKernelGGL((k1_local_merge<TH, NW, CONN8>), dim3(tiles), dim3(NW * 64), 0, stream, v);
    if (ev) (void)hipEventRecord(ev[1], stream);
    if (nH + nV > 0)
        hipLaunchKernelGGL((k2_boundary<TH, CONN8>), dim3((nH + nV + 3) / 4), dim3(256), 0, stream,
                           v, nH, nV);
    if (ev) (void)hipEventRecord(ev[2], stream);
    hipLaunchKernelGGL((k3_link<TH, NW, CONN8>), dim3(tiles), dim3(NW * 64), 0, stream, v);
    if (ev) (void)hipEventRecord(ev[3], stream);
    return hipGetLastError();
}

template <int TH, int NW>
static hipError_t launch_plain_c(const ImgView &v, int conn, hipStream_t s, hipEvent_t *ev) {
    return conn == 8 ? launch_plain_t<TH, NW, true>(v, s, ev) : launch_plain_t<TH, NW, false>(v, s, ev);
}

bool config_supported(int th, int nw) {
    switch (th) {
        case 16: return nw == 1 || nw == 2 || nw == 4 || nw == 8 || nw == 16;
        case 32: return nw == 1 || nw == 2 || nw == 4 || nw == 8 || nw == 16;
        case 64: return nw == 1 || nw == 2 || nw == 4 || nw == 8 || nw == 16;
        default: return false;
    }
}

hipError_t launch_plain(const ImgView &v, int th, int nw, int conn, hipStream_t s, hipEvent_t *ev) {
#define CCL_CASE(T, N) \
    if (th == T && nw == N) return launch_plain_c<T, N>(v, conn, s, ev);
    CCL_CASE(16, 1) CCL_CASE(16, 2) CCL_CASE(16, 4) CCL_CASE(16, 8) CCL_CASE(16, 16)
    CCL_CASE(32, 1) CCL_CASE(32, 2) CCL_CASE(32, 4) CCL_CASE(32, 8) CCL_CASE(32, 16)
    CCL_CASE(64, 1) CCL_CASE(64, 2) CCL_CASE(64, 4) CCL_CASE(64, 8) CCL_CASE(64, 16)
#undef CCL_CASE
    return hipErrorInvalidValue;
}

}  // namespace ccl
