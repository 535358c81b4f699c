// The three labeling kernels for one image (gfx950) and their launchers.
//
//   k1_local_merge     Sec. II-A (Kernel 1): tile-local merge with coarse
//                      labeling; writes the tile's edge masks and edge-cell
//                      roots to the workspace and seeds labels[root] = root+1
//                      for roots whose component touches a shared tile edge.
//   k2_boundary        Sec. II-B (Kernel 2): union-find on tile-edge cells
//                      only, one wavefront per tile edge; the only kernel
//                      with global atomics.
//   k3_link            Sec. II-C: reads each pixel's tile-local root from the
//                      workspace, resolves each edge-touching local root once
//                      in the global forest and writes the dense output
//                      labels (1 + root, 0 for background).
#include <map>
#include <mutex>
#include <utility>

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

// Local merge (Kernel 1).  Persistent: each workgroup walks tiles
// worker, worker + G, ... and issues the loads of its next tile before it
// starts merging the current one, so the image streams in while the LDS
// union-find runs.
template <int TH, int NW, bool CONN8>
__global__ void __launch_bounds__(NW * 64) k1_local_merge(ImgView v, uint32_t ntiles) {
    constexpr int RPW = TH / NW;
    constexpr int NT = NW * 64;
    constexpr int CH = TH * 4;                  // 16-byte chunks per tile
    constexpr int LPT = (CH + NT - 1) / NT;     // chunks per thread
    constexpr int NODES = TH * kSlotsPerRow;    // run-indexed nodes per tile
    constexpr int NPT = (NODES + NT - 1) / NT;  // nodes per thread
    __shared__ uint32_t par[NODES];
    __shared__ uint8_t col[NODES];
    __shared__ uint64_t msk[TH];
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t G = gridDim.x;
    uint32_t t = xcd_remap(blockIdx.x, G);
    const uint32_t TX = (uint32_t)v.tilesX;

    uint4 buf[LPT];
    if (t < ntiles) {
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            const int c = tid + i * NT;
            if (c < CH) buf[i] = load_chunk(v, (int)(t % TX), (int)(t / TX), TH, c >> 2, c & 3);
        }
    }
    for (; t < ntiles; t += G) {
        const int tx = (int)(t % TX), ty = (int)(t / TX);
        // row masks into LDS (16 pixels per chunk)
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            const int c = tid + i * NT;
            if (c < CH) ((uint16_t *)msk)[c] = (uint16_t)nonzero_bytes16(buf[i]);
        }
        __syncthreads();
        // prefetch the next tile while this one is merged
        const uint32_t tn = t + G;
        if (tn < ntiles) {
#pragma unroll
            for (int i = 0; i < LPT; ++i) {
                const int c = tid + i * NT;
                if (c < CH) buf[i] = load_chunk(v, (int)(tn % TX), (int)(tn / TX), TH, c >> 2, c & 3);
            }
        }
        sweep_band<TH, RPW, CONN8>(par, col, msk, wave, lane);
        if (NW > 1) {
            __syncthreads();
            if (wave > 0) merge_seam<CONN8>(par, msk, wave * RPW);
        }
        __syncthreads();

        // node-parallel finish: compress (each node written by its owner only, so
        // par[n] is the root afterwards), mark edge-touching roots, emit records
        const bool hasUp = ty > 0, hasDown = ty + 1 < v.tilesY;
        const bool hasLeft = tx > 0, hasRight = tx + 1 < v.tilesX;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int n = tid + i * NT;
            if (n >= NODES) break;
            const uint64_t d = msk[n >> 5];
            if ((n & 31) < __popcll(run_starts(d))) lds_st(&par[n], lds_root(par, (uint32_t)n));
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int n = tid + i * NT;
            if (n >= NODES) break;
            const int r = n >> 5, k = n & 31;
            const uint64_t d = msk[r];
            const int runs = __popcll(run_starts(d));
            if (k >= runs) continue;
            const bool edge = (r == 0 && hasUp) || (r == TH - 1 && hasDown) ||
                              (k == 0 && (d & 1ull) && hasLeft) ||
                              (k == runs - 1 && (d >> 63) && hasRight);
            if (edge) atomicOr(&par[lds_ld(&par[n]) & kIdx], kFlag);
        }
        __syncthreads();
        uint16_t *sl = v.slots + (size_t)t * TH * kSlotsPerRow;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int n = tid + i * NT;
            if (n >= NODES) break;
            const uint64_t d = msk[n >> 5];
            if ((n & 31) >= __popcll(run_starts(d))) continue;
            const uint32_t root = lds_ld(&par[n]) & kIdx;
            const uint32_t flag = lds_ld(&par[root]) & kFlag;
            const uint32_t rpix = (root >> 5) * kTileW + col[root];
            sl[n] = (uint16_t)(rpix | (flag ? kSlotFlag : 0u));
            if (root == (uint32_t)n && flag) {
                const uint32_t g = global_index(v, tx, ty, TH, rpix);
                v.labels[g] = g + 1u;
            }
        }
        if (tid < TH) v.rowmask[(size_t)t * TH + tid] = msk[tid];
        // edge masks and edge-cell roots for the boundary analysis
        if (wave == 0) {
            uint64_t *mk = v.masks + (size_t)t * 4;
            uint32_t *rt = v.roots + (size_t)t * roots_per_tile(TH);
            const uint64_t mTop = uniform64(msk[0]);
            const uint64_t mBot = uniform64(msk[TH - 1]);
            // root pixel (tile-local index) of run node n
            auto root_pix = [&](uint32_t n) {
                const uint32_t root = lds_ld(&par[n]) & kIdx;
                return (root >> 5) * kTileW + col[root];
            };
            if (hasUp && lane_in(mTop)) {
                const uint64_t S = run_starts(mTop);
                const uint32_t n = bits_below(S) - (lane_in(S) ? 0u : 1u);
                rt[roots_top(TH) + lane] = global_index(v, tx, ty, TH, root_pix(n));
            }
            if (hasDown && lane_in(mBot)) {
                const uint64_t S = run_starts(mBot);
                const uint32_t n = (uint32_t)((TH - 1) * kSlotsPerRow) + bits_below(S) -
                                   (lane_in(S) ? 0u : 1u);
                rt[roots_bottom(TH) + lane] = global_index(v, tx, ty, TH, root_pix(n));
            }
            const uint64_t mr = lane < TH ? msk[lane] : 0ull;
            const bool lb = (mr & 1ull) != 0, rb = (mr >> 63) != 0;
            const uint64_t mLeft = __ballot(lb), mRight = __ballot(rb);
            if (hasLeft && lb)
                rt[roots_left(TH) + lane] =
                    global_index(v, tx, ty, TH, root_pix((uint32_t)(lane * kSlotsPerRow)));
            if (hasRight && rb)
                rt[roots_right(TH) + lane] = global_index(
                    v, tx, ty, TH,
                    root_pix((uint32_t)(lane * kSlotsPerRow + __popcll(run_starts(mr)) - 1)));
            if (lane == 0) {
                mk[kMaskTop] = mTop;
                mk[kMaskBottom] = mBot;
                mk[kMaskLeft] = mLeft;
                mk[kMaskRight] = mRight;
            }
        }
        __syncthreads();  // LDS is reused by the next tile
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
    if (seg >= nH + nV) return;  // wave-uniform
    constexpr int RT = roots_per_tile(TH);
    const uint32_t TX = (uint32_t)v.tilesX;
    uint32_t a = kNone, b0 = kNone, b1 = kNone;
    if (seg < nH) {
        const uint32_t tx = seg % TX, ty = seg / TX + 1u;
        const uint32_t tl = ty * TX + tx, tu = tl - TX;
        const uint64_t d = v.masks[(size_t)tl * 4 + kMaskTop];
        const uint64_t u = v.masks[(size_t)tu * 4 + kMaskBottom];
        const bool hasL = tx > 0, hasR = tx + 1u < TX;
        const uint64_t uL = hasL ? v.masks[(size_t)(tu - 1) * 4 + kMaskBottom] : 0ull;
        const uint64_t uR = hasR ? v.masks[(size_t)(tu + 1) * 4 + kMaskBottom] : 0ull;
        if (bit(d, lane)) {
            const bool cL = lane > 0 ? bit(u, lane - 1) : (int)(uL >> 63);
            const bool cM = bit(u, lane);
            const bool cR = lane < 63 ? bit(u, lane + 1) : (int)(uR & 1ull);
            const bool start = !(lane > 0 && bit(d, lane - 1));
            const Plan p = plan_pairs<CONN8>(start, cL, cM, cR, lane > 0 && cL && cM,
                                             lane < 63 && cM && cR);
            const uint32_t *ru = v.roots + (size_t)tu * RT + roots_bottom(TH);
            if (p.l || p.m || p.r) a = v.roots[(size_t)tl * RT + roots_top(TH) + lane];
            // At lane 0 the above-left cell lies in the tile to the left, so
            // the left and middle requests can both be needed; otherwise at
            // most one of them is, and it never coexists with the right one
            // when both left and middle are set.
            if (p.l) b0 = lane > 0 ? ru[lane - 1] : ru[-RT + 63];
            else if (p.m) b0 = ru[lane];
            if (p.r) b1 = lane < 63 ? ru[lane + 1] : ru[RT];
            else if (p.l && p.m) b1 = ru[lane];
        }
    } else {
        const uint32_t s = seg - nH;
        const uint32_t tx = s % (TX - 1u) + 1u, ty = s / (TX - 1u);
        const uint32_t tr = ty * TX + tx, tlft = tr - 1u;
        const uint64_t d = v.masks[(size_t)tr * 4 + kMaskLeft];
        const uint64_t u = v.masks[(size_t)tlft * 4 + kMaskRight];
        if (lane < TH && bit(d, lane)) {
            const bool cL = lane > 0 && bit(u, lane - 1);
            const bool cM = bit(u, lane);
            const bool cR = lane + 1 < TH && bit(u, lane + 1);
            const bool start = !(lane > 0 && bit(d, lane - 1));
            const Plan p = plan_pairs<CONN8>(start, cL, cM, cR, cL && cM, cM && cR);
            const uint32_t *ru = v.roots + (size_t)tlft * RT + roots_right(TH);
            if (p.l || p.m || p.r) a = v.roots[(size_t)tr * RT + roots_left(TH) + lane];
            if (p.l) b0 = ru[lane - 1];
            else if (p.m) b0 = ru[lane];
            if (p.r) b1 = ru[lane + 1];
        }
    }
    bool keep0, keep1;
    dedupe_pairs(a, b0, b1, keep0, keep1);
    if (keep0) g_union(v.labels, v.n, a, b0);
    if (keep1) g_union(v.labels, v.n, a, b1);
}

// Link phase (Sec. II-C): the local merge left every tile's row masks and,
// per run, its tile-local root with an edge flag.  Each flagged local root
// is resolved once in the global forest (and, being rewritten with its final
// value, compressed for the tiles that still walk through it); unflagged
// roots are already final.  Output rows are written as full 256-byte lines.
template <int TH, int NW>
__global__ void __launch_bounds__(NW * 64) k3_link(ImgView v) {
    constexpr int RPW = TH / NW;
    __shared__ uint32_t fin[TH * kTileW];
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (uint32_t)v.tilesX), ty = (int)(t / (uint32_t)v.tilesX);
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const uint64_t *rm = v.rowmask + (size_t)t * TH;
    const uint16_t *sl = v.slots + (size_t)t * TH * kSlotsPerRow;
    uint64_t m[RPW];
    uint32_t rec[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) m[k] = rm[wave * RPW + k];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        rec[k] = kNone;
        if (bit(m[k], lane)) {
            const uint64_t starts = m[k] & ~(m[k] << 1);
            const int rank = __popcll(starts & ((2ull << lane) - 1ull)) - 1;
            rec[k] = sl[r * kSlotsPerRow + rank];
        }
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const uint32_t l = (uint32_t)((wave * RPW + k) * kTileW + lane);
        if (rec[k] != kNone && (rec[k] & kSlotFlag) && (rec[k] & ~(uint32_t)kSlotFlag) == l)
            fin[l] = g_find_final(v.labels, global_index(v, tx, ty, TH, l));
    }
    __syncthreads();
    const int x = tx * kTileW + lane;
    if (x >= v.W) return;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int y = ty * TH + wave * RPW + k;
        if (y >= v.H) break;
        uint32_t out = 0u;
        if (rec[k] != kNone) {
            const uint32_t root = rec[k] & ~(uint32_t)kSlotFlag;
            out = ((rec[k] & kSlotFlag) ? fin[root] : global_index(v, tx, ty, TH, root)) + 1u;
        }
        v.labels[(size_t)y * (size_t)v.W + (size_t)x] = out;
    }
}

// ---------------------------------------------------------------- launchers

// Resident workgroups of a persistent kernel on the current device
// (occupancy x compute units), cached per (device, kernel).
[[maybe_unused]] static uint32_t resident_groups(const void *kernel, int threads) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, uint32_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(std::make_pair(dev, kernel));
    if (it != cache.end()) return it->second;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0)
        return 1024;
    const uint32_t g = (uint32_t)cus * (uint32_t)per_cu;
    cache[std::make_pair(dev, kernel)] = g;
    return g;
}

template <int TH, int NW, bool CONN8>
static hipError_t launch_plain_t(const ImgView &v, hipStream_t stream, hipEvent_t *ev) {
    const uint32_t tiles = (uint32_t)v.tilesX * (uint32_t)v.tilesY;
    const uint32_t nH = (uint32_t)v.tilesX * (uint32_t)(v.tilesY - 1);
    const uint32_t nV = (uint32_t)(v.tilesX - 1) * (uint32_t)v.tilesY;
    // One workgroup per tile: with about as many tiles as resident slots, a
    // persistent grid leaves a second round of tiles on a few workgroups
    // while the rest of the chip idles.  The loop in the kernel only runs
    // more than once for grids capped below the tile count.
    const uint32_t grid1 = tiles;
    if (ev) (void)hipEventRecord(ev[0], stream);
    hipLaunchKernelGGL((k1_local_merge<TH, NW, CONN8>), dim3(grid1), dim3(NW * 64), 0, stream, v,
                       tiles);
    if (ev) (void)hipEventRecord(ev[1], stream);
    if (nH + nV > 0)
        hipLaunchKernelGGL((k2_boundary<TH, CONN8>), dim3((nH + nV + 3) / 4), dim3(256), 0, stream,
                           v, nH, nV);
    if (ev) (void)hipEventRecord(ev[2], stream);
    hipLaunchKernelGGL((k3_link<TH, NW>), dim3(tiles), dim3(NW * 64), 0, stream, v);
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
