// Device-side building blocks of the three labeling phases (gfx950, wave64).
//
// Tile model.  A tile is 64 pixels wide -- one lane of a 64-wide wavefront
// per column -- and TH rows tall (TH in {16, 32, 64}).  A workgroup of NW
// wavefronts owns one tile; wavefront w owns rows [w*RPW, (w+1)*RPW) with
// RPW = TH / NW.  Inside a tile, a row is a 64-bit foreground mask obtained
// with one ballot, so the paper's row scan plus row-column unification
// (Sec. II-A-2) collapses to: every pixel's provisional parent is the first
// pixel of its horizontal run, found in O(1) from the mask.  Only run starts
// are union-find nodes.  The local UF (Sec. II-A-3) then merges each run with
// the runs it touches in the row above through LDS atomicMin, always linking
// the larger index under the smaller.
//
// Forest encoding in global memory.  labels[p] holds 1 + parent(p); a root r
// holds r + 1 and background holds 0.  The final output is therefore itself a
// fully compressed forest, so the link phase can overwrite entries in place
// while other tiles still walk the forest.
//
// Workspace per tile (written by the local merge, read by the boundary
// analysis): four 64-bit edge masks (top row, bottom row, left column, right
// column) and, for every cell on those four edges, the global raster index of
// its tile-local root.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

constexpr int kTileW = 64;            // tile width == wavefront width
constexpr uint32_t kFlag = 0x80000000u;  // "touches a shared tile edge" mark in LDS parents
constexpr uint32_t kIdx = 0x7FFFFFFFu;

enum { kMaskTop = 0, kMaskBottom = 1, kMaskLeft = 2, kMaskRight = 3 };

__host__ __device__ constexpr int roots_per_tile(int th) { return 2 * kTileW + 2 * th; }
__host__ __device__ constexpr int roots_top(int) { return 0; }
__host__ __device__ constexpr int roots_bottom(int) { return kTileW; }
__host__ __device__ constexpr int roots_left(int) { return 2 * kTileW; }
__host__ __device__ constexpr int roots_right(int th) { return 2 * kTileW + th; }

// One image as the kernels see it.
struct ImgView {
    const uint8_t *img;
    uint32_t *labels;
    uint64_t *masks;   // [tiles][4]
    uint32_t *roots;   // [tiles][roots_per_tile(TH)]
    int64_t pitch;
    int32_t H, W;
    int32_t tilesX, tilesY;
    uint32_t n;        // H * W (<= 2^32 - 1)
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Smallest s <= j such that bits s..j of m are all set (bit j must be set).
__device__ __forceinline__ int run_start(uint64_t m, int j) {
    const uint64_t below = ~m & ((2ull << j) - 1ull);  // j == 63 wraps to all ones
    return below ? 64 - __clzll((long long)below) : 0;
}

__device__ __forceinline__ int bit(uint64_t m, int j) { return (int)((m >> j) & 1ull); }

// Foreground cell j of row mask m that begins a run.
__device__ __forceinline__ bool is_run_start(uint64_t m, int j) {
    return bit(m, j) && !(j > 0 && bit(m, j - 1));
}

template <typename T>
__device__ __forceinline__ T lds_ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void lds_st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Global forest accessors for the concurrent boundary phase.  Loads are
// agent-scope atomics so a wavefront on one XCD sees links made through the
// memory-side atomics of another XCD instead of a stale line in its own L2.
__device__ __forceinline__ uint32_t g_ld(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t g_min(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Which neighbours in the line above a cell must be merged with it so that
// every (lower run, upper run) pair that touches is merged exactly once: the
// pair is handled by the leftmost lower cell adjacent to the upper run.
//   start : the cell is the first of its run in its own line
//   cL/cM/cR : the cells above-left / above / above-right are foreground and
//              belong to this edge's candidate set
//   sameLM / sameMR : those upper neighbours belong to one run
struct Plan { bool l, m, r; };

template <bool CONN8>
__device__ __forceinline__ Plan plan_pairs(bool start, bool cL, bool cM, bool cR, bool sameLM,
                                           bool sameMR) {
    Plan p;
    if (CONN8) {
        p.l = start && cL;
        p.m = start && cM && !sameLM;
        p.r = cR && !sameMR;
    } else {
        p.l = false;
        p.m = cM && (start || !sameLM);
        p.r = false;
    }
    return p;
}

// ---------------------------------------------------------- LDS union-find

// Every parent is strictly smaller than its child, so `p >= x` both detects
// a root (p == x) and stops on anything that is not a valid parent; every
// loop below therefore strictly decreases its index and always terminates.
__device__ __forceinline__ uint32_t lds_find(uint32_t *par, uint32_t x) {
    // path halving; stores only ever replace a parent by an ancestor
    while (true) {
        const uint32_t p = lds_ld(&par[x]);
        if (p >= x) return x;
        const uint32_t gp = lds_ld(&par[p]);
        if (gp >= p) return p;
        lds_st(&par[x], gp);
        x = gp;
    }
}

// Link the two trees of a and b, the larger root under the smaller
// (Sec. II-A-3).  When the atomicMin finds that b stopped being a root in
// the meantime, the value it returns is b's new parent and the merge is
// retried from there, so no concurrent link is ever lost.
__device__ __forceinline__ void lds_union(uint32_t *par, uint32_t a, uint32_t b) {
    while (true) {
        a = lds_find(par, a);
        b = lds_find(par, b);
        if (a == b) return;
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicMin(&par[b], a);
        if (old >= b) return;
        b = old;
    }
}

// ------------------------------------------------------ global union-find

// Find with path halving for the concurrent boundary phase.  The halving
// write is an atomicMin, so it can only lower a parent to an ancestor.
__device__ __forceinline__ uint32_t g_find(uint32_t *L, uint32_t x) {
    while (true) {
        const uint32_t p = g_ld(&L[x]) - 1u;
        if (p >= x) return x;
        const uint32_t gp = g_ld(&L[p]) - 1u;
        if (gp >= p) return p;
        g_min(&L[x], gp + 1u);
        x = gp;
    }
}

__device__ __forceinline__ void g_union(uint32_t *L, uint32_t n, uint32_t a, uint32_t b) {
    if (a >= n || b >= n) return;
    while (true) {
        a = g_find(L, a);
        b = g_find(L, b);
        if (a == b) return;
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = g_min(&L[b], a + 1u);
        if (old - 1u >= b) return;
        b = old - 1u;
    }
}

// Find for the link phase.  No link is made any more, so every root is
// final and every path node may be overwritten with the root (full path
// compression with plain stores: all writers store the same value).
__device__ __forceinline__ uint32_t g_find_final(uint32_t *L, uint32_t x) {
    uint32_t r = x;
    uint32_t v = L[r] - 1u;
    while (v < r) { r = v; v = L[r] - 1u; }
    while (x > r) {
        const uint32_t nx = L[x] - 1u;
        if (nx >= x) break;
        if (nx != r) L[x] = r + 1u;
        x = nx;
    }
    return r;
}

// ------------------------------------------------------ tile-local labeling

template <int TH, int NW>
struct TileLds {
    uint32_t par[TH * kTileW];   // parents of run starts (local indices)
    uint64_t msk[TH];            // foreground mask of every tile row
};

// Per-lane state that the local merge leaves behind for the caller.
template <int RPW>
struct TileRegs {
    uint64_t m[RPW];      // row masks of this wavefront's rows (wave-uniform)
    uint32_t root[RPW];   // local root (index within the tile) of this lane's pixel
};

__device__ __forceinline__ uint32_t global_index(const ImgView &v, int tx, int ty, int th,
                                                 uint32_t l) {
    const uint64_t y = (uint64_t)ty * th + (l >> 6);
    const uint64_t x = (uint64_t)tx * kTileW + (l & 63u);
    return (uint32_t)(y * (uint64_t)v.W + x);
}

// Phase-1 body shared by the local merge and the link kernel: load the tile,
// label runs, merge runs across rows in LDS, compress, and mark the roots of
// components that touch a tile edge shared with another tile.
// Ends after a workgroup barrier; par[] then holds, for every run start, its
// root; roots carry kFlag when their component touches a shared edge.
template <int TH, int NW, bool CONN8>
__device__ __forceinline__ void tile_local(const ImgView &v, int tx, int ty, TileLds<TH, NW> &sh,
                                           TileRegs<TH / NW> &rg) {
    constexpr int RPW = TH / NW;
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int x = tx * kTileW + lane;
    const int y0 = ty * TH + wave * RPW;
    const bool xin = x < v.W;

    uint8_t pix[RPW];
    const uint8_t *src = v.img + (int64_t)y0 * v.pitch + x;
#pragma unroll
    for (int k = 0; k < RPW; ++k) pix[k] = (xin && (y0 + k) < v.H) ? src[(int64_t)k * v.pitch] : 0;

    uint32_t rs[RPW];  // local index of this lane's run start
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        const uint64_t m = __ballot(pix[k] != 0);
        rg.m[k] = m;
        if (lane == 0) lds_st(&sh.msk[r], m);
        const bool fg = bit(m, lane);
        const int s = fg ? run_start(m, lane) : lane;
        rs[k] = (uint32_t)(r * kTileW + s);
        if (fg && s == lane) lds_st(&sh.par[r * kTileW + lane], (uint32_t)(r * kTileW + lane));
    }
    __syncthreads();

    // merge each run with the runs it touches in the row above
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        if (r == 0) continue;
        const uint64_t d = rg.m[k];
        if (!bit(d, lane)) continue;
        const uint64_t u = (k > 0) ? rg.m[k - 1] : lds_ld(&sh.msk[r - 1]);
        const bool start = !(lane > 0 && bit(d, lane - 1));
        const bool cL = lane > 0 && bit(u, lane - 1);
        const bool cM = bit(u, lane);
        const bool cR = lane < 63 && bit(u, lane + 1);
        const Plan p = plan_pairs<CONN8>(start, cL, cM, cR, cL && cM, cM && cR);
        const uint32_t up = (uint32_t)((r - 1) * kTileW);
        if (p.l) lds_union(sh.par, rs[k], up + run_start(u, lane - 1));
        if (p.m) lds_union(sh.par, rs[k], up + run_start(u, lane));
        if (p.r) lds_union(sh.par, rs[k], up + run_start(u, lane + 1));
    }
    __syncthreads();

    // full compression: every run start points at its root
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        if (bit(rg.m[k], lane) && rs[k] == (uint32_t)(r * kTileW + lane))
            lds_st(&sh.par[rs[k]], lds_find(sh.par, rs[k]));
    }
    __syncthreads();

    // per-pixel root and edge marks (only edges shared with another tile)
    const bool hasUp = ty > 0, hasDown = ty + 1 < v.tilesY;
    const bool hasLeft = tx > 0, hasRight = tx + 1 < v.tilesX;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        const bool fg = bit(rg.m[k], lane);
        const uint32_t root = fg ? (lds_ld(&sh.par[rs[k]]) & kIdx) : 0u;
        rg.root[k] = root;
        if (!fg) continue;
        const bool isStart = rs[k] == (uint32_t)(r * kTileW + lane);
        const bool mark = ((r == 0 && hasUp) || (r == TH - 1 && hasDown)) ? isStart
                          : false;
        const bool markCol = (lane == 0 && hasLeft) || (lane == 63 && hasRight);
        if (mark || markCol) atomicOr(&sh.par[root], kFlag);
    }
    __syncthreads();
}

}  // namespace ccl
