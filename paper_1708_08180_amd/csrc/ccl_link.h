// Link phase (Sec. II-C) for one tile, shared by the labeling kernels and
// the kernel that also gathers component statistics.
//
// The local merge left the tile's row masks, the masks of its local roots
// whose components touch a shared tile edge ("flagged" roots), and per run
// (equal-value) or band interval (binary) its tile-local root pixel.  Every
// local root pixel first puts its final label - 1 into fin[]: unflagged
// roots are already final; flagged roots are resolved in the global forest
// (where a tile's stores of final labels compress the paths of the tiles
// that still walk through its pixels).  A wavefront resolves all flagged
// roots of its rows at once, lane i the i-th in row order (found from the
// rows' flag masks, with no list in LDS), so their walks overlap instead of
// following each other row by row.  Then every pixel reads its root's
// entry; output rows are full 256-byte lines.
#pragma once

#include "ccl_device.h"

namespace ccl {

// What one wavefront of the link holds for its rows once the roots are
// resolved (k3_resolve), and what the label writes (k3_write) consume.
template <int TH, int NW, bool EQ>
struct LinkRows {
    static constexpr int RPW = TH / NW;
    static_assert(EQ || RPW % 2 == 0, "a wavefront owns whole bands");
    static constexpr int BPW = EQ ? 1 : RPW / 2;
    // records: one per row (equal-value) or one per band, which both rows
    // of the band share (binary)
    static constexpr int NR = EQ ? RPW : BPW;
    uint64_t m[RPW];   // row foreground (equal-value: run starts)
    uint64_t be[BPW];  // band interval ends (binary)
    uint32_t rec[NR];  // this lane's tile-local root pixel, kNone for background
    uint32_t tx, ty;   // the tile's position in the tile grid
    int wave;          // this wavefront (wave-uniform)
};

// Offset (row << 6 | column, rows counted from the wavefront's first) of
// the i-th flagged local root, in row order, of a wavefront's RPW rows.  fv:
// lane k < RPW holds row k's flag mask, other lanes 0; fpre: the exclusive
// prefix count of fv's bits over the lanes.  The row is the last one whose
// prefix is at most i (a binary search over the lanes), the column a binary
// search by halves.  Call with every lane active (values move between
// lanes); a lane whose i is at or past the total gets some offset inside
// the rows.
template <int RPW>
__device__ __forceinline__ uint32_t nth_flagged(uint64_t fv, uint32_t fpre, uint32_t i) {
    static_assert((RPW & (RPW - 1)) == 0 && RPW <= 64, "a power of two up to the wave size");
    uint32_t row = 0, before = 0;
#pragma unroll
    for (int h = RPW / 2; h >= 1; h >>= 1) {
        const uint32_t p = (uint32_t)__shfl((int)fpre, (int)row + h, 64);
        if (i >= p) {
            row += (uint32_t)h;
            before = p;
        }
    }
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)fv, (int)row, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(fv >> 32), (int)row, 64);
    uint32_t n = i - before;
    uint32_t col = 0, w = lo;
    const uint32_t c = (uint32_t)__builtin_popcount(lo);
    if (n >= c) {
        n -= c;
        col = 32u;
        w = hi;
    }
#pragma unroll
    for (uint32_t h = 16u; h >= 1u; h >>= 1) {
        const uint32_t ch = (uint32_t)__builtin_popcount(w & ((1u << h) - 1u));
        if (n >= ch) {
            n -= ch;
            col += h;
            w >>= h;
        }
    }
    return row * (uint32_t)kTileW + col;
}

// First half of the link for tile t: loads the wavefront's rows and records
// and fills fin[] for every local root of the tile.  Ends after a workgroup
// barrier.  LANE_ENDS: the band ends are held in a vector register (lane k:
// band k) instead of scalar registers, for callers short of scalar
// registers.  `rw` / `sl`: the tile's row data and run records in the
// workspace (they depend on the tile only, so their loads need not wait for
// the image's descriptor in the batched form).
template <int TH, int NW, bool EQ, bool LANE_ENDS = false>
__device__ __forceinline__ void k3_resolve(const ImgView &v, uint32_t t, const uint64_t *rw,
                                           const uint16_t *sl, uint32_t *fin, LinkRows<TH, NW, EQ> &R) {
    using LR = LinkRows<TH, NW, EQ>;
    constexpr int SPR = slots_per_row<EQ>();
    constexpr int RPW = LR::RPW, BPW = LR::BPW, NR = LR::NR;
    const uint32_t TX = (uint32_t)v.tilesX;
    const uint32_t tx = t % TX, ty = t / TX;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    R.tx = tx;
    R.ty = ty;
    R.wave = wave;
    const uint32_t W = (uint32_t)v.W;
    const uint64_t *rm = rw + wave * RPW;
    // global index of the tile's pixel (0, 0); every label fits in 32 bits
    const uint32_t origin = ty * (uint32_t)TH * W + tx * (uint32_t)kTileW;
    // equal-value: every in-image pixel takes part (rows hold run starts)
    const int wlim = min(kTileW, v.W - (int)tx * kTileW);
    const uint64_t cols = wlim == 64 ? ~0ull : ((1ull << wlim) - 1ull);
    const int rows_in = v.H - (int)ty * TH - wave * RPW;
    // first record of this wave's rows or bands (lane k: row or band k of
    // the wave): equal-value records have 64 slots per row; binary records
    // are numbered densely by two-row band, and the local merge stored every
    // band's first record (a wavefront owns whole bands)
    uint32_t rbv;
    if (EQ) {
        rbv = (uint32_t)((wave * RPW + lane) * SPR);
    } else {
        const uint16_t *rbg = (const uint16_t *)(rw + rowmask_bases(TH));
        rbv = lane < BPW ? (uint32_t)rbg[wave * BPW + lane] : 0u;
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k) R.m[k] = uniform64(rm[k]);
    // flagged local roots of the rows, lane k holding row k's mask
    const uint64_t fv = lane < RPW ? rm[TH + lane] : 0ull;
    uint64_t ev = 0ull;
    if (!EQ) {
        if (LANE_ENDS) {
            if (lane < BPW) ev = rw[rowmask_ends(TH) + wave * BPW + lane];
        } else {
#pragma unroll
            for (int k = 0; k < BPW; ++k) R.be[k] = uniform64(rw[rowmask_ends(TH) + wave * BPW + k]);
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        // this lane's node (background lanes read some record of the tile
        // and discard it): equal-value, the rank among the row's run
        // starts at or below it; binary, the band's intervals ending before
        // it (lanes right of the band's last interval take that interval)
        uint32_t node;
        uint64_t d;
        if (EQ) {
            const uint64_t S = R.m[i];
            const uint32_t below = bits_below(S) + (lane_in(S) ? 1u : 0u);
            node = (uint32_t)__builtin_amdgcn_readlane((int)rbv, i) + (below ? below - 1u : 0u);
            d = i < rows_in ? cols : 0ull;
        } else {
            const uint64_t E = LANE_ENDS ? lane_value64(ev, i) : R.be[i];
            const uint32_t below = bits_below(E), last = (uint32_t)__popcll(E);
            node = (uint32_t)__builtin_amdgcn_readlane((int)rbv, i) + (below < last ? below : (last ? last - 1u : 0u));
            d = R.m[2 * i] | R.m[2 * i + 1];
        }
        const uint32_t r = sl[node];
        R.rec[i] = lane_in(d) ? r : kNone;
    }
    // unflagged local roots are final
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const uint32_t l = (uint32_t)((wave * RPW + k) * kTileW + lane);
        if (R.rec[EQ ? k : k / 2] == l && !lane_in(lane_value64(fv, k))) fin[l] = origin + (l >> 6) * W + (l & 63u);
    }
    // this wave's flagged roots
    uint32_t nf;
    const uint32_t fpre = wave_exclusive_scan((uint32_t)__popcll(fv), &nf);
    for (uint32_t b = 0; b < nf; b += 64u) {  // wave-uniform
        const uint32_t i = b + (uint32_t)lane;
        const uint32_t l = (uint32_t)(wave * RPW * kTileW) + nth_flagged<RPW>(fv, fpre, i);
        if (i < nf) fin[l] = g_root(v.labels, origin + (l >> 6) * W + (l & 63u));
    }
    __syncthreads();
}

// Second half: every pixel of the wavefront's rows gets 1 + its root's
// final label (0 for background).  Ends after a workgroup barrier.
template <int TH, int NW, bool EQ>
__device__ __forceinline__ void k3_write(const ImgView &v, const uint32_t *fin, const LinkRows<TH, NW, EQ> &R) {
    using LR = LinkRows<TH, NW, EQ>;
    constexpr int RPW = LR::RPW, NR = LR::NR;
    const uint32_t tx = R.tx, ty = R.ty;
    const int lane = lane_id();
    const int wave = R.wave;
    const uint32_t W = (uint32_t)v.W;
    const uint32_t origin = ty * (uint32_t)TH * W + tx * (uint32_t)kTileW;
    const uint32_t x = tx * (uint32_t)kTileW + (uint32_t)lane;
    const uint32_t y0 = ty * (uint32_t)TH + (uint32_t)(wave * RPW);
    uint32_t *out = v.labels + origin + (uint32_t)(wave * RPW) * W + (uint32_t)lane;
    const bool full = (tx + 1u) * kTileW <= W && y0 + RPW <= (uint32_t)v.H;
    // streaming stores: the output is not read again here, and keeping it
    // out of the L2 leaves the records and the forest cached for the tiles
    // still to run (a stale cached label is an ancestor)
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const uint32_t val = R.rec[i] != kNone ? fin[R.rec[i] & (TH * kTileW - 1)] + 1u : 0u;
        if (EQ) {
            if (full || (x < W && y0 + i < (uint32_t)v.H)) __builtin_nontemporal_store(val, &out[(size_t)i * W]);
        } else {
            const int k = 2 * i;
            const uint32_t v0 = lane_in(R.m[k]) ? val : 0u, v1 = lane_in(R.m[k + 1]) ? val : 0u;
            if (full || (x < W && y0 + k < (uint32_t)v.H)) __builtin_nontemporal_store(v0, &out[(size_t)k * W]);
            if (full || (x < W && y0 + k + 1 < (uint32_t)v.H)) __builtin_nontemporal_store(v1, &out[(size_t)(k + 1) * W]);
        }
    }
    __syncthreads();
}

// The whole link for tile t.
template <int TH, int NW, bool EQ>
__device__ __forceinline__ void k3_tile(const ImgView &v, uint32_t t, const uint64_t *rw,
                                        const uint16_t *sl, uint32_t *fin) {
    LinkRows<TH, NW, EQ> R;
    k3_resolve<TH, NW, EQ>(v, t, rw, sl, fin, R);
    k3_write<TH, NW, EQ>(v, fin, R);
}

// Waves per workgroup of the link kernel: 16 rows per wave whatever the
// local merge uses (measured best at 32 and 64 rows per tile).
template <int TH>
constexpr int link_waves() {
    return TH / 16;
}

}  // namespace ccl
