// Labels and per-component statistics in one call: the link phase (Sec.
// II-C) also gathers the size and location of every component (the
// quantities the paper's introduction lists as the uses of the labels),
// while it holds every band interval's final root in LDS, instead of a
// second pass that reads the label image back.
//
//   local merge, boundary analysis   unchanged (binary labeling)
//   k3_link_stats   the link for one tile.  Besides the labels it writes
//                   one 16-byte record per local component (its final label
//                   and tile-local statistics: pixel count, coordinate sums,
//                   extent), gathered from the band intervals in LDS, and
//                   per 64-pixel row word the mask of component roots (the
//                   pixels whose label is their own index + 1) and of those
//                   whose component reaches a shared tile edge.
//   st_band         per tile row (a few workgroups, each over a group of
//                   tile columns): the rank of every row word's first
//                   component root (components are numbered in raster order
//                   of their roots, i.e. in increasing label order), the
//                   component count, the output records of components inside
//                   one tile (complete in their single record), and the
//                   output records of the others, initialised.
//   st_span         per tile row (per 16 tiles of one under
//                   4-connectivity): the records of components that reach
//                   a tile edge, reduced by label in LDS, then added to the
//                   output records with global atomics.
#include <hip/hip_runtime.h>

#include "ccl.h"
#include "ccl_device.h"
#include "ccl_internal.h"
#include "ccl_link.h"

namespace ccl {

namespace {

// Local components of one tile are at most one per two pixels under
// 4-connectivity (a checkerboard) and one per 2 x 2 block under
// 8-connectivity.
constexpr int stats_rmax(int th, bool conn8) { return conn8 ? th * 16 : th * 32; }

struct StatsView {
    uint64_t *cm;        // [H][tilesX] component roots per 64-pixel row word
    uint64_t *sm;        // [H][tilesX] the subset whose component reaches a tile edge
    uint32_t *base;      // [H][tilesX] rank of the word's first component root
    uint32_t *tcnt;      // [tiles] component roots in the tile
    uint32_t *ncnt;      // [tiles] records: inside the tile | reaching an edge << 16
    uint4 *rec;          // [tiles][rmax] records (below)
    ccl_component *out;  // caller's output, cap records
    uint32_t *n_out;
    uint32_t cap;
};

// A record: x = final label; y = first row | last row << 6 | root pixel
// (tile-local) << 12; z, w = pixel count (13 bits) | column sum << 13 (18
// bits) | row sum << 31 (18 bits), tile-local coordinates, with the first
// and last columns in w's bits 17..22 and 23..28.  Tiles are at most 64
// pixels high and wide, so every field fits.  Records of components inside
// the tile fill the tile's slots from the front, the others from the back.

// Wavefronts of the statistics link: 16 rows each, as in the plain link.
// So that its scalar registers fit beside the statistics' own state, the
// link keeps the band ends in a vector register and the local-id loop is
// unrolled four rows at a time.
template <int TH>
constexpr int stats_waves() {
    return TH / 16;
}

// Accumulators for this many local components at a time: a tile with more
// local components takes several passes over its band intervals.
constexpr int kStatsChunk = 256;

// Sum of the column indices of the set bits of a and of b: the columns
// whose index has bit k set are those of the k-th mask.
__device__ __forceinline__ uint32_t column_sum2(uint64_t a, uint64_t b) {
    constexpr uint64_t P[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                               0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        s += ((uint32_t)__popcll(a & P[k]) + (uint32_t)__popcll(b & P[k])) << k;
    return s;
}

template <int TH, bool CONN8>
struct StatsLds {
    static constexpr int NW = stats_waves<TH>();
    static constexpr int RPW = TH / NW;
    static constexpr int RMAX = stats_rmax(TH, CONN8);
    // a wavefront's band intervals: at most 32 per band under
    // 8-connectivity (runs), 64 under 4-connectivity
    static constexpr int ILIST = RPW / 2 * (CONN8 ? 32 : 64);
    uint32_t fin[TH * kTileW];
    uint64_t rows[TH];                    // foreground per row
    uint64_t frows[TH];                   // flagged local roots per row
    uint64_t bends[TH / 2];               // band interval ends
    uint64_t rmask[TH];                   // local roots per row
    uint64_t fcm[TH];                     // flagged local roots that are component roots
    uint32_t rpre[TH + 1];                // local roots in the rows above; [TH]: all
    uint16_t rpos[RMAX];                  // local root pixel by local id; bit 15: flagged
    uint32_t ilist[NW][ILIST];            // first column | last << 6 | band << 12 | root << 15
    unsigned long long sums[kStatsChunk];  // packed count and sums (record layout)
    unsigned long long xm[kStatsChunk], ym[kStatsChunk];  // columns / rows holding pixels
    uint32_t nrec[2], ncomp;
};

template <int TH, bool CONN8>
__global__ void __launch_bounds__(stats_waves<TH>() * 64) k3_link_stats(ImgView v, StatsView s) {
    constexpr int NW = stats_waves<TH>(), NT = NW * 64;
    using LR = LinkRows<TH, NW, false>;
    constexpr int RPW = LR::RPW, BPW = LR::BPW;
    using Lds = StatsLds<TH, CONN8>;
    constexpr int RMAX = Lds::RMAX;
    static_assert(TH <= 64, "one mask word per tile row and 6-bit row offsets");
    __shared__ Lds sh;
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int tid = (int)threadIdx.x;
    const uint64_t *rw = v.rowmask + (size_t)t * rowmask_words(TH);
    // LDS copies of the tile's rows, flagged roots and band ends for the
    // statistics (kept in scalar registers across the link as well, the
    // masks of a wavefront's 16 rows would not fit)
    if (tid < TH) {
        sh.rows[tid] = rw[tid];
        sh.frows[tid] = rw[TH + tid];
        sh.fcm[tid] = 0ull;
        if (tid < TH / 2) sh.bends[tid] = rw[rowmask_ends(TH) + tid];
    }
    if (tid == 0) {
        sh.nrec[0] = 0u;
        sh.nrec[1] = 0u;
        sh.ncomp = 0u;
    }
    // accumulators of the first (usually only) chunk of local components
    for (int i = tid; i < kStatsChunk; i += NT) {
        sh.sums[i] = 0ull;
        sh.xm[i] = 0ull;
        sh.ym[i] = 0ull;
    }
    LR R;
    k3_resolve<TH, NW, false, true>(v, t, rw, v.slots + (size_t)t * TH * kSlotsPerRow, sh.fin, R);
    const int lane = tid & 63, wave = R.wave;
    const uint32_t W = (uint32_t)v.W, TX = (uint32_t)v.tilesX;
    const uint32_t tx = R.tx, ty = R.ty;
    const uint32_t origin = ty * (uint32_t)TH * W + tx * (uint32_t)kTileW;
    // the labels go out first
    k3_write<TH, NW, false>(v, sh.fin, R);  // ends after a barrier
    // flagged local roots that stayed roots of the forest are their
    // component's root (unflagged local roots always are)
    {
        const uint64_t fv = lane < RPW ? sh.frows[wave * RPW + lane] : 0ull;
        uint32_t nf;
        const uint32_t fpre = wave_exclusive_scan((uint32_t)__popcll(fv), &nf);
        for (uint32_t b = 0; b < nf; b += 64u) {  // wave-uniform
            const uint32_t i = b + (uint32_t)lane;
            const uint32_t l = (uint32_t)(wave * RPW * kTileW) + nth_flagged<RPW>(fv, fpre, i);
            if (i < nf && sh.fin[l] == origin + (l >> 6) * W + (l & 63u)) atomicOr(&sh.fcm[l >> 6], 1ull << (l & 63u));
        }
    }
    // local roots: the pixels that are their own interval's root
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const uint32_t l = (uint32_t)((wave * RPW + k) * kTileW + lane);
        const uint64_t rmk = __ballot(R.rec[k >> 1] == l);
        if (lane == 0) sh.rmask[wave * RPW + k] = rmk;
    }
    // this wavefront's band intervals, listed densely: their first lane
    // appends (first column, last column, band, root pixel)
    uint32_t nint = 0;
    uint32_t *il = sh.ilist[wave];
#pragma unroll
    for (int i = 0; i < BPW; ++i) {
        const int r0 = wave * RPW + 2 * i;
        const uint64_t d = uniform64(sh.rows[r0]) | uniform64(sh.rows[r0 + 1]);
        const uint64_t E = uniform64(sh.bends[wave * BPW + i]);
        const uint64_t starts = d & ~((d & ~E) << 1);
        if (lane_in(starts)) {
            const uint32_t e = (uint32_t)lane + (uint32_t)__builtin_ctzll(E >> lane);
            il[nint + bits_below(starts)] = (uint32_t)lane | (e << 6) | ((uint32_t)i << 12) | (R.rec[i] << 15);
        }
        nint += (uint32_t)__popcll(starts);
    }
    __syncthreads();
    // local roots in the rows above each row (lane = row), computed by every
    // wavefront for itself
    uint32_t nroots;
    const uint32_t rpre_l = wave_exclusive_scan(lane < TH ? (uint32_t)__popcll(sh.rmask[lane]) : 0u, &nroots);
    if (wave == 0) {
        if (lane < TH) sh.rpre[lane] = rpre_l;
        if (lane == 0) sh.rpre[TH] = nroots;
    }
    // local ids in raster order; component roots per row word
    uint32_t ncomp = 0;
#pragma unroll 4
    for (int k = 0; k < RPW; ++k) {
        const int row = wave * RPW + k;
        const uint64_t rmk = uniform64(sh.rmask[row]), fk = uniform64(sh.frows[row]);
        if (lane_in(rmk)) {
            const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)rpre_l, row) + bits_below(rmk);
            sh.rpos[id] = (uint16_t)((uint32_t)(row * kTileW + lane) | (lane_in(fk) ? 0x8000u : 0u));
        }
        const uint64_t cmk = (rmk & ~fk) | uniform64(sh.fcm[row]);
        const uint32_t y = ty * (uint32_t)TH + (uint32_t)row;
        if (lane == 0 && y < (uint32_t)v.H) {
            s.cm[(size_t)y * TX + tx] = cmk;
            s.sm[(size_t)y * TX + tx] = cmk & fk;
        }
        ncomp += (uint32_t)__popcll(cmk);
    }
    if (lane == 0 && ncomp) atomicAdd(&sh.ncomp, ncomp);
    uint4 *rec = s.rec + (size_t)t * RMAX;
    for (uint32_t c0 = 0; c0 < nroots; c0 += (uint32_t)kStatsChunk) {
        const uint32_t c1 = min(nroots, c0 + (uint32_t)kStatsChunk);
        if (c0 > 0) {
            for (uint32_t id = c0 + (uint32_t)tid; id < c1; id += NT) {
                sh.sums[id - c0] = 0ull;
                sh.xm[id - c0] = 0ull;
                sh.ym[id - c0] = 0ull;
            }
        }
        __syncthreads();  // accumulators cleared; rpre written
        // every interval adds its pixels to its local root's accumulators
        for (uint32_t j = (uint32_t)lane; j < nint; j += 64u) {
            const uint32_t q = il[j];
            const uint32_t c = q & 63u, e = (q >> 6) & 63u, i = (q >> 12) & 7u, r = q >> 15;
            const uint32_t rr = r >> 6;
            const uint32_t id = sh.rpre[rr] + (uint32_t)__popcll(sh.rmask[rr] & ((1ull << (r & 63u)) - 1ull));
            if (id < c0 || id >= c1) continue;
            const uint32_t yt = (uint32_t)(wave * RPW) + 2u * i, yb = yt + 1u;
            const uint64_t I = (~0ull >> (63u - e)) & (~0ull << c);
            const uint64_t at = sh.rows[yt] & I, ab = sh.rows[yb] & I;
            const uint32_t na = (uint32_t)__popcll(at), nb = (uint32_t)__popcll(ab);
            const uint64_t sx = column_sum2(at, ab);
            const uint64_t sy = yt * na + yb * nb;
            const uint64_t packed = (uint64_t)(na + nb) | (sx << 13) | (sy << 31);
            const uint64_t rows = (na ? 1ull << yt : 0ull) | (nb ? 1ull << yb : 0ull);
            atomicAdd(&sh.sums[id - c0], (unsigned long long)packed);
            atomicOr(&sh.xm[id - c0], (unsigned long long)I);
            atomicOr(&sh.ym[id - c0], (unsigned long long)rows);
        }
        __syncthreads();
        // one record per local component: those inside the tile from the
        // front of the tile's slots, the others from the back
        for (uint32_t b0 = c0; b0 < c1; b0 += NT) {
            const uint32_t id = b0 + (uint32_t)tid;
            const bool has = id < c1;
            const uint32_t p = has ? sh.rpos[id] : 0u;
            const bool spanning = (p & 0x8000u) != 0;
            const uint64_t mc = __ballot(has && !spanning), ms = __ballot(has && spanning);
            uint32_t fc = 0, fs = 0;
            if (lane == 0) {
                if (mc) fc = atomicAdd(&sh.nrec[0], (uint32_t)__popcll(mc));
                if (ms) fs = atomicAdd(&sh.nrec[1], (uint32_t)__popcll(ms));
            }
            fc = (uint32_t)__shfl((int)fc, 0, 64);
            fs = (uint32_t)__shfl((int)fs, 0, 64);
            if (!has) continue;
            const uint32_t pos = p & 0x7FFFu;
            const uint64_t su = sh.sums[id - c0], xm = sh.xm[id - c0], ym = sh.ym[id - c0];
            const uint32_t x0 = (uint32_t)__builtin_ctzll(xm), x1 = 63u - (uint32_t)__builtin_clzll(xm);
            const uint32_t y0 = (uint32_t)__builtin_ctzll(ym), y1 = 63u - (uint32_t)__builtin_clzll(ym);
            uint4 r;
            r.x = sh.fin[pos] + 1u;
            r.y = y0 | (y1 << 6) | (pos << 12);
            r.z = (uint32_t)su;
            r.w = (uint32_t)(su >> 32) | (x0 << 17) | (x1 << 23);
            const uint32_t slot = spanning ? (uint32_t)(RMAX - 1) - (fs + bits_below(ms)) : fc + bits_below(mc);
            if (slot < (uint32_t)RMAX) rec[slot] = r;  // always (at most RMAX local components)
        }
        __syncthreads();
    }
    if (tid == 0) {
        s.ncnt[t] = sh.nrec[0] | (sh.nrec[1] << 16);
        s.tcnt[t] = sh.ncomp;
    }
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// A record's statistics in image coordinates.
struct Part {
    uint32_t area, x0, x1, y0, y1;
    uint64_t sx, sy;
};

__device__ __forceinline__ Part unpack(uint4 r, uint32_t ox, uint32_t oy) {
    const uint64_t su = ((uint64_t)(r.w & 0x1FFFFu) << 32) | r.z;
    Part p;
    p.area = (uint32_t)(su & 0x1FFFu);
    p.x0 = ox + ((r.w >> 17) & 63u);
    p.x1 = ox + ((r.w >> 23) & 63u);
    p.y0 = oy + (r.y & 63u);
    p.y1 = oy + ((r.y >> 6) & 63u);
    p.sx = ((su >> 13) & 0x3FFFFull) + (uint64_t)p.area * ox;
    p.sy = ((su >> 31) & 0x3FFFFull) + (uint64_t)p.area * oy;
    return p;
}

// Tile columns whose records one st_band workgroup emits.
constexpr uint32_t kBandGroupTiles = 16;

// Workgroup (b, g): tile row b, tile columns [16 g, 16 g + 16).  Every
// workgroup of the row scans the whole row's words (their ranks depend on
// the words to their left in every image row of the tile row) and keeps
// the part of its columns; the counts it needs are all loaded up front, and
// the ranks of its own words stay in LDS for its records.
template <int TH, bool CONN8>
__global__ void __launch_bounds__(1024) st_band(ImgView v, StatsView s) {
    constexpr int RMAX = stats_rmax(TH, CONN8);
    constexpr uint32_t NT = 1024;
    constexpr uint32_t GW = (uint32_t)TH * kBandGroupTiles;  // the group's row words
    __shared__ uint32_t part[2][16];
    __shared__ uint32_t gpre[kBandGroupTiles + 1];
    __shared__ uint64_t gcm[GW];
    __shared__ uint32_t gbase[GW];
    const uint32_t TX = (uint32_t)v.tilesX, TY = (uint32_t)v.tilesY, H = (uint32_t)v.H, W = (uint32_t)v.W;
    const uint32_t ng = (TX + kBandGroupTiles - 1u) / kBandGroupTiles;
    const uint32_t b = blockIdx.x / ng, g = blockIdx.x % ng;
    const uint32_t gx0 = g * kBandGroupTiles, gx1 = min(TX, gx0 + kBandGroupTiles), gn = gx1 - gx0;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    // the tile row's words are consecutive in raster order; this thread's
    // share of them, the components of the tile rows above, and the group's
    // record counts, loaded together
    const uint32_t y0 = b * (uint32_t)TH, y1 = min(H, y0 + (uint32_t)TH);
    const size_t w0 = (size_t)y0 * TX;
    const uint32_t nw = (y1 - y0) * TX;
    const uint32_t per = (nw + NT - 1u) / NT;
    const uint32_t a0 = min(nw, tid * per), a1 = min(nw, a0 + per);
    uint32_t acc = 0, c = 0;
    for (uint32_t i = tid; i < b * TX; i += NT) acc += s.tcnt[i];
    for (uint32_t w = a0; w < a1; ++w) c += (uint32_t)__popcll(s.cm[w0 + w]);
    const uint32_t nrec = wave == 0 && lane < gn ? s.ncnt[b * TX + gx0 + lane] & 0xFFFFu : 0u;
    acc = wave_sum_u32(acc);
    uint32_t wtot;
    const uint32_t ex = wave_exclusive_scan(c, &wtot);
    if (lane == 0) {
        part[0][wave] = acc;
        part[1][wave] = wtot;
    }
    if (wave == 0) {
        uint32_t tot;
        const uint32_t p = wave_exclusive_scan(nrec, &tot);
        if (lane <= gn) gpre[lane] = lane < gn ? p : tot;
    }
    __syncthreads();
    uint32_t above = 0, run = ex, total = 0;
    for (uint32_t j = 0; j < 16u; ++j) {
        above += part[0][j];
        if (j < wave) run += part[1][j];
        total += part[1][j];
    }
    run += above;
    for (uint32_t w = a0; w < a1; ++w) {
        const size_t gw = w0 + w;
        const uint64_t m = s.cm[gw];
        const uint32_t wx = (uint32_t)(gw % TX);
        if (wx >= gx0 && wx < gx1) {
            const uint32_t li = (w / TX) * kBandGroupTiles + (wx - gx0);
            gcm[li] = m;
            gbase[li] = run;
            s.base[gw] = run;
            // components that reach a tile edge collect several records:
            // their output records start empty
            uint64_t sp = s.sm[gw];
            while (sp) {
                const uint32_t j = (uint32_t)__builtin_ctzll(sp);
                sp &= sp - 1ull;
                const uint32_t rank = run + (uint32_t)__popcll(m & ((1ull << j) - 1ull));
                if (rank < s.cap) {
                    const uint32_t y = (uint32_t)(gw / TX);
                    ccl_component &o = s.out[rank];
                    o.label = y * W + wx * (uint32_t)kTileW + j + 1u;
                    o.area = 0u;
                    o.x_min = 0xFFFFFFFFu;
                    o.y_min = 0xFFFFFFFFu;
                    o.x_max = 0u;
                    o.y_max = 0u;
                    o.sum_x = 0ull;
                    o.sum_y = 0ull;
                }
            }
        }
        run += (uint32_t)__popcll(m);
    }
    if (b + 1u == TY && g == 0 && tid == 0) *s.n_out = above + total;
    // components inside one tile: their single record is final.  The
    // group's records are numbered across its tiles (a prefix of their
    // counts), so all threads take part whatever the tiles hold.
    __syncthreads();
    const uint32_t nall = gpre[gn];
    for (uint32_t j = tid; j < nall; j += NT) {
        uint32_t k = 0;
        while (k + 1u < gn && gpre[k + 1u] <= j) ++k;
        const uint32_t tx = gx0 + k, t = b * TX + tx;
        const uint4 r = s.rec[(size_t)t * RMAX + (j - gpre[k])];
        const uint32_t pos = (r.y >> 12) & 0xFFFu;
        const uint32_t li = (pos >> 6) * kBandGroupTiles + k;
        const uint32_t rank = gbase[li] + (uint32_t)__popcll(gcm[li] & ((1ull << (pos & 63u)) - 1ull));
        if (rank >= s.cap) continue;
        const Part p = unpack(r, tx * (uint32_t)kTileW, y0);
        ccl_component o;
        o.label = r.x;
        o.area = p.area;
        o.x_min = p.x0;
        o.y_min = p.y0;
        o.x_max = p.x1;
        o.y_max = p.y1;
        o.sum_x = p.sx;
        o.sum_y = p.sy;
        s.out[rank] = o;
    }
}

// Rank of the component whose root is pixel r.
__device__ __forceinline__ uint32_t rank_of(const StatsView &s, uint32_t r, uint32_t W, uint32_t TX) {
    const uint32_t y = r / W, x = r - y * W;
    const size_t w = (size_t)y * TX + x / (uint32_t)kTileW;
    return s.base[w] + (uint32_t)__popcll(s.cm[w] & ((1ull << (x & 63u)) - 1ull));
}

__device__ __forceinline__ void add_global(ccl_component &o, const Part &p) {
    atomicAdd(&o.area, p.area);
    atomicMin(&o.x_min, p.x0);
    atomicMax(&o.x_max, p.x1);
    atomicMin(&o.y_min, p.y0);
    atomicMax(&o.y_max, p.y1);
    atomicAdd((unsigned long long *)&o.sum_x, (unsigned long long)p.sx);
    atomicAdd((unsigned long long *)&o.sum_y, (unsigned long long)p.sy);
}

constexpr int kSpanSlots = 2048;

// Tiles of one tile row whose edge-reaching records one st_span workgroup
// reduces.  Under 8-connectivity a whole tile row: a percolating component
// has records in most tiles, and each workgroup adds its part to that
// component's one output record with atomics.  Under 4-connectivity the
// crossing components are many and small (a tile row's distinct labels
// would overflow the table), so runs of 16 tiles (measured: 47 µs per
// launch with whole rows, 26 with 32 tiles, 15 with 16 or 8, at 4096² p=0.5).
template <bool CONN8>
__host__ __device__ constexpr uint32_t span_tiles(uint32_t tiles_x) {
    return CONN8 ? tiles_x : 16u;
}

constexpr uint32_t kEmpty = 0u;  // no component has label 0

struct SpanLds {
    uint32_t key[kSpanSlots], area[kSpanSlots], x0[kSpanSlots], x1[kSpanSlots], y0[kSpanSlots],
        y1[kSpanSlots];
    unsigned long long sx[kSpanSlots], sy[kSpanSlots];
    uint32_t tpre[1025];
    uint32_t wpart[16];
};

// One workgroup per span_tiles() tiles of a tile row: the records of their
// components that reach a tile edge, reduced by label in an LDS hash table,
// then added to the output records.  A component that crosses many tiles
// (one that percolates) has a record in most of them: the wavefront's
// smallest label is reduced across lanes first, so it costs one table
// update per wavefront pass, and one set of global atomics per workgroup.
template <int TH, bool CONN8>
__global__ void __launch_bounds__(1024) st_span(ImgView v, StatsView s) {
    constexpr int RMAX = stats_rmax(TH, CONN8);
    constexpr uint32_t NT = 1024;
    __shared__ SpanLds sh;
    const uint32_t TX = (uint32_t)v.tilesX, W = (uint32_t)v.W;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t per = span_tiles<CONN8>(TX), nch = (TX + per - 1u) / per;
    const uint32_t ty = blockIdx.x / nch, cx = (blockIdx.x % nch) * per, cend = min(TX, cx + per);
    for (uint32_t i = tid; i < (uint32_t)kSpanSlots; i += NT) {
        sh.key[i] = kEmpty;
        sh.area[i] = 0u;
        sh.x0[i] = sh.y0[i] = 0xFFFFFFFFu;
        sh.x1[i] = sh.y1[i] = 0u;
        sh.sx[i] = sh.sy[i] = 0ull;
    }
    auto add_lds = [&](uint32_t l, const Part &p) {
        uint32_t h = (l * 2654435761u) >> 21;  // 11 bits
        for (int probe = 0; probe < 8; ++probe) {
            const uint32_t kk = atomicCAS(&sh.key[h], kEmpty, l);
            if (kk == kEmpty || kk == l) {
                atomicAdd(&sh.area[h], p.area);
                atomicMin(&sh.x0[h], p.x0);
                atomicMax(&sh.x1[h], p.x1);
                atomicMin(&sh.y0[h], p.y0);
                atomicMax(&sh.y1[h], p.y1);
                atomicAdd(&sh.sx[h], (unsigned long long)p.sx);
                atomicAdd(&sh.sy[h], (unsigned long long)p.sy);
                return;
            }
            h = (h + 1u) & (uint32_t)(kSpanSlots - 1);
        }
        // table crowded around h: straight to the output record
        const uint32_t rank = rank_of(s, l - 1u, W, TX);
        if (rank < s.cap) add_global(s.out[rank], p);
    };
    __syncthreads();
    for (uint32_t c0 = cx; c0 < cend; c0 += NT) {
        // the next (at most 1024) tiles: prefix of their counts
        const uint32_t tcount = min(NT, cend - c0);
        const uint32_t mine = tid < tcount ? s.ncnt[ty * TX + c0 + tid] >> 16 : 0u;
        uint32_t wtot;
        const uint32_t ex = wave_exclusive_scan(mine, &wtot);
        if (lane == 0) sh.wpart[wave] = wtot;
        __syncthreads();
        uint32_t off = 0, total = 0;
        for (uint32_t j = 0; j < 16u; ++j) {
            if (j < wave) off += sh.wpart[j];
            total += sh.wpart[j];
        }
        sh.tpre[tid] = off + ex;
        __syncthreads();
        for (uint32_t j0 = 0; j0 < total; j0 += NT) {
            const uint32_t j = j0 + tid;
            const bool has = j < total;
            uint32_t l = 0xFFFFFFFFu;
            Part p{};
            if (has) {
                // tile of record j: the last tile whose prefix is <= j
                uint32_t lo = 0, hi = tcount - 1u;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1u) >> 1;
                    if (sh.tpre[mid] <= j) lo = mid;
                    else hi = mid - 1u;
                }
                const uint32_t tx = c0 + lo, t = ty * TX + tx;
                const uint32_t k = j - sh.tpre[lo];
                const uint4 r = s.rec[(size_t)t * RMAX + (RMAX - 1) - k];
                l = r.x;
                p = unpack(r, tx * (uint32_t)kTileW, ty * (uint32_t)TH);
            }
            const uint32_t hot = wave_min_u32(l);
            if (__ballot(has)) {  // wave-uniform
                const bool isHot = has && l == hot;
                Part q;
                q.area = wave_sum_u32(isHot ? p.area : 0u);
                q.x0 = wave_min_u32(isHot ? p.x0 : 0xFFFFFFFFu);
                q.x1 = wave_max_u32(isHot ? p.x1 : 0u);
                q.y0 = wave_min_u32(isHot ? p.y0 : 0xFFFFFFFFu);
                q.y1 = wave_max_u32(isHot ? p.y1 : 0u);
                q.sx = wave_sum_u64(isHot ? p.sx : 0ull);
                q.sy = wave_sum_u64(isHot ? p.sy : 0ull);
                if (lane == 0) add_lds(hot, q);
                if (has && !isHot) add_lds(l, p);
            }
        }
        __syncthreads();
    }
    for (uint32_t i = tid; i < (uint32_t)kSpanSlots; i += NT) {
        const uint32_t l = sh.key[i];
        if (l == kEmpty) continue;
        const uint32_t rank = rank_of(s, l - 1u, W, TX);
        if (rank >= s.cap) continue;
        Part p;
        p.area = sh.area[i];
        p.x0 = sh.x0[i];
        p.x1 = sh.x1[i];
        p.y0 = sh.y0[i];
        p.y1 = sh.y1[i];
        p.sx = sh.sx[i];
        p.sy = sh.sy[i];
        add_global(s.out[rank], p);
    }
}

struct StatsLayout {
    size_t words, tiles, rmax;
    size_t cm, sm, base, tcnt, ncnt, rec, total;
};

StatsLayout stats_layout(int H, int W, int th, int conn) {
    StatsLayout l;
    const size_t tx = ((size_t)W + kTileW - 1) / kTileW, ty = ((size_t)H + th - 1) / th;
    l.words = (size_t)H * tx;
    l.tiles = tx * ty;
    l.rmax = (size_t)stats_rmax(th, conn == 8);
    l.cm = align_up(l.words * sizeof(uint64_t), 256);
    l.sm = l.cm;
    l.base = align_up(l.words * sizeof(uint32_t), 256);
    l.tcnt = align_up(l.tiles * sizeof(uint32_t), 256);
    l.ncnt = l.tcnt;
    l.rec = align_up(l.tiles * l.rmax * sizeof(uint4), 256);
    l.total = l.cm + l.sm + l.base + l.tcnt + l.ncnt + l.rec;
    return l;
}

template <int TH, bool CONN8>
hipError_t launch_stats_t(const ImgView &v, const StatsView &s, hipStream_t st) {
    const uint32_t tiles = (uint32_t)v.tilesX * (uint32_t)v.tilesY;
    const uint32_t ng = ((uint32_t)v.tilesX + kBandGroupTiles - 1u) / kBandGroupTiles;
    hipLaunchKernelGGL((k3_link_stats<TH, CONN8>), dim3(tiles), dim3(stats_waves<TH>() * 64), 0, st, v, s);
    hipLaunchKernelGGL((st_band<TH, CONN8>), dim3((uint32_t)v.tilesY * ng), dim3(1024), 0, st, v, s);
    const uint32_t per = span_tiles<CONN8>((uint32_t)v.tilesX);
    hipLaunchKernelGGL((st_span<TH, CONN8>), dim3((uint32_t)v.tilesY * (((uint32_t)v.tilesX + per - 1u) / per)),
                       dim3(1024), 0, st, v, s);
    return hipGetLastError();
}

hipError_t launch_stats(const ImgView &v, const StatsView &s, int th, int conn, hipStream_t st) {
    const bool c8 = conn == 8;
    switch (th) {
        case 16: return c8 ? launch_stats_t<16, true>(v, s, st) : launch_stats_t<16, false>(v, s, st);
        case 32: return c8 ? launch_stats_t<32, true>(v, s, st) : launch_stats_t<32, false>(v, s, st);
        case 64: return c8 ? launch_stats_t<64, true>(v, s, st) : launch_stats_t<64, false>(v, s, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace ccl

using namespace ccl;

extern "C" int ccl_label_2d_stats(const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                                  int32_t connectivity, uint32_t *labels, ccl_component *out,
                                  int64_t capacity, uint32_t *n_out, const ccl_config *cfg,
                                  void *stream) {
    int rc = validate_image(img, H, W, pitch, labels);
    if (rc != CCL_OK) return rc;
    if (!n_out || capacity < 0 || (capacity > 0 && !out)) return CCL_ERR_INVALID_ARG;
    if (connectivity != 4 && connectivity != 8) return CCL_ERR_UNSUPPORTED;
    int th = 0, nw = 0;
    if (cfg && (cfg->tile_h != 0 || cfg->waves != 0)) {
        // the statistics link is compiled for tiles of at most 64 rows
        if (!config_supported(cfg->tile_h, cfg->waves) || cfg->tile_h > 64) return CCL_ERR_UNSUPPORTED;
        th = cfg->tile_h;
        nw = cfg->waves;
    } else {
        default_config(H, W, connectivity, &th, &nw);
        if (th > 64) {
            th = 64;
            nw = 4;
        }
    }
    const WsLayout wl = ws_layout(H, W, th);
    const StatsLayout sl = stats_layout(H, W, th, connectivity);
    hipStream_t st = (hipStream_t)stream;
    void *ws = nullptr;
    std::unique_lock<std::mutex> held;
    rc = stream_workspace(st, wl.total + sl.total, &ws, &held);
    if (rc != CCL_OK) return rc;
    const ImgView v = make_view(img, H, W, pitch, labels, ws, th);
    char *p = (char *)ws + wl.total;
    StatsView s;
    s.cm = (uint64_t *)p;
    p += sl.cm;
    s.sm = (uint64_t *)p;
    p += sl.sm;
    s.base = (uint32_t *)p;
    p += sl.base;
    s.tcnt = (uint32_t *)p;
    p += sl.tcnt;
    s.ncnt = (uint32_t *)p;
    p += sl.ncnt;
    s.rec = (uint4 *)p;
    s.out = out;
    s.n_out = n_out;
    s.cap = capacity > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)capacity;
    hipError_t e = launch_merge(v, th, nw, connectivity, st);
    if (e == hipSuccess) e = launch_stats(v, s, th, connectivity, st);
    if (e != hipSuccess) return fail_hip(e);
    return CCL_OK;
}
