// The three labeling kernels (gfx950) for one image and for a batch, and
// their launchers.
//
//   local merge        Sec. II-A (Kernel 1): tile-local merge with coarse
//                      labeling over two-row bands (equal-value: runs);
//                      writes the tile's edge masks and edge-cell roots, its
//                      row masks, band data and per-interval records to the
//                      workspace, and seeds labels[root] = root + 1 for roots
//                      whose component touches a shared tile edge.
//   boundary analysis  Sec. II-B (Kernel 2): union-find on tile-edge cells
//                      only, one wavefront per tile (its top and left
//                      edges); the only phase with global atomics.
//   link               Sec. II-C: reads each tile's row masks and records,
//                      resolves each edge-touching local root once in the
//                      global forest and writes the dense output labels
//                      (1 + root, 0 for background); its per-tile body is in
//                      ccl_link.h, shared with the statistics link.
//
// The per-tile bodies are device functions shared by the single-image
// kernels (one workgroup per tile; four tiles per workgroup for the
// boundary analysis) and the batch kernels (the same bodies over one global
// numbering of the tiles of all images).

#include <type_traits>

#include "ccl_device.h"
#include "ccl_internal.h"
#include "ccl_link.h"

namespace ccl {

// ------------------------------------------------------------- local merge

// Equal-value local merge (every value class labeled, Sec. II-A's
// "same property" test): nodes are the runs of equal values of every row,
// 64 slots per row, swept row by row (sweep_band_eq).
template <int TH>
struct K1EqLds {
    static constexpr int SPR = slots_per_row<true>();
    uint32_t par[TH * SPR];                // run-indexed parents
    uint8_t col[TH * SPR];                 // every run's first column (node n lies in row n / 64)
    uint64_t msk[TH];                      // per row: run starts
    uint64_t flg[TH];                      // per row: local roots of edge-touching components
    uint16_t rinfo[TH];                    // runs | 0x100: first run at column 0 | 0x200: last ends at 63
    alignas(16) uint8_t pix[TH * kTileW];  // the tile's bytes
};

// Kernel 1 body for tile t of image v, equal-value labeling.  Ends after a
// workgroup barrier, so the caller may reuse the LDS for another tile.
template <int TH, int NW, bool CONN8>
__device__ __forceinline__ void k1_tile_eq(const ImgView &v, uint32_t t, K1EqLds<TH> &sh) {
    constexpr int SPR = slots_per_row<true>();
    constexpr int RPW = TH / NW;
    constexpr int NT = NW * 64;
    constexpr int CH = TH * 4;                  // 16-byte chunks per tile
    constexpr int LPT = (CH + NT - 1) / NT;     // chunks per thread
    constexpr int NODES = TH * SPR;             // run-indexed nodes per tile
    constexpr int NPT = (NODES + NT - 1) / NT;  // nodes per thread
    uint32_t *par = sh.par;
    uint8_t *col = sh.col;
    uint64_t *msk = sh.msk;
    uint64_t *flg = sh.flg;
    uint16_t *rinfo = sh.rinfo;
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const uint32_t TX = (uint32_t)v.tilesX;
    const int tx = (int)(t % TX), ty = (int)(t / TX);
    const bool hasUp = ty > 0, hasDown = ty + 1 < v.tilesY;
    const bool hasLeft = tx > 0, hasRight = tx + 1 < v.tilesX;
    // columns / rows of the tile inside the image
    const int wlim = min(kTileW, v.W - tx * kTileW), hlim = min(TH, v.H - ty * TH);

#pragma unroll
    for (int i = 0; i < LPT; ++i) {
        const int c = tid + i * NT;
        if (c < CH) ((uint4 *)sh.pix)[c] = load_chunk(v, tx, ty, TH, c >> 2, c & 3);
    }
    if (tid < TH) flg[tid] = 0ull;
    __syncthreads();
    sweep_band_eq<TH, RPW, CONN8>(par, col, msk, rinfo, sh.pix, wave, lane, wlim, hlim);
    if (NW > 1) {
        __syncthreads();
        if (wave > 0) merge_seam_eq<CONN8>(par, msk, sh.pix, wave * RPW, lane, wlim, hlim);
    }
    __syncthreads();

    // node-parallel finish: every node finds its root (read-only walk) and
    // its owner alone stores it, so par[n] is the root afterwards; the run's
    // record (the root's tile-local pixel) goes out
    uint16_t *sl = v.slots + (size_t)t * TH * SPR;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int n = tid + i * NT;
        // the numbering leaves unused slots at the end of each row
        if (n % SPR >= (int)(rinfo[n / SPR] & 0x7Fu)) continue;
        const uint32_t root = lds_root(par, (uint32_t)n);
        if (root != (uint32_t)n) lds_st(&par[n], root);
        sl[n] = (uint16_t)((root / SPR) * kTileW + col[root]);
    }
    __syncthreads();
    if (tid < TH) v.rowmask[(size_t)t * rowmask_words(TH) + tid] = msk[tid];
    // edge masks and edge-cell roots for the boundary analysis; every such
    // root is seeded in the forest (lanes of one component store the same
    // word)
    if (wave == 0) {
        uint64_t *mk = v.masks + (size_t)t * mask_words(TH);
        uint32_t *rt = v.roots + (size_t)t * roots_per_tile(TH);
        // cells taking part in the top / bottom row, run starts of those rows
        const uint64_t cols = wlim == 64 ? ~0ull : ((1ull << wlim) - 1ull);
        const uint64_t mTop = cols, mBot = TH - 1 < hlim ? cols : 0ull;
        const uint64_t sTop = uniform64(msk[0]), sBot = uniform64(msk[TH - 1]);
        // global index of the root pixel of run node n; the root is marked
        // in the edge-root masks (its component touches a shared edge)
        auto root_g = [&](uint32_t n) {
            const uint32_t root = lds_ld(&par[n]);
            const uint32_t rr = root / SPR, rc = col[root];
            atomicOr((unsigned long long *)&flg[rr], 1ull << rc);
            return global_index(v, tx, ty, TH, rr * kTileW + rc);
        };
        auto put = [&](uint32_t *dst, uint32_t g) {
            *dst = g;
            v.labels[g] = g + 1u;
        };
        if (hasUp && lane_in(mTop)) {
            const uint32_t n = bits_below(sTop) - (lane_in(sTop) ? 0u : 1u);
            put(&rt[roots_top(TH) + lane], root_g(n));
        }
        if (hasDown && lane_in(mBot)) {
            const uint32_t n = (uint32_t)((TH - 1) * SPR) + bits_below(sBot) - (lane_in(sBot) ? 0u : 1u);
            put(&rt[roots_bottom(TH) + lane], root_g(n));
        }
        // per row (lane = row): cells in the left / right column, last run
        const uint64_t mr = lane < TH ? msk[lane] : 0ull;
        const bool rowIn = lane < hlim;
        const bool lb = rowIn, rb = rowIn && wlim == 64;
        const uint32_t first = (uint32_t)(lane * SPR), lastRun = (uint32_t)__popcll(mr) - 1u;
        const uint64_t mLeft = __ballot(lb), mRight = __ballot(rb);
        if (hasLeft && lb) put(&rt[roots_left(TH) + lane], root_g(first));
        if (hasRight && rb) put(&rt[roots_right(TH) + lane], root_g(first + lastRun));
        if (lane == 0) {
            mk[kMaskTop] = mTop;
            mk[kMaskBottom] = mBot;
            mk[kMaskLeft] = mLeft;
            mk[mask_right(TH)] = mRight;
        }
        // only this wavefront marks edge roots: once its own LDS operations
        // have completed, the masks are whole
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane < TH) v.rowmask[(size_t)t * rowmask_words(TH) + TH + lane] = flg[lane];
    }
    __syncthreads();  // LDS may be reused for another tile
}

// Binary local merge over two-row bands (see sweep_bands).
template <int TH>
struct K1BandLds {
    uint32_t par[TH * kSlotsPerRow];  // node keys (a band has at most 64 intervals)
    uint64_t msk[TH];                 // per row: foreground mask
    uint64_t ends[TH / 2];            // per band: interval ends
    uint64_t flg[TH];                 // per row: local roots of edge-touching components
    uint16_t bbase[TH / 2];           // first node of every band
};

// Kernel 1 body for tile t of image v, binary labeling.  Writes the tile's
// row masks, edge-root masks, band interval ends and band bases, one record
// per node (the tile-local pixel of its root), the edge masks and the roots
// of the edge cells, and seeds those roots in the forest.  Ends after a
// workgroup barrier.
template <int TH, int NW, bool CONN8>
__device__ __forceinline__ void k1_tile_bands(const ImgView &v, uint32_t t, K1BandLds<TH> &sh) {
    constexpr int RPW = TH / NW;
    static_assert(RPW % 2 == 0, "a wavefront owns whole bands");
    constexpr int BPW = RPW / 2;
    constexpr int NB = TH / 2;
    constexpr int NT = NW * 64;
    constexpr int CH = TH * 4;               // 16-byte chunks per tile
    constexpr int LPT = (CH + NT - 1) / NT;  // chunks per thread
    uint32_t *par = sh.par;
    uint64_t *msk = sh.msk;
    uint64_t *flg = sh.flg;
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const uint32_t TX = (uint32_t)v.tilesX;
    const int tx = (int)(t % TX), ty = (int)(t / TX);
    const bool hasUp = ty > 0, hasDown = ty + 1 < v.tilesY;
    const bool hasLeft = tx > 0, hasRight = tx + 1 < v.tilesX;

#pragma unroll
    for (int i = 0; i < LPT; ++i) {
        const int c = tid + i * NT;
        if (c < CH) ((uint16_t *)msk)[c] = (uint16_t)nonzero_bytes16(load_chunk(v, tx, ty, TH, c >> 2, c & 3));
    }
    for (int r = tid; r < TH; r += NT) flg[r] = 0ull;
    __syncthreads();
    // every band's intervals, one band per lane: nodes are numbered densely
    // (an exclusive scan of the bands' interval counts)
    uint32_t bbv, nodes;
    {
        const uint64_t bt = lane < NB ? msk[2 * lane] : 0ull, bb = lane < NB ? msk[2 * lane + 1] : 0ull;
        const uint64_t s = band_starts<CONN8>(bt, bb);
        bbv = wave_exclusive_scan((uint32_t)__popcll(s), &nodes);
        if (tid < NB) {
            sh.ends[tid] = band_ends(bt | bb, s);
            sh.bbase[tid] = (uint16_t)bbv;
        }
    }
    __syncthreads();
    sweep_bands<BPW, CONN8>(par, msk, sh.ends, wave, lane, bbv);
    if (NW > 1) {
        __syncthreads();
        if (wave > 0) {
            const int k = wave * BPW;
            merge_band_seam<CONN8>(par, msk, sh.ends, k, (uint32_t)__builtin_amdgcn_readlane((int)bbv, k),
                                   (uint32_t)__builtin_amdgcn_readlane((int)bbv, k - 1));
        }
    }
    __syncthreads();

    // node-parallel finish: every node finds its root (read-only walk) and
    // its owner alone stores it, so par[n] is the root's key afterwards; the
    // node's record (the root's tile-local pixel) goes out
    uint16_t *sl = v.slots + (size_t)t * TH * kSlotsPerRow;
    for (uint32_t n = (uint32_t)tid; n < nodes; n += NT) {
        const uint32_t e = lds_ld(&par[n]);
        const uint32_t root = key_root(par, e);
        if (root != e) lds_st(&par[n], root);
        sl[n] = (uint16_t)(root >> kNodeBits);
    }
    __syncthreads();
    uint64_t *rw = v.rowmask + (size_t)t * rowmask_words(TH);
    for (int r = tid; r < TH; r += NT) rw[r] = msk[r];
    if (tid < NB) {
        rw[rowmask_ends(TH) + tid] = sh.ends[tid];
        ((uint16_t *)(rw + rowmask_bases(TH)))[tid] = sh.bbase[tid];
    }
    // edge masks and edge-cell roots for the boundary analysis; every such
    // root is seeded in the forest (lanes of one component store the same
    // word) and marked in the edge-root masks.  The four edges go to four
    // wavefronts (edge k to wavefront k mod NW), so their root loads and
    // stores overlap.
    {
        uint64_t *mk = v.masks + (size_t)t * mask_words(TH);
        uint32_t *rt = v.roots + (size_t)t * roots_per_tile(TH);
        const uint64_t mTop = uniform64(msk[0]), mBot = uniform64(msk[TH - 1]);
        auto root_g = [&](uint32_t n) {
            const uint32_t pos = lds_ld(&par[n]) >> kNodeBits;
            atomicOr((unsigned long long *)&flg[pos >> 6], 1ull << (pos & 63u));
            return global_index(v, tx, ty, TH, pos);
        };
        auto put = [&](uint32_t *dst, uint32_t g) {
            *dst = g;
            v.labels[g] = g + 1u;
        };
        // first node of the last band, read while every lane is active (a
        // lane that is off inside the branch below may not hold it)
        const uint32_t bbLast = (uint32_t)__builtin_amdgcn_readlane((int)bbv, NB - 1);
        if (wave == 0) {
            if (hasUp && lane_in(mTop)) put(&rt[roots_top(TH) + lane], root_g(bits_below(uniform64(sh.ends[0]))));
            if (lane == 0) {
                mk[kMaskTop] = mTop;
                mk[kMaskBottom] = mBot;
            }
        }
        if (wave == 1 % NW && hasDown && lane_in(mBot))
            put(&rt[roots_bottom(TH) + lane], root_g(bbLast + bits_below(uniform64(sh.ends[NB - 1]))));
        // per row (lane = row, 64 rows at a time): the band's first / last
        // interval holds the row's cell in the left / right column
        if (wave == 2 % NW || wave == 3 % NW) {
#pragma unroll
            for (int h = 0; h < col_words(TH); ++h) {
                const int r = 64 * h + lane;
                const uint64_t mr = r < TH ? msk[r] : 0ull;
                const bool lb = (mr & 1ull) != 0, rb = (mr >> 63) != 0;
                const uint32_t bFirst = r < TH ? (uint32_t)sh.bbase[r >> 1] : 0u;
                const uint32_t nInt = r < TH ? (uint32_t)__popcll(sh.ends[r >> 1]) : 0u;
                const uint64_t mLeft = __ballot(lb), mRight = __ballot(rb);
                if (wave == 2 % NW) {
                    if (hasLeft && lb) put(&rt[roots_left(TH) + r], root_g(bFirst));
                    if (lane == 0) mk[kMaskLeft + h] = mLeft;
                }
                if (wave == 3 % NW) {
                    if (hasRight && rb) put(&rt[roots_right(TH) + r], root_g(bFirst + nInt - 1u));
                    if (lane == 0) mk[mask_right(TH) + h] = mRight;
                }
            }
        }
    }
    __syncthreads();  // every wavefront's marks are in
    for (int r = tid; r < TH; r += NT) rw[TH + r] = flg[r];
    __syncthreads();  // LDS may be reused for another tile
}

// ------------------------------------------------------ boundary analysis

// One wavefront per tile: the tile's top edge against the tile above (64
// lanes, one per column; it also takes the diagonal pairs that cross the
// tile's upper corners) and its left edge against the tile on its left (TH
// lanes, one per row; pairs inside one tile row only), so every adjacent
// foreground pair that crosses tiles is examined by exactly one edge.  All
// masks and edge-cell roots are loaded up front; the neighbours' roots come
// from lane shifts.  Each lane holds up to four merge requests (two per
// edge), which are deduplicated and merged together.
template <int TH, bool CONN8>
__device__ __forceinline__ void k2_tile(const ImgView &v, uint32_t t) {
    constexpr int RT = roots_per_tile(TH);
    constexpr int MW = mask_words(TH);
    constexpr int LH = col_words(TH);  // left-edge cells per lane
    const int lane = lane_id();
    const uint32_t TX = (uint32_t)v.tilesX;
    const uint32_t tx = t % TX, ty = t / TX;
    const bool hasT = ty > 0, hasL = tx > 0, hasR = tx + 1u < TX;
    const uint64_t *mk = v.masks;
    const uint32_t *rts = v.roots;
    uint64_t dT = 0, uT = 0, xl = 0, xr = 0, dL[LH], uL[LH];
    uint32_t aT = kNone, rT = kNone, eTL = kNone, eTR = kNone, aL[LH], rL[LH];
    if (hasT) {
        const uint32_t tu = t - TX;
        dT = mk[(size_t)t * MW + kMaskTop];
        uT = mk[(size_t)tu * MW + kMaskBottom];
        if (hasL) {
            xl = mk[(size_t)(tu - 1u) * MW + kMaskBottom] >> 63;
            eTL = rts[(size_t)(tu - 1u) * RT + roots_bottom(TH) + 63];
        }
        if (hasR) {
            xr = (mk[(size_t)(tu + 1u) * MW + kMaskBottom] & 1ull) << 63;
            eTR = rts[(size_t)(tu + 1u) * RT + roots_bottom(TH)];
        }
        aT = rts[(size_t)t * RT + roots_top(TH) + lane];
        rT = rts[(size_t)tu * RT + roots_bottom(TH) + lane];
    }
#pragma unroll
    for (int h = 0; h < LH; ++h) {
        const int r = 64 * h + lane;
        dL[h] = uL[h] = 0ull;
        aL[h] = rL[h] = kNone;
        if (hasL) {
            dL[h] = mk[(size_t)t * MW + kMaskLeft + h];
            uL[h] = mk[(size_t)(t - 1u) * MW + mask_right(TH) + h];
            if (r < TH) {
                aL[h] = rts[(size_t)t * RT + roots_left(TH) + r];
                rL[h] = rts[(size_t)(t - 1u) * RT + roots_right(TH) + r];
            }
        }
    }
    // roots of the cells above-left / above-right (left edge: above / below)
    const uint32_t bTl = from_left(rT, eTL), bTr = from_right(rT, eTR);
    uint32_t A[2 + 2 * LH], B[2 + 2 * LH];
    {
        const PairMasks p = pair_masks<CONN8>(dT, uT, xl, xr);
        // at lane 0 the above-left cell lies in the tile to the left, so
        // PL and PM can both hold there; elsewhere they exclude each other
        B[0] = lane_in(p.pl) ? bTl : (lane_in(p.pm) ? rT : kNone);
        B[1] = lane_in(p.pr) ? bTr : (lane_in(p.pl & p.pm) ? rT : kNone);
        A[0] = A[1] = aT;
    }
    // the left edge as lines of 64 rows; the rows next to a chunk boundary
    // come from the neighbouring chunk, the tile's own first and last rows
    // have none (their corner pairs belong to the top edges)
#pragma unroll
    for (int h = 0; h < LH; ++h) {
        const uint64_t cl = h > 0 ? uL[h - 1] >> 63 : 0ull;
        const uint64_t cr = h + 1 < LH ? (uL[h + 1] & 1ull) << 63 : 0ull;
        const uint32_t el = h > 0 ? (uint32_t)__builtin_amdgcn_readlane((int)rL[h - 1], 63) : kNone;
        const uint32_t er = h + 1 < LH ? (uint32_t)__builtin_amdgcn_readlane((int)rL[h + 1], 0) : kNone;
        const uint32_t bLl = from_left(rL[h], el), bLr = from_right(rL[h], er);
        const PairMasks p = pair_masks<CONN8>(dL[h], uL[h], cl, cr);
        B[2 + 2 * h] = lane_in(p.pl) ? bLl : (lane_in(p.pm) ? rL[h] : kNone);
        B[3 + 2 * h] = lane_in(p.pr) ? bLr : (lane_in(p.pl & p.pm) ? rL[h] : kNone);
        A[2 + 2 * h] = A[3 + 2 * h] = aL[h];
    }
    union_requests<2 + 2 * LH>(A, B, [&](uint32_t a, uint32_t b) { g_union(v.labels, v.n, a, b); });
}

// Equal-value boundary analysis for tile t: like k2_tile, but a pair of
// cells across the edge is merged when their image values are equal (read
// straight from the image), and every such pair is proposed -- the
// deduplication keeps one union per distinct pair of roots.
template <int TH, bool CONN8>
__device__ __forceinline__ void k2_tile_eq(const ImgView &v, uint32_t t) {
    constexpr int RT = roots_per_tile(TH);
    constexpr uint32_t kOut = 0x100u, kOutUp = 0x200u;  // no byte equals these
    const int lane = lane_id();
    const uint32_t TX = (uint32_t)v.tilesX;
    const uint32_t tx = t % TX, ty = t / TX;
    const bool hasT = ty > 0, hasL = tx > 0, hasR = tx + 1u < TX;
    const int x0 = (int)tx * kTileW, y0 = (int)ty * TH;
    const int wlim = min(kTileW, v.W - x0), hlim = min(TH, v.H - y0);
    const uint32_t *rts = v.roots;
    uint32_t vT = kOut, vU = kOutUp, vUL = kOutUp, vUR = kOutUp, vC = kOut, vN = kOutUp;
    uint32_t aT = kNone, rT = kNone, eTL = kNone, eTR = kNone, aL = kNone, rL = kNone;
    if (hasT) {
        const uint32_t tu = t - TX;
        const uint8_t *row = v.img + (int64_t)y0 * v.pitch + x0;  // this tile's top row
        const uint8_t *up = row - v.pitch;                         // the row above it
        if (lane < wlim) {
            vT = row[lane];
            vU = up[lane];
            aT = rts[(size_t)t * RT + roots_top(TH) + lane];
            rT = rts[(size_t)tu * RT + roots_bottom(TH) + lane];
        }
        if (hasL) {
            vUL = up[-1];
            eTL = rts[(size_t)(tu - 1u) * RT + roots_bottom(TH) + 63];
        }
        if (hasR) {
            vUR = up[kTileW];
            eTR = rts[(size_t)(tu + 1u) * RT + roots_bottom(TH)];
        }
    }
    if (hasL && lane < hlim) {
        const uint8_t *p = v.img + (int64_t)(y0 + lane) * v.pitch + x0;
        vC = p[0];
        vN = p[-1];
        aL = rts[(size_t)t * RT + roots_left(TH) + lane];
        rL = rts[(size_t)(t - 1u) * RT + roots_right(TH) + lane];
    }
    // neighbours across the edge: above-left / above-right (top edge), the
    // left cells of the rows above / below (left edge, inside the tile rows)
    const uint32_t vUl = from_left(vU, vUL), vUr = from_right(vU, vUR);
    const uint32_t bTl = from_left(rT, eTL), bTr = from_right(rT, eTR);
    const uint32_t vNu = from_left(vN, kOutUp), vNd = from_right(vN, kOutUp);
    const uint32_t bLu = from_left(rL, kNone), bLd = from_right(rL, kNone);
    uint32_t A[6], B[6];
    A[0] = A[1] = A[2] = aT;
    A[3] = A[4] = A[5] = aL;
    B[0] = vT == vU ? rT : kNone;
    B[1] = CONN8 && vT == vUl ? bTl : kNone;
    B[2] = CONN8 && vT == vUr ? bTr : kNone;
    B[3] = vC == vN ? rL : kNone;
    B[4] = CONN8 && vC == vNu ? bLu : kNone;
    B[5] = CONN8 && vC == vNd ? bLd : kNone;
    union_requests<6>(A, B, [&](uint32_t a, uint32_t b) { g_union(v.labels, v.n, a, b); });
}

// ------------------------------------------------------ single-image kernels

template <int TH, int NW, bool CONN8, bool EQ>
__global__ void __launch_bounds__(NW * 64) k1_local_merge(ImgView v) {
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    if constexpr (EQ) {
        __shared__ K1EqLds<TH> sh;
        k1_tile_eq<TH, NW, CONN8>(v, t, sh);
    } else {
        __shared__ K1BandLds<TH> sh;
        k1_tile_bands<TH, NW, CONN8>(v, t, sh);
    }
}

template <int TH, bool CONN8, bool EQ>
__global__ void __launch_bounds__(256) k2_boundary(ImgView v, uint32_t tiles) {
    // the same XCD-contiguous tile ranges as the local merge and the link:
    // the forest chains of a region's components stay in one XCD's L2
    const uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)(xcd_remap(blockIdx.x, gridDim.x) * 4u + (threadIdx.x >> 6)));
    if (t >= tiles) return;  // wave-uniform
    if (EQ) k2_tile_eq<TH, CONN8>(v, t);
    else k2_tile<TH, CONN8>(v, t);
}

template <int TH, int NW, bool EQ>
__global__ void __launch_bounds__(NW * 64) k3_link(ImgView v) {
    __shared__ uint32_t fin[TH * kTileW];
    constexpr int SPR = slots_per_row<EQ>();
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    k3_tile<TH, NW, EQ>(v, t, v.rowmask + (size_t)t * rowmask_words(TH), v.slots + (size_t)t * TH * SPR, fin);
}

// ------------------------------------------------------------ batch kernels

template <int TH>
__device__ __forceinline__ ImgView batch_view(const BatchImage &b, const BatchWs &w) {
    ImgView v;
    v.img = b.img;
    v.labels = b.labels;
    v.masks = w.masks + (size_t)b.tile_base * mask_words(TH);
    v.roots = w.roots + (size_t)b.tile_base * roots_per_tile(TH);
    v.rowmask = w.rowmask + (size_t)b.tile_base * rowmask_words(TH);
    v.slots = w.slots + (size_t)b.tile_base * TH * kSlotsPerRow;
    v.pitch = b.pitch;
    v.H = b.H;
    v.W = b.W;
    v.tilesX = b.tilesX;
    v.tilesY = b.tilesY;
    v.n = b.n;
    v.aligned16 = b.aligned16;
    return v;
}

// The batch kernels are the single-image ones over one global numbering of
// the tiles of all images: one workgroup per tile for the local merge and
// the link, four tiles per workgroup for the boundary analysis.  The host
// sizes the grids for every call.
template <int TH, int NW, bool CONN8>
__global__ void __launch_bounds__(NW * 64) k1_batch(BatchArgs a) {
    __shared__ K1BandLds<TH> sh;
    const uint32_t g = xcd_remap(blockIdx.x, gridDim.x);
    if (g >= a.tiles) return;  // workgroup-uniform
    const uint32_t i = batch_image_of(a, g);
    if (threadIdx.x == 0) a.w.tile_img[g] = i;
    const BatchImage &d = a.descs[i];
    k1_tile_bands<TH, NW, CONN8>(batch_view<TH>(d, a.w), g - d.tile_base, sh);
}

template <int TH, bool CONN8>
__global__ void __launch_bounds__(256) k2_batch(BatchArgs a) {
    const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)(xcd_remap(blockIdx.x, gridDim.x) * 4u + (threadIdx.x >> 6)));
    if (g >= a.tiles) return;  // wave-uniform
    const BatchImage &d = a.descs[a.w.tile_img[g]];
    k2_tile<TH, CONN8>(batch_view<TH>(d, a.w), g - d.tile_base);
}

template <int TH, int NW>
__global__ void __launch_bounds__(NW * 64) k3_batch(BatchArgs a) {
    __shared__ uint32_t fin[TH * kTileW];
    const uint32_t g = xcd_remap(blockIdx.x, gridDim.x);
    if (g >= a.tiles) return;  // workgroup-uniform
    const BatchImage &d = a.descs[a.w.tile_img[g]];
    k3_tile<TH, NW, false>(batch_view<TH>(d, a.w), g - d.tile_base, a.w.rowmask + (size_t)g * rowmask_words(TH),
                           a.w.slots + (size_t)g * TH * kSlotsPerRow, fin);
}

// ---------------------------------------------------------------- launchers

template <int TH, int NW, bool CONN8, bool EQ>
static hipError_t launch_plain_t(const ImgView &v, hipStream_t stream, hipEvent_t *ev) {
    const uint32_t tiles = (uint32_t)v.tilesX * (uint32_t)v.tilesY;
    if (ev) (void)hipEventRecord(ev[0], stream);
    hipLaunchKernelGGL((k1_local_merge<TH, NW, CONN8, EQ>), dim3(tiles), dim3(NW * 64), 0, stream, v);
    if (ev) (void)hipEventRecord(ev[1], stream);
    if (tiles > 1)
        hipLaunchKernelGGL((k2_boundary<TH, CONN8, EQ>), dim3((tiles + 3) / 4), dim3(256), 0, stream,
                           v, tiles);
    if (ev) (void)hipEventRecord(ev[2], stream);
    constexpr int NW3 = link_waves<TH>();
    hipLaunchKernelGGL((k3_link<TH, NW3, EQ>), dim3(tiles), dim3(NW3 * 64), 0, stream, v);
    if (ev) (void)hipEventRecord(ev[3], stream);
    return hipGetLastError();
}

// Local merge and boundary analysis only (binary labeling): the phases
// before a link kernel that the caller launches.
template <int TH, int NW, bool CONN8>
static hipError_t launch_merge_t(const ImgView &v, hipStream_t stream) {
    const uint32_t tiles = (uint32_t)v.tilesX * (uint32_t)v.tilesY;
    hipLaunchKernelGGL((k1_local_merge<TH, NW, CONN8, false>), dim3(tiles), dim3(NW * 64), 0, stream, v);
    if (tiles > 1)
        hipLaunchKernelGGL((k2_boundary<TH, CONN8, false>), dim3((tiles + 3) / 4), dim3(256), 0, stream,
                           v, tiles);
    return hipGetLastError();
}

template <int TH, int NW, bool CONN8>
static void batch_kernels_t(BatchKernels *k) {
    k->k1 = (const void *)k1_batch<TH, NW, CONN8>;
    k->k2 = (const void *)k2_batch<TH, CONN8>;
    k->k3 = (const void *)k3_batch<TH, link_waves<TH>()>;
    k->block1 = NW * 64;
    k->block3 = link_waves<TH>() * 64;
    k->block2 = 256;
    k->tiles_per_group2 = 4;
}

bool config_supported(int th, int nw) {
    switch (th) {
        case 16: return nw == 1 || nw == 2 || nw == 4 || nw == 8;
        case 32: return nw == 1 || nw == 2 || nw == 4 || nw == 8 || nw == 16;
        case 64: return nw == 1 || nw == 2 || nw == 4 || nw == 8 || nw == 16;
        case 128: return nw == 2 || nw == 4 || nw == 8 || nw == 16;
        default: return false;
    }
}

#define CCL_FOR_EACH_CONFIG(X)                                                              \
    X(16, 1) X(16, 2) X(16, 4) X(16, 8) X(32, 1) X(32, 2) X(32, 4) X(32, 8) X(32, 16) \
        X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(64, 16) X(128, 2) X(128, 4) X(128, 8) X(128, 16)

// Tile configurations compiled for equal-value labeling.
#define CCL_FOR_EACH_EQ_CONFIG(X) X(16, 4) X(32, 2) X(32, 8) X(64, 4) X(64, 8)

bool config_supported_equal(int th, int nw) {
#define CCL_CASE(T, N) \
    if (th == T && nw == N) return true;
    CCL_FOR_EACH_EQ_CONFIG(CCL_CASE)
#undef CCL_CASE
    return false;
}

hipError_t launch_plain(const ImgView &v, int th, int nw, int conn, hipStream_t s, hipEvent_t *ev,
                        bool equal) {
    if (equal) {
#define CCL_CASE(T, N)                                                        \
    if (th == T && nw == N)                                                   \
        return conn == 8 ? launch_plain_t<T, N, true, true>(v, s, ev)         \
                         : launch_plain_t<T, N, false, true>(v, s, ev);
        CCL_FOR_EACH_EQ_CONFIG(CCL_CASE)
#undef CCL_CASE
        return hipErrorInvalidValue;
    }
#define CCL_CASE(T, N)                                                        \
    if (th == T && nw == N)                                                   \
        return conn == 8 ? launch_plain_t<T, N, true, false>(v, s, ev)        \
                         : launch_plain_t<T, N, false, false>(v, s, ev);
    CCL_FOR_EACH_CONFIG(CCL_CASE)
#undef CCL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_merge(const ImgView &v, int th, int nw, int conn, hipStream_t s) {
#define CCL_CASE(T, N)                                                        \
    if (th == T && nw == N)                                                   \
        return conn == 8 ? launch_merge_t<T, N, true>(v, s) : launch_merge_t<T, N, false>(v, s);
    CCL_FOR_EACH_CONFIG(CCL_CASE)
#undef CCL_CASE
    return hipErrorInvalidValue;
}

bool batch_kernels(int th, int nw, int conn, BatchKernels *out) {
#define CCL_CASE(T, N)                                                                   \
    if (th == T && nw == N) {                                                            \
        if (conn == 8) batch_kernels_t<T, N, true>(out);                                 \
        else batch_kernels_t<T, N, false>(out);                                          \
        return true;                                                                     \
    }
    CCL_FOR_EACH_CONFIG(CCL_CASE)
#undef CCL_CASE
    return false;
}

}  // namespace ccl
