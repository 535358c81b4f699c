// Device-side building blocks of the three labeling phases (gfx950, wave64).
//
// Tile model.  A tile is 64 pixels wide -- one lane of a 64-wide wavefront
// per column -- and TH rows tall (TH in {16, 32, 64, 128}).  A workgroup of NW
// wavefronts owns one tile at a time; wavefront w owns rows [w*RPW,
// (w+1)*RPW) with RPW = TH / NW.  A tile row is a 64-bit foreground mask, so
// the paper's row scan plus row-column unification (Sec. II-A-2) collapses
// to mask arithmetic: binary labeling takes two rows at a time, and the
// components of such a band are column intervals found from its two masks
// (see sweep_bands); those intervals are the union-find nodes.  The local
// UF (Sec. II-A-3) then merges each interval with the intervals of the band
// above that it touches through LDS atomicMin, always linking the node with
// the larger smallest pixel under the other.  Equal-value labeling keeps one
// node per run of equal values in a row.
//
// Forest encoding in global memory.  labels[p] holds 1 + parent(p); a root r
// holds r + 1 and background holds 0.  The final output is therefore itself a
// fully compressed forest, so the link phase can overwrite entries in place
// while other tiles still walk the forest.
//
// Workspace per tile, written by the local merge:
//   masks[...]      top-row, bottom-row, left-column, right-column foreground
//                   masks (boundary analysis; mask_words)
//   roots[...]      global raster index of the tile-local root of every cell
//                   on those four edges (boundary analysis)
//   rowmask[...]    the 64-bit foreground mask of every tile row, then per
//                   row the mask of the local root pixels whose component
//                   touches a shared tile edge, then (binary labeling) every
//                   two-row band's interval ends and first node (link)
//   slots[...]      one 16-bit record per union-find node (binary: per band
//                   interval; equal-value: per run, 64 slots per row): the
//                   tile-local pixel of the node's local root (link)
// Every root of an edge-touching component is also seeded in the forest,
// labels[root] = root + 1, before the boundary analysis runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

constexpr int kTileW = 64;               // tile width == wavefront width
constexpr uint32_t kNone = 0xFFFFFFFFu;  // "no node"

// Edge masks of a tile: the top and bottom rows (one word each), then the
// left and the right column, one bit per row (one word per 64 rows each).
enum { kMaskTop = 0, kMaskBottom = 1, kMaskLeft = 2 };
__host__ __device__ constexpr int col_words(int th) { return (th + 63) / 64; }
__host__ __device__ constexpr int mask_words(int th) { return 2 + 2 * col_words(th); }
__host__ __device__ constexpr int mask_right(int th) { return kMaskLeft + col_words(th); }

// Run records per tile row: a 64-pixel row has at most 32 foreground runs,
// and at most 64 equal-value runs.
template <bool EQ>
__host__ __device__ constexpr int slots_per_row() { return EQ ? 64 : 32; }
constexpr int kSlotsPerRow = slots_per_row<false>();

__host__ __device__ constexpr int roots_per_tile(int th) { return 2 * kTileW + 2 * th; }
// 64-bit words per tile of the row data: TH row masks, TH edge-root masks,
// TH / 2 band interval-end masks, then TH / 2 16-bit band bases (first
// record of every band)
__host__ __device__ constexpr int rowmask_words(int th) { return 2 * th + th / 2 + th / 8; }
__host__ __device__ constexpr int rowmask_ends(int th) { return 2 * th; }
__host__ __device__ constexpr int rowmask_bases(int th) { return 2 * th + th / 2; }
__host__ __device__ constexpr int roots_top(int) { return 0; }
__host__ __device__ constexpr int roots_bottom(int) { return kTileW; }
__host__ __device__ constexpr int roots_left(int) { return 2 * kTileW; }
__host__ __device__ constexpr int roots_right(int th) { return 2 * kTileW + th; }

// One image as the kernels see it.
struct ImgView {
    const uint8_t *img;
    uint32_t *labels;
    uint64_t *masks;    // [tiles][mask_words(TH)]
    uint32_t *roots;    // [tiles][roots_per_tile(TH)]
    uint64_t *rowmask;  // [tiles][rowmask_words(TH)]: row masks, edge-root masks, row bases
    uint16_t *slots;    // [tiles][TH][slots_per_row]
    int64_t pitch;
    int32_t H, W;
    int32_t tilesX, tilesY;
    uint32_t n;         // H * W (<= 2^32 - 1)
    int32_t aligned16;  // img and pitch are multiples of 16 bytes
};

// One image of a batch as the batch kernels see it (device descriptor).
// Tiles of all images are numbered consecutively: image i owns global tiles
// [tile_base, tile_base + tilesX*tilesY), and its workspace lives at those
// tile offsets.
struct BatchImage {
    const uint8_t *img;
    uint32_t *labels;
    int64_t pitch;
    int32_t H, W;
    int32_t tilesX, tilesY;
    uint32_t n;
    int32_t aligned16;
    uint32_t tile_base, pad;
};

// Workspace of a batch context, indexed by global tile.  tile_img[g] is the
// image that owns global tile g (written by the local merge, read by the
// two later phases).
struct BatchWs {
    uint64_t *masks;
    uint32_t *roots;
    uint64_t *rowmask;
    uint16_t *slots;
    uint32_t *tile_img;
};

// Kernel argument of the three batch kernels (one call).  tile_base holds
// the n images' first global tiles (ascending) and coarse every 64th of
// them, so the local merge finds a tile's image with two coalesced reads.
struct BatchArgs {
    const BatchImage *descs;
    const uint32_t *tile_base;
    const uint32_t *coarse;
    BatchWs w;
    uint32_t n, tiles;
};

// ---------------------------------------------------------- launch helpers

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

// ------------------------------------------------------------------ helpers

// Image that owns global tile g: the last image whose tile_base is <= g,
// i.e. the number of bases <= g minus one.  First among the coarse bases
// (every 64th image), then among the 64 images of that group; each lane
// compares one base.
__device__ __forceinline__ uint32_t batch_image_of(const BatchArgs &a, uint32_t g) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nc = (a.n + 63u) >> 6;
    uint32_t cnt = 0;
    for (uint32_t j = 0; j < nc; j += 64) {
        const uint32_t k = j + lane;
        cnt += (uint32_t)__popcll(__ballot(k < nc && a.coarse[k] <= g));
    }
    const uint32_t k = ((cnt - 1u) << 6) + lane;
    return ((cnt - 1u) << 6) + (uint32_t)__popcll(__ballot(k < a.n && a.tile_base[k] <= g)) - 1u;
}


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

// Global forest accessors for the concurrent boundary phase.  Links are
// made with agent-scope atomicMin, which acts on the one coherent copy.
// Finds read through the caches (g_ld): a read may return an older parent
// than the current one, but the forest only ever gets coarser -- a parent
// is only replaced by one of its own ancestors, always a smaller index --
// so an old parent is still an ancestor, every walk still ends, and a node
// taken for a root by mistake is caught by the value the linking atomicMin
// returns (the link is then retried from there).  Reading the hot roots of
// large components from the caches instead of memory is what keeps the
// phase from serializing on them.
__device__ __forceinline__ uint32_t g_ld(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t g_min(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------- LDS union-find

// Every parent is strictly smaller than its child, so `p >= x` both detects
// a root (p == x) and stops on anything that is not a valid parent; every
// loop below therefore strictly decreases its index and always terminates.

// Find without writes.  Compression is done by the owner of each node only
// (see the finish pass of the local merge): a path-halving store by one
// thread can land after another thread stored the final root into the same
// node and leave a non-root ancestor there, which breaks every later reader
// that takes par[n] to be the root.
__device__ __forceinline__ uint32_t lds_root(const uint32_t *par, uint32_t x) {
    while (true) {
        const uint32_t p = lds_ld(&par[x]);
        if (p >= x) return x;
        x = p;
    }
}

// Join the trees of a and b (Sec. II-A-3), the larger index under the
// smaller, without finding the roots first: the atomicMin lowers the larger
// node's parent to the smaller node and returns the parent it had.  If that
// was the node itself, a root was linked and the join is done; otherwise the
// node is now the smaller one's child, its old parent still has to be joined
// to it, and the step repeats on that pair.  The larger index of the pair
// drops every step, so the walk ends; every parent only ever moves to a
// smaller node connected to it, so no concurrent link is lost.  Callers
// mostly pass roots, which makes this a single atomic.
__device__ __forceinline__ void lds_link(uint32_t *par, uint32_t a, uint32_t b) {
    while (a != b) {
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicMin(&par[b], a);
        if (old >= b) return;
        b = old;
    }
}

// ------------------------------------------------------ global union-find

// Find steps after which a join also points its starting nodes at the root.
constexpr uint32_t kLongWalk = 256u;

// Roots of a and b in the global forest, found together so that the loads
// of both walks are in flight at once.  Path halving: a node whose parent
// is not a root is pointed at its grandparent with an atomicMin, which can
// only lower a parent to an ancestor.  steps counts the loop's passes.
__device__ __forceinline__ void g_find2(uint32_t *L, uint32_t &a, uint32_t &b, uint32_t &steps) {
    // every step issues both walks' loads unconditionally (a root re-reads
    // its own entry), so the two loads are in flight together and the
    // wavefront waits once per step
    while (true) {
        ++steps;
        uint32_t pa = g_ld(&L[a]) - 1u, pb = g_ld(&L[b]) - 1u;
        bool ra = pa >= a, rb = pb >= b;
        if (ra && rb) return;
        pa = ra ? a : pa;
        pb = rb ? b : pb;
        const uint32_t ga = g_ld(&L[pa]) - 1u, gb = g_ld(&L[pb]) - 1u;
        if (!ra) {
            if (ga >= pa) {
                a = pa;
                ra = true;
            } else {
                g_min(&L[a], ga + 1u);
                a = ga;
            }
        }
        if (!rb) {
            if (gb >= pb) {
                b = pb;
                rb = true;
            } else {
                g_min(&L[b], gb + 1u);
                b = gb;
            }
        }
        if (ra && rb) return;
    }
}

// Link the trees of a and b, the larger root under the smaller (Sec. II-B).
// When the atomicMin shows that b stopped being a root meanwhile, the value
// it returns is b's new parent and the link is retried from there, so no
// concurrent link is lost.
//
// A join whose walks took many steps (a long chain, as a spiral or a
// serpentine builds across tiles) points both of its starting nodes straight
// at the final root, so the next join along the same chain starts next to
// the root instead of walking it again.  Path halving alone only halves such
// a chain per walk.  Joins that found their roots quickly skip this.
__device__ __forceinline__ void g_union(uint32_t *L, uint32_t n, uint32_t a, uint32_t b) {
    if (a >= n || b >= n) return;
    const uint32_t a0 = a, b0 = b;
    uint32_t steps = 0;
    while (true) {
        g_find2(L, a, b, steps);
        if (a == b) break;
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = g_min(&L[b], a + 1u) - 1u;
        if (old >= b) break;
        b = old;
    }
    if (steps > kLongWalk) {
        g_min(&L[a0], a + 1u);
        g_min(&L[b0], a + 1u);
    }
}

// Merge requests of one wavefront: every lane holds NS (a, b) slots (b ==
// kNone: empty).  Along a tile edge most requests repeat the same pair of
// tile-local roots, so the distinct pairs are collected first (one per
// lane, at most 64 at a time) and then merged by all lanes concurrently
// with join(a, b) (a lane without a pair gets kNone for both).
template <int NS, class Union>
__device__ __forceinline__ void union_requests(const uint32_t (&A)[NS], const uint32_t (&B)[NS],
                                               Union &&join) {
    const int lane = (int)(threadIdx.x & 63);
    uint64_t pend[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) pend[s] = __ballot(B[s] != kNone);
    bool more = true;
    while (more) {  // rounds of up to 64 distinct pairs, one per lane
        more = false;
        uint32_t ma = kNone, mb = kNone;
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            while (pend[s] && cnt < 64) {
                const int lead = __builtin_ctzll(pend[s]);
                const uint32_t PA = (uint32_t)__builtin_amdgcn_readlane((int)A[s], lead);
                const uint32_t PB = (uint32_t)__builtin_amdgcn_readlane((int)B[s], lead);
                if (lane == cnt) {
                    ma = PA;
                    mb = PB;
                }
#pragma unroll
                for (int q = s; q < NS; ++q) pend[q] &= ~__ballot(A[q] == PA && B[q] == PB);
                ++cnt;
            }
            more = more || pend[s] != 0ull;
        }
        join(ma, mb);  // one call site: lanes without a pair return at once
    }
}

// Root of x once no link is made any more (link phase).  A long walk (a
// component threaded through many tiles, such as a one-pixel-wide spiral)
// then points every node it passed at the root, so the tiles that walk
// there later stop short; a short one writes nothing.  The stores are the
// final root, the value every other writer of those entries stores too.
__device__ __forceinline__ uint32_t g_root(uint32_t *L, uint32_t x0) {
    uint32_t x = x0, v = L[x] - 1u, steps = 0;
    while (v < x) {
        x = v;
        v = L[x] - 1u;
        ++steps;
    }
    if (steps > 8u) {
        uint32_t y = x0;
        while (y > x) {
            const uint32_t ny = L[y] - 1u;
            if (ny >= y) break;
            L[y] = x + 1u;
            y = ny;
        }
    }
    return x;
}

// ------------------------------------------------------ tile-local labeling

__device__ __forceinline__ uint32_t global_index(const ImgView &v, int tx, int ty, int th,
                                                 uint32_t l) {
    const uint64_t y = (uint64_t)ty * th + (l >> 6);
    const uint64_t x = (uint64_t)tx * kTileW + (l & 63u);
    return (uint32_t)(y * (uint64_t)v.W + x);
}

// Bit i (i < 4) set iff byte i of w is nonzero: fold every byte onto its low
// bit, then gather the four low bits into bits 28..31 with one multiply (the
// shifted copies land on distinct bits below 24, so nothing carries).
__device__ __forceinline__ uint32_t nonzero_bytes4(uint32_t w) {
    uint32_t t = w | (w >> 4);
    t |= t >> 2;
    t |= t >> 1;
    t &= 0x01010101u;
    return (t * 0x10204080u) >> 28;
}

__device__ __forceinline__ uint32_t nonzero_bytes16(uint4 b) {
    return nonzero_bytes4(b.x) | (nonzero_bytes4(b.y) << 4) | (nonzero_bytes4(b.z) << 8) |
           (nonzero_bytes4(b.w) << 12);
}

// 16 pixels of one tile row: row `row` of tile (tx, ty), columns
// [16q, 16q + 16).  One 16-byte load when the chunk is aligned and inside
// the image, byte loads with zero fill otherwise.
template <class V>
__device__ __forceinline__ uint4 load_chunk(const V &v, int tx, int ty, int th, int row, int q) {
    const int y = ty * th + row;
    const int x = tx * kTileW + q * 16;
    uint4 b = make_uint4(0u, 0u, 0u, 0u);
    if (y >= v.H) return b;
    const uint8_t *p = v.img + (int64_t)y * v.pitch + x;
    if (v.aligned16 && x + 16 <= v.W) return *(const uint4 *)p;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (x + i < v.W) w[i >> 2] |= (uint32_t)p[i] << (8 * (i & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// ------------------------------------------------- run-indexed local forest
//
// Inside K1 the union-find nodes are runs: run k (0-based, left to right) of
// tile row r is node r*32 + k.  Run order within a row follows the columns
// and rows follow each other, so node order is raster order of run starts
// and the smallest node of a component is the run holding its smallest
// pixel.  col[node] keeps the run's first column.

// Lane predicate from a wave-uniform 64-bit mask (no VALU work).
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Number of set bits of m strictly below this lane.
__device__ __forceinline__ uint32_t bits_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// acc + the set bits of m below this lane
__device__ __forceinline__ uint32_t bits_below_plus(uint64_t m, uint32_t acc) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, acc));
}

// Value of lane-1 / lane+1 (whole-wave DPP shifts; lane 0 / 63 get `edge`).
__device__ __forceinline__ uint32_t from_left(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_right(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130, 0xF, 0xF, false);
}
// The same shifts for callers that never read lane 0's / lane 63's result:
// those lanes get 0 (one instruction, no edge value to set up).
__device__ __forceinline__ uint32_t from_left_any(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t from_right_any(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true);
}

__device__ __forceinline__ uint64_t run_starts(uint64_t d) { return d & ~(d << 1); }
// last cell of every run
__device__ __forceinline__ uint64_t run_ends(uint64_t d) { return d & ~(d >> 1); }

// Exclusive prefix sum over the 64 lanes of a wavefront; *total gets the
// sum of all lanes.  DPP row shifts scan each 16-lane row, then the last
// lane of row 0 / row 1 is broadcast into rows 1 and 3 / 2 and 3.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t x, uint32_t *total) {
    uint32_t v = x;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    *total = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    return v - x;
}

// A value every lane holds identically, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Lane k's value of x (k wave-uniform), in scalar registers.
__device__ __forceinline__ uint64_t lane_value64(uint64_t x, int k) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), k);
    return ((uint64_t)hi << 32) | lo;
}

// Which (lower run, upper run) pairs of two adjacent lines are merged, as
// lane masks over the lower line d with the upper line u: every pair of runs
// that touch is taken exactly once, by the leftmost lower cell adjacent to
// the upper run.  8-connectivity: PL = the upper run containing column j-1
// (only at a lower run start), PM = the upper run starting at j (only at a
// lower run start whose above-left is empty), PR = the upper run starting at
// j+1.  4-connectivity: PM = the upper run containing j, at the lower run
// start or where the upper run starts.  On a tile's top edge the upper line
// continues into the neighbouring tiles: xl (bit 0 only) is set when the
// cell above-left of column 0 is foreground, xr (bit 63 only) when the cell
// above-right of column 63 is; inside a tile both are 0.
struct PairMasks { uint64_t pl, pm, pr; };

template <bool CONN8>
__device__ __forceinline__ PairMasks pair_masks(uint64_t d, uint64_t u, uint64_t xl = 0,
                                                uint64_t xr = 0) {
    const uint64_t S = run_starts(d);
    PairMasks p;
    if (CONN8) {
        p.pl = S & ((u << 1) | xl);
        p.pm = S & u & ~(u << 1);
        p.pr = d & (((u >> 1) & ~u) | xr);
    } else {
        p.pl = 0;
        p.pm = d & u & (S | ~(u << 1));
        p.pr = 0;
    }
    return p;
}

// Sweep of one wavefront's band of rows, top to bottom (Sec. II-A-2/3).
// `ra` carries, per lane, the root node of the pixel above (kNone for
// background), so the roots a run touches come from neighbouring lanes'
// registers.  A run's parent becomes the smallest of those roots (one LDS
// atomicMin per lane on its node).  Every other root it touches is then
// linked under that one; they were roots when the row began, so one
// atomicMin per link normally does it, and only a link that finds its root
// already linked elsewhere in this row continues as a walk up both trees.  After
// a row with links the row's roots are re-resolved, so `ra` always holds
// true roots.
//
// Node numbering: the first node of tile row j is lane j's value of `rbv`
// (a row's nodes are consecutive and rows follow each other, so nodes stay
// in raster order of run starts): either dense, an exclusive scan of the
// rows' run counts, or sparse, j * 32.  A foreground cell's run follows the
// runs that end before it.  cr[node] = first column | row << 8.
template <int TH, int RPW, bool CONN8>
__device__ __forceinline__ void sweep_band(uint32_t *par, uint16_t *cr, const uint64_t *msk,
                                           int wave, int lane, uint32_t rbv) {
    uint32_t ra = kNone;
    uint64_t u = 0;
    uint64_t m[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) m[k] = uniform64(msk[wave * RPW + k]);
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        const uint64_t d = m[k];
        const uint64_t S = run_starts(d);
        const bool fg = lane_in(d), isS = lane_in(S);
        const uint32_t rb = (uint32_t)__builtin_amdgcn_readlane((int)rbv, r);
        const uint32_t node = bits_below_plus(run_ends(d), rb);
        uint32_t *pn = &par[node];
        if (isS) {
            lds_st(pn, node);
            cr[node] = (uint16_t)(lane | (r << 8));
        }
        uint32_t md = fg ? node : kNone;
        if (k > 0) {
            const PairMasks p = pair_masks<CONN8>(d, u);
            const uint32_t rL = from_left(ra, kNone), rR = from_right(ra, kNone);
            // PL and PM are disjoint
            const uint32_t t0 = lane_in(p.pm) ? ra : (lane_in(p.pl) ? rL : kNone);
            const uint32_t t1 = lane_in(p.pr) ? rR : kNone;
            const uint32_t tm = t0 < t1 ? t0 : t1;
            if (tm != kNone) atomicMin(pn, tm);
            if (fg) md = lds_ld(pn);  // the smallest root the run touches
            const bool n0 = t0 != kNone && t0 != md;
            const bool n1 = t1 != kNone && t1 != md;
            if (__ballot(n0 || n1)) {
                uint32_t o0 = 0, o1 = 0;
                if (n0) o0 = atomicMin(&par[t0], md);
                if (n1) o1 = atomicMin(&par[t1], md);
                const bool r0 = n0 && o0 < t0 && o0 != md, r1 = n1 && o1 < t1 && o1 != md;
                if (__ballot(r0 || r1)) {
                    if (r0) lds_link(par, md, o0);
                    if (r1) lds_link(par, md, o1);
                }
                if (fg) md = lds_root(par, md);
                if (isS) lds_st(pn, md);
            }
        }
        ra = md;
        u = d;
    }
}

// ------------------------------------------------- two-row band nodes
//
// The binary local merge takes the tile two rows at a time.  Inside such a
// band every connected component is one contiguous interval of columns:
// under 8-connectivity the intervals are the runs of t | b (t the band's top
// row, b its bottom row); under 4-connectivity they are those runs split
// wherever neither row continues across the column boundary.  So the row
// scan and the row-column unification of Sec. II-A-2 reduce to a few 64-bit
// operations per band, and the union-find of Sec. II-A-3 runs over intervals
// and over half as many steps as rows.
//
// Node n of a tile is its n-th interval in band order, left to right inside
// a band.  Every parent entry holds a key, the node's smallest pixel (tile
// row << 6 | column) above its node's byte offset in the parent array
// (node << 2, so a key addresses its entry with one mask): an atomicMin on
// keys links the tree whose node holds the larger pixel under the other, so
// the root of every tree is the node holding the component's smallest pixel
// (the linking rule of Sec. II-A-3, with pixels as the order).  A root's
// entry is its own key.

constexpr uint32_t kNodeBits = 14;  // the byte offsets of at most 4096 nodes per tile (64 intervals per band)
constexpr uint32_t kNodeMask = ((1u << 12) - 1u) << 2;

// Key of node n whose smallest pixel is pos.
__device__ __forceinline__ uint32_t node_key(uint32_t pos, uint32_t n) { return (pos << kNodeBits) | (n << 2); }

// Parent entry of the node that key k names.
__device__ __forceinline__ uint32_t *key_entry(uint32_t *par, uint32_t k) {
    return (uint32_t *)((char *)par + (k & kNodeMask));
}
__device__ __forceinline__ const uint32_t *key_entry(const uint32_t *par, uint32_t k) {
    return (const uint32_t *)((const char *)par + (k & kNodeMask));
}

// First column of every interval of the band (t above b).
template <bool CONN8>
__device__ __forceinline__ uint64_t band_starts(uint64_t t, uint64_t b) {
    const uint64_t m = t | b;
    uint64_t s = m & ~(m << 1);
    if (!CONN8) s |= m & (m << 1) & ~(t & (t << 1)) & ~(b & (b << 1));
    return s;
}

// Last column of every interval, from the band's columns m = t | b and the
// interval starts s.
__device__ __forceinline__ uint64_t band_ends(uint64_t m, uint64_t s) { return m & (~(m >> 1) | (s >> 1)); }

// Root key of the tree holding key k (read-only walk; see lds_root).
__device__ __forceinline__ uint32_t key_root(const uint32_t *par, uint32_t k) {
    while (true) {
        const uint32_t p = lds_ld(key_entry(par, k));
        if (p >= k) return k;
        k = p;
    }
}

// Join the trees of the nodes with keys a and b (or of any of their
// ancestors), as lds_link does with node numbers.
__device__ __forceinline__ void key_link(uint32_t *par, uint32_t a, uint32_t b) {
    while (a != b) {
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicMin(key_entry(par, b), a);
        if (old >= b) return;
        b = old;
    }
}

// Sweep of one wavefront's bands, top to bottom, as sweep_band does for
// rows: `ra` carries per lane the root key of the interval holding the
// pixel above the band's top row (kNone for background); a band's
// interval takes the smallest root its top row touches (one LDS atomicMin
// per lane on its node), every other touched root is linked under it, and
// the bottom row's pixels hand the interval's root on to the next band.
// The first node of band j is lane j's value of `bbv`; ends[j] holds the
// band's interval ends.  Touching pairs come from pair_masks over the top
// row and the row above; several of them may name the same two intervals.
template <int BPW, bool CONN8>
__device__ __forceinline__ void sweep_bands(uint32_t *par, const uint64_t *msk, const uint64_t *ends,
                                            int wave, int lane, uint32_t bbv) {
    uint32_t ra = kNone;
    uint64_t u = 0;
    uint64_t m[2 * BPW], e[BPW];
#pragma unroll
    for (int k = 0; k < 2 * BPW; ++k) m[k] = uniform64(msk[wave * 2 * BPW + k]);
#pragma unroll
    for (int k = 0; k < BPW; ++k) e[k] = uniform64(ends[wave * BPW + k]);
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
        const int band = wave * BPW + k;
        const uint64_t t = m[2 * k], b = m[2 * k + 1];
        const uint64_t M = t | b, E = e[k];
        const uint64_t S = band_starts<CONN8>(t, b);
        const bool in = lane_in(M);
        const uint32_t rb = (uint32_t)__builtin_amdgcn_readlane((int)bbv, band);
        const uint32_t node = bits_below_plus(E, rb);
        uint32_t *pn = &par[node];
        if (lane_in(S)) {
            // the interval's smallest pixel: its first top-row pixel, else
            // its first pixel (a bottom-row one, at the start column).  Seen
            // from the start column, the first top-row pixel belongs to the
            // interval when it comes no later than the interval's end (the
            // first end at or after the start, so er != 0)
            const uint64_t tr = t >> lane, er = E >> lane;
            const uint32_t dt = tr ? (uint32_t)__builtin_ctzll(tr) : 64u;
            const bool top = dt <= (uint32_t)__builtin_ctzll(er);
            const uint32_t row = (uint32_t)(2 * band) + (top ? 0u : 1u);
            const uint32_t col = (uint32_t)lane + (top ? dt : 0u);
            lds_st(pn, node_key((row << 6) | col, node));
        }
        uint32_t md = kNone;
        if (k > 0) {
            const PairMasks p = pair_masks<CONN8>(t, u);
            // PL never holds lane 0 and PR never lane 63 (no column beyond the tile)
            const uint32_t rL = from_left_any(ra), rR = from_right_any(ra);
            const uint32_t t0 = lane_in(p.pm) ? ra : (lane_in(p.pl) ? rL : kNone);
            const uint32_t t1 = lane_in(p.pr) ? rR : kNone;
            const uint32_t tm = t0 < t1 ? t0 : t1;
            if (tm != kNone) atomicMin(pn, tm);
            if (in) md = lds_ld(pn);
            const bool n0 = t0 != kNone && t0 != md;
            const bool n1 = t1 != kNone && t1 != md;
            if (__ballot(n0 || n1)) {
                uint32_t o0 = 0, o1 = 0;
                if (n0) o0 = atomicMin(key_entry(par, t0), md);
                if (n1) o1 = atomicMin(key_entry(par, t1), md);
                const bool r0 = n0 && o0 < t0 && o0 != md, r1 = n1 && o1 < t1 && o1 != md;
                if (__ballot(r0 || r1)) {
                    if (r0) key_link(par, md, o0);
                    if (r1) key_link(par, md, o1);
                }
                // under 8-connectivity the walk to the current root pays:
                // dense images link many roots per band, and carrying a
                // root that was just linked elsewhere deepens the trees the
                // next bands walk; under 4-connectivity it does not pay
                // (measured), and key_link tolerates a stale root
                if (CONN8) {
                    if (in) md = key_root(par, md);
                    if (lane_in(S)) lds_st(pn, md);
                }
            }
        } else if (in) {
            md = lds_ld(pn);
        }
        ra = lane_in(b) ? md : kNone;
        u = b;
    }
}

// Band seam of a multi-wavefront tile: the top row of band k against the
// bottom row of band k - 1, any forest state.  bk / bu: first node of band
// k / k - 1.
template <bool CONN8>
__device__ __forceinline__ void merge_band_seam(uint32_t *par, const uint64_t *msk, const uint64_t *ends,
                                                int k, uint32_t bk, uint32_t bu) {
    const uint64_t t = uniform64(msk[2 * k]), u = uniform64(msk[2 * k - 1]);
    const uint64_t E = uniform64(ends[k]), Eu = uniform64(ends[k - 1]);
    const uint32_t node = bk + bits_below(E);
    const uint32_t upC = bu + bits_below(Eu);  // interval of the upper cell in this column
    auto join = [&](uint32_t a, uint32_t b) { key_link(par, lds_ld(&par[a]), lds_ld(&par[b])); };
    const PairMasks p = pair_masks<CONN8>(t, u);
    if (CONN8) {
        if (lane_in(p.pl)) join(node, bu + bits_below(Eu << 1));
        else if (lane_in(p.pm)) join(node, upC);
        if (lane_in(p.pr)) join(node, upC + (uint32_t)bit(Eu, (int)(threadIdx.x & 63)));
    } else {
        if (lane_in(p.pm)) join(node, upC);
    }
}

// ------------------------------------------- equal-value labeling (K1 part)
//
// Every in-image pixel takes part and a pixel joins the neighbours whose
// image value equals its own (the kernels' literal test in Sec. II-A, all
// value classes labeled).  Runs are maximal horizontal segments of one
// value, so a row holds up to 64 of them.  `v` is a lane's pixel value, or
// a value no byte can equal for lanes outside the image.

// Sweep of one wavefront's band for equal-value labeling.  Each lane links
// its run to the runs of the equal-valued cells above it (every such lane
// proposes; the LDS atomicMin keeps the smallest root and the rare other
// roots are joined by real unions).  Writes msk[r] = the row's run starts
// and rinfo[r] (runs | 0x100: first run at column 0 | 0x200: last run ends
// at column 63).
template <int TH, int RPW, bool CONN8>
__device__ __forceinline__ void sweep_band_eq(uint32_t *par, uint8_t *col, uint64_t *msk,
                                              uint16_t *rinfo, const uint8_t *pix, int wave,
                                              int lane, int wlim, int hlim) {
    constexpr int SPR = slots_per_row<true>();
    constexpr uint32_t kOut = 0x100u, kOutUp = 0x200u;
    uint32_t ra = kNone, vu = kOutUp;
    uint32_t pv[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) pv[k] = pix[(wave * RPW + k) * kTileW + lane];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wave * RPW + k;
        const bool in = lane < wlim && r < hlim;
        const uint32_t vv = in ? pv[k] : kOut;
        const uint32_t vl = from_left(vv, kOut);
        const uint64_t S = __ballot(in && (lane == 0 || vv != vl));
        const bool isS = lane_in(S);
        const uint32_t node = (uint32_t)(r * SPR) + bits_below(S) - (isS ? 0u : 1u);
        uint32_t *pn = &par[node];
        if (isS) {
            lds_st(pn, node);
            col[node] = (uint8_t)lane;
        }
        if (lane == 0) {
            msk[r] = S;
            rinfo[r] = (uint16_t)(__popcll(S) | ((S & 1ull) ? 0x100 : 0) | (wlim == 64 ? 0x200 : 0));
        }
        uint32_t md = in ? node : kNone;
        if (k > 0) {
            const uint32_t tM = in && vv == vu ? ra : kNone;
            uint32_t tL = kNone, tR = kNone;
            if (CONN8) {
                const uint32_t vuL = from_left(vu, kOutUp), vuR = from_right(vu, kOutUp);
                const uint32_t rL = from_left(ra, kNone), rR = from_right(ra, kNone);
                tL = in && vv == vuL ? rL : kNone;
                tR = in && vv == vuR ? rR : kNone;
            }
            const uint32_t tm = tM < tL ? (tM < tR ? tM : tR) : (tL < tR ? tL : tR);
            if (tm != kNone) atomicMin(pn, tm);
            if (in) md = lds_ld(pn);
            const bool nM = tM != kNone && tM != md;
            const bool nL = tL != kNone && tL != md;
            const bool nR = tR != kNone && tR != md;
            if (__ballot(nM || nL || nR)) {
                // as in the binary sweep: one atomicMin per link, a general
                // join only where the root was already linked elsewhere (a
                // lane that finds md there met a duplicate of its own link)
                uint32_t oM = 0, oL = 0, oR = 0;
                if (nM) oM = atomicMin(&par[tM], md);
                if (nL) oL = atomicMin(&par[tL], md);
                if (nR) oR = atomicMin(&par[tR], md);
                const bool rM = nM && oM < tM && oM != md;
                const bool rL = nL && oL < tL && oL != md;
                const bool rR = nR && oR < tR && oR != md;
                if (__ballot(rM || rL || rR)) {
                    if (rM) lds_link(par, md, oM);
                    if (rL) lds_link(par, md, oL);
                    if (rR) lds_link(par, md, oR);
                }
                if (in) md = lds_root(par, md);
                if (isS) lds_st(pn, md);
            }
        }
        ra = md;
        vu = in ? vv : kOutUp;
    }
}

// Band seam for equal-value labeling: the first row r of a band against the
// last row of the band above (run starts already in msk), any forest state.
template <bool CONN8>
__device__ __forceinline__ void merge_seam_eq(uint32_t *par, const uint64_t *msk, const uint8_t *pix,
                                              int r, int lane, int wlim, int hlim) {
    constexpr int SPR = slots_per_row<true>();
    constexpr uint32_t kOut = 0x100u, kOutUp = 0x200u;
    if (r >= hlim) return;  // wave-uniform: the whole band lies below the image
    const bool in = lane < wlim;
    const uint32_t vv = in ? pix[r * kTileW + lane] : kOut;
    const uint32_t vu = in ? pix[(r - 1) * kTileW + lane] : kOutUp;
    const uint64_t S = uniform64(msk[r]), Su = uniform64(msk[r - 1]);
    const uint32_t node = (uint32_t)(r * SPR) + bits_below(S) - (lane_in(S) ? 0u : 1u);
    const uint32_t up = (uint32_t)((r - 1) * SPR) + bits_below(Su) - (lane_in(Su) ? 0u : 1u);
    if (in && vv == vu) lds_link(par, node, up);
    if (CONN8) {
        const uint32_t vuL = from_left(vu, kOutUp), vuR = from_right(vu, kOutUp);
        const uint32_t upL = from_left(up, kNone), upR = from_right(up, kNone);
        if (in && vv == vuL) lds_link(par, node, upL);
        if (in && vv == vuR) lds_link(par, node, upR);
    }
}

}  // namespace ccl
