// Row-parallel tiles: the data layout shared by the three kernels of the
// row-parallel path and by the host code that sizes and launches them.
//
// A tile is 64 columns wide and TH = 64 * R rows tall.  The local merge runs
// one 64-lane wavefront per tile and gives each lane R consecutive rows, each
// row held as one 64-bit foreground mask, so the bit tricks that find runs
// and the pairs of touching runs (Sec. II-A-2) act on a whole row at once.
// Union-find nodes are runs, numbered densely in raster order of their
// starts; a parent entry packs the parent's node number above its tile-local
// pixel position (row * 64 + column), so comparing entries compares node
// numbers, which is raster order, and the root of every tree is the run
// holding the smallest pixel of the tree (the linking rule of Sec. II-A-3).
//
// Only the local roots of components that touch a shared tile edge
// ("flagged" roots) enter the global union-find of the boundary analysis
// (Sec. II-B).  They live in a compact forest: tile g has FMAX slots, and
// slot g * FMAX + f holds, for the f-th flagged root of the tile in raster
// order, the 64-bit entry (global pixel index of its parent << 32 | the
// parent's slot).  A root holds its own pixel and slot, so an atomicMin on
// an entry links by pixel index and the root of every global tree is the
// smallest pixel of the component.  The link (Sec. II-C) resolves each
// flagged root once in that forest; every other label is arithmetic.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace ccl {
namespace rp {

constexpr int kPB = 14;                         // bits of the packed pixel position
constexpr uint32_t kPosMask = (1u << kPB) - 1u;
constexpr uint16_t kFlagged = 0x8000u;          // record: flagged root, low bits = flag index

// Flagged roots per tile, at most: every run of the top and bottom rows
// (32 each) and every row of the left and right columns.
__host__ __device__ constexpr int fmax_tile(int th) { return 64 + 2 * th; }
// Edge masks per tile: top row, bottom row, then the left column and the
// right column as th / 64 words each (bit k of word w = row 64 w + k).
__host__ __device__ constexpr int emask_words(int th) { return 2 + 2 * (th / 64); }
__host__ __device__ constexpr int em_left(int) { return 2; }
__host__ __device__ constexpr int em_right(int th) { return 2 + th / 64; }
// Edge-cell roots per tile (forest slots): top row, bottom row, left
// column, right column.
__host__ __device__ constexpr int eroot_words(int th) { return 128 + 2 * th; }
__host__ __device__ constexpr int er_top(int) { return 0; }
__host__ __device__ constexpr int er_bottom(int) { return 64; }
__host__ __device__ constexpr int er_left(int) { return 128; }
__host__ __device__ constexpr int er_right(int th) { return 128 + th; }
// Run records per tile (a 64-pixel row holds at most 32 runs).
__host__ __device__ constexpr int nodes_tile(int th) { return th * 32; }

// Per-tile workspace arrays (all indexed by the tile number t of the view).
struct RpWs {
    uint64_t *emask;   // [t][emask_words]
    uint32_t *eroot;   // [t][eroot_words]: forest slot of the root of every edge cell
    uint64_t *rows;    // [t][th]: foreground mask of every row
    uint16_t *rbase;   // [t][th]: first run record of every row
    uint32_t *nflag;   // [t]: number of flagged roots
    uint16_t *rec;     // [t][nodes]: per run, its root's tile-local pixel, or kFlagged | flag index
};

// Workspace layout of one image (or of the tiles of a batch).
struct RpLayout {
    size_t tiles;
    size_t off_emask, off_eroot, off_rows, off_rbase, off_nflag, off_rec, off_forest;
    size_t total;
};

inline size_t rp_align(size_t v) { return (v + 255) / 256 * 256; }

inline RpLayout rp_layout(size_t tiles, int th) {
    RpLayout l;
    l.tiles = tiles;
    size_t o = 0;
    l.off_emask = o;
    o += rp_align(tiles * (size_t)emask_words(th) * 8);
    l.off_eroot = o;
    o += rp_align(tiles * (size_t)eroot_words(th) * 4);
    l.off_rows = o;
    o += rp_align(tiles * (size_t)th * 8);
    l.off_rbase = o;
    o += rp_align(tiles * (size_t)th * 2);
    l.off_nflag = o;
    o += rp_align(tiles * 4);
    l.off_rec = o;
    o += rp_align(tiles * (size_t)nodes_tile(th) * 2);
    l.off_forest = o;
    o += rp_align(tiles * (size_t)fmax_tile(th) * 8);
    l.total = o;
    return l;
}

inline RpWs rp_ws(void *base, const RpLayout &l) {
    char *b = (char *)base;
    RpWs w;
    w.emask = (uint64_t *)(b + l.off_emask);
    w.eroot = (uint32_t *)(b + l.off_eroot);
    w.rows = (uint64_t *)(b + l.off_rows);
    w.rbase = (uint16_t *)(b + l.off_rbase);
    w.nflag = (uint32_t *)(b + l.off_nflag);
    w.rec = (uint16_t *)(b + l.off_rec);
    return w;
}

// One image as the row-parallel kernels see it.  The per-tile arrays of `w`
// start at the image's tile 0; `forest` is the base of the whole forest and
// `gtile0` the global number of the image's tile 0 (slots are global).
struct RpView {
    const uint8_t *img;
    uint32_t *labels;
    RpWs w;
    uint64_t *forest;
    int64_t pitch;
    int32_t H, W;
    int32_t tilesX, tilesY;
    uint32_t n;
    int32_t aligned16;
    uint32_t gtile0;
};

}  // namespace rp
}  // namespace ccl
