// 3D volume labeling (the paper's method on a 3D grid): the same three
// phases over 3D tiles of 64 (x) x 16 (y) x 4 (z) voxels.
//
//   local merge   one wavefront per slice of the tile sweeps its 16 rows
//                 with the 2D run union-find (4-connectivity inside a slice
//                 for 6-connectivity, 8 for 18 and 26); every run then takes
//                 its slice root, and every row is joined with the rows of
//                 the previous slice it touches (pair masks, one LDS
//                 atomicMin per pair of roots; the four wavefronts share
//                 these joins by rows).  Every foreground
//                 voxel gets labels[p] = 1 + its tile-local root (a dense
//                 store, as in the paper's Kernel 1), which is already a
//                 valid forest.
//   boundary      every voxel on a tile face proposes its raster-earlier
//                 neighbours that lie in another tile (each such pair is
//                 proposed by its later voxel, once); requests are
//                 deduplicated along a face and merged with the global
//                 union-find of the 2D path.
//   link          every voxel is resolved to its root and stores its final
//                 label.
#include <hip/hip_runtime.h>

#include "ccl.h"
#include "ccl_device.h"
#include "ccl_internal.h"

namespace ccl {

namespace {

constexpr int kTY = 16, kTZ = 4, kRows = kTY * kTZ;  // 64 tile rows

struct Vol {
    const uint8_t *vol;
    uint32_t *labels;
    int64_t pitch_y, pitch_z;
    int32_t D, H, W;
    int32_t tilesX, tilesY, tilesZ;
    uint32_t n;
    int32_t aligned16;
};

__device__ __forceinline__ uint4 load_chunk3d(const Vol &v, int x0, int y, int z, int q) {
    uint4 b = make_uint4(0u, 0u, 0u, 0u);
    if (y >= v.H || z >= v.D) return b;
    const int x = x0 + q * 16;
    const uint8_t *p = v.vol + (int64_t)z * v.pitch_z + (int64_t)y * v.pitch_y + x;
    if (v.aligned16 && x + 16 <= v.W) return *(const uint4 *)p;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (x + i < v.W) w[i >> 2] |= (uint32_t)p[i] << (8 * (i & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ void tile_of(const Vol &v, uint32_t t, int &tx, int &ty, int &tz) {
    const uint32_t TX = (uint32_t)v.tilesX, TY = (uint32_t)v.tilesY;
    tx = (int)(t % TX);
    ty = (int)((t / TX) % TY);
    tz = (int)(t / (TX * TY));
}

// Every run node's parent becomes its root (read-only walk; the owner alone
// stores).  Nodes: 32 slots per tile row, the row's runs first.
__device__ __forceinline__ void compress_nodes(uint32_t *par, const uint64_t *msk, int tid) {
    for (int n = tid; n < kRows * kSlotsPerRow; n += 256) {
        if ((n % kSlotsPerRow) >= __popcll(run_starts(msk[n / kSlotsPerRow]))) continue;
        const uint32_t root = lds_root(par, (uint32_t)n);
        if (root != (uint32_t)n) lds_st(&par[n], root);
    }
}

// Nodes of the runs of tile row ru that this lane's cell (row mask d) pairs
// with, at most two (kNone: none): each pair of touching runs is taken by
// one lane only (pair_masks).  Nodes: 32 slots per row.
template <bool CONN8>
__device__ __forceinline__ void upper_runs(uint64_t d, const uint64_t *msk, int ru, uint32_t &q0,
                                           uint32_t &q1) {
    const uint64_t u = uniform64(msk[ru]);
    const uint64_t Su = run_starts(u);
    const uint32_t up = (uint32_t)(ru * kSlotsPerRow) + bits_below(Su);
    const PairMasks p = pair_masks<CONN8>(d, u);
    if (CONN8) {
        // PL: upper run containing j-1; PM / PR: upper run starting at j / j+1
        q0 = lane_in(p.pl) ? up - 1u : (lane_in(p.pm) ? up : kNone);
        q1 = lane_in(p.pr) ? up : kNone;
    } else {
        q0 = lane_in(p.pm) ? up - (lane_in(Su) ? 0u : 1u) : kNone;
        q1 = kNone;
    }
}

template <int CONN>
__global__ void __launch_bounds__(256) k1_local_merge3d(Vol v) {
    constexpr bool CONN8 = CONN != 6;  // neighbours inside a slice
    __shared__ uint32_t par[kRows * kSlotsPerRow];
    __shared__ uint16_t cr[kRows * kSlotsPerRow];
    __shared__ uint64_t msk[kRows];
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int tx, ty, tz;
    tile_of(v, xcd_remap(blockIdx.x, gridDim.x), tx, ty, tz);
    const int x0 = tx * kTileW, y0 = ty * kTY, z0 = tz * kTZ;
    {
        const int r = tid >> 2, q = tid & 3;  // 64 rows x 4 chunks, one per thread
        ((uint16_t *)msk)[tid] =
            (uint16_t)nonzero_bytes16(load_chunk3d(v, x0, y0 + (r % kTY), z0 + r / kTY, q));
    }
    __syncthreads();
    // wavefront w sweeps slice w (rows w*16 .. w*16+15)
    sweep_band<kRows, kTY, CONN8>(par, cr, msk, wave, lane, (uint32_t)(lane * kSlotsPerRow));
    __syncthreads();
    // every run node takes its slice root (read-only walk, owner store), so
    // the slice merges below start from roots
    compress_nodes(par, msk, tid);
    __syncthreads();
    {
        // rows of slice z against the rows of slice z-1 they touch: the
        // straight row (with diagonals unless 6-connectivity) and, for 18 /
        // 26, the rows above and below it (straight / with diagonals).  The
        // roots of all upper runs a lane touches are read together and
        // joined with its own run's root by one atomicMin each; only a join
        // whose root was linked elsewhere meanwhile continues as a walk.
        // Wavefront w takes rows 4w .. 4w+3 of every slice pair, so all
        // four share the joins.
        constexpr int NQ = CONN == 6 ? 1 : 6;
        constexpr int RJ = kTY / 4;
        for (int j = 0; j < (kTZ - 1) * RJ; ++j) {
            const int sz = 1 + j / RJ, yi = wave * RJ + j % RJ;
            const int r = sz * kTY + yi, ru = (sz - 1) * kTY + yi;
            const uint64_t d = uniform64(msk[r]);
            const uint64_t S = run_starts(d);
            const bool fg = lane_in(d);
            const uint32_t node = (uint32_t)(r * kSlotsPerRow) + bits_below(S) - (lane_in(S) ? 0u : 1u);
            uint32_t q[NQ];
            if (CONN == 6) {
                uint32_t none;
                upper_runs<false>(d, msk, ru, q[0], none);
            } else {
                upper_runs<true>(d, msk, ru, q[0], q[1]);
                q[2] = q[3] = q[4] = q[5] = kNone;
                if (yi > 0) upper_runs<CONN == 26>(d, msk, ru - 1, q[2], q[3]);
                if (yi + 1 < kTY) upper_runs<CONN == 26>(d, msk, ru + 1, q[4], q[5]);
            }
            bool want = false;
#pragma unroll
            for (int i = 0; i < NQ; ++i) want = want || q[i] != kNone;
            if (__ballot(fg && want)) {
                const uint32_t a = fg ? lds_ld(&par[node]) : kNone;
                uint32_t lo[NQ], o[NQ];
                bool again[NQ];
#pragma unroll
                for (int i = 0; i < NQ; ++i) {
                    const uint32_t b = q[i] != kNone ? lds_ld(&par[q[i]]) : kNone;
                    const bool go = fg && b != kNone && b != a;
                    lo[i] = a < b ? a : b;
                    const uint32_t hi = a < b ? b : a;
                    o[i] = go ? atomicMin(&par[hi], lo[i]) : hi;
                    again[i] = go && o[i] < hi && o[i] != lo[i];
                }
                bool any = false;
#pragma unroll
                for (int i = 0; i < NQ; ++i) any = any || again[i];
                if (__ballot(any)) {
#pragma unroll
                    for (int i = 0; i < NQ; ++i)
                        if (again[i]) lds_link(par, lo[i], o[i]);
                }
            }
        }
    }
    __syncthreads();
    compress_nodes(par, msk, tid);
    __syncthreads();
    // dense store: 1 + the global index of every foreground voxel's local root
    const int x = x0 + lane;
    for (int k = 0; k < kTY; ++k) {
        const int r = wave * kTY + k;
        const int y = y0 + k, z = z0 + wave;
        if (y >= v.H || z >= v.D) break;  // wave-uniform
        const uint64_t d = uniform64(msk[r]);
        if (x >= v.W) continue;
        uint32_t out = 0u;
        if (lane_in(d)) {
            const uint64_t S = run_starts(d);
            const uint32_t node = (uint32_t)(r * kSlotsPerRow) + bits_below(S) - (lane_in(S) ? 0u : 1u);
            const uint32_t c = cr[lds_ld(&par[node])];
            const uint32_t rr = c >> 8;
            const uint64_t g = ((uint64_t)(z0 + rr / kTY) * v.H + (uint64_t)(y0 + rr % kTY)) * v.W +
                               (uint64_t)(x0 + (c & 0xFFu));
            out = (uint32_t)g + 1u;
        }
        v.labels[((uint64_t)z * v.H + y) * v.W + x] = out;
    }
}

// Raster-earlier neighbour offsets (dz, dy, dx) for 26-connectivity; the
// first `count` of them for each connectivity.
struct Off { int8_t dz, dy, dx, steps; };
__constant__ Off kBack[13] = {
    {0, 0, -1, 1}, {0, -1, 0, 1}, {-1, 0, 0, 1},                                     // faces
    {0, -1, -1, 2}, {0, -1, 1, 2}, {-1, 0, -1, 2}, {-1, 0, 1, 2}, {-1, -1, 0, 2},
    {-1, 1, 0, 2},                                                                   // edges
    {-1, -1, -1, 3}, {-1, -1, 1, 3}, {-1, 1, -1, 3}, {-1, 1, 1, 3}};                 // corners

// Boundary analysis of tile t.  A pair of neighbours in different tiles is
// proposed by its raster-later voxel p.  The candidates are split so that
// every pair is seen once and requests along a face are deduplicated across
// a whole wavefront:
//   x-lines (lane = column): the 22 tile rows on the front face (first
//     slice) or on the top / bottom row of a slice, for the neighbours that
//     leave the tile through y or z;
//   x-faces (lane = tile row): the first and the last column of the tile,
//     for the neighbours that leave it through x only.
template <int CONN>
__global__ void __launch_bounds__(256) k2_boundary3d(Vol v) {
    constexpr int NOFF = CONN == 6 ? 3 : (CONN == 18 ? 9 : 13);
    constexpr int kLines = kTY + 2 * (kTZ - 1);  // 22 x-lines per tile
    int tx, ty, tz;
    tile_of(v, xcd_remap(blockIdx.x, gridDim.x), tx, ty, tz);
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int x0 = tx * kTileW, y0 = ty * kTY, z0 = tz * kTZ;
    const uint32_t *L = v.labels;
    const uint64_t HW = (uint64_t)v.H * v.W;
    auto at = [&](int z, int y, int x) { return L[(uint64_t)z * HW + (uint64_t)y * v.W + (uint64_t)x]; };
    for (int task = wave; task < kLines + 2; task += 4) {
        int z, y, x;
        bool xface;
        if (task < kLines) {
            // rows 0..15: the first slice; then the top and bottom rows of slices 1..3
            const int r = task < kTY ? task : (task - kTY) / 2 * kTY + kTY + ((task - kTY) & 1) * (kTY - 1);
            z = z0 + r / kTY;
            y = y0 + r % kTY;
            x = x0 + lane;
            xface = false;
        } else {
            z = z0 + lane / kTY;
            y = y0 + lane % kTY;
            x = task == kLines ? x0 : x0 + kTileW - 1;
            xface = true;
        }
        const bool in = z < v.D && y < v.H && x < v.W;
        const uint32_t lp = in ? at(z, y, x) : 0u;
        // every neighbour's label first (the loads overlap), then all the
        // task's merge requests together
        uint32_t A[NOFF], B[NOFF];
#pragma unroll
        for (int o = 0; o < NOFF; ++o) {
            const Off d = kBack[o];
            const bool dirOk = !xface || d.dx == (task == kLines ? -1 : 1);  // wave-uniform
            const int qz = z + d.dz, qy = y + d.dy, qx = x + d.dx;
            const bool outYZ = qz < z0 || qy < y0 || qy >= y0 + kTY;
            const bool outX = qx < x0 || qx >= x0 + kTileW;
            const bool mine = xface ? (outX && !outYZ) : outYZ;
            const bool valid = dirOk && lp != 0u && mine && qz >= 0 && qy >= 0 && qy < v.H && qx >= 0 &&
                               qx < v.W;
            const uint32_t lq = valid ? at(qz, qy, qx) : 0u;
            A[o] = lp - 1u;
            B[o] = lq != 0u ? lq - 1u : kNone;
        }
        union_requests<NOFF>(A, B, [&](uint32_t a, uint32_t b) { g_union(v.labels, v.n, a, b); });
    }
}

__global__ void __launch_bounds__(256) k3_link3d(uint32_t *L, uint32_t n) {
    const uint64_t p = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (p >= n) return;
    const uint32_t lp = L[p];
    if (lp == 0u) return;
    // the voxel's root (long walks also repoint the nodes they pass), then
    // its final label as a streaming store: the output is not read again
    // beyond the other voxels' walks, for which any ancestor will do
    const uint32_t r = g_root(L, lp - 1u);
    if (r + 1u != lp) __builtin_nontemporal_store(r + 1u, &L[p]);
}

}  // namespace

}  // namespace ccl

using namespace ccl;

extern "C" int ccl_label_3d(const uint8_t *vol, int32_t D, int32_t H, int32_t W, int64_t pitch_y,
                            int64_t pitch_z, int32_t connectivity, uint32_t *labels, void *stream) {
    if (!vol || !labels || D <= 0 || H <= 0 || W <= 0) return CCL_ERR_INVALID_ARG;
    if (pitch_y < (int64_t)W || pitch_z < (int64_t)H * pitch_y) return CCL_ERR_INVALID_ARG;
    if (connectivity != 6 && connectivity != 18 && connectivity != 26) return CCL_ERR_UNSUPPORTED;
    const uint64_t n = (uint64_t)D * (uint64_t)H * (uint64_t)W;
    if (n > 0xFFFFFFFFull) return CCL_ERR_TOO_LARGE;
    const unsigned __int128 vol_bytes = (unsigned __int128)(D - 1) * (uint64_t)pitch_z +
                                        (unsigned __int128)(H - 1) * (uint64_t)pitch_y + (uint64_t)W;
    if (byte_ranges_overlap(vol, vol_bytes, labels, (unsigned __int128)n * 4u)) return CCL_ERR_INVALID_ARG;
    Vol v;
    v.vol = vol;
    v.labels = labels;
    v.pitch_y = pitch_y;
    v.pitch_z = pitch_z;
    v.D = D;
    v.H = H;
    v.W = W;
    v.tilesX = (W + kTileW - 1) / kTileW;
    v.tilesY = (H + kTY - 1) / kTY;
    v.tilesZ = (D + kTZ - 1) / kTZ;
    v.n = (uint32_t)n;
    v.aligned16 = (((uintptr_t)vol & 15u) == 0 && (pitch_y & 15) == 0 && (pitch_z & 15) == 0) ? 1 : 0;
    const uint64_t tiles = (uint64_t)v.tilesX * v.tilesY * v.tilesZ;
    if (tiles * kRows > 0x7FFFFFFFull) return CCL_ERR_TOO_LARGE;
    hipStream_t s = (hipStream_t)stream;
    switch (connectivity) {
        case 6:
            hipLaunchKernelGGL(k1_local_merge3d<6>, dim3((uint32_t)tiles), dim3(256), 0, s, v);
            hipLaunchKernelGGL(k2_boundary3d<6>, dim3((uint32_t)tiles), dim3(256), 0, s, v);
            break;
        case 18:
            hipLaunchKernelGGL(k1_local_merge3d<18>, dim3((uint32_t)tiles), dim3(256), 0, s, v);
            hipLaunchKernelGGL(k2_boundary3d<18>, dim3((uint32_t)tiles), dim3(256), 0, s, v);
            break;
        default:
            hipLaunchKernelGGL(k1_local_merge3d<26>, dim3((uint32_t)tiles), dim3(256), 0, s, v);
            hipLaunchKernelGGL(k2_boundary3d<26>, dim3((uint32_t)tiles), dim3(256), 0, s, v);
            break;
    }
    hipLaunchKernelGGL(k3_link3d, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, labels,
                       (uint32_t)n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e);
    return CCL_OK;
}
