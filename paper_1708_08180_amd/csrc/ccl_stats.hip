// Per-component statistics of a canonical labeling: area, inclusive
// bounding box and the sums of the pixels' column and row indices (the
// size and location of every component, which is what the applications in
// the paper's introduction use the labels for).
//
// A component's root is the pixel whose label is its own raster index + 1.
// Roots are numbered in raster order, so records come out in increasing
// label order:
//   st_roots     one 64-bit root mask per 64-pixel row word (lane = pixel)
//                and the number of roots per block of 64 words;
//   st_scan      exclusive scan of the block counts (one workgroup), total;
//   st_bases     exclusive scan inside each block: the first record index
//                of every word, and the records of its roots initialised;
//   st_accum     every run of equal labels in a row adds its length,
//                extent and coordinate sums to its component's record: first
//                into a hash table in LDS keyed by label per 64 x 256 block
//                (a large component has thousands of runs, which would
//                otherwise all hit one record), then once per table slot
//                with global atomics.
#include <hip/hip_runtime.h>

#include "ccl.h"
#include "ccl_device.h"
#include "ccl_internal.h"

namespace ccl {

namespace {

constexpr int kWordsPerBlock = 64;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

__global__ void __launch_bounds__(256) st_roots(const uint32_t *L, uint32_t W, uint32_t WW,
                                                 uint32_t words, uint64_t *mask, uint32_t *bsum) {
    __shared__ uint32_t part[4];
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    uint32_t cnt = 0;
    for (int i = 0; i < kWordsPerBlock / 4; ++i) {
        const uint32_t w = blockIdx.x * kWordsPerBlock + (uint32_t)(wave * (kWordsPerBlock / 4) + i);
        if (w >= words) break;  // wave-uniform
        const uint32_t y = w / WW, x = (w % WW) * (uint32_t)kTileW + (uint32_t)lane;
        bool root = false;
        if (x < W) {
            const uint32_t p = y * W + x;
            root = L[p] == p + 1u;
        }
        const uint64_t m = __ballot(root);
        if (lane == 0) mask[w] = m;
        cnt += (uint32_t)__popcll(m);
    }
    if (lane == 0) part[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ void __launch_bounds__(1024) st_scan(uint32_t *bsum, uint32_t nb, uint32_t *n_out) {
    __shared__ uint32_t s[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (nb + 1023u) / 1024u;
    const uint32_t b0 = tid * per, b1 = min(nb, b0 + per);
    uint32_t acc = 0;
    for (uint32_t b = b0; b < b1; ++b) acc += bsum[b];
    s[tid] = acc;
    __syncthreads();
    for (uint32_t off = 1; off < 1024u; off <<= 1) {
        const uint32_t v = tid >= off ? s[tid - off] : 0u;
        __syncthreads();
        s[tid] += v;
        __syncthreads();
    }
    uint32_t run = s[tid] - acc;
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t t = bsum[b];
        bsum[b] = run;
        run += t;
    }
    if (tid == 1023u) *n_out = s[1023];
}

__global__ void __launch_bounds__(64) st_bases(const uint64_t *mask, const uint32_t *bsum,
                                                uint32_t words, uint32_t W, uint32_t WW,
                                                uint32_t *base, ccl_component *out, uint32_t cap) {
    const int lane = (int)(threadIdx.x & 63);
    const uint32_t w = blockIdx.x * kWordsPerBlock + (uint32_t)lane;
    const uint64_t m = w < words ? mask[w] : 0ull;
    const uint32_t c = (uint32_t)__popcll(m);
    uint32_t x = c;  // inclusive scan over the 64 words of the block
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)x, off, 64);
        if (lane >= off) x += t;
    }
    if (w >= words) return;
    const uint32_t b = bsum[blockIdx.x] + x - c;
    base[w] = b;
    const uint32_t p0 = (w / WW) * W + (w % WW) * (uint32_t)kTileW;
    uint64_t mm = m;
    uint32_t id = b;
    while (mm) {
        const uint32_t j = (uint32_t)__builtin_ctzll(mm);
        mm &= mm - 1ull;
        if (id < cap) {
            ccl_component &r = out[id];
            r.label = p0 + j + 1u;
            r.area = 0u;
            r.x_min = 0xFFFFFFFFu;
            r.y_min = 0xFFFFFFFFu;
            r.x_max = 0u;
            r.y_max = 0u;
            r.sum_x = 0ull;
            r.sum_y = 0ull;
        }
        ++id;
    }
}

__device__ __forceinline__ void add_global(ccl_component &r, uint32_t len, uint32_t xmn, uint32_t xmx,
                                           uint32_t ymn, uint32_t ymx, uint64_t sxv, uint64_t syv) {
    atomicAdd(&r.area, len);
    atomicMin(&r.x_min, xmn);
    atomicMax(&r.x_max, xmx);
    atomicMin(&r.y_min, ymn);
    atomicMax(&r.y_max, ymx);
    atomicAdd((unsigned long long *)&r.sum_x, (unsigned long long)sxv);
    atomicAdd((unsigned long long *)&r.sum_y, (unsigned long long)syv);
}

// Reductions over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
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

// Record index of the component whose root pixel is r (its label - 1).
__device__ __forceinline__ uint32_t record_of(uint32_t r, uint32_t W, uint32_t WW,
                                              const uint64_t *mask, const uint32_t *base) {
    const uint32_t rx = r % W;
    const uint32_t w = (r / W) * WW + rx / (uint32_t)kTileW;
    return base[w] + (uint32_t)__popcll(mask[w] & ((1ull << (rx & 63u)) - 1ull));
}

// Block of 64 columns x kAccRows rows, 16 wavefronts of 16 rows each.  The
// hash table is keyed by label, so a run needs no global read; the record
// index is looked up once per table slot when the block flushes.
constexpr int kAccWaves = 16, kAccRowsPerWave = 16, kAccRows = kAccWaves * kAccRowsPerWave;
constexpr int kAccSlots = 1024;

__global__ void __launch_bounds__(kAccWaves * 64) st_accum(const uint32_t *L, uint32_t H, uint32_t W,
                                                          uint32_t WW, const uint64_t *mask,
                                                          const uint32_t *base, ccl_component *out,
                                                          uint32_t cap) {
    __shared__ uint32_t key[kAccSlots], area[kAccSlots], xmn[kAccSlots], ymn[kAccSlots],
        xmx[kAccSlots], ymx[kAccSlots];
    __shared__ unsigned long long sx[kAccSlots], sy[kAccSlots];
    constexpr int NT = kAccWaves * 64;
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < kAccSlots; i += NT) {
        key[i] = kEmpty;
        area[i] = 0u;
        xmn[i] = ymn[i] = 0xFFFFFFFFu;
        xmx[i] = ymx[i] = 0u;
        sx[i] = sy[i] = 0ull;
    }
    __syncthreads();
    const uint32_t x0 = blockIdx.x * (uint32_t)kTileW, y0 = blockIdx.y * (uint32_t)kAccRows;
    const uint32_t n = H * W;
    const uint32_t x = x0 + (uint32_t)lane;
    const bool xin = x < W;
    // Adds one run (or a wave's partial record) to the LDS table.
    auto add_lds = [&](uint32_t l, uint32_t len, uint32_t xa, uint32_t xb, uint32_t ya, uint32_t yb,
                       uint64_t sxv, uint64_t syv) {
        uint32_t h = (l * 2654435761u) >> 22;  // 10 bits
        for (int probe = 0; probe < 16; ++probe) {
            const uint32_t kk = atomicCAS(&key[h], kEmpty, l);
            if (kk == kEmpty || kk == l) {
                atomicAdd(&area[h], len);
                atomicMin(&xmn[h], xa);
                atomicMax(&xmx[h], xb);
                atomicMin(&ymn[h], ya);
                atomicMax(&ymx[h], yb);
                atomicAdd(&sx[h], (unsigned long long)sxv);
                atomicAdd(&sy[h], (unsigned long long)syv);
                return;
            }
            h = (h + 1u) & (uint32_t)(kAccSlots - 1);
        }
        // table full around h: straight to the record
        const uint32_t id = record_of(l - 1u, W, WW, mask, base);
        if (id < cap) add_global(out[id], len, xa, xb, ya, yb, sxv, syv);
    };
    // A large component has runs in most rows, which would all meet on one
    // table slot: the runs of the wavefront's "hot" label (the smallest
    // label starting a run in its first row with one, which is a large
    // component's in noise) add into per-lane registers instead, reduced
    // over the wavefront once at the end.
    uint32_t hot = kEmpty;
    uint32_t hA = 0u, hXa = 0xFFFFFFFFu, hXb = 0u, hYa = 0xFFFFFFFFu, hYb = 0u;
    uint64_t hSx = 0ull, hSy = 0ull;
    // all the wavefront's rows are loaded first, so the loads overlap
    uint32_t lv[kAccRowsPerWave];
#pragma unroll
    for (int k = 0; k < kAccRowsPerWave; ++k) {
        const uint32_t y = y0 + (uint32_t)(wave * kAccRowsPerWave + k);
        lv[k] = xin && y < H ? L[y * W + x] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kAccRowsPerWave; ++k) {
        const uint32_t y = y0 + (uint32_t)(wave * kAccRowsPerWave + k);
        if (y >= H) break;  // wave-uniform
        const uint32_t l = lv[k];
        const uint32_t ll = from_left(l, 0u), lr = from_right(l, 0u);
        const bool start = l != 0u && l != ll && l <= n;  // (labels above H*W: not canonical)
        const uint64_t S = __ballot(start);
        const uint64_t E = __ballot(l != 0u && l != lr);
        if (hot == kEmpty && S) hot = wave_min_u32(start ? l : kEmpty);  // wave-uniform
        if (!start) continue;
        // this lane starts a run of equal labels; it ends at the first run
        // end at or after it
        const uint32_t e = (uint32_t)lane + (uint32_t)__builtin_ctzll(E >> lane);
        const uint32_t len = e - (uint32_t)lane + 1u, x1 = x0 + e;
        const uint64_t sxv = (uint64_t)len * ((uint64_t)x + (uint64_t)x1) / 2u;
        const uint64_t syv = (uint64_t)len * (uint64_t)y;
        if (l == hot) {
            hA += len;
            hXa = min(hXa, x);
            hXb = max(hXb, x1);
            hYa = min(hYa, y);
            hYb = max(hYb, y);
            hSx += sxv;
            hSy += syv;
        } else {
            add_lds(l, len, x, x1, y, y, sxv, syv);
        }
    }
    if (hot != kEmpty) {  // wave-uniform
        hA = wave_sum_u32(hA);
        hXa = wave_min_u32(hXa);
        hXb = wave_max_u32(hXb);
        hYa = wave_min_u32(hYa);
        hYb = wave_max_u32(hYb);
        hSx = wave_sum_u64(hSx);
        hSy = wave_sum_u64(hSy);
        if (lane == 0 && hA != 0u) add_lds(hot, hA, hXa, hXb, hYa, hYb, hSx, hSy);
    }
    __syncthreads();
    for (int i = tid; i < kAccSlots; i += NT) {
        const uint32_t l = key[i];
        if (l == kEmpty) continue;
        const uint32_t id = record_of(l - 1u, W, WW, mask, base);
        if (id < cap) add_global(out[id], area[i], xmn[i], xmx[i], ymn[i], ymx[i], sx[i], sy[i]);
    }
}

}  // namespace

size_t stats_workspace_bytes(int32_t H, int32_t W) {
    const size_t WW = ((size_t)W + kTileW - 1) / kTileW;
    const size_t words = (size_t)H * WW;
    const size_t nb = (words + kWordsPerBlock - 1) / kWordsPerBlock;
    return align_up(words * sizeof(uint64_t), 256) + align_up(words * sizeof(uint32_t), 256) +
           align_up(nb * sizeof(uint32_t), 256);
}

}  // namespace ccl

using namespace ccl;

extern "C" int ccl_component_stats(const uint32_t *labels, int32_t H, int32_t W,
                                   ccl_component *out, int64_t capacity, uint32_t *n_out,
                                   void *stream) {
    if (!labels || !n_out || H <= 0 || W <= 0 || capacity < 0 || (capacity > 0 && !out))
        return CCL_ERR_INVALID_ARG;
    if ((uint64_t)H * (uint64_t)W > 0xFFFFFFFFull) return CCL_ERR_TOO_LARGE;
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    std::unique_lock<std::mutex> held;
    int rc = stream_workspace(s, stats_workspace_bytes(H, W), &ws, &held);
    if (rc != CCL_OK) return rc;
    const uint32_t WW = (uint32_t)((W + kTileW - 1) / kTileW);
    const uint32_t words = (uint32_t)H * WW;
    const uint32_t nb = (words + kWordsPerBlock - 1) / kWordsPerBlock;
    char *p = (char *)ws;
    uint64_t *mask = (uint64_t *)p;
    uint32_t *base = (uint32_t *)(p + align_up((size_t)words * sizeof(uint64_t), 256));
    uint32_t *bsum = (uint32_t *)((char *)base + align_up((size_t)words * sizeof(uint32_t), 256));
    const uint32_t cap = capacity > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)capacity;
    hipLaunchKernelGGL(st_roots, dim3(nb), dim3(256), 0, s, labels, (uint32_t)W, WW, words, mask, bsum);
    hipLaunchKernelGGL(st_scan, dim3(1), dim3(1024), 0, s, bsum, nb, n_out);
    hipLaunchKernelGGL(st_bases, dim3(nb), dim3(64), 0, s, mask, bsum, words, (uint32_t)W, WW, base,
                       out, cap);
    hipLaunchKernelGGL(st_accum, dim3(WW, ((uint32_t)H + kAccRows - 1u) / kAccRows), dim3(kAccWaves * 64),
                       0, s, labels,
                       (uint32_t)H, (uint32_t)W, WW, mask, base, out, cap);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e);
    return CCL_OK;
}
