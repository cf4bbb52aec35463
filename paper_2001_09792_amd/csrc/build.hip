// build.hip -- linear BVH construction for gfx950 and the bottom/top-level
// entry points.
//
// The paper builds its two-layered structure from the models' vertex data
// (bottom level) and from instances with transformation matrices (top level)
// inside the RTX driver (section 1).  Here both levels use one pipeline:
//   1. primitive boxes and the bounds of their centres,
//   2. 63-bit Morton codes of the quantised centres,
//   3. a stable LSD radix sort of (key, id), 8-bit digits, ranked in LDS,
//   4. Karras's parallel radix-tree construction (HPG 2012), or
//      locally-ordered clustering (Meister & Bittner 2018),
//   5. box refit level by level from the deepest (the inner nodes grouped
//      by their depth from the root), then optionally rounds of treelet
//      restructuring (Karras & Aila 2013),
//   6. top-down collapse into W-wide nodes (repeatedly opening the inner
//      child with the largest surface area), leaves of <= leaf_max prims,
// followed by reordering the primitives into leaf order.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "rg_internal.h"

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

namespace {

constexpr int kThreads = 256;
// radix sort tiles: kSortThreads threads of kSortItems keys.  A compute
// unit keeps only so many loads in flight, so the tiles have to be spread
// over all of them (2,048 keys: 307 tiles for a mesh of 627,200 triangles).
constexpr int kSortThreads = 512;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kCountCopies = 8;  // copies of the digit counts, spread over the tiles (fewer atomics per word)
constexpr int kScanThreads = 1024;

// --------------------------------------------------------------- helpers

// The value that lane (this lane ^ J) of the wave holds, J = 1 .. 32, with
// every lane active: DPP quad permutes and row mirrors below 16 (4 = half-row
// mirror then quad reversal, 8 = row mirror then half-row mirror), the
// gfx950 row swaps for 16 and 32 (each returns both swapped operands; a lane
// takes the half that came from the other row).
template <int J>
__device__ inline uint32_t lane_xor(uint32_t v) {
    if constexpr (J == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    else if constexpr (J == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    else if constexpr (J == 4)
        return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
    else if constexpr (J == 8)
        return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false), 0x141, 0xF, 0xF, false);
    else if constexpr (J == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (__lane_id() & 16) ? r[0] : r[1];
    } else {
        static_assert(J == 32, "lane distance");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (__lane_id() & 32) ? r[0] : r[1];
    }
}
__device__ inline uint32_t lane_xor(uint32_t v, int j) {  // j a constant after unrolling
    switch (j) {
        case 1: return lane_xor<1>(v);
        case 2: return lane_xor<2>(v);
        case 4: return lane_xor<4>(v);
        case 8: return lane_xor<8>(v);
        case 16: return lane_xor<16>(v);
        default: return lane_xor<32>(v);
    }
}
__device__ inline float lane_xor(float v, int j) { return __uint_as_float(lane_xor(__float_as_uint(v), j)); }

__device__ inline float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, lane_xor(v, o));
    return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, lane_xor(v, o));
    return v;
}

// ------------------------------------------------- 1. primitive boxes
// flags bit 0: an index out of range; bit 1: a non-finite coordinate.
__global__ void k_tri_boxes(const float *__restrict__ verts, int64_t n_verts,
                            const uint32_t *__restrict__ idx, int64_t n, float *__restrict__ box,
                            uint32_t *__restrict__ flags) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t a = idx[3 * i], b = idx[3 * i + 1], c = idx[3 * i + 2];
    uint32_t bad = 0;
    if ((int64_t)a >= n_verts || (int64_t)b >= n_verts || (int64_t)c >= n_verts) {
        bad |= 1u;
        a = b = c = 0;
    }
    float v[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = verts[3 * (int64_t)a + k];
        v[3 + k] = verts[3 * (int64_t)b + k];
        v[6 + k] = verts[3 * (int64_t)c + k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k)
        if (!isfinite(v[k])) bad |= 2u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        box[6 * i + k] = fminf(fminf(v[k], v[3 + k]), v[6 + k]);
        box[6 * i + 3 + k] = fmaxf(fmaxf(v[k], v[3 + k]), v[6 + k]);
    }
    if (bad) atomicOr(flags, bad);
}

// Bounds of the box centres c = 0.5 (lo + hi): one partial per block,
// part[6 b .. 6 b + 5] = min xyz, max xyz (k_morton reduces them, so no
// atomics and no initialised bounds are needed).  Also clears zero[0, nz):
// the sort's digit counts, tickets and tile status words.
constexpr int kBoundParts = 512;  // largest grid of k_centre_bounds
__global__ void __launch_bounds__(kThreads) k_centre_bounds(const float *__restrict__ box, int64_t n,
                                                            float *__restrict__ part, uint32_t *__restrict__ zero,
                                                            int64_t nz) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t j = i0; j < nz; j += stride) zero[j] = 0u;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll 4
    for (int64_t i = i0; i < n; i += stride) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float c = (box[6 * i + k] + box[6 * i + 3 + k]) * 0.5f;
            mn[k] = fminf(mn[k], c);
            mx[k] = fmaxf(mx[k], c);
        }
    }
    __shared__ float red[6][kThreads / 64];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        mn[k] = wave_min(mn[k]);
        mx[k] = wave_max(mx[k]);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            red[k][wv] = mn[k];
            red[3 + k][wv] = mx[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float v = red[k][0];
        for (int q = 1; q < kThreads / 64; ++q) v = k < 3 ? fminf(v, red[k][q]) : fmaxf(v, red[k][q]);
        part[6 * blockIdx.x + k] = v;
    }
}

// ------------------------------------------------------ 2. Morton codes
__device__ inline uint64_t spread21(uint64_t x) {
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// The key of one primitive box from the centre bounds lo[3], hi[3].
__device__ inline uint64_t morton_key(const float *__restrict__ b, const float *lo3, const float *hi3) {
#pragma clang fp contract(off)
    uint64_t q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float lo = lo3[k], hi = hi3[k];
        float ext = hi - lo;
        float s = ext > 0.0f ? 2097152.0f / ext : 0.0f;
        float c = (b[k] + b[3 + k]) * 0.5f;
        float x = (c - lo) * s;
        x = floorf(x);
        uint64_t v = (x > 0.0f) ? (uint64_t)x : 0ull;  // NaN -> 0
        q[k] = v > 2097151ull ? 2097151ull : v;
    }
    return (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
}
// The same from bounds held as order-preserving uints (lo[0..2], hi[3..5]).
__device__ inline uint64_t morton_key(const float *__restrict__ b, const uint32_t *bounds) {
    float lo[3], hi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = rg_ord2f(bounds[k]);
        hi[k] = rg_ord2f(bounds[3 + k]);
    }
    return morton_key(b, lo, hi);
}

// Keys and ids of one tile of kSortTile boxes per block, and the counts of
// every 8-bit digit of the keys for all eight sort passes, added into
// count[copy][pass][digit] (copy = block mod kCountCopies; cleared by
// k_centre_bounds).  The centre bounds are the reduction of
// k_centre_bounds' nparts partials.
__global__ void __launch_bounds__(kSortThreads) k_morton(const float *__restrict__ box, int64_t n,
                                                         const float *__restrict__ part, int nparts, int key_shift,
                                                         uint64_t *__restrict__ keys, uint32_t *__restrict__ ids,
                                                         uint32_t *__restrict__ count) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t h[8 * 256];
    __shared__ float red[6][kWaves];
    __shared__ float bnd[6];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int j = t; j < 8 * 256; j += kSortThreads) h[j] = 0u;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int j = t; j < nparts; j += kSortThreads) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mn[k] = fminf(mn[k], part[6 * j + k]);
            mx[k] = fmaxf(mx[k], part[6 * j + 3 + k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        mn[k] = wave_min(mn[k]);
        mx[k] = wave_max(mx[k]);
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            red[k][w] = mn[k];
            red[3 + k][w] = mx[k];
        }
    }
    __syncthreads();
    if (t < 6) {
        float v = red[t][0];
        for (int q = 1; q < kWaves; ++q) v = t < 3 ? fminf(v, red[t][q]) : fmaxf(v, red[t][q]);
        bnd[t] = v;
    }
    __syncthreads();
    const float lo[3] = {bnd[0], bnd[1], bnd[2]}, hi[3] = {bnd[3], bnd[4], bnd[5]};
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    float b[kSortItems][6];  // every box load in flight before the first is used
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = base + it * kSortThreads + t;
#pragma unroll
        for (int k = 0; k < 6; ++k) b[it][k] = i < n ? box[6 * i + k] : 0.0f;
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = base + it * kSortThreads + t;
        const bool valid = i < n;
        uint64_t key = 0ull;
        if (valid) {
            key = morton_key(b[it], lo, hi) >> key_shift;
            keys[i] = key;
            ids[i] = (uint32_t)i;
        }
        const uint64_t vm = __ballot(valid);
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t d = (uint32_t)(key >> (8 * p)) & 255u;
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);  // lane 0: valid whenever vm != 0
            if (__ballot(valid && d != d0) == 0ull) {  // one digit across the wave (the high digits)
                if (lane == 0) atomicAdd(&h[256 * p + d0], (uint32_t)__popcll(vm));
            } else if (valid) {
                atomicAdd(&h[256 * p + d], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *cc = count + 2048 * (blockIdx.x % kCountCopies);
    for (int j = t; j < 8 * 256; j += kSortThreads) {
        const uint32_t c = h[j];
        if (c) atomicAdd(&cc[j], c);
    }
}

// -------------------------------------------------- 3. LSD radix sort
// Three launches per pass of 8 bits, each spread over every compute unit
// (a unit keeps only so many loads in flight, so a tile of 2,048 keys per
// workgroup): the digit counts of every tile (k_sort_count, digit-major),
// their exclusive scan per digit plus the pass's count of all smaller
// digits (k_sort_scan, one workgroup per digit; the totals of every pass
// were counted with the keys), and the stable scatter (k_sort_scatter).  A
// single launch per pass with a look-back over earlier tiles' counts was
// slower here: with ~300 tiles finishing at once its chain of cross-die
// reads outlasts the two extra launches.

// Ranks a tile's items by digit, tile order = (wave, item, lane): rk[k] =
// count of equal digits before item k within its wave; wcnt[w][d] (zero on
// entry) ends as wave w's count of digit d.  Lanes with equal digits are
// matched with 8 ballots (one when the wave shares one digit).
template <typename K>
__device__ inline void rank_items(const K (&key)[kSortItems], int in_tile, int shift, uint32_t (&rk)[kSortItems],
                                  uint32_t (*wcnt)[256]) {
    constexpr int kPerWave = kSortTile / (kSortThreads / 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const bool valid = w * kPerWave + k * 64 + lane < in_tile;
        const uint32_t dg = (uint32_t)(key[k] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
        if (__ballot(valid && dg != d0) != 0ull) {  // uniform; else every valid lane shares one digit
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (dg >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        const uint32_t c = wcnt[w][dg];  // LDS accesses of one wave complete in order
        rk[k] = c + before;
        if (valid && before == 0u) wcnt[w][dg] = c + (uint32_t)__popcll(peers);
    }
}

// Loads tile blockIdx.x: wave w holds elements [w kPerWave, (w + 1)
// kPerWave), item k at k * 64 + lane; every load issued before any is used.
template <typename K>
__device__ inline int load_tile(const K *__restrict__ keys, int64_t n, K (&key)[kSortItems]) {
    constexpr int kPerWave = kSortTile / (kSortThreads / 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int in_tile = (int)(n - base < kSortTile ? n - base : kSortTile);
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int e = w * kPerWave + k * 64 + lane;
        key[k] = e < in_tile ? keys[base + e] : (K)0;
    }
    return in_tile;
}

// cnt[d * nb + tile] = the tile's count of digit d.
template <typename K>
__global__ void __launch_bounds__(kSortThreads) k_sort_count(const K *__restrict__ keys, int64_t n, int shift,
                                                             uint32_t *__restrict__ cnt, int nb) {
    constexpr int kWaves = kSortThreads / 64;
    static_assert(kSortThreads >= 256, "a thread per digit");
    __shared__ uint32_t wcnt[kWaves][256];
    const int t = threadIdx.x;
    for (int j = t; j < kWaves * 256; j += kSortThreads) (&wcnt[0][0])[j] = 0u;
    K key[kSortItems];
    uint32_t rk[kSortItems];
    const int in_tile = load_tile(keys, n, key);
    __syncthreads();
    rank_items(key, in_tile, shift, rk, wcnt);
    __syncthreads();
    if (t < 256) {
        uint32_t tot = 0u;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) tot += wcnt[q][t];
        cnt[(int64_t)t * nb + blockIdx.x] = tot;
    }
}

// Exclusive scan in place.  A block scans a chunk of kScanChunk elements at
// a time: each thread takes kScanPer consecutive elements (their loads in
// flight together), scans them serially, and the block scans the per-thread
// totals.
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;

// Scans data[base, base + kScanChunk) (clipped to m), adding `carry`;
// returns the chunk's total (every thread of the block).
__device__ inline uint32_t scan_chunk(uint32_t *data, int64_t m, int64_t base, uint32_t carry, uint32_t *wsum) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t i0 = base + (int64_t)t * kScanPer;
    uint32_t v[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v[k] = (i0 + k < m) ? data[i0 + k] : 0u;
    uint32_t tot = 0u;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) tot += v[k];
    uint32_t x = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        uint32_t s = lane < kScanThreads / 64 ? wsum[lane] : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(s, o, 64);
            if (lane >= o) s += y;
        }
        if (lane < kScanThreads / 64) wsum[lane] = s;  // inclusive wave totals
    }
    __syncthreads();
    uint32_t run = carry + (w > 0 ? wsum[w - 1] : 0u) + x - tot;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (i0 + k < m) data[i0 + k] = run;
        run += v[k];
    }
    const uint32_t total = wsum[kScanThreads / 64 - 1];
    __syncthreads();
    return total;
}

// The whole array by one block, chunk after chunk.
__global__ void __launch_bounds__(kScanThreads) k_scan_excl(uint32_t *data, int64_t m) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    uint32_t carry = 0u;
    for (int64_t base = 0; base < m; base += kScanChunk) carry += scan_chunk(data, m, base, carry, wsum);
}


// One workgroup per digit d: cnt[d][*] becomes the exclusive scan over the
// tiles plus the pass's count of all smaller digits (total: the pass's
// digit counts, kCountCopies copies 2,048 words apart).
__global__ void __launch_bounds__(kScanThreads) k_sort_scan(uint32_t *cnt, int nb, const uint32_t *__restrict__ total) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    __shared__ uint32_t below;
    const int d = blockIdx.x, t = threadIdx.x;
    if (t < 256) {
        uint32_t x = 0u;
        if (t < d) {
#pragma unroll
            for (int c = 0; c < kCountCopies; ++c) x += total[2048 * c + t];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((t & 63) == 0) wsum[t >> 6] = x;
    }
    __syncthreads();
    if (t == 0) below = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    uint32_t carry = below;
    __syncthreads();  // wsum is reused by the scan
    uint32_t *col = cnt + (int64_t)d * nb;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanChunk) carry += scan_chunk(col, nb, b0, carry, wsum);
}

// Stable scatter of tile blockIdx.x: its keys ranked by digit, put in digit
// order in LDS, then written out with consecutive threads on consecutive
// positions of each digit's run, from the tile's first position per digit
// in goff[d * nb + tile].
template <typename K>
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const K *__restrict__ keys_in,
                                                               const uint32_t *__restrict__ ids_in,
                                                               K *__restrict__ keys_out,
                                                               uint32_t *__restrict__ ids_out, int64_t n, int shift,
                                                               const uint32_t *__restrict__ goff, int nb) {
    constexpr int kWaves = kSortThreads / 64, kPerWave = kSortTile / kWaves;
    __shared__ K skey[kSortTile];
    __shared__ uint32_t sid[kSortTile];
    __shared__ uint32_t wcnt[kWaves][256];  // per wave: digit counts, then offsets within the tile's digit
    __shared__ uint32_t dstart[256], gpos[256];
    __shared__ uint32_t wsum[kWaves];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int j = t; j < kWaves * 256; j += kSortThreads) (&wcnt[0][0])[j] = 0u;
    if (t < 256) gpos[t] = goff[(int64_t)t * nb + blockIdx.x];
    K key[kSortItems];
    uint32_t id[kSortItems], rk[kSortItems];
    const int in_tile = load_tile(keys_in, n, key);
    load_tile(ids_in, n, id);
    __syncthreads();
    rank_items(key, in_tile, shift, rk, wcnt);
    __syncthreads();
    // thread t < 256 = digit t: offsets of the waves within the tile's digit,
    // then the digit's first position in the tile
    uint32_t tot = 0u;
    if (t < 256) {
        for (int q = 0; q < kWaves; ++q) {
            const uint32_t c = wcnt[q][t];
            wcnt[q][t] = tot;
            tot += c;
        }
    }
    uint32_t x = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t pre = 0u;
    for (int q = 0; q < w; ++q) pre += wsum[q];
    if (t < 256) dstart[t] = pre + x - tot;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int e = w * kPerWave + k * 64 + lane;
        if (e < in_tile) {
            const uint32_t dg = (uint32_t)(key[k] >> shift) & 255u;
            const uint32_t p = dstart[dg] + wcnt[w][dg] + rk[k];
            skey[p] = key[k];
            sid[p] = id[k];
        }
    }
    __syncthreads();
    for (int j = t; j < in_tile; j += kSortThreads) {
        const K kk = skey[j];
        const uint32_t dg = (uint32_t)(kk >> shift) & 255u;
        const uint32_t o = gpos[dg] + ((uint32_t)j - dstart[dg]);
        if (o < (uint64_t)n) {  // always true for consistent counts
            keys_out[o] = kk;
            ids_out[o] = sid[j];
        }
    }
}

// ------------------------------------------------- 4. Karras hierarchy
// Index arithmetic in 32 bits: n <= RG_MAX_TRIS = 2^28, so every probe
// i + m * d below stays within (-2^30, 2^30).
__device__ inline int k_delta(const uint64_t *k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    const uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
    return __clzll((long long)(a ^ b));
}

// Inner node i of the radix tree over n sorted keys (keys may be in LDS):
// its children (>= 0 inner, < 0 leaf -(j+1)), parent links and leaf range.
__device__ inline void karras_node(const uint64_t *keys, int64_t n64, int64_t i64, int32_t *__restrict__ left,
                                   int32_t *__restrict__ right, int32_t *__restrict__ parent_int,
                                   int32_t *__restrict__ parent_leaf, int32_t *__restrict__ first,
                                   int32_t *__restrict__ last) {
    static_assert(RG_MAX_TRIS <= (1ll << 28), "32-bit index arithmetic");
    const int n = (int)n64, i = (int)i64;
    const int d = (k_delta(keys, n, i, i + 1) - k_delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = k_delta(keys, n, i, i - d);
    int lmax = 2;
    while (k_delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (k_delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = k_delta(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (k_delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int g = i + s * d + (d < 0 ? -1 : 0);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    if (g < 0 || g + 1 > n - 1 || lo < 0 || hi > n - 1) return;  // unreachable for sorted keys
    if (lo == g) {
        left[i] = -(g + 1);
        parent_leaf[g] = i;
    } else {
        left[i] = g;
        parent_int[g] = i;
    }
    if (hi == g + 1) {
        right[i] = -(g + 2);
        parent_leaf[g + 1] = i;
    } else {
        right[i] = g + 1;
        parent_int[g + 1] = i;
    }
    first[i] = lo;
    last[i] = hi;
    if (i == 0) parent_int[0] = -1;
}

__global__ void k_karras(const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ left,
                         int32_t *__restrict__ right, int32_t *__restrict__ parent_int,
                         int32_t *__restrict__ parent_leaf, int32_t *__restrict__ first,
                         int32_t *__restrict__ last) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    karras_node(keys, n, i, left, right, parent_int, parent_leaf, first, last);
}

// -------------------------------------------------------- 5. box refit
// Inner boxes come from the leaf ranges (k_range_* below), after
// k_leaf_boxes has gathered the leaf boxes in leaf order.

// --------------------------------------------------- 6. wide collapse
__device__ inline float surface_area(const float *b) {
    float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return 2.0f * (dx * dy + dy * dz + dz * dx);
}

constexpr int kCollapseRing = 24;   // per-level bookkeeping slots on the device
constexpr int kCollapseBatch = 8;   // levels launched between host reads after the first batch
constexpr int kCollapseFirstMax = kCollapseRing - 3;  // the first batch (sized from n) at most

// The children of the wide node that stands for binary inner node b: b's
// two children, then repeatedly the inner one of largest surface area opened
// into its two children, up to W (each candidate's area computed once, when
// it joins).  C[k] >= 0 an inner node, < 0 leaf -(j+1).  Returns the count.
template <int W>
__device__ inline int collapse_children(int32_t b, const int32_t *__restrict__ left,
                                        const int32_t *__restrict__ right, const float *__restrict__ int_box,
                                        int32_t C[W]) {
    float A[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        C[k] = -1;
        A[k] = -1.0f;
    }
    C[0] = left[b];
    C[1] = right[b];
    int m = 2;
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (C[k] >= 0) A[k] = surface_area(int_box + 6 * (int64_t)C[k]);
    while (m < W) {
        int best = -1;
        float bsa = -1.0f;
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (k < m && C[k] >= 0 && A[k] > bsa) {
                bsa = A[k];
                best = k;
            }
        if (best < 0) break;
        int32_t c = 0;
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (k == best) c = C[k];
        const int32_t l = left[c], r = right[c];
        const float al = l >= 0 ? surface_area(int_box + 6 * (int64_t)l) : -1.0f;
        const float ar = r >= 0 ? surface_area(int_box + 6 * (int64_t)r) : -1.0f;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (k == best) {
                C[k] = l;
                A[k] = al;
            }
            if (k == m) {
                C[k] = r;
                A[k] = ar;
            }
        }
        ++m;
    }
    return m;
}

// Links of the m children: a leaf (a binary leaf, or an inner node whose
// range holds at most leaf_max primitives), RG_EMPTY past m; returns the
// mask of the children that stay inner nodes (their links set by the caller).
template <int W>
__device__ inline uint32_t collapse_links(const int32_t C[W], int m, const int32_t *__restrict__ first,
                                          const int32_t *__restrict__ last, int leaf_max, uint32_t link[W]) {
    uint32_t inner = 0u;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        link[k] = RG_EMPTY;
        if (k >= m) continue;
        const int32_t c = C[k];
        if (c < 0) {
            link[k] = rg_leaf((uint32_t)(-c - 1), 1u);
        } else {
            const int32_t f = first[c], size = last[c] - f + 1;
            if (size <= leaf_max) link[k] = rg_leaf((uint32_t)f, (uint32_t)size);
            else inner |= 1u << k;
        }
    }
    return inner;
}

// Writes a wide node: the children's boxes (empty slots inverted) and links,
// assembled in registers and stored 16 bytes at a time (a node is 64-byte
// aligned): 2W stores per node instead of 8W.
template <int W>
__device__ inline void write_wide_node(RgNode<W> *nd, const int32_t C[W], int m, const uint32_t link[W],
                                       const float *__restrict__ int_box, const float *__restrict__ leaf_box) {
    uint32_t w[8 * W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        if (k < m) {
            const int32_t c = C[k];
            const float *src = c < 0 ? leaf_box + 6 * (int64_t)(-c - 1) : int_box + 6 * (int64_t)c;
#pragma unroll
            for (int z = 0; z < 6; ++z) b[z] = src[z];
        }
#pragma unroll
        for (int z = 0; z < 6; ++z) w[z * W + k] = __float_as_uint(b[z]);
        w[6 * W + k] = link[k];
        w[7 * W + k] = 0u;
    }
    uint4 *dst = reinterpret_cast<uint4 *>(nd);
#pragma unroll
    for (int q = 0; q < 2 * W; ++q) dst[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// The children every inner node of the binary hierarchy would get as the
// root of a wide node (the opening order depends on that node alone), for
// all m inner nodes at once: binary ids (wch), the links of the children
// that end as leaves (wlink, RG_EMPTY past the last child) and the mask of
// those that stay inner nodes (winner).  The level-by-level collapse then
// waits on one load round for them instead of the whole opening sequence.
template <int W>
__global__ void k_wide_plan(const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                            const int32_t *__restrict__ first, const int32_t *__restrict__ last,
                            const float *__restrict__ int_box, int leaf_max, int64_t m, int32_t *__restrict__ wch,
                            uint32_t *__restrict__ wlink, uint8_t *__restrict__ winner) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t C[W];
    uint32_t link[W];
    const int n_ch = collapse_children<W>((int32_t)i, left, right, int_box, C);
    winner[i] = (uint8_t)collapse_links<W>(C, n_ch, first, last, leaf_max, link);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        wch[W * i + k] = k < n_ch ? C[k] : 0;
        wlink[W * i + k] = link[k];
    }
}

// One thread per node of the level (queue items: node index, binary node it
// stands for).  Children that stay inner nodes join the next level's queue:
// one counter add per wave, and a child's node index is the next level's
// first index plus its queue slot.
template <int W>
__global__ void k_collapse(const int32_t *__restrict__ wch, const uint32_t *__restrict__ wlink,
                           const uint8_t *__restrict__ winner, const float *__restrict__ int_box,
                           const float *__restrict__ leaf_box, const uint2 *__restrict__ q_in,
                           uint2 *__restrict__ q_out, uint32_t *ring, int level, RgNode<W> *__restrict__ nodes,
                           uint32_t *__restrict__ parents, uint32_t *__restrict__ levels, uint32_t cap) {
    // ring: [0, R) node count of level l at l % R, [R, 2R) first node index of
    // level l at R + l % R, [2R] error flags.  A level's kernel sets up the
    // next level's first index and clears the count two levels ahead, so
    // levels can be launched back to back with no host step between them.
    uint32_t *count_in = ring + level % kCollapseRing, *q_out_count = ring + (level + 1) % kCollapseRing;
    uint32_t cnt = *count_in;
    if (cnt > cap) cnt = cap;
    const uint32_t next_base = ring[kCollapseRing + level % kCollapseRing] + cnt;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ring[kCollapseRing + (level + 1) % kCollapseRing] = next_base;
        ring[(level + 2) % kCollapseRing] = 0u;
        // the level table (first node of each level, then the node count):
        // launches past the last level write the node count again
        if (levels && level + 1 <= RG_LEVELS_CAP) levels[level + 1] = next_base;
    }
    uint32_t *err = ring + 2 * kCollapseRing;
    const int lane = threadIdx.x & 63;
    // the loop bound is the same for every lane of a block, so whole waves
    // take part in the scan below
    for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
        const uint32_t qi = base + threadIdx.x;
        const bool active = qi < cnt;
        int32_t C[W];
        uint32_t link[W];
        uint2 item = make_uint2(0u, 0u);
        int m = 0;
        uint32_t inner = 0u;
        if (active) {
            item = q_in[qi];
            const int64_t b = item.y;
            inner = winner[b];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                C[k] = wch[W * b + k];
                link[k] = wlink[W * b + k];
                if (((inner >> k) & 1u) || link[k] != RG_EMPTY) m = k + 1;
            }
        }
        // queue slots: an exclusive scan of the inner-child counts over the wave
        const uint32_t nc = __popc(inner);
        uint32_t incl = nc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        const uint32_t total = __shfl(incl, 63, 64);
        uint32_t wbase = 0u;
        if (lane == 63 && total) wbase = atomicAdd(q_out_count, total);
        wbase = __shfl(wbase, 63, 64);
        uint32_t slot = wbase + incl - nc;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (!((inner >> k) & 1u)) continue;
            const uint32_t nn = next_base + slot;
            if (nn < cap && slot < cap) {  // a BVH2 has n-1 inner nodes: never exceeded
                q_out[slot] = make_uint2(nn, (uint32_t)C[k]);
                if (parents) parents[nn] = (item.x << 3) | (uint32_t)k;
                link[k] = nn;
            } else {
                atomicOr(err, 4u);
            }
            ++slot;
        }
        if (!active) continue;
        write_wide_node<W>(nodes + item.x, C, m, link, int_box, leaf_box);
    }
}

// Single-primitive structure: one root node with one leaf child.
template <int W>
__global__ void k_single_root(const float *__restrict__ leaf_box, RgNode<W> *nodes) {
    int k = threadIdx.x;
    if (k >= W) return;
    RgNode<W> *nd = nodes;
    if (k == 0) {
        nd->lo_x[0] = leaf_box[0]; nd->lo_y[0] = leaf_box[1]; nd->lo_z[0] = leaf_box[2];
        nd->hi_x[0] = leaf_box[3]; nd->hi_y[0] = leaf_box[4]; nd->hi_z[0] = leaf_box[5];
        nd->child[0] = rg_leaf(0u, 1u);
    } else {
        nd->lo_x[k] = INFINITY; nd->lo_y[k] = INFINITY; nd->lo_z[k] = INFINITY;
        nd->hi_x[k] = -INFINITY; nd->hi_y[k] = -INFINITY; nd->hi_z[k] = -INFINITY;
        nd->child[k] = RG_EMPTY;
    }
    nd->pad[k] = 0u;
}

__global__ void k_collapse_init(uint2 *q, uint32_t *ring, uint32_t *parents, uint32_t *levels) {
    q[0] = make_uint2(0u, 0u);
    for (int k = 0; k <= 2 * kCollapseRing; ++k) ring[k] = 0u;
    ring[0] = 1u;  // level 0: the root, node 0
    if (parents) parents[0] = RG_MISS;  // the root
    if (levels) levels[0] = 0u;
}

// ------------------------------------------------ top-level instances
struct BlasInfo {
    uint64_t nodes, tris, hdr;
};

__device__ inline float round_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}
__device__ inline float round_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

// Instance i: its world box (the 8 transformed corners of the bottom level's
// root box, in double, rounded outward), its record (the world->object
// inverse in double, stored as float) and a copy of its matrix.  The bottom
// level's root box and the status of its last refit come from its header on
// the device (a refit updates them without a host round trip).
struct InstTables {
    const float *xform;
    const uint32_t *blas_id, *inst_mat, *inst_flags;  // inst_flags nullable
    const BlasInfo *blas;
    uint32_t *flags;   // bit 0: a bottom level's last refit saw invalid input
    float *xf_keep;
};

// A top level of up to kResidentMax instances built in one launch with its
// instance step (RgLbvhOut::tlas_fuse points to one).
struct TlasFuse {
    InstTables T;
    RgInst *rec_tmp, *recs_out;
    uint32_t *rec_of;
};

__device__ inline void inst_setup_one(const InstTables &T, int64_t i, float box[6], RgInst &r) {
    double m[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        m[k] = (double)T.xform[12 * i + k];
        T.xf_keep[12 * i + k] = T.xform[12 * i + k];
    }
    const BlasInfo &BI = T.blas[T.blas_id[i]];
    const RgBlasHdr &B = *reinterpret_cast<const RgBlasHdr *>(BI.hdr);
    if (B.status != 0u) atomicOr(T.flags, 1u);
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int c = 0; c < 8; ++c) {
        double p[3] = {(double)((c & 1) ? B.hi[0] : B.lo[0]), (double)((c & 2) ? B.hi[1] : B.lo[1]),
                       (double)((c & 4) ? B.hi[2] : B.lo[2])};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double w = m[4 * q] * p[0] + m[4 * q + 1] * p[1] + m[4 * q + 2] * p[2] + m[4 * q + 3];
            mn[q] = fmin(mn[q], w);
            mx[q] = fmax(mx[q], w);
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        box[q] = round_down(mn[q]);
        box[3 + q] = round_up(mx[q]);
    }
    // inverse of the linear part (adjugate over determinant), in double
    double a = m[0], b = m[1], c = m[2], d = m[4], e = m[5], f = m[6], g = m[8], h = m[9], k = m[10];
    double A = e * k - f * h, Bc = -(d * k - f * g), Cc = d * h - e * g;
    double det = a * A + b * Bc + c * Cc;
    const double rdet = 1.0 / det;  // one division; the entries differ from x / det by an ulp of double at most
    double inv[9] = {A * rdet, -(b * k - c * h) * rdet, (b * f - c * e) * rdet,
                     Bc * rdet, (a * k - c * g) * rdet, -(a * f - c * d) * rdet,
                     Cc * rdet, -(a * h - b * g) * rdet, (a * e - b * d) * rdet};
#pragma unroll
    for (int q = 0; q < 9; ++q) r.inv[q] = (float)inv[q];
    r.p[0] = T.xform[12 * i + 3];
    r.p[1] = T.xform[12 * i + 7];
    r.p[2] = T.xform[12 * i + 11];
    r.nodes = BI.nodes;
    r.tris = BI.tris;
    r.hdr = BI.hdr;
    r.mat = T.inst_mat[i];
    r.inst = (uint32_t)i;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        r.blo[q] = B.lo[q];
        r.bhi[q] = B.hi[q];
    }
    r.flags = (T.inst_flags ? T.inst_flags[i] : RG_INST_MASK_ALL) | (B.alpha ? RG_INST_ALPHA : 0u);
    r.pad = 0u;
}

__global__ void k_inst_setup(InstTables T, int64_t n, float *__restrict__ box, RgInst *__restrict__ recs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float b[6];
    RgInst r;
    inst_setup_one(T, i, b, r);
#pragma unroll
    for (int q = 0; q < 6; ++q) box[6 * i + q] = b[q];
    recs[i] = r;
}

// ------------------------------------- whole build in one workgroup
// For up to kSmallMax primitives (top levels, small meshes) the steps above
// run in one workgroup of one launch, the keys in LDS: the same centre
// bounds and Morton codes, a bitonic sort by (key, input index) -- the order
// of the stable sort --, the same radix tree and box unions (boxes round by
// round: a node's box once both children's are known), and the same wide
// collapse level by level (a queue slot per inner child from an LDS
// counter).  No host step in between; the result summary goes to `res`.
constexpr int kSmallThreads = 1024;
constexpr int kSmallMax = 4096;
struct SmallResult {
    uint32_t depth, n_nodes, err, flag;  // flag: a copy of *SmallArgs::flag_in (0 without)
    float lo[3], hi[3];
};

struct SmallArgs {
    const float *prim_box;
    int32_t n, leaf_max;
    uint64_t *keys_out;             // sorted keys (nullable: only for the stage check)
    uint32_t *ids;                  // sorted primitive order
    int32_t *left, *right, *pint, *pleaf, *first, *last;
    float *int_box, *leaf_box;
    uint2 *q[2];
    void *nodes;                    // nullable: binary hierarchy only
    uint32_t *parents, *levels;     // nullable
    const uint32_t *flag_in;        // nullable: a word of an earlier step (or of this kernel) returned with the summary
    int32_t key_shift;              // 0 (63-bit keys) or 33 (their top 30 bits)
    SmallResult *res;
    // a top level built in the same launch (TLAS): each primitive is an
    // instance whose box and record the kernel computes from the tables; the
    // records land in rec_tmp (input order), then recs_out (leaf order) with
    // rec_of (each instance's record)
    InstTables inst;
    RgInst *rec_tmp, *recs_out;
    uint32_t *rec_of;
};

// LDS of the one-workgroup build (dynamic).  Up to kResidentMax primitives
// everything the steps read again and again stays in LDS: keys, order, tree
// links, ranges and parents, inner boxes, the primitive boxes in input and in
// leaf order (108 bytes per primitive).  Above that: the keys and the order.
constexpr int kResidentMax = 1024;
constexpr size_t kSmallLdsResident = (size_t)kResidentMax * (8 + 4 + 6 * 4 + 3 * 24);
constexpr size_t kSmallLdsGlobal = (size_t)kSmallMax * (8 + 4);
size_t small_lds_bytes(int64_t n) { return n <= kResidentMax ? kSmallLdsResident : kSmallLdsGlobal; }
static_assert(8 * 2 + 1 <= 24, "the wide-children table fits the primitive-box area (W <= 8)");

template <int W, bool RESIDENT, bool TLAS = false>
__global__ void __launch_bounds__(kSmallThreads) k_small_build(SmallArgs a) {
    static_assert(RESIDENT || !TLAS, "a fused top level is built resident");
    extern __shared__ uint64_t small_lds[];
    __shared__ uint32_t bnd[6];
    __shared__ uint32_t done[2][kSmallMax / 32];
    __shared__ uint32_t qcnt[3], lstart[RG_LEVELS_CAP + 2];
    const int t = threadIdx.x, n = a.n, lane = t & 63;
    constexpr int cap = RESIDENT ? kResidentMax : kSmallMax;
    uint64_t *key = small_lds;
    uint32_t *id = reinterpret_cast<uint32_t *>(key + cap);
    // tree links, ranges, parents and boxes: LDS when resident, else the
    // scratch arrays.  Once the tree is built the key area holds the arrival
    // counters and the collapse queues (resident).
    int32_t *left = a.left, *right = a.right, *first = a.first, *last = a.last, *pint = a.pint, *pleaf = a.pleaf;
    float *int_box = a.int_box, *lbox = a.leaf_box, *pbox = nullptr;
    uint32_t *arrive = reinterpret_cast<uint32_t *>(key);
    uint32_t *const lq = arrive + cap;  // two queues of cap items (by offset: the pointer stays an LDS one)
    if (RESIDENT) {
        left = reinterpret_cast<int32_t *>(id + cap);
        right = left + cap;
        first = right + cap;
        last = first + cap;
        pint = last + cap;
        pleaf = pint + cap;
        int_box = reinterpret_cast<float *>(pleaf + cap);
        pbox = int_box + 6 * cap;
        lbox = pbox + 6 * cap;
    }
    if (t < 3) bnd[t] = 0xFFFFFFFFu;
    else if (t < 6) bnd[t] = 0u;
    if (t < 3) qcnt[t] = t == 0 ? 1u : 0u;  // the collapse starts from the root
    for (int i = t; i < kSmallMax / 32; i += kSmallThreads) done[0][i] = done[1][i] = 0u;
    __syncthreads();
    // centre bounds (exact min / max, any order): per wave, then LDS atomics;
    // resident, each thread keeps its primitive's box in LDS
    {
        float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = t; i < n; i += kSmallThreads) {
            float b[6];
            if (TLAS) {
                RgInst r;
                inst_setup_one(a.inst, i, b, r);
                a.rec_tmp[i] = r;
            } else {
#pragma unroll
                for (int q = 0; q < 6; ++q) b[q] = a.prim_box[6 * i + q];
            }
            if (RESIDENT) {
#pragma unroll
                for (int q = 0; q < 6; ++q) pbox[6 * i + q] = b[q];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float c = (b[k] + b[3 + k]) * 0.5f;
                mn[k] = fminf(mn[k], c);
                mx[k] = fmaxf(mx[k], c);
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mn[k] = wave_min(mn[k]);
            mx[k] = wave_max(mx[k]);
        }
        if (lane == 0 && mn[0] <= mx[0]) {  // a wave with elements
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                atomicMin(&bnd[k], rg_f2ord(mn[k]));
                atomicMax(&bnd[3 + k], rg_f2ord(mx[k]));
            }
        }
    }
    __syncthreads();
    if (RESIDENT) {
        // one element per thread (padding past n sorts last): bitonic sort by
        // (key, index) in registers, partners within a wave by shuffles,
        // across waves through LDS
        uint64_t k0 = t < n ? morton_key(pbox + 6 * t, bnd) >> a.key_shift : ~0ull;
        uint32_t v0 = (uint32_t)t;
#pragma unroll
        for (int kk = 2; kk <= kResidentMax; kk <<= 1) {
#pragma unroll
            for (int j = kk >> 1; j > 0; j >>= 1) {
                uint64_t ko;
                uint32_t vo;
                if (j >= 64) {
                    __syncthreads();
                    key[t] = k0;
                    id[t] = v0;
                    __syncthreads();
                    ko = key[t ^ j];
                    vo = id[t ^ j];
                } else {
                    ko = ((uint64_t)lane_xor((uint32_t)(k0 >> 32), j) << 32) | lane_xor((uint32_t)k0, j);
                    vo = lane_xor(v0, j);
                }
                // the lower end of an ascending run keeps the smaller one: take
                // the partner's when greater, with the sense flipped where
                // exactly one of "descending run" and "upper end" holds
                // (pairs are distinct); selects, not branches
                const bool gt = k0 > ko || (k0 == ko && v0 > vo);
                const bool take = gt != (((t & kk) != 0) != ((t & j) != 0));
                k0 = take ? ko : k0;
                v0 = take ? vo : v0;
            }
        }
        __syncthreads();
        key[t] = k0;
        if (t < n) {
            a.ids[t] = v0;
            if (a.keys_out) a.keys_out[t] = k0;
            if (TLAS) {  // the record of the instance at leaf position t (written above, before the barriers)
                a.recs_out[t] = a.rec_tmp[v0];
                a.rec_of[v0] = (uint32_t)t;
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float b = pbox[6 * v0 + q];
                lbox[6 * t + q] = b;
                a.leaf_box[6 * t + q] = b;
            }
        }
        __syncthreads();
    } else {
        int P = 1;
        while (P < n) P <<= 1;
        for (int i = t; i < P; i += kSmallThreads) {
            key[i] = i < n ? morton_key(a.prim_box + 6 * i, bnd) >> a.key_shift : ~0ull;  // padding sorts last
            id[i] = (uint32_t)i;
        }
        // bitonic sort by (key, index)
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                __syncthreads();
                for (int i = t; i < P; i += kSmallThreads) {
                    const int l = i ^ j;
                    if (l <= i) continue;
                    const uint64_t ki = key[i], kl = key[l];
                    const uint32_t ii = id[i], il = id[l];
                    const bool gt = ki > kl || (ki == kl && ii > il);
                    if (((i & k) == 0) == gt) {
                        key[i] = kl; key[l] = ki;
                        id[i] = il; id[l] = ii;
                    }
                }
            }
        }
        __syncthreads();
        for (int i = t; i < n; i += kSmallThreads) {
            a.ids[i] = id[i];
            if (a.keys_out) a.keys_out[i] = key[i];
#pragma unroll
            for (int q = 0; q < 6; ++q) a.leaf_box[6 * i + q] = a.prim_box[6 * (int64_t)id[i] + q];
        }
    }
    for (int i = t; i < n - 1; i += kSmallThreads) karras_node(key, n, i, left, right, pint, pleaf, first, last);
    __syncthreads();
    if (RESIDENT) {
        // inner boxes bottom-up: each leaf's thread climbs; at a node the
        // first child to arrive stops, the second takes the union of both
        // children's boxes (written before their arrival was counted)
        for (int i = t; i < cap; i += kSmallThreads) arrive[i] = 0u;
        __syncthreads();
        if (t < n && n > 1) {
            int32_t node = pleaf[t];
            for (int guard = 0; node >= 0 && guard < n; ++guard) {
                __threadfence_block();  // this thread's box writes before its arrival
                if (atomicAdd(&arrive[node], 1u) == 0u) break;  // the sibling's thread continues
                __threadfence_block();  // the sibling's box reads after its arrival
                const int32_t c[2] = {left[node], right[node]};
                float b[12];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const float *src = c[q] < 0 ? lbox + 6 * (-c[q] - 1) : int_box + 6 * c[q];
#pragma unroll
                    for (int z = 0; z < 6; ++z) b[6 * q + z] = src[z];
                }
#pragma unroll
                for (int z = 0; z < 3; ++z) {
                    int_box[6 * node + z] = fminf(b[z], b[6 + z]);
                    int_box[6 * node + 3 + z] = fmaxf(b[3 + z], b[9 + z]);
                }
                if (node == 0) {
                    atomicOr(&done[0][0], 1u);  // the root is final
                    break;
                }
                node = pint[node];
            }
        }
        __syncthreads();
    } else {
        // inner boxes, round by round: a node whose children were final at the
        // start of the round takes the union of their boxes
        for (int round = 0; n > 1 && round < n; ++round) {
            for (int i = t; i < n - 1; i += kSmallThreads) {
                if ((done[0][i >> 5] >> (i & 31)) & 1u) continue;
                const int32_t c[2] = {left[i], right[i]};
                bool ready = true;
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    if (c[q] >= 0 && !((done[0][c[q] >> 5] >> (c[q] & 31)) & 1u)) ready = false;
                if (!ready) continue;
                float b[12];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const float *src = c[q] < 0 ? a.leaf_box + 6 * (int64_t)(-c[q] - 1) : int_box + 6 * (int64_t)c[q];
#pragma unroll
                    for (int z = 0; z < 6; ++z) b[6 * q + z] = src[z];
                }
#pragma unroll
                for (int z = 0; z < 3; ++z) {
                    int_box[6 * i + z] = fminf(b[z], b[6 + z]);
                    int_box[6 * i + 3 + z] = fmaxf(b[3 + z], b[9 + z]);
                }
                atomicOr(&done[1][i >> 5], 1u << (i & 31));
            }
            __syncthreads();
            for (int i = t; i < kSmallMax / 32; i += kSmallThreads) done[0][i] |= done[1][i];
            __syncthreads();
            if (done[0][0] & 1u) break;  // the root
        }
    }
    if (RESIDENT && a.keys_out) {  // the stage check reads the binary tree from the scratch arrays
        for (int i = t; i < n - 1; i += kSmallThreads) {
            a.left[i] = left[i];
            a.right[i] = right[i];
#pragma unroll
            for (int q = 0; q < 6; ++q) a.int_box[6 * i + q] = int_box[6 * i + q];
        }
    }
    const float *root = n > 1 ? int_box : lbox;
    if (t == 0) {
#pragma unroll
        for (int z = 0; z < 3; ++z) {
            a.res->lo[z] = root[z];
            a.res->hi[z] = root[3 + z];
        }
        a.res->err = (n > 1 && !(done[0][0] & 1u)) ? 1u : 0u;
        a.res->flag = a.flag_in ? __hip_atomic_load(a.flag_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    }
    if (!a.nodes) return;
    RgNode<W> *nodes = reinterpret_cast<RgNode<W> *>(a.nodes);
    if (n == 1) {
        if (t < W) {
            RgNode<W> *nd = nodes;
            const int k = t;
            if (k == 0) {
                nd->lo_x[0] = lbox[0]; nd->lo_y[0] = lbox[1]; nd->lo_z[0] = lbox[2];
                nd->hi_x[0] = lbox[3]; nd->hi_y[0] = lbox[4]; nd->hi_z[0] = lbox[5];
                nd->child[0] = rg_leaf(0u, 1u);
            } else {
                nd->lo_x[k] = INFINITY; nd->lo_y[k] = INFINITY; nd->lo_z[k] = INFINITY;
                nd->hi_x[k] = -INFINITY; nd->hi_y[k] = -INFINITY; nd->hi_z[k] = -INFINITY;
                nd->child[k] = RG_EMPTY;
            }
            nd->pad[k] = 0u;
        }
        if (t == 0) {
            if (a.parents) a.parents[0] = RG_MISS;
            if (a.levels) {
                a.levels[0] = 0u;
                a.levels[1] = 1u;
            }
            a.res->depth = 1u;
            a.res->n_nodes = 1u;
        }
        return;
    }
    // resident: the children every inner node would get as the root of a wide
    // node (the opening order depends on that node alone), all at once, into
    // the primitive-box area (dead since the leaf boxes were gathered):
    // binary node ids as int16 (leaves negative, 0x7FFF past the last child)
    // and the mask of the children that stay inner nodes
    int16_t *wch = reinterpret_cast<int16_t *>(pbox);
    uint8_t *winner = reinterpret_cast<uint8_t *>(wch + W * cap);
    if (RESIDENT) {
        for (int i = t; i < n - 1; i += kSmallThreads) {
            int32_t C[W];
            uint32_t link[W];
            const int m = collapse_children<W>(i, left, right, int_box, C);
            winner[i] = (uint8_t)collapse_links<W>(C, m, first, last, a.leaf_max, link);
#pragma unroll
            for (int k = 0; k < W; ++k) wch[W * i + k] = k < m ? (int16_t)C[k] : (int16_t)0x7FFF;
        }
        __syncthreads();
    }
    // wide collapse, level by level; queue items (node, binary node): packed
    // 16 + 16 bits in LDS when resident, else the scratch queues.  Three
    // counters rotate: level L reads its size from qcnt[L % 3], appends to
    // qcnt[(L + 1) % 3] and clears qcnt[(L + 2) % 3] (read by every thread
    // at the start of level L - 1), so one barrier per level suffices.
    if (t == 0) {
        if (RESIDENT) lq[0] = 0u;
        else a.q[0][0] = make_uint2(0u, 0u);
        if (a.parents) a.parents[0] = RG_MISS;
        lstart[0] = 0u;
    }
    uint32_t start = 0u;
    int level = 0;
    __syncthreads();
    for (;;) {
        const uint32_t count = qcnt[level % 3];
        if (count == 0u) break;
        if (t == 0) qcnt[(level + 2) % 3] = 0u;
        const uint32_t next_base = start + count;
        for (uint32_t base = 0; base < count; base += kSmallThreads) {
            const uint32_t qi = base + t;
            const bool active = qi < count;
            uint32_t ix = 0u, iy = 0u;
            int32_t C[W];
            int m = 0;
            uint32_t link[W], inner = 0u;
            if (active) {
                if (RESIDENT) {
                    const uint32_t w = lq[(level & 1) * cap + qi];
                    ix = w >> 16;
                    iy = w & 0xFFFFu;
                    m = W;
#pragma unroll
                    for (int k = W - 1; k >= 0; --k) {
                        C[k] = wch[W * iy + k];
                        if (C[k] == 0x7FFF) m = k;
                    }
                    inner = winner[iy];
#pragma unroll
                    for (int k = 0; k < W; ++k) {  // the links of the children that end as leaves
                        link[k] = RG_EMPTY;
                        if (k >= m || ((inner >> k) & 1u)) continue;
                        if (C[k] < 0) {
                            link[k] = rg_leaf((uint32_t)(-C[k] - 1), 1u);
                        } else {
                            const int32_t f = first[C[k]];
                            link[k] = rg_leaf((uint32_t)f, (uint32_t)(last[C[k]] - f + 1));
                        }
                    }
                } else {
                    const uint2 item = a.q[level & 1][qi];
                    ix = item.x;
                    iy = item.y;
                    m = collapse_children<W>((int32_t)iy, left, right, int_box, C);
                    inner = collapse_links<W>(C, m, first, last, a.leaf_max, link);
                }
            }
            // queue slots: a scan of the inner-child counts over the wave, one
            // LDS add per wave
            const uint32_t nc = __popc(inner);
            uint32_t incl = nc;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            const uint32_t total = __shfl(incl, 63, 64);
            uint32_t wbase = 0u;
            if (lane == 63 && total) wbase = atomicAdd(&qcnt[(level + 1) % 3], total);
            wbase = __shfl(wbase, 63, 64);
            uint32_t slot = wbase + incl - nc;
            if (active) {
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    if (!((inner >> k) & 1u)) continue;
                    const uint32_t nn = next_base + slot;
                    if (RESIDENT) lq[((level + 1) & 1) * cap + slot] = (nn << 16) | (uint32_t)C[k];
                    else a.q[(level + 1) & 1][slot] = make_uint2(nn, (uint32_t)C[k]);
                    if (a.parents) a.parents[nn] = (ix << 3) | (uint32_t)k;
                    link[k] = nn;
                    ++slot;
                }
                write_wide_node<W>(nodes + ix, C, m, link, int_box, lbox);
            }
        }
        start = next_base;
        ++level;
        if (t == 0 && level <= RG_LEVELS_CAP) lstart[level] = start;
        __syncthreads();
    }
    // `level` levels, nodes [0, start)
    if (t == 0) {
        a.res->depth = (uint32_t)level;
        a.res->n_nodes = start;
    }
    if (a.levels && level <= RG_LEVELS_CAP)
        for (int l = t; l <= level; l += kSmallThreads) a.levels[l] = lstart[l];
}

// ------------------------------------ 5'. locally-ordered clustering
// Alternative to steps 4-5 (Meister & Bittner 2018): the Morton-sorted
// leaves start as clusters; each round every cluster finds its nearest
// neighbour within `radius` positions (distance: surface area of the union
// box, float32, ties to the smaller position), mutual nearest pairs merge
// into a new inner node at the lower position, and the clusters are compacted
// in order.  Inner nodes are numbered n-2, n-3, ... in merge order, so the
// root is 0 and children carry larger indices than their parents.
constexpr int kPlocT = 256;
constexpr int kPlocMaxRadius = 32;

__device__ inline float union_area(const float *a, const float *b) {
#pragma clang fp contract(off)
    const float dx = fmaxf(a[3], b[3]) - fminf(a[0], b[0]);
    const float dy = fmaxf(a[4], b[4]) - fminf(a[1], b[1]);
    const float dz = fmaxf(a[5], b[5]) - fminf(a[2], b[2]);
    return 2.0f * ((dx * dy + dy * dz) + dz * dx);
}

__global__ void k_ploc_init(const float *__restrict__ prim_box, const uint32_t *__restrict__ ids, int64_t n,
                            float *__restrict__ leaf_box, int32_t *__restrict__ cid, float *__restrict__ cbox) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t src = ids[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float v = prim_box[6 * (int64_t)src + k];
        leaf_box[6 * i + k] = v;
        cbox[6 * i + k] = v;
    }
    cid[i] = -(int32_t)(i + 1);
}

// nearest[i] for m clusters; the block's boxes and a halo of `radius` on each
// side are staged in LDS
__global__ void __launch_bounds__(kPlocT) k_ploc_nearest(const float *__restrict__ cbox, int64_t m, int radius,
                                                         int32_t *__restrict__ nearest) {
    __shared__ float tile[(kPlocT + 2 * kPlocMaxRadius) * 6];
    const int64_t base = (int64_t)blockIdx.x * kPlocT - radius;
    const int span = (kPlocT + 2 * radius) * 6;
    for (int t = threadIdx.x; t < span; t += kPlocT) {
        const int64_t g = base + t / 6;
        tile[t] = (g >= 0 && g < m) ? cbox[6 * g + t % 6] : 0.0f;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kPlocT + threadIdx.x;
    if (i >= m) return;
    const float *bi = tile + 6 * (threadIdx.x + radius);
    float best = INFINITY;
    int64_t bj = m;
    for (int o = -radius; o <= radius; ++o) {
        const int64_t j = i + o;
        if (o == 0 || j < 0 || j >= m) continue;
        const float d = union_area(bi, tile + 6 * (threadIdx.x + radius + o));
        if (d < best) {  // ascending j: a tie keeps the smaller position
            best = d;
            bj = j;
        }
    }
    nearest[i] = (int32_t)bj;
}

// Per block: merges (i < nearest, mutual) and kept clusters (all but the
// upper partner of a mutual pair).  counts[nb] and counts2[nb] are zeroed
// so that their exclusive scans end in the totals.
__global__ void __launch_bounds__(kPlocT) k_ploc_flags(const int32_t *__restrict__ nearest, int64_t m,
                                                       uint32_t *__restrict__ merges, uint32_t *__restrict__ keeps,
                                                       int nb) {
    __shared__ uint32_t sm[kPlocT / 64], sk[kPlocT / 64];
    const int64_t i = (int64_t)blockIdx.x * kPlocT + threadIdx.x;
    bool merge = false, keep = false;
    if (i < m) {
        const int32_t j = nearest[i];
        const bool mutual = j >= 0 && j < m && nearest[j] == (int32_t)i;
        merge = mutual && i < j;
        keep = !(mutual && i > j);
    }
    const uint64_t bm = __ballot(merge), bk = __ballot(keep);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sm[w] = (uint32_t)__popcll(bm);
        sk[w] = (uint32_t)__popcll(bk);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int k = 0; k < kPlocT / 64; ++k) {
            a += sm[k];
            b += sk[k];
        }
        merges[blockIdx.x] = a;
        keeps[blockIdx.x] = b;
        if (blockIdx.x == 0) {
            merges[nb] = 0u;
            keeps[nb] = 0u;
        }
    }
}

// Writes the next round's clusters (order kept) and the new inner nodes.
__global__ void __launch_bounds__(kPlocT) k_ploc_write(
    const int32_t *__restrict__ nearest, int64_t m, const uint32_t *__restrict__ merge_off,
    const uint32_t *__restrict__ keep_off, int64_t next_id, const int32_t *__restrict__ cid,
    const float *__restrict__ cbox, int32_t *__restrict__ out_cid, float *__restrict__ out_cbox,
    int32_t *__restrict__ left, int32_t *__restrict__ right, float *__restrict__ int_box,
    int32_t *__restrict__ parent_int, int32_t *__restrict__ parent_leaf) {
    __shared__ uint32_t sm[kPlocT / 64], sk[kPlocT / 64];
    const int64_t i = (int64_t)blockIdx.x * kPlocT + threadIdx.x;
    int32_t j = 0;
    bool merge = false, keep = false;
    if (i < m) {
        j = nearest[i];
        const bool mutual = j >= 0 && j < m && nearest[j] == (int32_t)i;
        merge = mutual && i < j;
        keep = !(mutual && i > j);
    }
    const uint64_t bm = __ballot(merge), bk = __ballot(keep);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
        sm[w] = (uint32_t)__popcll(bm);
        sk[w] = (uint32_t)__popcll(bk);
    }
    __syncthreads();
    uint32_t rm = (uint32_t)__popcll(bm & lt), rk = (uint32_t)__popcll(bk & lt);
    for (int k = 0; k < w; ++k) {
        rm += sm[k];
        rk += sk[k];
    }
    if (!keep) return;
    const int64_t at = (int64_t)keep_off[blockIdx.x] + rk;
    if (!merge) {
        out_cid[at] = cid[i];
#pragma unroll
        for (int k = 0; k < 6; ++k) out_cbox[6 * at + k] = cbox[6 * i + k];
        return;
    }
    const int32_t node = (int32_t)(next_id - (int64_t)(merge_off[blockIdx.x] + rm));
    const int32_t a = cid[i], b = cid[j];
    left[node] = a;
    right[node] = b;
    if (a < 0) parent_leaf[-a - 1] = node;
    else parent_int[a] = node;
    if (b < 0) parent_leaf[-b - 1] = node;
    else parent_int[b] = node;
    float box[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        box[k] = fminf(cbox[6 * i + k], cbox[6 * (int64_t)j + k]);
        box[3 + k] = fmaxf(cbox[6 * i + 3 + k], cbox[6 * (int64_t)j + 3 + k]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int_box[6 * (int64_t)node + k] = box[k];
        out_cbox[6 * at + k] = box[k];
    }
    out_cid[at] = node;
}

// Rank of each leaf in the tree's left-to-right order: the leaves of the
// left siblings along its path to the root come before it.  The leaf is the
// leftmost of the ancestors reached from left children only, whose leaf range
// starts at its rank.  Triangle order and leaf boxes follow the ranks.
__global__ void k_ploc_ranks(int64_t n, const int32_t *__restrict__ left, const int32_t *__restrict__ parent_int,
                             const int32_t *__restrict__ parent_leaf, const int32_t *__restrict__ size,
                             const uint32_t *__restrict__ ids, const float *__restrict__ leaf_box,
                             int32_t *__restrict__ rank, int32_t *__restrict__ first, int32_t *__restrict__ last,
                             uint32_t *__restrict__ ids_out, float *__restrict__ leaf_box_out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t me = -(int32_t)(i + 1);
    int32_t r = 0;
    int32_t c = me, p = parent_leaf[i];
    for (int64_t guard = 0; p >= 0 && guard < n; ++guard) {
        const int32_t l = left[p];
        if (l != c) r += l < 0 ? 1 : size[l];
        c = p;
        p = parent_int[p];
    }
    if (r >= n) return;  // only for an inconsistent hierarchy, which the collapse reports
    rank[i] = r;
    c = me;
    p = parent_leaf[i];
    for (int64_t guard = 0; p >= 0 && guard < n && left[p] == c; ++guard) {
        first[p] = r;
        last[p] = r + size[p] - 1;
        c = p;
        p = parent_int[p];
    }
    ids_out[r] = ids[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) leaf_box_out[6 * (int64_t)r + k] = leaf_box[6 * i + k];
}

// Leaf children re-encoded by rank.
__global__ void k_ploc_relabel(int64_t n, int32_t *__restrict__ left, int32_t *__restrict__ right,
                               const int32_t *__restrict__ rank) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (x >= n - 1) return;
    const int32_t a = left[x], b = right[x];
    if (a < 0) left[x] = -(rank[-a - 1] + 1);
    if (b < 0) right[x] = -(rank[-b - 1] + 1);
}

// ------------------------------------ 5''. treelet restructuring
// Karras & Aila 2013 over the binary hierarchy.  A round visits every inner
// node with at least three leaves below it after the nodes below it (a node
// with two leaf children has one topology and is skipped): depths from the
// root are taken when the round begins, deepest first, one launch per depth
// and one wave per node; nodes of one depth have disjoint subtrees, and a
// restructure never changes the set of leaves below its node, so the result
// is that of any order that puts every node after those below it.
// The treelet starts as the node's children; its inner leaf of largest
// surface area (first on ties) is replaced in place by its left child and its
// right child appended, up to kTreelet leaves.  The topology of least total
// surface area comes from a dynamic program over the leaf subsets (float32,
// no fused multiply-add, splits holding the subset's lowest leaf tried in
// increasing bit order, the first minimum kept); the node keeps its index and
// the other inner nodes take the opened nodes' indices, ascending, in
// pre-order (left subtree first).
constexpr int kTreelet = 7;
constexpr int kTreeletMaxRounds = 8;

// The 127 non-empty subsets of 7 leaves ordered by size, then by value, and
// where each size starts.  Subsets within the low m bits precede the others
// of their size, so for a treelet of m leaves the subsets of size k are the
// first C(m, k) entries of block k.
struct TreeletSubsets {
    uint8_t s[(1 << kTreelet) - 1];
    uint8_t off[kTreelet + 2];
    uint8_t binom[kTreelet + 1][kTreelet + 1];
};

constexpr int popc_const(int v) { return v ? (v & 1) + popc_const(v >> 1) : 0; }

constexpr TreeletSubsets make_treelet_subsets() {
    TreeletSubsets t{};
    int n = 0;
    for (int k = 1; k <= kTreelet; ++k) {
        t.off[k] = (uint8_t)n;
        for (int S = 1; S < (1 << kTreelet); ++S)
            if (popc_const(S) == k) t.s[n++] = (uint8_t)S;
    }
    t.off[kTreelet + 1] = (uint8_t)n;
    for (int m = 0; m <= kTreelet; ++m)
        for (int k = 0; k <= kTreelet; ++k) {
            int c = 0;
            for (int S = 0; S < (1 << m); ++S) c += popc_const(S) == k;
            t.binom[m][k] = (uint8_t)c;
        }
    return t;
}

__constant__ TreeletSubsets kSubsets = make_treelet_subsets();

// The j-th subset of `mask` in increasing order: the bits of j placed on the
// set bits of mask, lowest first.
__device__ inline uint32_t deposit(uint32_t j, uint32_t mask) {
    uint32_t r = 0u;
    for (uint32_t b = mask; b; b &= b - 1u, j >>= 1)
        if (j & 1u) r |= b & (0u - b);
    return r;
}

__device__ inline float area32(const float *lo, const float *hi) {
#pragma clang fp contract(off)
    const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0f * ((dx * dy + dy * dz) + dz * dx);
}

// Depth of every inner node (the root 0) by walking its parent links, and
// the count of nodes per depth; counts of depths below kDepthBins are summed
// per block in LDS first, so the global counters take one atomic per block
// and depth.
constexpr int kDepthBins = 256;

__global__ void __launch_bounds__(kThreads) k_depths(int64_t m, const int32_t *__restrict__ parent_int,
                                                     int32_t *__restrict__ depth, uint32_t *hcount, uint32_t *hmax) {
    __shared__ uint32_t bins[kDepthBins];
    __shared__ uint32_t bmax;
    for (int k = threadIdx.x; k < kDepthBins; k += blockDim.x) bins[k] = 0u;
    if (threadIdx.x == 0) bmax = 0u;
    __syncthreads();
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (x < m) {
        int32_t d = 0, p = parent_int[x];
        // a consistent tree has fewer than m inner nodes above any node
        for (; p >= 0 && p < m && d < m; p = parent_int[p]) ++d;
        depth[x] = d;
        if (d < kDepthBins) atomicAdd(&bins[d], 1u);
        else if (d < m) atomicAdd(&hcount[d], 1u);
        atomicMax(&bmax, (uint32_t)d);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kDepthBins; k += blockDim.x)
        if (bins[k]) atomicAdd(&hcount[k], bins[k]);
    if (threadIdx.x == 0) atomicMax(hmax, bmax);
}

// Inner nodes grouped by depth: order[hstart[d] ...] holds depth d (in no
// particular order within a depth).  Positions are handed out per block and
// depth, then per node within the block.
__global__ void __launch_bounds__(kThreads) k_depth_scatter(int64_t m, const int32_t *__restrict__ depth,
                                                            const uint32_t *__restrict__ hstart, uint32_t *hcursor,
                                                            int32_t dmax, int32_t *__restrict__ order) {
    __shared__ uint32_t bins[kDepthBins], base[kDepthBins];
    for (int k = threadIdx.x; k < kDepthBins; k += blockDim.x) bins[k] = 0u;
    __syncthreads();
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t d = -1;
    uint32_t local = 0u;
    if (x < m) {
        d = depth[x];
        if (d < 0 || d > dmax) d = -1;  // never once the host has checked the counts
        else if (d < kDepthBins) local = atomicAdd(&bins[d], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kDepthBins; k += blockDim.x)
        if (bins[k]) base[k] = atomicAdd(&hcursor[k], bins[k]);
    __syncthreads();
    if (d < 0) return;
    const uint32_t at = d < kDepthBins ? base[d] + local : atomicAdd(&hcursor[d], 1u);
    order[hstart[d] + at] = (int32_t)x;
}

// Per-depth pass over the nodes of one depth (order[0 .. count)), run
// deepest first: the children of a node are deeper, so their sizes are final.
__global__ void k_sizes_at(const int32_t *__restrict__ order, int64_t count, const int32_t *__restrict__ left,
                           const int32_t *__restrict__ right, int32_t *size) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int32_t x = order[i];
    const int32_t a = left[x], b = right[x];
    size[x] = (a < 0 ? 1 : size[a]) + (b < 0 ? 1 : size[b]);
}

__global__ void k_leaf_boxes(const float *__restrict__ prim_box, const uint32_t *__restrict__ ids, int64_t n,
                             float *__restrict__ leaf_box) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t src = ids[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) leaf_box[6 * i + k] = prim_box[6 * (int64_t)src + k];
}

// ---------------------------------------------- inner boxes from ranges
// Every inner node of the radix tree covers a contiguous range of leaves
// (first .. last, leaf order), and its box is the union of their boxes.  The
// unions come from three tables, so the boxes are computed in three kinds of
// launches with no dependence on the tree's depth: per block of
// kRangeLeaves leaves, the prefix and the suffix unions inside the block;
// a sparse table over the blocks (level j: the union of 2^j consecutive
// blocks); then one thread per inner node combines at most four entries (or
// loops over the at most kRangeLeaves leaves of a range inside one block).
// min / max are exact, so the boxes are the same as any order of unions.
constexpr int kRangeLeaves = 16;

__device__ inline void box_union(float u[6], const float *__restrict__ b) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        u[k] = fminf(u[k], b[k]);
        u[3 + k] = fmaxf(u[3 + k], b[3 + k]);
    }
}

__global__ void __launch_bounds__(kThreads) k_range_blocks(const float *__restrict__ leaf_box, int64_t n,
                                                           float *__restrict__ pre, float *__restrict__ suf,
                                                           float *__restrict__ table) {
    __shared__ float b[kThreads * 6];
    const int t = threadIdx.x;
    const int64_t i = blockIdx.x * (int64_t)kThreads + t;
#pragma unroll
    for (int k = 0; k < 6; ++k) b[6 * t + k] = i < n ? leaf_box[6 * i + k] : (k < 3 ? INFINITY : -INFINITY);
    __syncthreads();
    if (i >= n) return;
    const int g0 = t & ~(kRangeLeaves - 1), r = t & (kRangeLeaves - 1);
    float p[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    float q[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k <= r; ++k) box_union(p, b + 6 * (g0 + k));
    for (int k = r; k < kRangeLeaves; ++k) box_union(q, b + 6 * (g0 + k));  // past n: empty boxes
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        pre[6 * i + k] = p[k];
        suf[6 * i + k] = q[k];
    }
    if (r == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) table[6 * (i / kRangeLeaves) + k] = q[k];  // the whole block
    }
}

// Levels j0 + 1 .. j0 + kRangeStride of the sparse table over nb blocks
// from level j0 (one launch): entry b of level j0 + r (b + 2^(j0 + r) <= nb)
// is the union of level j0's entries b + k 2^j0, k < 2^r.  Thread
// (r - 1, b).
constexpr int kRangeStride = 4;
__global__ void k_range_levels(float *table, int64_t nb, int j0, int top) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int r = (int)(x / nb) + 1;
    const int64_t b = x % nb;
    const int j = j0 + r;
    if (r > kRangeStride || j > top || b + (1ll << j) > nb) return;
    const int64_t step = 1ll << j0;
    const float *src = table + 6 * ((int64_t)j0 * nb + b);
    float u[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < (1 << r); ++k) box_union(u, src + 6 * step * k);
    float *y = table + 6 * ((int64_t)j * nb + b);
#pragma unroll
    for (int k = 0; k < 6; ++k) y[k] = u[k];
}

__global__ void k_range_boxes(const int32_t *__restrict__ first, const int32_t *__restrict__ last, int64_t m,
                              const float *__restrict__ leaf_box, const float *__restrict__ pre,
                              const float *__restrict__ suf, const float *__restrict__ table, int64_t nb,
                              float *__restrict__ int_box) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t f = first[i], l = last[i];
    const int32_t bf = f / kRangeLeaves, bl = l / kRangeLeaves;
    float u[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (bf == bl) {
        for (int32_t k = f; k <= l; ++k) box_union(u, leaf_box + 6 * (int64_t)k);
    } else {
        box_union(u, suf + 6 * (int64_t)f);
        box_union(u, pre + 6 * (int64_t)l);
        if (bl - bf >= 2) {  // whole blocks bf + 1 .. bl - 1: two overlapping table entries
            const int32_t a = bf + 1, len = bl - 1 - a + 1;
            const int j = 31 - __clz(len);
            box_union(u, table + 6 * ((int64_t)j * nb + a));
            box_union(u, table + 6 * ((int64_t)j * nb + (a + len - (1 << j))));
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) int_box[6 * i + k] = u[k];
}

int64_t range_levels(int64_t nb) {
    int64_t L = 1;
    while ((1ll << L) <= nb) ++L;
    return L;  // levels 0 .. L - 1: 2^(L-1) <= nb
}

__global__ void __launch_bounds__(64) k_treelet(const int32_t *__restrict__ order, int32_t *left, int32_t *right,
                                                int32_t *parent_int, int32_t *parent_leaf, float *int_box,
                                                const float *__restrict__ leaf_box) {
    __shared__ float ulo[1 << kTreelet][3], uhi[1 << kTreelet][3];
    __shared__ float area[1 << kTreelet], cost[1 << kTreelet];
    __shared__ uint8_t split[1 << kTreelet];
    __shared__ int32_t leaves[kTreelet], opened[kTreelet];
    __shared__ float lbox[kTreelet][6], larea[kTreelet];
    __shared__ int n_leaves, n_opened;
    const int lane = threadIdx.x;
    const int32_t node = order[blockIdx.x];
    if (left[node] < 0 && right[node] < 0) return;  // two leaves: one topology, nothing to change
    if (lane == 0) {
        // Each treelet leaf's box and area are read once, when it joins, and
        // kept in LDS: a growth step then waits on two loads (the opened
        // node's children, then both their boxes) whatever the leaf count.
        auto join = [&](int k0, int32_t c0, int k1, int32_t c1) {
            const float *p0 = c0 < 0 ? leaf_box + 6 * (int64_t)(-c0 - 1) : int_box + 6 * (int64_t)c0;
            const float *p1 = c1 < 0 ? leaf_box + 6 * (int64_t)(-c1 - 1) : int_box + 6 * (int64_t)c1;
            float b0[6], b1[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                b0[q] = p0[q];
                b1[q] = p1[q];
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                lbox[k0][q] = b0[q];
                lbox[k1][q] = b1[q];
            }
            leaves[k0] = c0;
            leaves[k1] = c1;
            larea[k0] = area32(b0, b0 + 3);
            larea[k1] = area32(b1, b1 + 3);
        };
        int m = 2, r = 0;
        join(0, left[node], 1, right[node]);
        while (m < kTreelet) {
            int bk = -1;
            float ba = -INFINITY;
            for (int k = 0; k < m; ++k) {
                if (leaves[k] < 0) continue;   // a primitive cannot be opened
                if (larea[k] > ba) {
                    ba = larea[k];
                    bk = k;
                }
            }
            if (bk < 0) break;
            const int32_t c = leaves[bk];
            opened[r++] = c;
            join(bk, left[c], m, right[c]);
            ++m;
        }
        for (int k = 1; k < r; ++k)  // ascending: the order the indices are handed out in
            for (int q = k; q > 0 && opened[q - 1] > opened[q]; --q) {
                const int32_t t = opened[q];
                opened[q] = opened[q - 1];
                opened[q - 1] = t;
            }
        n_leaves = m;
        n_opened = r;
    }
    __syncthreads();
    const int m = n_leaves;
    const uint32_t full = (1u << m) - 1u;
    for (uint32_t S = (uint32_t)lane + 1u; S <= full; S += 64u) {
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < m; ++k) {
            if (!((S >> k) & 1u)) continue;
            const float *b = lbox[k];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                lo[q] = fminf(lo[q], b[q]);
                hi[q] = fmaxf(hi[q], b[3 + q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            ulo[S][q] = lo[q];
            uhi[S][q] = hi[q];
        }
        area[S] = area32(lo, hi);
        cost[S] = 0.0f;
        split[S] = 0;
    }
    __syncthreads();
    // Subsets of one size at a time.  A subset S splits into P (holding its
    // lowest leaf) and S \ P; P = low | Q for the proper subsets Q of the rest,
    // Q the j-th in increasing order.  The first cheapest split in that order
    // is kept.  The subsets of a size share the wave: g lanes per subset,
    // each taking every g-th j, then the least (cost, j) over the group.
    for (int k = 2; k <= m; ++k) {
        const int nk = kSubsets.binom[m][k];
        const uint32_t np = (1u << (k - 1)) - 1u;   // splits of a k-subset
        int g = 1;
        while (2 * g * nk <= 64 && (uint32_t)g < np) g *= 2;
        const int si = lane / g, part = lane % g;
        uint32_t S = 0u, low = 0u, rest = 0u, bj = 0xFFFFFFFFu;
        float best = INFINITY;
        if (si < nk) {
            S = kSubsets.s[kSubsets.off[k] + si];
            low = S & (0u - S);
            rest = S ^ low;
            for (uint32_t j = (uint32_t)part; j < np; j += (uint32_t)g) {
                const uint32_t P = low | deposit(j, rest);
                const float v = cost[P] + cost[S ^ P];
                if (v < best) {
                    best = v;
                    bj = j;
                }
            }
        }
        for (int d = 1; d < g; d <<= 1) {
            const float ov = __shfl_xor(best, d);
            const uint32_t oj = __shfl_xor(bj, d);
            if (ov < best || (ov == best && oj < bj)) {
                best = ov;
                bj = oj;
            }
        }
        if (si < nk && part == 0) {
            cost[S] = area[S] + best;
            split[S] = (uint8_t)(bj == 0xFFFFFFFFu ? 0u : (low | deposit(bj, rest)));
        }
        __syncthreads();
    }
    if (lane != 0) return;
    // rebuild: entries (subset, parent, side) popped in pre-order; the stack
    // lives in LDS, which keeps the kernel's registers low enough for more
    // waves per SIMD (the walk is one lane's)
    __shared__ uint32_t st_set[2 * kTreelet];
    __shared__ int32_t st_parent[2 * kTreelet];
    __shared__ int32_t st_side[2 * kTreelet];
    int sp = 0, next = 0;
    st_set[sp] = full ^ split[full]; st_parent[sp] = node; st_side[sp] = 1; ++sp;
    st_set[sp] = split[full]; st_parent[sp] = node; st_side[sp] = 0; ++sp;
    while (sp > 0) {
        --sp;
        const uint32_t T = st_set[sp];
        const int32_t parent = st_parent[sp];
        const int side = st_side[sp];
        int32_t child;
        if ((T & (T - 1u)) == 0u) {
            child = leaves[__ffs((int)T) - 1];
        } else {
            if (next >= n_opened || sp + 2 > 2 * kTreelet) return;  // never: m - 2 opened nodes, depth < m
            child = opened[next++];
            float *b = int_box + 6 * (int64_t)child;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                b[q] = ulo[T][q];
                b[3 + q] = uhi[T][q];
            }
            st_set[sp] = T ^ split[T]; st_parent[sp] = child; st_side[sp] = 1; ++sp;
            st_set[sp] = split[T]; st_parent[sp] = child; st_side[sp] = 0; ++sp;
        }
        if (side == 0) left[parent] = child;
        else right[parent] = child;
        if (child < 0) parent_leaf[-child - 1] = parent;
        else parent_int[child] = parent;
    }
}

// ------------------------------------------------------ reordering
// An index out of range reads vertex 0 instead (the input check then fails
// the call; a build in one workgroup reorders before the check is read).
__global__ void k_reorder_tris(const float *__restrict__ verts, int64_t n_verts, const uint32_t *__restrict__ idx,
                               const uint32_t *__restrict__ ids, int64_t n, const uint16_t *__restrict__ pm,
                               RgTri *__restrict__ tris, uint16_t *__restrict__ mats, uint32_t *__restrict__ slots) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t s = ids[i];
    RgTri t;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        uint32_t vi = idx[3 * (int64_t)s + v];
        if ((int64_t)vi >= n_verts) vi = 0u;
#pragma unroll
        for (int k = 0; k < 3; ++k) t.v[3 * v + k] = verts[3 * (int64_t)vi + k];
    }
    t.prim = s;
    tris[i] = t;
    mats[i] = pm ? pm[s] : (uint16_t)0;
    slots[s] = (uint32_t)i;
}

// root: the root box (lo xyz, hi xyz) as the build left it on the device
__global__ void k_blas_header(RgBlasHdr *h, uint64_t nodes, uint64_t tris, uint64_t mats, uint64_t slots,
                              const float *root) {
    h->nodes = nodes;
    h->tris = tris;
    h->mats = mats;
    h->slots = slots;
    h->lo[0] = root[0]; h->lo[1] = root[1]; h->lo[2] = root[2];
    h->hi[0] = root[3]; h->hi[1] = root[4]; h->hi[2] = root[5];
    h->status = 0u;
    h->pad = 0u;
    h->alpha = 0ull;
    h->alpha_level = 0u;
}

__global__ void k_blas_alpha(RgBlasHdr *h, uint64_t alpha, uint32_t level) {
    h->alpha = alpha;
    h->alpha_level = level;
}

// --------------------------------------------------------------- refit
// Built bottom levels over new positions of the same triangles keep their
// hierarchies: the leaf-order triangle copies are rewritten, then every box
// is recomputed bottom-up.  Boxes are min / max of vertex coordinates, which
// are exact, so refitting to unchanged vertices reproduces the build bit for
// bit.  Several bottom levels are refitted together: each launch covers one
// level of every one of them (blockIdx.y picks the bottom level), so the
// per-launch latency of a level is paid once for the whole set.
constexpr int kRefitBatch = 32;
struct RefitJob {
    void *nodes;
    RgTri *tris;
    const uint32_t *levels, *parents;
    RgBlasHdr *hdr;
    const float *verts;
    const uint32_t *idx;
    int64_t n_verts, n_tris;
    int32_t depth, pad;
};
struct RefitJobs {
    RefitJob j[kRefitBatch];
};

__global__ void k_refit_begin(RefitJobs jobs, int n) {
    if ((int)threadIdx.x < n) jobs.j[threadIdx.x].hdr->status = 0u;
}

// New leaf-order triangle copies; an index out of range or a non-finite
// coordinate sets the header's status word (flags as for k_tri_boxes) and
// leaves that triangle as it was.
__global__ void k_refit_tris(RefitJobs jobs) {
    const RefitJob &J = jobs.j[blockIdx.y];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < J.n_tris;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t prim = J.tris[s].prim;
        uint32_t bad = 0;
        uint32_t v3[3] = {0u, 0u, 0u};
        if ((int64_t)prim >= J.n_tris) {
            bad |= 1u;
        } else {
            v3[0] = J.idx[3 * (int64_t)prim];
            v3[1] = J.idx[3 * (int64_t)prim + 1];
            v3[2] = J.idx[3 * (int64_t)prim + 2];
            if ((int64_t)v3[0] >= J.n_verts || (int64_t)v3[1] >= J.n_verts || (int64_t)v3[2] >= J.n_verts) {
                bad |= 1u;
                v3[0] = v3[1] = v3[2] = 0u;
            }
        }
        float v[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k) v[3 * a + k] = J.verts[3 * (int64_t)v3[a] + k];
#pragma unroll
        for (int k = 0; k < 9; ++k)
            if (!isfinite(v[k])) bad |= 2u;
        if (bad) {
            atomicOr(&J.hdr->status, bad);
            continue;
        }
        // the 40-byte record (nine coordinates, then prim unchanged) as five
        // 8-byte stores: records are 8-byte aligned
        uint2 *dst = reinterpret_cast<uint2 *>(&J.tris[s]);
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[k] = make_uint2(__float_as_uint(v[2 * k]), __float_as_uint(v[2 * k + 1]));
        dst[4] = make_uint2(__float_as_uint(v[8]), prim);
    }
}

// Stores W floats at a 16-byte aligned address with 16-byte stores (W >= 4)
// or one 8-byte store (W = 2).
template <int W>
__device__ inline void store_row(float *dst, const float *v) {
    if constexpr (W == 2) {
        *reinterpret_cast<float2 *>(dst) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int q = 0; q < W; q += 4)
            *reinterpret_cast<float4 *>(dst + q) = make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]);
    }
}

// Level `level` (counted from the root) of every bottom level deep enough,
// its node range from the level table, deepest levels first (launch order
// orders them; no atomics).  Each node's inner children have already put
// their boxes into its rows (one launch earlier, see below); the node
// computes the boxes of its leaf children from their triangles, writes its
// rows back if it has any leaf child (vector stores), and puts the union of
// its child boxes into its own slot of its parent's rows: so a level reads
// only its own nodes, not its children's.  The root's union goes to the
// header.  Boxes are min / max of coordinates, exact in any order.
template <int W>
__device__ inline void refit_node(const RefitJob &J, RgNode<W> *nodes, uint32_t x) {
    {
        RgNode<W> &nd = nodes[x];
        float bx[6][W];
        uint32_t ch[W];
        bool any_leaf = false;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            ch[k] = nd.child[k];
            bx[0][k] = nd.lo_x[k]; bx[1][k] = nd.lo_y[k]; bx[2][k] = nd.lo_z[k];
            bx[3][k] = nd.hi_x[k]; bx[4][k] = nd.hi_y[k]; bx[5][k] = nd.hi_z[k];
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const uint32_t c = ch[k];
            if (c == RG_EMPTY || !rg_is_leaf(c)) continue;
            any_leaf = true;
            float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
            const uint32_t first = rg_leaf_first(c), cnt = rg_leaf_count(c);
            for (uint32_t j = 0; j < cnt; ++j) {
                const RgTri &t = J.tris[first + j];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    b[a] = fminf(b[a], fminf(fminf(t.v[a], t.v[3 + a]), t.v[6 + a]));
                    b[3 + a] = fmaxf(b[3 + a], fmaxf(fmaxf(t.v[a], t.v[3 + a]), t.v[6 + a]));
                }
            }
#pragma unroll
            for (int a = 0; a < 6; ++a) bx[a][k] = b[a];
        }
        float u[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (ch[k] == RG_EMPTY) continue;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u[a] = fminf(u[a], bx[a][k]);
                u[3 + a] = fmaxf(u[3 + a], bx[3 + a][k]);
            }
        }
        if (any_leaf) {
            store_row<W>(nd.lo_x, bx[0]);
            store_row<W>(nd.lo_y, bx[1]);
            store_row<W>(nd.lo_z, bx[2]);
            store_row<W>(nd.hi_x, bx[3]);
            store_row<W>(nd.hi_y, bx[4]);
            store_row<W>(nd.hi_z, bx[5]);
        }
        const uint32_t p = J.parents[x];
        if (p == RG_MISS) {  // the root
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                J.hdr->lo[k] = u[k];
                J.hdr->hi[k] = u[3 + k];
            }
        } else {
            RgNode<W> &pd = nodes[p >> 3];
            const uint32_t ps = p & 7u;
            pd.lo_x[ps] = u[0]; pd.lo_y[ps] = u[1]; pd.lo_z[ps] = u[2];
            pd.hi_x[ps] = u[3]; pd.hi_y[ps] = u[4]; pd.hi_z[ps] = u[5];
        }
    }
}

template <int W>
__global__ void k_refit_level(RefitJobs jobs, int level) {
    const RefitJob &J = jobs.j[blockIdx.y];
    if (level >= J.depth) return;
    RgNode<W> *nodes = reinterpret_cast<RgNode<W> *>(J.nodes);
    const uint32_t lo = J.levels[level], hi = J.levels[level + 1];
    for (uint32_t x = lo + blockIdx.x * blockDim.x + threadIdx.x; x < hi; x += gridDim.x * blockDim.x)
        refit_node<W>(J, nodes, x);
}

// The levels near the root hold few nodes (at most W^l at level l), too few
// to fill the GPU, yet a launch per level costs its start and end: levels
// top - 1 .. 0 of every bottom level are refitted in one launch, one
// workgroup per bottom level stepping up to the root with a workgroup
// barrier between levels.  A level's writes into its parents' rows are read
// by the next level's threads of the same workgroup after the barrier.
constexpr int kRefitTopThreads = 1024;
constexpr uint32_t kRefitTopNodes = 4096;  // the widest level the one-workgroup launch takes (W^l)
template <int W>
__global__ void __launch_bounds__(kRefitTopThreads) k_refit_top(RefitJobs jobs, int top) {
    const RefitJob &J = jobs.j[blockIdx.x];
    RgNode<W> *nodes = reinterpret_cast<RgNode<W> *>(J.nodes);
    for (int level = top - 1; level >= 0; --level) {
        if (level < J.depth) {  // the same for the whole workgroup
            const uint32_t lo = J.levels[level], hi = J.levels[level + 1];
            for (uint32_t x = lo + threadIdx.x; x < hi; x += blockDim.x) refit_node<W>(J, nodes, x);
        }
        __syncthreads();
    }
}

// Hierarchies deeper than the level table: bottom-up with arrival counters.
// The boxes of each node's leaf children and the number of inner children
// the node waits for before its own box is known.
template <int W>
__global__ void k_refit_leaves(RgNode<W> *__restrict__ nodes, int64_t n_nodes, const RgTri *__restrict__ tris,
                               uint32_t *__restrict__ need, uint32_t *__restrict__ arrived) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (x >= n_nodes) return;
    RgNode<W> &nd = nodes[x];
    uint32_t inner = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const uint32_t c = nd.child[k];
        if (c == RG_EMPTY) continue;
        if (!rg_is_leaf(c)) {
            ++inner;
            continue;
        }
        const uint32_t first = rg_leaf_first(c), cnt = rg_leaf_count(c);
        float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (uint32_t j = 0; j < cnt; ++j) {
            const RgTri &t = tris[first + j];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                b[a] = fminf(b[a], fminf(fminf(t.v[a], t.v[3 + a]), t.v[6 + a]));
                b[3 + a] = fmaxf(b[3 + a], fmaxf(fmaxf(t.v[a], t.v[3 + a]), t.v[6 + a]));
            }
        }
        nd.lo_x[k] = b[0]; nd.lo_y[k] = b[1]; nd.lo_z[k] = b[2];
        nd.hi_x[k] = b[3]; nd.hi_y[k] = b[4]; nd.hi_z[k] = b[5];
    }
    need[x] = inner;
    arrived[x] = 0u;
}

// From the nodes without inner children upwards: a node whose children are
// all final writes the union of its child boxes into its parent's slot; the
// last child to arrive at a parent continues with the parent (acquire /
// release at agent scope).  The root's box goes to the header.
template <int W>
__global__ void k_refit_up(RgNode<W> *nodes, int64_t n_nodes, const uint32_t *__restrict__ parents,
                           const uint32_t *__restrict__ need, uint32_t *arrived, RgBlasHdr *hdr) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (x >= n_nodes || need[x] != 0u) return;
    uint32_t node = (uint32_t)x;
    for (int64_t guard = 0; guard <= n_nodes; ++guard) {
        const RgNode<W> &nd = nodes[node];
        float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (nd.child[k] == RG_EMPTY) continue;
            b[0] = fminf(b[0], nd.lo_x[k]); b[1] = fminf(b[1], nd.lo_y[k]); b[2] = fminf(b[2], nd.lo_z[k]);
            b[3] = fmaxf(b[3], nd.hi_x[k]); b[4] = fmaxf(b[4], nd.hi_y[k]); b[5] = fmaxf(b[5], nd.hi_z[k]);
        }
        const uint32_t p = parents[node];
        if (p == RG_MISS) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                hdr->lo[k] = b[k];
                hdr->hi[k] = b[3 + k];
            }
            return;
        }
        const uint32_t pn = p >> 3, ps = p & 7u;
        if ((int64_t)pn >= n_nodes || ps >= (uint32_t)W) return;  // never for a structure this library built
        RgNode<W> &pd = nodes[pn];
        pd.lo_x[ps] = b[0]; pd.lo_y[ps] = b[1]; pd.lo_z[ps] = b[2];
        pd.hi_x[ps] = b[3]; pd.hi_y[ps] = b[4]; pd.hi_z[ps] = b[5];
        const uint32_t old = __hip_atomic_fetch_add(&arrived[pn], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u < need[pn]) return;  // a sibling subtree is still being refitted
        node = pn;
    }
}

template <int W>
void refit_levels(const RefitJobs &jobs, int n, int max_depth, unsigned blocks, hipStream_t st) {
    // levels 0 .. top - 1 hold at most W^(top - 1) <= kRefitTopNodes nodes
    int top = 1;
    for (uint64_t c = W; c <= kRefitTopNodes && top < max_depth; c *= W) ++top;
    for (int l = max_depth - 1; l >= top; --l)
        k_refit_level<W><<<dim3(blocks, (unsigned)n), kThreads, 0, st>>>(jobs, l);
    k_refit_top<W><<<(unsigned)n, kRefitTopThreads, 0, st>>>(jobs, top);
}

template <int W>
void refit_deep(const rg_blas &b, uint32_t *need, uint32_t *arrived, hipStream_t st) {
    char *base = (char *)b.buf;
    RgNode<W> *nd = reinterpret_cast<RgNode<W> *>(base + b.nodes_off);
    const RgTri *tris = (const RgTri *)(base + b.tris_off);
    const uint32_t *parents = (const uint32_t *)(base + b.parents_off);
    k_refit_leaves<W><<<rg_blocks(b.n_nodes, kThreads), kThreads, 0, st>>>(nd, b.n_nodes, tris, need, arrived);
    k_refit_up<W><<<rg_blocks(b.n_nodes, kThreads), kThreads, 0, st>>>(nd, b.n_nodes, parents, need, arrived,
                                                                         (RgBlasHdr *)base);
}

// ----------------------------------------------------------- top level
__global__ void k_reorder_inst(const RgInst *__restrict__ in, const uint32_t *__restrict__ ids, int64_t n,
                               RgInst *__restrict__ out, uint32_t *__restrict__ rec_of) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = in[ids[i]];
    rec_of[ids[i]] = (uint32_t)i;
}

int node_bytes(int w) { return 32 * w; }

struct Opts {
    int32_t w, leaf, builder, radius, bits;
    int32_t key_shift() const { return bits == 10 ? 33 : 0; }  // the 30-bit key: top bits of the 63-bit one
    bool fits(int64_t n) const { return bits != 10 || n <= RG_MORTON_BITS_COMPACT_MAX_PRIMS; }
};

bool opts_ok(const rg_build_opts *o, Opts *out) {
    Opts r{4, 4, RG_BUILDER_LBVH, 0, 21};
    if (o) r = Opts{o->width, o->leaf_max, o->builder, o->radius, o->morton_bits == 0 ? 21 : o->morton_bits};
    if (!(r.bits == 21 || r.bits == 10)) return false;
    if (!(r.w == 2 || r.w == 4 || r.w == 8)) return false;
    if (r.leaf < 1 || r.leaf > 8) return false;
    if (r.builder == RG_BUILDER_TREELET) {
        if (r.radius == 0) r.radius = RG_TREELET_ROUNDS_DEFAULT;
        if (r.radius < 1 || r.radius > kTreeletMaxRounds) return false;
    } else {
        if (r.builder != RG_BUILDER_LBVH && r.builder != RG_BUILDER_PLOC) return false;
        if (r.radius == 0) r.radius = RG_PLOC_RADIUS_DEFAULT;
        if (r.radius < 1 || r.radius > kPlocMaxRadius) return false;
    }
    *out = r;
    return true;
}

uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t(255); }

struct LbvhScratch {
    float *leaf_box, *int_box;
    uint64_t *keys, *keys2;
    uint32_t *ids, *ids2, *qcount, *flags;
    // sort: the digit counts of the eight passes (kCountCopies x 2048,
    // cleared by k_centre_bounds), per-tile digit counts of one pass
    uint32_t *sortz, *count, *cnt;
    int64_t sortz_words;
    float *part;  // centre-bound partials, 6 per block of k_centre_bounds
    int32_t *left, *right, *pint, *pleaf, *first, *last;
    uint2 *q0, *q1;
    int32_t *wch;       // wide-node plan: W children, W links per inner node (W up to 8), inner masks
    uint32_t *wlink;
    uint8_t *winner;
    // clustering only
    int32_t *cid[2], *nearest, *rank, *size;
    float *cbox[2];
    uint32_t *n_merge, *n_keep;
    // inner nodes grouped by depth (depth, order, counts); treelet
    // restructuring also takes rank, size and cbox[0]
    int32_t *height, *order;
    uint32_t *hcount, *hcursor, *hstart, *hmax;
    // inner boxes from leaf ranges (radix tree): prefix / suffix unions,
    // sparse table over blocks of kRangeLeaves leaves
    float *pre, *suf, *rtab;
    SmallResult *small;  // summary of a one-workgroup build
};

bool carve(RgArena &a, int64_t n, int32_t builder, LbvhScratch &s) {
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    int64_t ni = n > 1 ? n - 1 : 1;
    s.leaf_box = a.take<float>(6 * n);
    s.int_box = a.take<float>(6 * ni);
    s.keys = a.take<uint64_t>(n);
    s.keys2 = a.take<uint64_t>(n);
    s.ids = a.take<uint32_t>(n);
    s.ids2 = a.take<uint32_t>(n);
    s.sortz_words = 2048 * kCountCopies;
    s.sortz = a.take<uint32_t>(s.sortz_words);
    s.count = s.sortz;
    s.cnt = a.take<uint32_t>(256 * nb);
    s.part = a.take<float>(6 * kBoundParts);
    s.qcount = a.take<uint32_t>(2 * kCollapseRing + 8);
    s.flags = a.take<uint32_t>(8);
    s.left = a.take<int32_t>(ni);
    s.right = a.take<int32_t>(ni);
    s.pint = a.take<int32_t>(ni);
    s.pleaf = a.take<int32_t>(n);
    s.first = a.take<int32_t>(ni);
    s.last = a.take<int32_t>(ni);
    s.q0 = a.take<uint2>(ni);
    s.q1 = a.take<uint2>(ni);
    s.wch = a.take<int32_t>(8 * ni);
    s.wlink = a.take<uint32_t>(8 * ni);
    s.winner = a.take<uint8_t>(ni);
    if (builder == RG_BUILDER_PLOC) {
        int64_t pb = (n + kPlocT - 1) / kPlocT + 1;
        for (int k = 0; k < 2; ++k) {
            s.cid[k] = a.take<int32_t>(n);
            s.cbox[k] = a.take<float>(6 * n);
        }
        s.nearest = a.take<int32_t>(n);
        s.rank = a.take<int32_t>(n);
        s.size = a.take<int32_t>(ni);
        s.n_merge = a.take<uint32_t>(pb);
        s.n_keep = a.take<uint32_t>(pb);
    }
    if (builder == RG_BUILDER_TREELET) {
        s.cbox[0] = a.take<float>(6 * n);
        s.rank = a.take<int32_t>(n);
        s.size = a.take<int32_t>(ni);
    }
    s.height = a.take<int32_t>(ni);
    s.order = a.take<int32_t>(ni);
    s.hcount = a.take<uint32_t>(n + 1);
    s.hcursor = a.take<uint32_t>(n + 1);
    s.hstart = a.take<uint32_t>(n + 1);
    s.hmax = a.take<uint32_t>(8);
    if (builder != RG_BUILDER_PLOC) {
        const int64_t nbr = (n + kRangeLeaves - 1) / kRangeLeaves;
        s.pre = a.take<float>(6 * n);
        s.suf = a.take<float>(6 * n);
        s.rtab = a.take<float>(6 * nbr * range_levels(nbr));
    }
    s.small = a.take<SmallResult>(1);
    return !a.overflow();
}

// The m >= 1 inner nodes of the binary hierarchy in s grouped by depth from
// the root: s.order[start[d] .. start[d] + cnt[d]) holds depth d.
struct DepthOrder {
    uint32_t dmax = 0;
    std::vector<uint32_t> cnt, start;
};

rg_status depth_order(LbvhScratch &s, int64_t m, hipStream_t st, DepthOrder &o) {
    k_fill_u32<<<rg_blocks(m + 2, kThreads), kThreads, 0, st>>>(s.hcount, 0u, m + 2);
    k_fill_u32<<<1, 64, 0, st>>>(s.hmax, 0u, 1);
    k_depths<<<rg_blocks(m, kThreads), kThreads, 0, st>>>(m, s.pint, s.height, s.hcount, s.hmax);
    RG_LAUNCH_CHECK();
    RG_HIP(hipMemcpyAsync(&o.dmax, s.hmax, 4, hipMemcpyDeviceToHost, st));
    RG_HIP(hipStreamSynchronize(st));
    if ((int64_t)o.dmax >= m) return RG_ERR_HIP;  // never: a depth is below the inner node count
    o.cnt.assign(o.dmax + 1, 0u);
    o.start.assign(o.dmax + 1, 0u);
    RG_HIP(hipMemcpyAsync(o.cnt.data(), s.hcount, 4 * (o.dmax + 1), hipMemcpyDeviceToHost, st));
    RG_HIP(hipStreamSynchronize(st));
    uint64_t total = 0;
    for (uint32_t d = 0; d <= o.dmax; ++d) {
        o.start[d] = (uint32_t)total;
        total += o.cnt[d];
    }
    if ((int64_t)total != m) return RG_ERR_HIP;  // never: every inner node has one depth
    RG_HIP(hipMemcpyAsync(s.hstart, o.start.data(), 4 * (o.dmax + 1), hipMemcpyHostToDevice, st));
    k_fill_u32<<<rg_blocks(o.dmax + 1, kThreads), kThreads, 0, st>>>(s.hcursor, 0u, o.dmax + 1);
    k_depth_scatter<<<rg_blocks(m, kThreads), kThreads, 0, st>>>(m, s.height, s.hstart, s.hcursor, (int32_t)o.dmax,
                                                                  s.order);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

// Renumbers the leaves of the binary hierarchy in s (n >= 2) in the tree's
// left-to-right order: triangle order ids -> ids_out, leaf boxes to box_out
// (which then replaces s.leaf_box), inner leaf ranges first / last.
rg_status relabel_leaves(LbvhScratch &s, int64_t n, const uint32_t *ids, uint32_t *ids_out, float *box_out,
                         hipStream_t st) {
    DepthOrder o;
    rg_status r = depth_order(s, n - 1, st, o);
    if (r != RG_OK) return r;
    for (int64_t d = o.dmax; d >= 0; --d)
        k_sizes_at<<<rg_blocks(o.cnt[d], kThreads), kThreads, 0, st>>>(s.order + o.start[d], o.cnt[d], s.left,
                                                                        s.right, s.size);
    RG_LAUNCH_CHECK();
    RG_HIP(hipStreamSynchronize(st));  // the host vectors of `o` go away on return
    k_ploc_ranks<<<rg_blocks(n, kThreads), kThreads, 0, st>>>(n, s.left, s.pint, s.pleaf, s.size, ids,
                                                               s.leaf_box, s.rank, s.first, s.last, ids_out,
                                                               box_out);
    k_ploc_relabel<<<rg_blocks(n - 1, kThreads), kThreads, 0, st>>>(n, s.left, s.right, s.rank);
    RG_LAUNCH_CHECK();
    s.leaf_box = box_out;
    return RG_OK;
}

// Clustering over the n >= 2 sorted leaves (`ids`): fills left, right,
// parents, inner boxes, first / last; leaves, leaf boxes (s.leaf_box) and
// the triangle order (*ids_out) in the tree's left-to-right order.
rg_status ploc_build(const float *prim_box, int64_t n, int radius, const uint32_t *ids, uint32_t *ids_out,
                     LbvhScratch &s, hipStream_t st) {
    k_ploc_init<<<rg_blocks(n, kThreads), kThreads, 0, st>>>(prim_box, ids, n, s.leaf_box, s.cid[0], s.cbox[0]);
    k_fill_u32<<<rg_blocks(n - 1, kThreads), kThreads, 0, st>>>((uint32_t *)s.pint, 0xFFFFFFFFu, n - 1);
    RG_LAUNCH_CHECK();
    int64_t m = n, next = n - 2;
    int cur = 0;
    for (int64_t its = 0; m > 1; ++its) {
        if (its > n) return RG_ERR_HIP;  // every round merges at least one pair
        const int nb = (int)((m + kPlocT - 1) / kPlocT);
        k_ploc_nearest<<<nb, kPlocT, 0, st>>>(s.cbox[cur], m, radius, s.nearest);
        k_ploc_flags<<<nb, kPlocT, 0, st>>>(s.nearest, m, s.n_merge, s.n_keep, nb);
        RG_LAUNCH_CHECK();
        rg_status r = rg_scan_excl_u32(s.n_merge, nb + 1, st);
        if (r == RG_OK) r = rg_scan_excl_u32(s.n_keep, nb + 1, st);
        if (r != RG_OK) return r;
        k_ploc_write<<<nb, kPlocT, 0, st>>>(s.nearest, m, s.n_merge, s.n_keep, next, s.cid[cur], s.cbox[cur],
                                            s.cid[cur ^ 1], s.cbox[cur ^ 1], s.left, s.right, s.int_box, s.pint,
                                            s.pleaf);
        RG_LAUNCH_CHECK();
        uint32_t tot[2];
        RG_HIP(hipMemcpyAsync(tot, s.n_merge + nb, 4, hipMemcpyDeviceToHost, st));
        RG_HIP(hipMemcpyAsync(tot + 1, s.n_keep + nb, 4, hipMemcpyDeviceToHost, st));
        RG_HIP(hipStreamSynchronize(st));
        if (tot[0] == 0u || (int64_t)tot[1] != m - (int64_t)tot[0]) return RG_ERR_HIP;
        next -= tot[0];
        m = tot[1];
        cur ^= 1;
    }
    if (next != -1) return RG_ERR_HIP;
    return relabel_leaves(s, n, ids, ids_out, s.cbox[cur], st);
}

// Rounds of treelet restructuring over the binary hierarchy in s (n >= 2),
// then the leaves renumbered in left-to-right order (ids -> ids_out).
rg_status treelet_build(int64_t n, int rounds, const uint32_t *ids, uint32_t *ids_out, LbvhScratch &s,
                        hipStream_t st) {
    const int64_t m = n - 1;
    for (int round = 0; round < rounds; ++round) {
        DepthOrder o;
        rg_status r = depth_order(s, m, st, o);
        if (r != RG_OK) return r;
        if (o.dmax < 1u) break;  // only the root: no inner node has three leaves below it
        const std::vector<uint32_t> &cnt = o.cnt, &start = o.start;
        const uint32_t dmax = o.dmax;
        // deepest first: a node's descendants are deeper, nodes of one depth
        // have disjoint subtrees
        for (int64_t d = dmax; d >= 0; --d) {
            if (cnt[d] == 0u) continue;
            k_treelet<<<cnt[d], 64, 0, st>>>(s.order + start[d], s.left, s.right, s.pint, s.pleaf, s.int_box,
                                             s.leaf_box);
        }
        RG_LAUNCH_CHECK();
        RG_HIP(hipStreamSynchronize(st));  // the host vectors above are reused next round
    }
    return relabel_leaves(s, n, ids, ids_out, s.cbox[0], st);
}

// A level-by-level collapse between host reads.  Levels go in batches; the
// host learns their sizes after each batch (the counts in the device ring).
// A level's size is at most W times the one before, which bounds the grids
// of the levels launched before their sizes are known; levels launched after
// the last one find an empty queue and return.
struct CollapseState {
    int32_t width = 4;
    int32_t d = 0;         // first level of the next batch
    int32_t batch = 0;     // levels in the batch last launched
    int32_t depth = 0;     // the number of levels, once known
    uint32_t known = 1;    // size of level d
    uint32_t cap = 0;
    uint64_t n_nodes = 1;  // nodes of the levels known so far
    const int32_t *wch;
    const uint32_t *wlink;
    const uint8_t *winner;
    const float *int_box, *leaf_box;
    uint2 *q[2];
    uint32_t *ring;
    void *nodes;
    uint32_t *parents, *levels;
};
constexpr int kRingWords = 2 * kCollapseRing + 1;  // what the host reads after a batch

template <int W>
void collapse_batch(const CollapseState &c, hipStream_t st) {
    uint64_t bound = c.known;
    for (int j = 0; j < c.batch; ++j) {
        unsigned blocks = rg_blocks((int64_t)(bound ? bound : 1), kThreads);
        if (blocks > 1024) blocks = 1024;
        const int level = c.d + j;
        k_collapse<W><<<blocks, kThreads, 0, st>>>(c.wch, c.wlink, c.winner, c.int_box, c.leaf_box, c.q[level & 1],
                                                    c.q[(level + 1) & 1], c.ring, level,
                                                    reinterpret_cast<RgNode<W> *>(c.nodes), c.parents, c.levels,
                                                    c.cap);
        bound = std::min<uint64_t>((uint64_t)c.cap, bound * (uint64_t)W);
    }
}

rg_status collapse_launch(const CollapseState &c, hipStream_t st) {
    if (c.width == 2) collapse_batch<2>(c, st);
    else if (c.width == 4) collapse_batch<4>(c, st);
    else collapse_batch<8>(c, st);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

// Takes in the counts read after a batch: the depth once a level comes out
// empty, else the next batch (kCollapseBatch levels) to launch.
rg_status collapse_absorb(CollapseState &c, const uint32_t *hr) {
    if (hr[2 * kCollapseRing] != 0u) return RG_ERR_HIP;  // inconsistent hierarchy: never expected
    for (int j = 0; j < c.batch; ++j) {
        const uint32_t cnt = hr[(c.d + j + 1) % kCollapseRing];  // nodes of level d + j + 1
        if (cnt == 0u) {
            c.depth = c.d + j + 1;
            return RG_OK;
        }
        c.n_nodes += cnt;
        c.known = cnt;
    }
    c.d += c.batch;
    c.batch = kCollapseBatch;
    if (c.d > 4096 || c.n_nodes > c.cap) return RG_ERR_HIP;  // never expected
    return RG_OK;
}

// Launches the plan and the first batch (sized to cover the depth a tree of
// n leaves usually reaches, 1.6 log_W n + 2 levels, so that most builds read
// the counts once).  n == 1: the single root, depth known at once.
template <int W>
rg_status collapse_begin(const LbvhScratch &s, int64_t n, int leaf_max, void *nodes, uint32_t *parents,
                         uint32_t *levels, hipStream_t st, CollapseState &c) {
    c = CollapseState{};
    c.width = W;
    if (n == 1) {
        k_single_root<W><<<1, 64, 0, st>>>(s.leaf_box, reinterpret_cast<RgNode<W> *>(nodes));
        if (parents) k_fill_u32<<<1, 64, 0, st>>>(parents, RG_MISS, 1);
        if (levels) {
            k_fill_u32<<<1, 64, 0, st>>>(levels, 0u, 1);
            k_fill_u32<<<1, 64, 0, st>>>(levels + 1, 1u, 1);
        }
        RG_LAUNCH_CHECK();
        c.depth = 1;
        return RG_OK;
    }
    c.cap = (uint32_t)(n - 1);
    c.wch = s.wch;
    c.wlink = s.wlink;
    c.winner = s.winner;
    c.int_box = s.int_box;
    c.leaf_box = s.leaf_box;
    c.q[0] = s.q0;
    c.q[1] = s.q1;
    c.ring = s.qcount;
    c.nodes = nodes;
    c.parents = parents;
    c.levels = levels;
    k_wide_plan<W><<<rg_blocks(n - 1, kThreads), kThreads, 0, st>>>(s.left, s.right, s.first, s.last, s.int_box,
                                                                     leaf_max, n - 1, s.wch, s.wlink, s.winner);
    k_collapse_init<<<1, 1, 0, st>>>(s.q0, c.ring, parents, levels);
    RG_LAUNCH_CHECK();
    const int b = (int)std::ceil(1.6 * std::log((double)n) / std::log((double)W)) + 2;
    c.batch = std::max(kCollapseBatch, std::min(kCollapseFirstMax, b));
    return collapse_launch(c, st);
}

// Reads the counts of the batch in flight (into hr, pinned or not) and goes
// on until the depth is known; waits for `st` at each read.
rg_status collapse_finish(CollapseState &c, hipStream_t st, uint32_t *hr) {
    while (c.depth == 0) {
        RG_HIP(hipMemcpyAsync(hr, c.ring, kRingWords * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        RG_HIP(hipStreamSynchronize(st));
        rg_status r = collapse_absorb(c, hr);
        if (r != RG_OK) return r;
        if (c.depth == 0 && (r = collapse_launch(c, st)) != RG_OK) return r;
    }
    return RG_OK;
}

template <int W>
rg_status collapse(const LbvhScratch &s, int64_t n, int leaf_max, void *nodes, uint32_t *parents,
                   uint32_t *levels, hipStream_t st, int32_t *depth, int64_t *n_nodes) {
    CollapseState c;
    rg_status r = collapse_begin<W>(s, n, leaf_max, nodes, parents, levels, st, c);
    if (r != RG_OK) return r;
    uint32_t hr[kRingWords];
    if ((r = collapse_finish(c, st, hr)) != RG_OK) return r;
    *depth = c.depth;
    *n_nodes = (int64_t)c.n_nodes;
    return RG_OK;
}

}  // namespace

uint64_t rg_lbvh_scratch_bytes(int64_t n, int32_t builder) {
    RgArena a{nullptr, 0, 0};
    LbvhScratch s;
    carve(a, n, builder, s);
    return a.used;
}

rg_status rg_lbvh_build(const float *prim_box, int64_t n, int32_t width, int32_t leaf_max, int32_t builder,
                        int32_t radius, void *nodes, uint32_t *parents, uint32_t *levels, RgArena &arena,
                        hipStream_t st, RgLbvhOut *out, bool keep_stages, uint64_t *keys_out, int32_t *left_out,
                        int32_t *right_out, float *boxes_out) {
    LbvhScratch s;
    if (!carve(arena, n, builder, s)) return RG_ERR_OUT_OF_MEMORY;
    if (builder == RG_BUILDER_LBVH && n <= kSmallMax) {
        // the whole build in one workgroup, one host wait for its summary
        SmallArgs sa;
        sa.prim_box = prim_box;
        sa.n = (int32_t)n;
        sa.leaf_max = leaf_max;
        sa.keys_out = keep_stages ? keys_out : nullptr;
        sa.ids = s.ids;
        sa.left = s.left; sa.right = s.right; sa.pint = s.pint; sa.pleaf = s.pleaf;
        sa.first = s.first; sa.last = s.last;
        sa.int_box = s.int_box;
        sa.leaf_box = s.leaf_box;
        sa.q[0] = s.q0;
        sa.q[1] = s.q1;
        sa.nodes = nodes;
        sa.parents = parents;
        sa.levels = levels;
        sa.flag_in = out->flag_in;
        sa.key_shift = out->key_shift;
        sa.res = s.small;
        const size_t lds = small_lds_bytes(n);
        const TlasFuse *fuse = reinterpret_cast<const TlasFuse *>(out->tlas_fuse);
        if (fuse && n <= kResidentMax) {
            sa.inst = fuse->T;
            sa.rec_tmp = fuse->rec_tmp;
            sa.recs_out = fuse->recs_out;
            sa.rec_of = fuse->rec_of;
            if (width == 2) k_small_build<2, true, true><<<1, kSmallThreads, lds, st>>>(sa);
            else if (width == 4) k_small_build<4, true, true><<<1, kSmallThreads, lds, st>>>(sa);
            else k_small_build<8, true, true><<<1, kSmallThreads, lds, st>>>(sa);
        } else if (fuse) {
            return RG_ERR_HIP;  // never: the top level fuses only up to kResidentMax instances
        } else if (n <= kResidentMax) {
            if (width == 2) k_small_build<2, true><<<1, kSmallThreads, lds, st>>>(sa);
            else if (width == 4) k_small_build<4, true><<<1, kSmallThreads, lds, st>>>(sa);
            else k_small_build<8, true><<<1, kSmallThreads, lds, st>>>(sa);
        } else {
            if (width == 2) k_small_build<2, false><<<1, kSmallThreads, lds, st>>>(sa);
            else if (width == 4) k_small_build<4, false><<<1, kSmallThreads, lds, st>>>(sa);
            else k_small_build<8, false><<<1, kSmallThreads, lds, st>>>(sa);
        }
        RG_LAUNCH_CHECK();
        if (keep_stages) {
            if (n > 1) {
                RG_HIP(hipMemcpyAsync(left_out, s.left, 4 * (n - 1), hipMemcpyDeviceToDevice, st));
                RG_HIP(hipMemcpyAsync(right_out, s.right, 4 * (n - 1), hipMemcpyDeviceToDevice, st));
                RG_HIP(hipMemcpyAsync(boxes_out, s.int_box, 24 * (n - 1), hipMemcpyDeviceToDevice, st));
            }
            RG_HIP(hipMemcpyAsync(boxes_out + 6 * (n - 1), s.leaf_box, 24 * n, hipMemcpyDeviceToDevice, st));
        }
        static_assert(sizeof(SmallResult) == 10 * sizeof(uint32_t), "summary layout");
        out->ids = s.ids;
        out->root_dev = s.small->lo;
        if (out->deferred) {
            RG_HIP(hipMemcpyAsync(out->deferred, s.small, sizeof(SmallResult), hipMemcpyDeviceToHost, st));
            out->pending = true;
            return RG_OK;
        }
        uint32_t res[10];
        out->deferred = res;
        RG_HIP(hipMemcpyAsync(res, s.small, sizeof(SmallResult), hipMemcpyDeviceToHost, st));
        RG_HIP(hipStreamSynchronize(st));
        out->pending = true;
        rg_status r = rg_lbvh_finish(out, nodes != nullptr);
        out->deferred = nullptr;
        return r;
    }
    const int nblocks = (int)((n + kSortTile - 1) / kSortTile);
    // centre bounds (partials; the sort's counters cleared), keys with the
    // digit counts of every pass, then one launch per pass
    int64_t bparts = (n + kThreads - 1) / kThreads;
    if (bparts > kBoundParts) bparts = kBoundParts;
    k_centre_bounds<<<(unsigned)bparts, kThreads, 0, st>>>(prim_box, n, s.part, s.sortz, s.sortz_words);
    RG_LAUNCH_CHECK();
    k_morton<<<nblocks, kSortThreads, 0, st>>>(prim_box, n, s.part, (int)bparts, out->key_shift, s.keys, s.ids,
                                               s.count);
    RG_LAUNCH_CHECK();
    // 8 passes of 8 bits (4 for 30-bit keys); the result lands in ka / ia
    uint64_t *ka = s.keys, *kb = s.keys2;
    uint32_t *ia = s.ids, *ib = s.ids2;
    const int passes = out->key_shift ? 4 : 8;
    for (int p = 0; p < passes; ++p) {
        k_sort_count<uint64_t><<<nblocks, kSortThreads, 0, st>>>(ka, n, 8 * p, s.cnt, nblocks);
        k_sort_scan<<<256, kScanThreads, 0, st>>>(s.cnt, nblocks, s.count + 256 * p);
        k_sort_scatter<uint64_t><<<nblocks, kSortThreads, 0, st>>>(ka, ia, kb, ib, n, 8 * p, s.cnt, nblocks);
        RG_LAUNCH_CHECK();
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *ti = ia; ia = ib; ib = ti;
    }
    if (builder == RG_BUILDER_PLOC && n > 1) {
        rg_status r = ploc_build(prim_box, n, radius, ia, ib, s, st);
        if (r != RG_OK) return r;
        ia = ib;
    } else {
        if (n > 1) {
            k_karras<<<rg_blocks(n - 1, kThreads), kThreads, 0, st>>>(ka, n, s.left, s.right, s.pint, s.pleaf,
                                                                      s.first, s.last);
            RG_LAUNCH_CHECK();
        }
        k_leaf_boxes<<<rg_blocks(n, kThreads), kThreads, 0, st>>>(prim_box, ia, n, s.leaf_box);
        RG_LAUNCH_CHECK();
        if (n > 1) {  // inner boxes from the leaf ranges: no host step
            const int64_t nbr = (n + kRangeLeaves - 1) / kRangeLeaves;
            k_range_blocks<<<rg_blocks(n, kThreads), kThreads, 0, st>>>(s.leaf_box, n, s.pre, s.suf, s.rtab);
            const int top = (int)range_levels(nbr) - 1;
            for (int j0 = 0; j0 < top; j0 += kRangeStride)
                k_range_levels<<<rg_blocks(kRangeStride * nbr, kThreads), kThreads, 0, st>>>(s.rtab, nbr, j0, top);
            k_range_boxes<<<rg_blocks(n - 1, kThreads), kThreads, 0, st>>>(s.first, s.last, n - 1, s.leaf_box,
                                                                            s.pre, s.suf, s.rtab, nbr, s.int_box);
            RG_LAUNCH_CHECK();
        }
        if (builder == RG_BUILDER_TREELET && n > 1) {
            rg_status r = treelet_build(n, radius, ia, ib, s, st);
            if (r != RG_OK) return r;
            ia = ib;
        }
    }
    if (keep_stages) {
        RG_HIP(hipMemcpyAsync(keys_out, ka, 8 * n, hipMemcpyDeviceToDevice, st));
        if (n > 1) {
            RG_HIP(hipMemcpyAsync(left_out, s.left, 4 * (n - 1), hipMemcpyDeviceToDevice, st));
            RG_HIP(hipMemcpyAsync(right_out, s.right, 4 * (n - 1), hipMemcpyDeviceToDevice, st));
            RG_HIP(hipMemcpyAsync(boxes_out, s.int_box, 24 * (n - 1), hipMemcpyDeviceToDevice, st));
        }
        RG_HIP(hipMemcpyAsync(boxes_out + 6 * (n - 1), s.leaf_box, 24 * n, hipMemcpyDeviceToDevice, st));
    }
    out->ids = ia;
    rg_status r = RG_OK;
    if (nodes && out->coll_async) {  // the first batch only; the caller completes the collapse
        CollapseState &c = *static_cast<CollapseState *>(out->coll_async);
        if (width == 2) r = collapse_begin<2>(s, n, leaf_max, nodes, parents, levels, st, c);
        else if (width == 4) r = collapse_begin<4>(s, n, leaf_max, nodes, parents, levels, st, c);
        else r = collapse_begin<8>(s, n, leaf_max, nodes, parents, levels, st, c);
        if (r != RG_OK) return r;
        if (c.depth == 0)
            RG_HIP(hipMemcpyAsync(out->coll_hr, c.ring, kRingWords * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    } else if (nodes) {
        if (width == 2) r = collapse<2>(s, n, leaf_max, nodes, parents, levels, st, &out->depth, &out->n_nodes);
        else if (width == 4) r = collapse<4>(s, n, leaf_max, nodes, parents, levels, st, &out->depth, &out->n_nodes);
        else r = collapse<8>(s, n, leaf_max, nodes, parents, levels, st, &out->depth, &out->n_nodes);
        if (r != RG_OK) return r;
    }
    out->root_dev = n > 1 ? s.int_box : s.leaf_box;
    if (out->deferred) {  // the root box comes back with the caller's wait, into the summary's box words
        static_assert(offsetof(SmallResult, lo) == 16, "summary layout");
        RG_HIP(hipMemcpyAsync(out->deferred + 4, out->root_dev, 24, hipMemcpyDeviceToHost, st));
        out->pending_box = true;
        return RG_OK;
    }
    float rb[6];
    RG_HIP(hipMemcpyAsync(rb, out->root_dev, 24, hipMemcpyDeviceToHost, st));
    RG_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < 3; ++k) {
        out->lo[k] = rb[k];
        out->hi[k] = rb[3 + k];
    }
    return RG_OK;
}

// A pinned host buffer per calling thread, grown on demand and kept for the
// thread's life: host tables go to the device and build summaries come back
// through it with asynchronous copies, so a build waits for its stream once.
// nullptr if pinned memory cannot be had (callers then copy from pageable
// memory, which waits at each copy).
static char *pinned_staging(size_t bytes) {
    thread_local char *buf = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        const size_t want = ((bytes > (64u << 10) ? bytes : (64u << 10)) + 4095u) & ~(size_t)4095u;
        void *p = nullptr;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
        buf = (char *)p;
        cap = want;
    }
    return buf;
}

rg_status rg_lbvh_finish(RgLbvhOut *out, bool with_nodes) {
    if (out->pending_box) {
        out->pending_box = false;
        float rb[6];
        memcpy(rb, out->deferred + 4, sizeof(rb));
        for (int k = 0; k < 3; ++k) {
            out->lo[k] = rb[k];
            out->hi[k] = rb[3 + k];
        }
    }
    if (!out->pending) return RG_OK;
    out->pending = false;
    SmallResult res;
    memcpy(&res, out->deferred, sizeof(res));
    if (res.err) return RG_ERR_HIP;  // never: every inner node gets a box
    out->flag = res.flag;
    out->depth = with_nodes ? (int32_t)res.depth : 0;
    out->n_nodes = with_nodes ? (int64_t)res.n_nodes : 0;
    for (int k = 0; k < 3; ++k) {
        out->lo[k] = res.lo[k];
        out->hi[k] = res.hi[k];
    }
    return RG_OK;
}

rg_status rg_scan_excl_u32(uint32_t *data, int64_t m, hipStream_t st) {
    k_scan_excl<<<1, kScanThreads, 0, st>>>(data, m);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

// ================================================================ ABI
namespace {

uint64_t blas_out_bytes(int64_t n, int w, uint64_t *nodes_off, uint64_t *tris_off, uint64_t *mats_off,
                        uint64_t *slots_off, uint64_t *parents_off, uint64_t *levels_off) {
    int64_t max_nodes = n > 1 ? n - 1 : 1;
    uint64_t off = 256;  // header
    *nodes_off = off;
    off = align256(off + (uint64_t)max_nodes * node_bytes(w));
    *tris_off = off;
    off = align256(off + (uint64_t)n * sizeof(RgTri));
    *mats_off = off;
    off = align256(off + (uint64_t)n * 2u);
    *slots_off = off;
    off = align256(off + (uint64_t)n * 4u);
    *parents_off = off;
    off = align256(off + (uint64_t)max_nodes * 4u);
    *levels_off = off;
    off = align256(off + (uint64_t)(RG_LEVELS_CAP + 1) * 4u);
    return off;
}

uint64_t blas_scratch_bytes(int64_t n, int32_t builder) {
    RgArena a{nullptr, 0, 0};
    a.take<float>(6 * n);  // primitive boxes
    a.take<uint32_t>(8);   // flags
    return a.used + rg_lbvh_scratch_bytes(n, builder);
}

uint64_t tlas_out_bytes(int64_t n, int w, uint64_t *nodes_off, uint64_t *inst_off, uint64_t *rec_off,
                        uint64_t *xf_off) {
    int64_t max_nodes = n > 1 ? n - 1 : 1;
    uint64_t off = 0;
    *nodes_off = off;
    off = align256(off + (uint64_t)max_nodes * node_bytes(w));
    *inst_off = off;
    off = align256(off + (uint64_t)n * sizeof(RgInst));
    *rec_off = off;
    off = align256(off + (uint64_t)n * 4u);
    *xf_off = off;
    off = align256(off + (uint64_t)n * 48u);
    return off;
}

uint64_t tlas_scratch_bytes(int64_t n, int32_t n_blas, int32_t builder) {
    RgArena a{nullptr, 0, 0};
    const size_t t4 = (4 * (size_t)n + 7) & ~size_t(7);
    // host tables: matrices, three uint32 tables, bottom-level addresses, flag word
    a.take<char>(48 * (size_t)n + 3 * t4 + sizeof(BlasInfo) * (size_t)(n_blas > 0 ? n_blas : 1) + 8);
    a.take<float>(6 * n);       // instance boxes
    a.take<RgInst>(n);          // unsorted records
    return a.used + rg_lbvh_scratch_bytes(n, builder);
}

}  // namespace

namespace {
thread_local char g_last_error[256] = "";
}

void rg_set_error(const char *file, int line, const char *what) {
    const char *base = file;
    for (const char *p = file; *p; ++p)
        if (*p == '/') base = p + 1;
    snprintf(g_last_error, sizeof(g_last_error), "%s:%d: %s", base, line, what);
}

rg_status rg_debug_done(rg_status r, hipStream_t st) {
    static const bool on = [] {
        const char *v = getenv("RG_DEBUG");
        return v && v[0] && !(v[0] == '0' && v[1] == 0);
    }();
    if (!on || r != RG_OK) return r;
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        rg_set_error(__FILE__, __LINE__, hipGetErrorName(e));
        return RG_ERR_HIP;
    }
    return RG_OK;
}

extern "C" {

const char *rg_last_error(void) { return g_last_error; }

const char *rg_status_string(rg_status s) {
    switch (s) {
        case RG_OK: return "ok";
        case RG_ERR_INVALID_ARG: return "invalid argument";
        case RG_ERR_OUT_OF_MEMORY: return "buffer too small";
        case RG_ERR_HIP: return "HIP runtime error";
        case RG_ERR_UNSUPPORTED: return "unsupported";
        case RG_ERR_UNIMPLEMENTED: return "unimplemented";
        default: return "unknown status";
    }
}

rg_status rg_blas_sizes(int64_t n_tris, const rg_build_opts *opts, rg_sizes *out) {
    Opts o;
    if (!out || n_tris < 1 || n_tris > RG_MAX_TRIS || !opts_ok(opts, &o) || !o.fits(n_tris)) return RG_ERR_INVALID_ARG;
    uint64_t a, b, c, d, e, f;
    out->bytes = blas_out_bytes(n_tris, o.w, &a, &b, &c, &d, &e, &f);
    out->scratch_bytes = blas_scratch_bytes(n_tris, o.builder);
    return RG_OK;
}

rg_status rg_build_blas(const float *verts, int64_t n_verts, const uint32_t *idx, int64_t n_tris,
                        const uint16_t *prim_material, const rg_build_opts *opts, void *out_buf,
                        uint64_t out_bytes, void *scratch, uint64_t scratch_bytes, void *stream, rg_blas *out) {
    Opts o;
    if (!verts || !idx || !out_buf || !scratch || !out) return RG_ERR_INVALID_ARG;
    if (n_verts < 1 || n_verts > (1ll << 32) || n_tris < 1 || n_tris > RG_MAX_TRIS) return RG_ERR_INVALID_ARG;
    if (!opts_ok(opts, &o) || !o.fits(n_tris)) return RG_ERR_INVALID_ARG;
    const int32_t w = o.w, l = o.leaf;
    uint64_t no, to, mo, so, po, lvo;
    uint64_t need = blas_out_bytes(n_tris, w, &no, &to, &mo, &so, &po, &lvo);
    if (out_bytes < need || scratch_bytes < blas_scratch_bytes(n_tris, o.builder)) return RG_ERR_OUT_OF_MEMORY;
    hipStream_t st = (hipStream_t)stream;
    RgArena arena{(char *)scratch, scratch_bytes, 0};
    float *pbox = arena.take<float>(6 * n_tris);
    uint32_t *flags = arena.take<uint32_t>(8);
    k_fill_u32<<<1, 64, 0, st>>>(flags, 0u, 1);
    k_tri_boxes<<<rg_blocks(n_tris, kThreads), kThreads, 0, st>>>(verts, n_verts, idx, n_tris, pbox, flags);
    RG_LAUNCH_CHECK();
    // the build's summary (one-workgroup builds) or root box, then the flags
    // word: pinned, so the copies back do not wait
    uint32_t local[11] = {};
    uint32_t *summary = (uint32_t *)pinned_staging(64);
    if (!summary) summary = local;
    summary[10] = 0u;
    // the linear build runs on whatever the boxes hold (out-of-range indices
    // were clamped, and its steps stay in bounds for any key values): the
    // input check comes back with the call's last wait.  The clustering and
    // restructuring builders take only checked input.
    if (o.builder != RG_BUILDER_LBVH) {
        RG_HIP(hipMemcpyAsync(summary + 10, flags, 4, hipMemcpyDeviceToHost, st));
        RG_HIP(hipStreamSynchronize(st));
        if (summary[10]) return RG_ERR_INVALID_ARG;
    }
    char *base = (char *)out_buf;
    RgLbvhOut lo;
    lo.deferred = summary;
    lo.key_shift = o.key_shift();
    rg_status r = rg_lbvh_build(pbox, n_tris, w, l, o.builder, o.radius, base + no, (uint32_t *)(base + po),
                                (uint32_t *)(base + lvo), arena, st, &lo, false, nullptr, nullptr, nullptr, nullptr);
    if (r != RG_OK) {
        // an invalid input is reported as such, also when it upset the build
        const hipError_t fe = hipMemcpyAsync(summary + 10, flags, 4, hipMemcpyDeviceToHost, st);
        (void)hipStreamSynchronize(st);  // the summary copies target this frame
        if (fe == hipSuccess && summary[10]) return RG_ERR_INVALID_ARG;
        return r;
    }
    k_reorder_tris<<<rg_blocks(n_tris, kThreads), kThreads, 0, st>>>(
        verts, n_verts, idx, lo.ids, n_tris, prim_material, (RgTri *)(base + to), (uint16_t *)(base + mo),
        (uint32_t *)(base + so));
    k_blas_header<<<1, 1, 0, st>>>((RgBlasHdr *)base, (uint64_t)(base + no), (uint64_t)(base + to),
                                   (uint64_t)(base + mo), (uint64_t)(base + so), lo.root_dev);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = le == hipSuccess ? hipMemcpyAsync(summary + 10, flags, 4, hipMemcpyDeviceToHost, st) : le;
    RG_HIP(hipStreamSynchronize(st));
    RG_HIP(ce);
    if ((r = rg_lbvh_finish(&lo, true)) != RG_OK) return r;
    if (summary[10]) return RG_ERR_INVALID_ARG;
    out->buf = out_buf;
    out->nodes_off = no;
    out->tris_off = to;
    out->mats_off = mo;
    out->slots_off = so;
    out->parents_off = po;
    out->levels_off = lvo;
    out->n_tris = n_tris;
    out->n_nodes = lo.n_nodes;
    out->width = w;
    out->leaf_max = l;
    out->depth = lo.depth;
    out->has_mats = prim_material ? 1 : 0;
    for (int k = 0; k < 3; ++k) {
        out->lo[k] = lo.lo[k];
        out->hi[k] = lo.hi[k];
    }
    out->has_alpha = 0;
    out->alpha_level = 0;
    return RG_OK;
}

// The state of an asynchronous bottom-level build, kept in the caller's
// pinned ticket: the device summaries land in it by asynchronous copies.
struct BlasTicket {
    uint64_t magic;
    hipStream_t st;
    hipEvent_t done;
    uint32_t summary[12];    // one-workgroup summary (10 words) or the root box at 4..9; input flags at 10
    uint32_t hr[kRingWords];  // the collapse's level counts after its first batch
    RgLbvhOut lo;
    CollapseState coll;
    rg_blas desc;            // what is known at enqueue time
};
constexpr uint64_t kTicketMagic = 0x7267424c41534174ull;
static_assert(sizeof(BlasTicket) <= RG_BUILD_TICKET_BYTES, "ticket size");

rg_status rg_build_blas_async(const float *verts, int64_t n_verts, const uint32_t *idx, int64_t n_tris,
                              const uint16_t *prim_material, const rg_build_opts *opts, void *out_buf,
                              uint64_t out_bytes, void *scratch, uint64_t scratch_bytes, void *stream, void *ticket) {
    Opts o;
    if (!verts || !idx || !out_buf || !scratch || !ticket || ((uintptr_t)ticket & 15u)) return RG_ERR_INVALID_ARG;
    if (n_verts < 1 || n_verts > (1ll << 32) || n_tris < 1 || n_tris > RG_MAX_TRIS) return RG_ERR_INVALID_ARG;
    if (!opts_ok(opts, &o) || !o.fits(n_tris)) return RG_ERR_INVALID_ARG;
    if (o.builder != RG_BUILDER_LBVH) return RG_ERR_UNSUPPORTED;  // the others step their rounds from the host
    const int32_t w = o.w, l = o.leaf;
    uint64_t no, to, mo, so, po, lvo;
    const uint64_t need = blas_out_bytes(n_tris, w, &no, &to, &mo, &so, &po, &lvo);
    if (out_bytes < need || scratch_bytes < blas_scratch_bytes(n_tris, o.builder)) return RG_ERR_OUT_OF_MEMORY;
    hipStream_t st = (hipStream_t)stream;
    BlasTicket *T = new (ticket) BlasTicket();
    T->st = st;
    RG_HIP(hipEventCreateWithFlags(&T->done, hipEventDisableTiming));  // before anything is enqueued
    RgArena arena{(char *)scratch, scratch_bytes, 0};
    float *pbox = arena.take<float>(6 * n_tris);
    uint32_t *flags = arena.take<uint32_t>(8);
    k_fill_u32<<<1, 64, 0, st>>>(flags, 0u, 1);
    k_tri_boxes<<<rg_blocks(n_tris, kThreads), kThreads, 0, st>>>(verts, n_verts, idx, n_tris, pbox, flags);
    RG_LAUNCH_CHECK();
    char *base = (char *)out_buf;
    T->lo.deferred = T->summary;
    T->lo.key_shift = o.key_shift();
    T->lo.coll_async = &T->coll;
    T->lo.coll_hr = T->hr;
    rg_status r = rg_lbvh_build(pbox, n_tris, w, l, o.builder, o.radius, base + no, (uint32_t *)(base + po),
                                (uint32_t *)(base + lvo), arena, st, &T->lo, false, nullptr, nullptr, nullptr,
                                nullptr);
    hipError_t e = hipSuccess;
    if (r == RG_OK) {
        k_reorder_tris<<<rg_blocks(n_tris, kThreads), kThreads, 0, st>>>(
            verts, n_verts, idx, T->lo.ids, n_tris, prim_material, (RgTri *)(base + to), (uint16_t *)(base + mo),
            (uint32_t *)(base + so));
        k_blas_header<<<1, 1, 0, st>>>((RgBlasHdr *)base, (uint64_t)(base + no), (uint64_t)(base + to),
                                       (uint64_t)(base + mo), (uint64_t)(base + so), T->lo.root_dev);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(T->summary + 10, flags, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(T->done, st);
    }
    if (r != RG_OK || e != hipSuccess) {
        (void)hipStreamSynchronize(st);  // copies into the ticket may be in flight
        (void)hipEventDestroy(T->done);
        T->magic = 0;
        if (r != RG_OK) return r;
        RG_HIP(e);
    }
    rg_blas &d = T->desc;
    d = rg_blas{};
    d.buf = out_buf;
    d.nodes_off = no;
    d.tris_off = to;
    d.mats_off = mo;
    d.slots_off = so;
    d.parents_off = po;
    d.levels_off = lvo;
    d.n_tris = n_tris;
    d.width = w;
    d.leaf_max = l;
    d.has_mats = prim_material ? 1 : 0;
    T->magic = kTicketMagic;
    return RG_OK;
}

rg_status rg_build_blas_finish(void *ticket, rg_blas *out) {
    if (!ticket || !out || ((uintptr_t)ticket & 15u)) return RG_ERR_INVALID_ARG;
    BlasTicket *T = static_cast<BlasTicket *>(ticket);
    if (T->magic != kTicketMagic) return RG_ERR_INVALID_ARG;
    T->magic = 0;  // a ticket completes once
    const hipError_t we = hipEventSynchronize(T->done);
    (void)hipEventDestroy(T->done);
    RG_HIP(we);
    rg_status r = RG_OK;
    if (T->lo.pending) {  // one-workgroup build: everything is in the summary
        r = rg_lbvh_finish(&T->lo, true);
    } else {
        r = rg_lbvh_finish(&T->lo, true);  // the root box
        if (r == RG_OK && T->coll.depth == 0) {
            r = collapse_absorb(T->coll, T->hr);
            if (r == RG_OK && T->coll.depth == 0) {  // deeper than the first batch: the rest, waiting here
                if ((r = collapse_launch(T->coll, T->st)) == RG_OK) r = collapse_finish(T->coll, T->st, T->hr);
            }
        }
        T->lo.depth = T->coll.depth;
        T->lo.n_nodes = (int64_t)T->coll.n_nodes;
    }
    if (r != RG_OK) return r;
    if (T->summary[10]) return RG_ERR_INVALID_ARG;
    rg_blas d = T->desc;
    d.n_nodes = T->lo.n_nodes;
    d.depth = T->lo.depth;
    for (int k = 0; k < 3; ++k) {
        d.lo[k] = T->lo.lo[k];
        d.hi[k] = T->lo.hi[k];
    }
    *out = d;
    return RG_OK;
}

rg_status rg_refit_sizes(const rg_blas *blas, uint64_t *scratch_bytes) {
    if (!blas || !scratch_bytes || blas->n_nodes < 1) return RG_ERR_INVALID_ARG;
    RgArena a{nullptr, 0, 0};
    a.take<uint32_t>(blas->n_nodes);  // inner children per node (hierarchies deeper than the level table)
    a.take<uint32_t>(blas->n_nodes);  // arrivals
    *scratch_bytes = a.used;
    return RG_OK;
}

rg_status rg_refit_blas_many(rg_blas *blas, int32_t n_blas, const float *const *verts, const int64_t *n_verts,
                             const uint32_t *const *idx, const int64_t *n_tris, void *scratch,
                             uint64_t scratch_bytes, void *stream) {
    if (!blas || !verts || !n_verts || !idx || !n_tris || n_blas < 1) return RG_ERR_INVALID_ARG;
    const int32_t w = blas[0].width;
    if (!(w == 2 || w == 4 || w == 8)) return RG_ERR_INVALID_ARG;
    uint64_t scratch_need = 0;
    for (int32_t b = 0; b < n_blas; ++b) {
        const rg_blas &B = blas[b];
        if (!B.buf || !verts[b] || !idx[b] || B.width != w || B.n_nodes < 1 || B.depth < 1) return RG_ERR_INVALID_ARG;
        if (n_tris[b] != B.n_tris || n_verts[b] < 1 || n_verts[b] > (1ll << 32)) return RG_ERR_INVALID_ARG;
        if (B.depth > RG_LEVELS_CAP) {
            uint64_t need = 0;
            rg_refit_sizes(&B, &need);
            if (need > scratch_need) scratch_need = need;
        }
    }
    if (scratch_need > 0 && (!scratch || scratch_bytes < scratch_need)) return RG_ERR_OUT_OF_MEMORY;
    hipStream_t st = (hipStream_t)stream;
    for (int32_t b0 = 0; b0 < n_blas; b0 += kRefitBatch) {
        const int n = n_blas - b0 < kRefitBatch ? n_blas - b0 : kRefitBatch;
        RefitJobs jobs;
        std::memset(&jobs, 0, sizeof(jobs));
        int64_t max_tris = 0;
        int max_depth = 0;
        for (int k = 0; k < n; ++k) {
            const rg_blas &B = blas[b0 + k];
            char *base = (char *)B.buf;
            RefitJob &J = jobs.j[k];
            J.nodes = base + B.nodes_off;
            J.tris = (RgTri *)(base + B.tris_off);
            J.levels = (const uint32_t *)(base + B.levels_off);
            J.parents = (const uint32_t *)(base + B.parents_off);
            J.hdr = (RgBlasHdr *)base;
            J.verts = verts[b0 + k];
            J.idx = idx[b0 + k];
            J.n_verts = n_verts[b0 + k];
            J.n_tris = B.n_tris;
            J.depth = B.depth <= RG_LEVELS_CAP ? B.depth : 0;  // deeper ones: refit_deep below
            if (B.n_tris > max_tris) max_tris = B.n_tris;
            if (J.depth > max_depth) max_depth = J.depth;
        }
        k_refit_begin<<<1, 64, 0, st>>>(jobs, n);
        unsigned tb = rg_blocks(max_tris, kThreads);
        if (tb > 1024) tb = 1024;
        k_refit_tris<<<dim3(tb, (unsigned)n), kThreads, 0, st>>>(jobs);
        RG_LAUNCH_CHECK();
        // grid per level: enough blocks for the widest level of any of them
        int64_t max_nodes = 0;
        for (int k = 0; k < n; ++k)
            if (blas[b0 + k].n_nodes > max_nodes) max_nodes = blas[b0 + k].n_nodes;
        unsigned lb = rg_blocks(max_nodes, kThreads);
        if (lb > 512) lb = 512;
        if (max_depth > 0) {
            if (w == 2) refit_levels<2>(jobs, n, max_depth, lb, st);
            else if (w == 4) refit_levels<4>(jobs, n, max_depth, lb, st);
            else refit_levels<8>(jobs, n, max_depth, lb, st);
        }
        RG_LAUNCH_CHECK();
        for (int k = 0; k < n; ++k) {
            const rg_blas &B = blas[b0 + k];
            if (B.depth <= RG_LEVELS_CAP) continue;
            RgArena arena{(char *)scratch, scratch_bytes, 0};
            uint32_t *need = arena.take<uint32_t>(B.n_nodes);
            uint32_t *arrived = arena.take<uint32_t>(B.n_nodes);
            if (w == 2) refit_deep<2>(B, need, arrived, st);
            else if (w == 4) refit_deep<4>(B, need, arrived, st);
            else refit_deep<8>(B, need, arrived, st);
            RG_LAUNCH_CHECK();
        }
    }
    return rg_debug_done(RG_OK, st);
}

rg_status rg_refit_blas(rg_blas *blas, const float *verts, int64_t n_verts, const uint32_t *idx, int64_t n_tris,
                        void *scratch, uint64_t scratch_bytes, void *stream) {
    if (!blas || !verts || !idx) return RG_ERR_INVALID_ARG;
    return rg_refit_blas_many(blas, 1, &verts, &n_verts, &idx, &n_tris, scratch, scratch_bytes, stream);
}

rg_status rg_blas_state(const rg_blas *blas, float *lo, float *hi, uint32_t *status, void *stream) {
    if (!blas || !blas->buf || !lo || !hi || !status) return RG_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    RgBlasHdr h;
    RG_HIP(hipMemcpyAsync(&h, blas->buf, sizeof(RgBlasHdr), hipMemcpyDeviceToHost, st));
    RG_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < 3; ++k) {
        lo[k] = h.lo[k];
        hi[k] = h.hi[k];
    }
    *status = h.status;
    return RG_OK;
}

rg_status rg_blas_set_alpha(rg_blas *blas, const uint64_t *alpha, int32_t level, void *stream) {
    if (!blas || !blas->buf || (alpha && (level < 0 || level > RG_ALPHA_LEVEL_MAX))) return RG_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    k_blas_alpha<<<1, 1, 0, st>>>((RgBlasHdr *)blas->buf, (uint64_t)alpha, alpha ? (uint32_t)level : 0u);
    RG_LAUNCH_CHECK();
    blas->has_alpha = alpha ? 1 : 0;
    blas->alpha_level = alpha ? level : 0;
    return rg_debug_done(RG_OK, st);
}

rg_status rg_tlas_sizes(int64_t n_inst, const rg_build_opts *opts, rg_sizes *out) {
    Opts o;
    if (!out || n_inst < 1 || n_inst > RG_MAX_TRIS || !opts_ok(opts, &o) || !o.fits(n_inst)) return RG_ERR_INVALID_ARG;
    uint64_t a, b, c, d;
    out->bytes = tlas_out_bytes(n_inst, o.w, &a, &b, &c, &d);
    out->scratch_bytes = tlas_scratch_bytes(n_inst, 4096, o.builder);
    return RG_OK;
}

}  // extern "C"

namespace {

// Host tables of a top-level build, copied to the device in one piece
// (byte offsets, 8-aligned): matrices, blas ids, materials, flags,
// bottom-level addresses, a zero word (the invalid-bottom-level flag); the
// build's summary comes back behind them (stage = the whole staging area).
struct TlasLayout {
    size_t off_bid, off_mat, off_fl, off_info, off_flag, t_bytes, stage;
};
TlasLayout tlas_layout(int64_t n_inst, int32_t n_blas, bool with_flags) {
    const size_t n8 = (size_t)n_inst, t4 = (4 * n8 + 7) & ~size_t(7);
    TlasLayout L;
    L.off_bid = 48 * n8;
    L.off_mat = L.off_bid + t4;
    L.off_fl = L.off_mat + t4;
    L.off_info = L.off_fl + (with_flags ? t4 : 0);
    L.off_flag = L.off_info + sizeof(BlasInfo) * (size_t)n_blas;
    L.t_bytes = L.off_flag + 8;
    L.stage = L.t_bytes + 64;
    return L;
}

// A top-level build between enqueue and completion (the caller's pinned
// ticket for rg_build_tlas_async, a local for the synchronous call).
struct TlasTicket {
    uint64_t magic = 0;
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;   // nullptr: complete by waiting for the stream
    uint32_t *summary = nullptr;  // in the staging area: a one-workgroup summary, or the flag word
    bool deferred = false;
    RgLbvhOut lo;
    CollapseState coll;
    uint32_t hr[kRingWords];
    rg_tlas desc;
};
constexpr size_t kTlasTicketHead = (sizeof(TlasTicket) + 255) & ~size_t(255);
constexpr uint64_t kTlasTicketMagic = 0x7267544c41534174ull;

// Validates and enqueues a top-level build; T holds what completing it
// needs.  stage: host staging of tlas_stage_bytes (pinned for an
// asynchronous build), reused only after completion; async: the collapse
// goes no further than its first batch and nothing waits (the clustering and
// treelet builders, which step their rounds from the host, are refused).
// The synchronous top-level build's upload of its host tables: into a device
// buffer of the library's own (one per thread and device: the call waits for
// its summary before it returns, so the buffer is free again by then), on a
// stream of its own (default priority, not ordered with the null stream).
// The caller's stream waits for the copy's event just before the build reads
// the tables, so the copy overlaps whatever that stream still runs, such as
// the refit of the bottom levels the instances refer to, instead of queueing
// behind it (used only when that stream has work queued).  nullptr: no such
// buffer (the copy then goes on the caller's stream, into its scratch).
struct TableUpload {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    char *buf = nullptr;
    size_t cap = 0;
};
constexpr int kUploadDevices = 16;
TableUpload *table_upload(size_t bytes) {
    thread_local TableUpload per_dev[kUploadDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kUploadDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    TableUpload &U = per_dev[dev];
    if (!U.st && hipStreamCreateWithFlags(&U.st, hipStreamNonBlocking) != hipSuccess) {
        U.st = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    if (!U.done && hipEventCreateWithFlags(&U.done, hipEventDisableTiming) != hipSuccess) {
        U.done = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    if (bytes > U.cap) {
        if (U.buf) (void)hipFree(U.buf);
        U.buf = nullptr;
        U.cap = 0;
        const size_t want = ((bytes > (64u << 10) ? bytes : (64u << 10)) + 4095u) & ~(size_t)4095u;
        void *p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        U.buf = (char *)p;
        U.cap = want;
    }
    return &U;
}

rg_status tlas_enqueue(const rg_blas *blas, int32_t n_blas, const float *xform, const uint32_t *blas_id,
                       const uint32_t *inst_material, const uint32_t *inst_flags, int64_t n_inst,
                       const rg_build_opts *opts, void *out_buf, uint64_t out_bytes, void *scratch,
                       uint64_t scratch_bytes, hipStream_t st, char *stage, uint64_t stage_bytes, bool async,
                       TlasTicket *Tk, bool side_upload) {
    Opts o;
    if (!blas || !xform || !blas_id || !inst_material || !out_buf || !scratch) return RG_ERR_INVALID_ARG;
    if (n_blas < 1 || n_blas > 4096 || n_inst < 1 || n_inst > RG_MAX_TRIS) return RG_ERR_INVALID_ARG;
    if (!opts_ok(opts, &o) || !o.fits(n_inst)) return RG_ERR_INVALID_ARG;
    if (async && o.builder != RG_BUILDER_LBVH) return RG_ERR_UNSUPPORTED;
    const int32_t w = o.w;
    int32_t max_depth = 0;
    std::vector<BlasInfo> info((size_t)n_blas);
    for (int32_t b = 0; b < n_blas; ++b) {
        if (!blas[b].buf || blas[b].width != w) return RG_ERR_INVALID_ARG;
        if (blas[b].depth > max_depth) max_depth = blas[b].depth;
        info[b].nodes = (uint64_t)((char *)blas[b].buf + blas[b].nodes_off);
        info[b].tris = (uint64_t)((char *)blas[b].buf + blas[b].tris_off);
        info[b].hdr = (uint64_t)blas[b].buf;
    }
    const uint32_t known = 0xFFu | RG_INST_CULL_DISABLE | RG_INST_FLIP_FACING;
    if (inst_flags)
        for (int64_t i = 0; i < n_inst; ++i)
            if (inst_flags[i] & ~known) return RG_ERR_INVALID_ARG;
    for (int64_t i = 0; i < n_inst; ++i) {
        if (blas_id[i] >= (uint32_t)n_blas) return RG_ERR_INVALID_ARG;
        const float *m = xform + 12 * i;
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(m[k])) return RG_ERR_INVALID_ARG;
        double a = m[0], b = m[1], c = m[2], d = m[4], e = m[5], f = m[6], g = m[8], h = m[9], k = m[10];
        double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
        if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return RG_ERR_INVALID_ARG;
    }
    uint64_t no, io, ro, xo;
    uint64_t need = tlas_out_bytes(n_inst, w, &no, &io, &ro, &xo);
    if (out_bytes < need || scratch_bytes < tlas_scratch_bytes(n_inst, n_blas, o.builder))
        return RG_ERR_OUT_OF_MEMORY;
    const TlasLayout L = tlas_layout(n_inst, n_blas, inst_flags != nullptr);
    if (stage && stage_bytes < L.stage) return RG_ERR_OUT_OF_MEMORY;
    RgArena arena{(char *)scratch, scratch_bytes, 0};
    float *d_xf = (float *)((char *)out_buf + xo);  // kept: the trace calls recompute hits from it
    // everything from the host goes over in one copy, in this layout (byte
    // offsets, 8-aligned): matrices, blas ids, materials, flags, bottom-level
    // addresses, a zero word (the invalid-bottom-level flag); the summary of
    // the build comes back behind it
    const size_t n8 = (size_t)n_inst;
    const size_t off_bid = L.off_bid, off_mat = L.off_mat, off_fl = L.off_fl, off_info = L.off_info;
    const size_t off_flag = L.off_flag, t_bytes = L.t_bytes;
    char *d_tab = arena.take<char>(t_bytes);
    // only worth it while the caller's stream still has work queued: on an
    // idle stream the cross-stream wait costs more than the copy it hides
    bool busy = false;
    if (side_upload && !async) {
        busy = hipStreamQuery(st) == hipErrorNotReady;
        (void)hipGetLastError();  // "not ready" is an answer, not an error
    }
    TableUpload *up = busy ? table_upload(t_bytes) : nullptr;
    if (up) d_tab = up->buf;
    float *d_box = arena.take<float>(6 * n_inst);
    RgInst *d_rec = arena.take<RgInst>(n_inst);
    char *tab = stage;
    memcpy(tab, xform, 48 * n8);
    memcpy(tab + off_bid, blas_id, 4 * n8);
    memcpy(tab + off_mat, inst_material, 4 * n8);
    if (inst_flags) memcpy(tab + off_fl, inst_flags, 4 * n8);
    memcpy(tab + off_info, info.data(), sizeof(BlasInfo) * (size_t)n_blas);
    memset(tab + off_flag, 0, 8);
    uint32_t *summary = (uint32_t *)(tab + t_bytes);  // a one-workgroup build's summary, or the flag word
    uint32_t *d_flag = (uint32_t *)(d_tab + off_flag);
    if (async) RG_HIP(hipEventCreateWithFlags(&Tk->done, hipEventDisableTiming));  // before anything is enqueued
    if (up) {
        hipError_t e = hipMemcpyAsync(d_tab, tab, t_bytes, hipMemcpyHostToDevice, up->st);
        if (e == hipSuccess) e = hipEventRecord(up->done, up->st);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, up->done, 0);
        if (e != hipSuccess) (void)hipStreamSynchronize(up->st);  // the staging buffer may still be read
        RG_HIP(e);
    } else {
        RG_HIP(hipMemcpyAsync(d_tab, tab, t_bytes, hipMemcpyHostToDevice, st));
    }
    InstTables T;
    T.xform = (const float *)d_tab;
    T.blas_id = (const uint32_t *)(d_tab + off_bid);
    T.inst_mat = (const uint32_t *)(d_tab + off_mat);
    T.inst_flags = inst_flags ? (const uint32_t *)(d_tab + off_fl) : nullptr;
    T.blas = (const BlasInfo *)(d_tab + off_info);
    T.flags = d_flag;
    T.xf_keep = d_xf;
    char *base = (char *)out_buf;
    // up to kResidentMax instances (linear BVH): the instance step, the
    // build and the record reordering in one launch
    const bool fused = o.builder == RG_BUILDER_LBVH && n_inst <= kResidentMax;
    const TlasFuse F{T, d_rec, (RgInst *)(base + io), (uint32_t *)(base + ro)};
    if (!fused) {
        k_inst_setup<<<rg_blocks(n_inst, kThreads), kThreads, 0, st>>>(T, n_inst, d_box, d_rec);
        RG_LAUNCH_CHECK();
    }
    Tk->st = st;
    Tk->summary = summary;
    RgLbvhOut &lo = Tk->lo;
    lo.deferred = summary;
    lo.flag_in = d_flag;
    lo.key_shift = o.key_shift();
    lo.tlas_fuse = fused ? &F : nullptr;
    if (async) {
        lo.coll_async = &Tk->coll;
        lo.coll_hr = Tk->hr;
    }
    rg_status r = rg_lbvh_build(d_box, n_inst, w, 1, o.builder, o.radius, base + no, nullptr, nullptr, arena, st, &lo,
                                false, nullptr, nullptr, nullptr, nullptr);
    lo.tlas_fuse = nullptr;  // it pointed at this frame
    if (r != RG_OK) {
        (void)hipStreamSynchronize(st);  // the staging buffer may still be in use by a copy
        return r;
    }
    if (!fused)
        k_reorder_inst<<<rg_blocks(n_inst, kThreads), kThreads, 0, st>>>(d_rec, lo.ids, n_inst,
                                                                          (RgInst *)(base + io),
                                                                          (uint32_t *)(base + ro));
    Tk->deferred = lo.pending;  // else the flag word comes back on its own
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && !Tk->deferred) e = hipMemcpyAsync(summary, d_flag, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && async) e = hipEventRecord(Tk->done, st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        RG_HIP(e);
    }
    rg_tlas &d = Tk->desc;
    d = rg_tlas{};
    d.buf = out_buf;
    d.nodes_off = no;
    d.inst_off = io;
    d.rec_off = ro;
    d.xf_off = xo;
    d.n_inst = n_inst;
    d.width = w;
    d.max_blas_depth = max_depth;
    for (int32_t b = 0; b < n_blas; ++b)
        if (blas[b].has_alpha) d.has_inst_flags = 1;
    if (inst_flags)
        for (int64_t i = 0; i < n_inst; ++i)
            if (inst_flags[i] != RG_INST_MASK_ALL) d.has_inst_flags = 1;
    return RG_OK;
}

// Completes an enqueued top-level build: waits (for its event, else its
// stream), finishes a collapse left after its first batch, fills *out.
rg_status tlas_complete(TlasTicket *Tk, rg_tlas *out) {
    if (Tk->done) {
        const hipError_t we = hipEventSynchronize(Tk->done);
        (void)hipEventDestroy(Tk->done);
        Tk->done = nullptr;
        RG_HIP(we);
    } else {
        RG_HIP(hipStreamSynchronize(Tk->st));
    }
    RgLbvhOut &lo = Tk->lo;
    rg_status r = rg_lbvh_finish(&lo, true);
    if (r == RG_OK && !Tk->deferred && lo.coll_async) {
        if (Tk->coll.depth == 0) {
            r = collapse_absorb(Tk->coll, Tk->hr);
            if (r == RG_OK && Tk->coll.depth == 0 && (r = collapse_launch(Tk->coll, Tk->st)) == RG_OK)
                r = collapse_finish(Tk->coll, Tk->st, Tk->hr);
        }
        lo.depth = Tk->coll.depth;
        lo.n_nodes = (int64_t)Tk->coll.n_nodes;
    }
    if (r != RG_OK) return r;
    if (Tk->deferred ? lo.flag : Tk->summary[0]) return RG_ERR_INVALID_ARG;  // a bottom level was refitted to invalid vertex data
    rg_tlas d = Tk->desc;
    d.n_nodes = lo.n_nodes;
    d.depth = lo.depth;
    for (int k = 0; k < 3; ++k) {
        d.lo[k] = lo.lo[k];
        d.hi[k] = lo.hi[k];
    }
    *out = d;
    return RG_OK;
}

}  // namespace

extern "C" {

rg_status rg_build_tlas_ex(const rg_blas *blas, int32_t n_blas, const float *xform, const uint32_t *blas_id,
                           const uint32_t *inst_material, const uint32_t *inst_flags, int64_t n_inst,
                           const rg_build_opts *opts, void *out_buf, uint64_t out_bytes, void *scratch,
                           uint64_t scratch_bytes, void *stream, rg_tlas *out) {
    if (!out || n_inst < 1 || n_inst > RG_MAX_TRIS || n_blas < 1 || n_blas > 4096) return RG_ERR_INVALID_ARG;
    const TlasLayout L = tlas_layout(n_inst, n_blas, inst_flags != nullptr);
    std::vector<char> fallback;
    char *tab = pinned_staging(L.stage);
    if (!tab) {
        fallback.resize(L.stage);
        tab = fallback.data();
    }
    TlasTicket T;
    rg_status r = tlas_enqueue(blas, n_blas, xform, blas_id, inst_material, inst_flags, n_inst, opts, out_buf,
                               out_bytes, scratch, scratch_bytes, (hipStream_t)stream, tab, L.stage, false, &T,
                               fallback.empty());
    if (r != RG_OK) return r;
    return tlas_complete(&T, out);
}

rg_status rg_tlas_ticket_bytes(int64_t n_inst, int32_t n_blas, int32_t with_flags, uint64_t *bytes) {
    if (!bytes || n_inst < 1 || n_inst > RG_MAX_TRIS || n_blas < 1 || n_blas > 4096) return RG_ERR_INVALID_ARG;
    *bytes = kTlasTicketHead + tlas_layout(n_inst, n_blas, with_flags != 0).stage;
    return RG_OK;
}

rg_status rg_build_tlas_async(const rg_blas *blas, int32_t n_blas, const float *xform, const uint32_t *blas_id,
                              const uint32_t *inst_material, const uint32_t *inst_flags, int64_t n_inst,
                              const rg_build_opts *opts, void *out_buf, uint64_t out_bytes, void *scratch,
                              uint64_t scratch_bytes, void *stream, void *ticket, uint64_t ticket_bytes) {
    if (!ticket || ((uintptr_t)ticket & 255u) || ticket_bytes < kTlasTicketHead) return RG_ERR_INVALID_ARG;
    TlasTicket *T = new (ticket) TlasTicket();
    rg_status r = tlas_enqueue(blas, n_blas, xform, blas_id, inst_material, inst_flags, n_inst, opts, out_buf,
                               out_bytes, scratch, scratch_bytes, (hipStream_t)stream,
                               (char *)ticket + kTlasTicketHead, ticket_bytes - kTlasTicketHead, true, T, false);
    if (r != RG_OK) {
        if (T->done) (void)hipEventDestroy(T->done);
        T->magic = 0;
        return r;
    }
    T->magic = kTlasTicketMagic;
    return RG_OK;
}

rg_status rg_build_tlas_finish(void *ticket, rg_tlas *out) {
    if (!ticket || !out || ((uintptr_t)ticket & 255u)) return RG_ERR_INVALID_ARG;
    TlasTicket *T = static_cast<TlasTicket *>(ticket);
    if (T->magic != kTlasTicketMagic) return RG_ERR_INVALID_ARG;
    T->magic = 0;  // a ticket completes once
    return tlas_complete(T, out);
}

rg_status rg_build_tlas(const rg_blas *blas, int32_t n_blas, const float *xform, const uint32_t *blas_id,
                        const uint32_t *inst_material, int64_t n_inst, const rg_build_opts *opts, void *out_buf,
                        uint64_t out_bytes, void *scratch, uint64_t scratch_bytes, void *stream, rg_tlas *out) {
    return rg_build_tlas_ex(blas, n_blas, xform, blas_id, inst_material, nullptr, n_inst, opts, out_buf, out_bytes,
                            scratch, scratch_bytes, stream, out);
}

rg_status rg_lbvh_stages(const float *verts, int64_t n_verts, const uint32_t *idx, int64_t n_tris,
                         const rg_build_opts *opts, uint64_t *keys, uint32_t *ids, int32_t *left, int32_t *right,
                         float *boxes, void *scratch, uint64_t scratch_bytes, void *stream) {
    Opts o;
    if (!verts || !idx || !keys || !ids || !boxes || !scratch) return RG_ERR_INVALID_ARG;
    if (n_tris > 1 && (!left || !right)) return RG_ERR_INVALID_ARG;
    if (n_verts < 1 || n_tris < 1 || n_tris > RG_MAX_TRIS || !opts_ok(opts, &o) || !o.fits(n_tris))
        return RG_ERR_INVALID_ARG;
    if (scratch_bytes < blas_scratch_bytes(n_tris, o.builder)) return RG_ERR_OUT_OF_MEMORY;
    hipStream_t st = (hipStream_t)stream;
    RgArena arena{(char *)scratch, scratch_bytes, 0};
    float *pbox = arena.take<float>(6 * n_tris);
    uint32_t *flags = arena.take<uint32_t>(8);
    k_fill_u32<<<1, 64, 0, st>>>(flags, 0u, 1);
    k_tri_boxes<<<rg_blocks(n_tris, kThreads), kThreads, 0, st>>>(verts, n_verts, idx, n_tris, pbox, flags);
    RG_LAUNCH_CHECK();
    uint32_t hflags = 0;
    RG_HIP(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, st));
    RG_HIP(hipStreamSynchronize(st));
    if (hflags) return RG_ERR_INVALID_ARG;
    RgLbvhOut lo;
    lo.key_shift = o.key_shift();
    rg_status r = rg_lbvh_build(pbox, n_tris, o.w, o.leaf, o.builder, o.radius, nullptr, nullptr, nullptr, arena,
                                st, &lo, true, keys, left, right, boxes);
    if (r != RG_OK) return r;
    RG_HIP(hipMemcpyAsync(ids, lo.ids, 4 * n_tris, hipMemcpyDeviceToDevice, st));
    RG_HIP(hipStreamSynchronize(st));
    return RG_OK;
}

}  // extern "C"
