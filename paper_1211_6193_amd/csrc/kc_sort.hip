// LDS-staged LSD radix sort of 64-bit access records on gfx950.
//
// Large inputs: one pass per 8-bit digit over the requested bit range, three
// kernels per pass:
//   k_rs_hist     per-tile digit histograms, digit-major ([digit][tile])
//   k_rs_scan     one workgroup per digit: exclusive scan of the digit's
//                 column over the tiles, and the digit's total
//   k_rs_scatter  digit bases (scan of the 256 totals), stable rank inside the
//                 tile (wave-level 8-ballot digit match), reorder the tile in
//                 LDS, write each digit's run contiguously.
// A tile is 4 waves x 64 lanes x ITEMS keys; wave w owns a contiguous quarter
// of the tile so ranks need no cross-wave synchronisation until the end.
// Small inputs (a replay's records): k_rs_small sorts in one workgroup of 16
// waves, all passes in one launch, ping-ponging between the two buffers.
#include "kc_internal.h"

#include <mutex>

namespace kc {

namespace {

constexpr int WAVE = 64;
constexpr int WG = 256;
constexpr int NW = WG / WAVE;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// The sort orders records by a virtual key that drops the unused high bits of
// the epoch field: V = (k >> s_blk) . (epoch low ueb bits) . (low pb payload bits).
__device__ __forceinline__ uint64_t vkey(uint64_t k, const VKey &v) {
    const uint64_t hi = (k >> v.s_blk) << (v.ueb + v.pb);
    const uint64_t ep = v.ueb ? ((k >> v.s_ep) & ((1ull << v.ueb) - 1ull)) << v.pb : 0ull;
    const uint64_t lo = v.pb ? (k & ((1ull << v.pb) - 1ull)) : 0ull;
    return hi | ep | lo;
}
__device__ __forceinline__ uint32_t digit_of(uint64_t k, const VKey &v, uint32_t shift, uint32_t bits) {
    return (uint32_t)(vkey(k, v) >> shift) & ((1u << bits) - 1u);
}

template <int ITEMS>
__global__ void __launch_bounds__(WG) k_rs_hist(const uint64_t *__restrict__ keys, uint64_t n, VKey vk, uint32_t shift,
                                                uint32_t bits, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[NW][256];
    for (int i = threadIdx.x; i < NW * 256; i += WG) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t w = threadIdx.x / WAVE;
    const uint64_t tile0 = (uint64_t)blockIdx.x * (WG * ITEMS);
    const uint64_t seg0 = tile0 + (uint64_t)w * (WAVE * ITEMS);
#pragma unroll 4
    for (int j = 0; j < ITEMS; j++) {
        uint64_t idx = seg0 + (uint64_t)j * WAVE + lane_id();
        if (idx < n) atomicAdd(&h[w][digit_of(keys[idx], vk, shift, bits)], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < 256; d += WG) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < NW; q++) s += h[q][d];
        hist[(size_t)d * gridDim.x + blockIdx.x] = s;
    }
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp, uint32_t &total) {
    const uint32_t t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    uint32_t x = v;
    for (uint32_t o = 1; o < WG; o <<= 1) {
        const uint32_t y = t >= o ? tmp[t - o] : 0;
        __syncthreads();
        x += y;
        tmp[t] = x;
        __syncthreads();
    }
    total = tmp[WG - 1];
    __syncthreads();
    return x - v;
}

// Column scan of one digit (blockIdx.x): hist[d][t] becomes the exclusive
// start of tile t within digit d, tot[d] the digit's total.
__global__ void __launch_bounds__(WG) k_rs_scan(uint32_t *__restrict__ hist, uint32_t n_tiles,
                                                uint32_t *__restrict__ tot) {
    __shared__ uint32_t tmp[WG];
    uint32_t *col = hist + (size_t)blockIdx.x * n_tiles;
    const uint32_t per = (n_tiles + WG - 1) / WG;
    const uint32_t c0 = min(n_tiles, threadIdx.x * per), c1 = min(c0 + per, n_tiles);
    uint32_t sum = 0;
    for (uint32_t c = c0; c < c1; c++) sum += col[c];
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, tmp, total);
    for (uint32_t c = c0; c < c1; c++) {
        const uint32_t v = col[c];
        col[c] = run;
        run += v;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

template <int ITEMS>
__global__ void __launch_bounds__(WG) k_rs_scatter(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                   uint64_t n, VKey vk, uint32_t shift, uint32_t bits,
                                                   const uint32_t *__restrict__ offs,
                                                   const uint32_t *__restrict__ tot) {
    constexpr int TILE = WG * ITEMS;
    __shared__ uint64_t buf[TILE];
    __shared__ uint32_t wc[NW][256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t goff[256];
    const uint32_t w = threadIdx.x / WAVE;
    const uint32_t lane = lane_id();
    for (int i = threadIdx.x; i < NW * 256; i += WG) (&wc[0][0])[i] = 0;
    {   // global start of each digit's run of this tile: digit base + tiles before
        const uint32_t d = threadIdx.x;
        uint32_t all;
        const uint32_t base = block_exclusive_scan(tot[d], tstart, all);
        goff[d] = base + offs[(size_t)d * gridDim.x + blockIdx.x];
    }
    __syncthreads();

    const uint64_t tile0 = (uint64_t)blockIdx.x * TILE;
    const uint64_t seg0 = tile0 + (uint64_t)w * (WAVE * ITEMS);
    uint64_t k[ITEMS];
    uint32_t rank[ITEMS];
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint64_t idx = seg0 + (uint64_t)j * WAVE + lane;
        const bool valid = idx < n;
        k[j] = valid ? in[idx] : 0ull;
        const uint32_t d = digit_of(k[j], vk, shift, bits);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; b++) {
            if (b < bits) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(valid && bit);
                peers &= bit ? bb : ~bb;
            }
        }
        const uint32_t leader = valid ? (uint32_t)__ffsll((long long)peers) - 1 : 0;
        uint32_t old = 0;
        if (valid && lane == leader) {
            old = wc[w][d];
            wc[w][d] = old + (uint32_t)__popcll(peers);
        }
        old = __shfl(old, (int)leader);
        rank[j] = valid ? old + (uint32_t)__popcll(peers & lt) : 0xFFFFFFFFu;
    }
    __syncthreads();
    // per digit: tile-local start and per-wave base positions
    {
        const uint32_t d = threadIdx.x;     // WG == 256 digits
        uint32_t c[NW], tot = 0;
#pragma unroll
        for (int q = 0; q < NW; q++) { c[q] = wc[q][d]; tot += c[q]; }
        tstart[d] = tot;
        __syncthreads();
        uint32_t x = tot;
        for (uint32_t o = 1; o < 256; o <<= 1) {
            uint32_t y = d >= o ? tstart[d - o] : 0;
            __syncthreads();
            x += y;
            tstart[d] = x;
            __syncthreads();
        }
        const uint32_t start = x - tot;
        __syncthreads();
        tstart[d] = start;
        uint32_t run = start;
#pragma unroll
        for (int q = 0; q < NW; q++) { wc[q][d] = run; run += c[q]; }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        if (rank[j] != 0xFFFFFFFFu) {
            const uint32_t d = digit_of(k[j], vk, shift, bits);
            buf[wc[w][d] + rank[j]] = k[j];
        }
    }
    __syncthreads();
    const uint64_t tile_n = (n - tile0) < (uint64_t)TILE ? (n - tile0) : (uint64_t)TILE;
    for (uint32_t p = threadIdx.x; p < tile_n; p += WG) {
        const uint64_t key = buf[p];
        const uint32_t d = digit_of(key, vk, shift, bits);
        out[(uint64_t)goff[d] + (p - tstart[d])] = key;
    }
}

template <int ITEMS>
hipError_t sort_passes(uint64_t *keys, uint64_t n, const VKey &vk, uint32_t hi, uint32_t digit, SortScratch &sc,
                       hipStream_t s, uint64_t **out) {
    constexpr uint64_t TILE = WG * ITEMS;
    const uint32_t n_tiles = (uint32_t)((n + TILE - 1) / TILE);
    uint64_t *a = keys, *b = sc.alt;
    for (uint32_t sh = 0; sh < hi; sh += digit) {
        const uint32_t bits = (hi - sh) < digit ? (hi - sh) : digit;
        hipLaunchKernelGGL(k_rs_hist<ITEMS>, dim3(n_tiles), dim3(WG), 0, s, a, n, vk, sh, bits, sc.hist);
        hipLaunchKernelGGL(k_rs_scan, dim3(256), dim3(WG), 0, s, sc.hist, n_tiles, sc.part);
        hipLaunchKernelGGL(k_rs_scatter<ITEMS>, dim3(n_tiles), dim3(WG), 0, s, a, b, n, vk, sh, bits, sc.hist,
                           sc.part);
        uint64_t *t = a; a = b; b = t;
    }
    *out = a;
    return hipGetLastError();
}

// ---- one-workgroup sort of small inputs --------------------------------------
constexpr int SWG = 1024;
constexpr int SNW = SWG / WAVE;
constexpr uint64_t SMALL_N = 16384;     // keys staged in LDS: 128 KiB

__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (uint32_t b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(valid && bit);
        peers &= bit ? bb : ~bb;
    }
    return peers;
}

// All passes over keys[0..n) (n <= SMALL_N) ping-ponging with alt; the
// result is in keys when the number of passes is even, else in alt.  Each pass
// stages the input in LDS (coalesced, every load in flight at once), counts
// digits per wave over the wave's contiguous chunk (8-ballot match), scans the
// counters digit-major / wave-minor and writes every wave's keys in order
// (stable) to the other buffer: one round trip to memory per pass.
__global__ void __launch_bounds__(SWG) k_rs_small(uint64_t *__restrict__ keys, uint64_t *__restrict__ alt, uint32_t n,
                                                  VKey vk, uint32_t hi) {
    extern __shared__ uint64_t stage[];     // n keys
    __shared__ uint32_t wc[SNW][256];
    __shared__ uint32_t wtot[4];
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    const uint32_t per = (n + SNW - 1) / SNW;
    const uint32_t c0 = min(n, w * per), c1 = min(n, c0 + per);
    const uint64_t lt = (1ull << lane) - 1ull;
    uint64_t *a = keys, *b = alt;
    for (uint32_t sh = 0; sh < hi; sh += 8) {
        const uint32_t bits = (hi - sh) < 8 ? (hi - sh) : 8;
        {   // all loads in flight before the first LDS store
            constexpr int R = (int)(SMALL_N / SWG);
            uint64_t v[R];
#pragma unroll
            for (int j = 0; j < R; j++) {
                const uint32_t i = threadIdx.x + (uint32_t)j * SWG;
                v[j] = i < n ? a[i] : 0ull;
            }
#pragma unroll
            for (int j = 0; j < R; j++) {
                const uint32_t i = threadIdx.x + (uint32_t)j * SWG;
                if (i < n) stage[i] = v[j];
            }
        }
        for (uint32_t d = lane; d < 256; d += WAVE) wc[w][d] = 0;
        __syncthreads();
        for (uint32_t base = c0; base < c1; base += WAVE) {
            const bool valid = base + lane < c1;
            const uint32_t d = valid ? digit_of(stage[base + lane], vk, sh, bits) : 0u;
            const uint64_t peers = digit_peers(d, valid);
            if (valid && lane == (uint32_t)__ffsll((long long)peers) - 1) wc[w][d] += (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // thread d < 256: digit d summed over the waves, exclusive scan over
        // digits (waves of 64 digits, then the four wave totals), and the
        // per-wave starts of digit d in wave order
        uint32_t dsum = 0, dincl = 0;
        if (threadIdx.x < 256) {
#pragma unroll
            for (int q = 0; q < SNW; q++) dsum += wc[q][threadIdx.x];
            dincl = dsum;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const uint32_t y = __shfl_up(dincl, o);
                if ((int)lane >= o) dincl += y;
            }
            if (lane == WAVE - 1) wtot[w] = dincl;
        }
        __syncthreads();
        if (threadIdx.x < 256) {
            uint32_t run = dincl - dsum;
            for (uint32_t q = 0; q < w; q++) run += wtot[q];
#pragma unroll
            for (int q = 0; q < SNW; q++) {
                const uint32_t x = wc[q][threadIdx.x];
                wc[q][threadIdx.x] = run;
                run += x;
            }
        }
        __syncthreads();
        for (uint32_t base = c0; base < c1; base += WAVE) {
            const bool valid = base + lane < c1;
            const uint64_t key = valid ? stage[base + lane] : 0ull;
            const uint32_t d = valid ? digit_of(key, vk, sh, bits) : 0u;
            const uint64_t peers = digit_peers(d, valid);
            const uint32_t leader = valid ? (uint32_t)__ffsll((long long)peers) - 1 : 0u;
            uint32_t old = 0;
            if (valid && lane == leader) {
                old = wc[w][d];
                wc[w][d] = old + (uint32_t)__popcll(peers);
            }
            old = __shfl(old, (int)leader);
            if (valid) b[old + (uint32_t)__popcll(peers & lt)] = key;
        }
        __syncthreads();        // the next pass reads what other waves wrote (one CU: the barrier suffices)
        uint64_t *t = a; a = b; b = t;
    }
}

}  // namespace

// Raise the small sort's dynamic LDS limit, once per device (batch worker
// threads may sort for the first time together).
static hipError_t raise_small_lds_limit() {
    constexpr int kMaxDevices = 64;
    static std::once_flag once[kMaxDevices];
    static hipError_t result[kMaxDevices];
    int dev = 0;
    const hipError_t eg = hipGetDevice(&dev);
    if (eg != hipSuccess) return eg;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(once[dev], [dev] {
        result[dev] = hipFuncSetAttribute((const void *)k_rs_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)(SMALL_N * 8));
    });
    return result[dev];
}

size_t radix_hist_entries(uint64_t n, uint32_t tile) {
    const uint64_t n_tiles = (n + tile - 1) / tile;
    return (size_t)(n_tiles ? n_tiles : 1) * 256;
}

hipError_t radix_sort(uint64_t *keys, uint64_t n, const VKey &vk, SortScratch &sc, uint32_t tile,
                      hipStream_t s, uint64_t **out, uint32_t digit) {
    if (digit < 4 || digit > 8) digit = 8;
    *out = keys;
    if (n <= 1 || vk.vbits == 0) return hipSuccess;
    if (n <= SMALL_N) {
        const hipError_t ea = raise_small_lds_limit();
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(k_rs_small, dim3(1), dim3(SWG), n * 8, s, keys, sc.alt, (uint32_t)n, vk, vk.vbits);
        *out = ((vk.vbits + 7) / 8) % 2 ? sc.alt : keys;
        return hipGetLastError();
    }
    switch (tile) {
    case 1024: return sort_passes<4>(keys, n, vk, vk.vbits, digit, sc, s, out);
    case 2048: return sort_passes<8>(keys, n, vk, vk.vbits, digit, sc, s, out);
    case 8192: return sort_passes<32>(keys, n, vk, vk.vbits, digit, sc, s, out);
    case 4096: return sort_passes<16>(keys, n, vk, vk.vbits, digit, sc, s, out);
    default: return sort_passes<8>(keys, n, vk, vk.vbits, digit, sc, s, out);
    }
}

}  // namespace kc
