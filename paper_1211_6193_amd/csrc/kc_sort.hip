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
//
// Single-pass digit scatter (SortScratch::os set, large inputs): one kernel
// counts the digits of every pass in one read of the keys (k_os_hist), one
// workgroup per pass scans the counts into digit bases (k_os_bases), then one
// kernel per pass (k_os_scatter) reads and writes each key once.  Workgroup
// t ranks tile t like k_rs_scatter, publishes its per-digit counts, and finds
// the keys of each digit in earlier tiles by walking back over the published
// words (a count, or an inclusive prefix that ends the walk) before
// publishing its own inclusive prefix.  The tile is the workgroup index, not
// a ticket from a global counter: on this chip one atomic counter for every
// workgroup costs about 57 ns per tile, serialised (3.7 ms a pass over 66k
// tiles).  The dispatcher hands out workgroups in index order, so the lowest
// unfinished tile's workgroup is always running and every wait ends; each
// wait is still bounded (should dispatch ever run out of order), and a
// wait that runs out marks the pass stalled (the stall word holds the pass +
// 1): later passes do nothing, and the host finishes the sort with
// three-kernel passes from the stalled pass's input, which no kernel has
// overwritten.
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
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    const uint64_t tile0 = (uint64_t)blockIdx.x * (WG * ITEMS);
    const uint64_t seg0 = tile0 + (uint64_t)w * (WAVE * ITEMS);
    uint64_t k[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {       // every load in flight before the first count
        const uint64_t idx = seg0 + (uint64_t)j * WAVE + lane;
        k[j] = idx < n ? keys[idx] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const bool valid = seg0 + (uint64_t)j * WAVE + lane < n;
        const uint64_t vm = __ballot(valid);
        if (vm == 0) break;                 // valid lanes form a prefix: lane 0 holds a key
        const uint32_t d = digit_of(k[j], vk, shift, bits);
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
        // a wave of one digit (the high digits of one block's records) counts once
        if (__ballot(valid && d != d0) == 0) {
            if (lane == 0) atomicAdd(&h[w][d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[w][d], 1u);
        }
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

// Exclusive scan of one value per thread over a workgroup of NWAVES waves:
// wave scans, then the wave totals through LDS (two barriers).
template <int NWAVES>
__device__ __forceinline__ uint32_t block_exclusive_scan_waves(uint32_t v, uint32_t *wtot, uint32_t &total) {
    const uint32_t lane = lane_id(), w = threadIdx.x / WAVE;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if ((int)lane >= o) x += y;
    }
    if (lane == WAVE - 1) wtot[w] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NWAVES; q++) {
        const uint32_t t = wtot[q];
        pre += (uint32_t)q < w ? t : 0u;
        tot += t;
    }
    __syncthreads();                        // wtot is rewritten by the next call
    total = tot;
    return pre + x - v;
}

// Column scan of one digit (blockIdx.x): hist[d][t] becomes the exclusive
// start of tile t within digit d, tot[d] the digit's total.  One workgroup of
// SCAN_WG threads per digit takes the column in chunks of SCAN_WG x SCAN_K
// entries, SCAN_K consecutive ones per thread; the next chunk's loads are in
// flight while the current one is scanned.
constexpr int SCAN_WG = 1024;
constexpr int SCAN_K = 16;
__global__ void __launch_bounds__(SCAN_WG) k_rs_scan(uint32_t *__restrict__ hist, uint32_t n_tiles,
                                                     uint32_t *__restrict__ tot) {
    __shared__ uint32_t wtot[SCAN_WG / WAVE];
    uint32_t *col = hist + (size_t)blockIdx.x * n_tiles;
    constexpr uint32_t CHUNK = SCAN_WG * SCAN_K;
    uint32_t cur[SCAN_K], nxt[SCAN_K] = {};
    auto load = [&](uint32_t base, uint32_t *v) {
        const uint32_t c0 = base + threadIdx.x * SCAN_K;
#pragma unroll
        for (int i = 0; i < SCAN_K; i++) v[i] = c0 + i < n_tiles ? col[c0 + i] : 0u;
    };
    load(0, cur);
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n_tiles; base += CHUNK) {
        if (base + CHUNK < n_tiles) load(base + CHUNK, nxt);
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < SCAN_K; i++) sum += cur[i];
        uint32_t total;
        uint32_t run = carry + block_exclusive_scan_waves<SCAN_WG / WAVE>(sum, wtot, total);
        const uint32_t c0 = base + threadIdx.x * SCAN_K;
#pragma unroll
        for (int i = 0; i < SCAN_K; i++) {
            if (c0 + i < n_tiles) col[c0 + i] = run;
            run += cur[i];
        }
        carry += total;
#pragma unroll
        for (int i = 0; i < SCAN_K; i++) cur[i] = nxt[i];
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8); the
// scatter gives each XCD a contiguous range of tiles instead, so the runs that
// neighbouring tiles write for one digit, which share cache lines at their
// ends, meet in one XCD's L2 before they reach HBM.
constexpr uint32_t N_XCD = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t x = b % N_XCD, per = n / N_XCD, rem = n % N_XCD;
    return x * per + (x < rem ? x : rem) + b / N_XCD;
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
    __shared__ uint32_t wtot[NW];
    const uint32_t w = threadIdx.x / WAVE;
    const uint32_t lane = lane_id();
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    for (int i = threadIdx.x; i < NW * 256; i += WG) (&wc[0][0])[i] = 0;
    {   // global start of each digit's run of this tile: digit base + tiles before
        const uint32_t d = threadIdx.x;
        uint32_t all;
        const uint32_t base = block_exclusive_scan_waves<NW>(tot[d], wtot, all);
        goff[d] = base + offs[(size_t)d * gridDim.x + tile];
    }
    __syncthreads();

    const uint64_t tile0 = (uint64_t)tile * TILE;
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
        uint32_t all;
        const uint32_t start = block_exclusive_scan_waves<NW>(tot, wtot, all);
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

// Passes from digit shift sh0 up, reading a first (b: the other buffer).
template <int ITEMS>
hipError_t sort_passes(uint64_t *a, uint64_t *b, uint64_t n, const VKey &vk, uint32_t sh0, uint32_t hi,
                       uint32_t digit, SortScratch &sc, hipStream_t s, uint64_t **out) {
    constexpr uint64_t TILE = WG * ITEMS;
    const uint32_t n_tiles = (uint32_t)((n + TILE - 1) / TILE);
    for (uint32_t sh = sh0; sh < hi; sh += digit) {
        const uint32_t bits = (hi - sh) < digit ? (hi - sh) : digit;
        hipLaunchKernelGGL(k_rs_hist<ITEMS>, dim3(n_tiles), dim3(WG), 0, s, a, n, vk, sh, bits, sc.hist);
        hipLaunchKernelGGL(k_rs_scan, dim3(256), dim3(SCAN_WG), 0, s, sc.hist, n_tiles, sc.part);
        hipLaunchKernelGGL(k_rs_scatter<ITEMS>, dim3(n_tiles), dim3(WG), 0, s, a, b, n, vk, sh, bits, sc.hist,
                           sc.part);
        uint64_t *t = a; a = b; b = t;
    }
    *out = a;
    return hipGetLastError();
}

// ---- single-pass digit scatter ---------------------------------------------------
constexpr uint32_t OS_AGG = 1u << 30;        // published: the tile's own count
constexpr uint32_t OS_INC = 2u << 30;        // published: inclusive prefix over tiles 0..t
constexpr uint32_t OS_FLAGS = 3u << 30;
constexpr uint32_t OS_VALUE = OS_AGG - 1u;
constexpr int OS_WINDOW = 16;                // predecessors read per look-back step

// Digit counts of every pass: workgroup-private counters in LDS, one global
// add per counter at the end.  A wave whose valid lanes share a digit (the
// high digits of runs of one block's records) adds once.
__global__ void __launch_bounds__(WG) k_os_hist(const uint64_t *__restrict__ keys, uint64_t n, VKey vk, uint32_t hi,
                                                uint32_t digit, uint32_t passes, uint32_t *__restrict__ ghist) {
    __shared__ uint32_t h[RADIX_OS_PASSES * 256];
    for (uint32_t i = threadIdx.x; i < passes * 256; i += WG) h[i] = 0;
    __syncthreads();
    const uint64_t per = ((n + gridDim.x - 1) / gridDim.x + WAVE - 1) / WAVE * WAVE;
    const uint64_t c0 = (uint64_t)blockIdx.x * per;
    const uint64_t c1 = c0 + per < n ? c0 + per : n;
    const uint32_t lane = lane_id();
    constexpr int U = 4;
    for (uint64_t base = c0 + (threadIdx.x / WAVE) * WAVE; base < c1; base += (uint64_t)WG * U) {
        uint64_t v[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t i = base + (uint64_t)u * WG + lane;
            ok[u] = i < c1;
            v[u] = ok[u] ? vkey(keys[i], vk) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t vm = __ballot(ok[u]);
            if (vm == 0) continue;          // lane 0 holds a key whenever any lane does
            for (uint32_t p = 0; p < passes; p++) {
                const uint32_t sh = p * digit;
                const uint32_t bits = (hi - sh) < digit ? (hi - sh) : digit;
                const uint32_t d = (uint32_t)(v[u] >> sh) & ((1u << bits) - 1u);
                const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
                if (__ballot(ok[u] && d != d0) == 0) {
                    if (lane == 0) atomicAdd(&h[p * 256 + d0], (uint32_t)__popcll(vm));
                } else if (ok[u]) {
                    atomicAdd(&h[p * 256 + d], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < passes * 256; i += WG)
        if (h[i]) atomicAdd(&ghist[i], h[i]);
}

// Pass blockIdx.x: exclusive scan of its 256 digit counts.
__global__ void __launch_bounds__(WG) k_os_bases(const uint32_t *__restrict__ ghist, uint32_t *__restrict__ gbase) {
    __shared__ uint32_t tmp[WG];
    const uint32_t off = blockIdx.x * 256 + threadIdx.x;
    uint32_t total;
    gbase[off] = block_exclusive_scan(ghist[off], tmp, total);
}

template <int ITEMS>
__global__ void __launch_bounds__(WG) k_os_scatter(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                   uint64_t n, VKey vk, uint32_t shift, uint32_t bits, uint32_t pass,
                                                   const uint32_t *__restrict__ gbase, uint32_t *status,
                                                   uint32_t *__restrict__ status_next, uint32_t *stall,
                                                   uint32_t spin_limit) {
    constexpr int TILE = WG * ITEMS;
    __shared__ uint64_t buf[TILE];
    __shared__ uint32_t wc[NW][256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t wtot[NW];
    __shared__ uint32_t skip_sh;
    const uint32_t w = threadIdx.x / WAVE;
    const uint32_t lane = lane_id();
    for (int i = threadIdx.x; i < NW * 256; i += WG) (&wc[0][0])[i] = 0;
    if (threadIdx.x == 0) skip_sh = __hip_atomic_load(stall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (skip_sh) return;                        // an earlier pass stalled: its input stays as it is
    const uint32_t tile = blockIdx.x;
    status_next[(size_t)tile * 256 + threadIdx.x] = 0u;     // the next pass's words of this tile index

    const uint64_t tile0 = (uint64_t)tile * TILE;
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
    {
        const uint32_t d = threadIdx.x;     // WG == 256 digits
        uint32_t c[NW], tot = 0;
#pragma unroll
        for (int q = 0; q < NW; q++) { c[q] = wc[q][d]; tot += c[q]; }
        uint32_t *mine = status + (size_t)tile * 256 + d;
        __hip_atomic_store(mine, (tile == 0 ? OS_INC : OS_AGG) | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // tile-local start of each digit and per-wave bases
        uint32_t all;
        const uint32_t start = block_exclusive_scan_waves<NW>(tot, wtot, all);
        tstart[d] = start;
        uint32_t run = start;
#pragma unroll
        for (int q = 0; q < NW; q++) { wc[q][d] = run; run += c[q]; }
        // keys of digit d in earlier tiles: OS_WINDOW predecessors read at
        // once (every load in flight together), consumed nearest first up to
        // an inclusive prefix; a word not yet published is polled again
        uint32_t excl = 0;
        if (tile > 0) {
            int64_t j = (int64_t)tile - 1;          // nearest predecessor not yet consumed
            uint32_t spins = 0;
            bool stalled = false;
            for (;;) {
                uint32_t v[OS_WINDOW];
#pragma unroll
                for (int u = 0; u < OS_WINDOW; u++)
                    v[u] = j - u >= 0 ? __hip_atomic_load(status + (size_t)(j - u) * 256 + d, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : OS_INC;     // never consumed: tile 0 publishes an inclusive prefix
                bool done = false;
                int used = 0;
#pragma unroll
                for (int u = 0; u < OS_WINDOW; u++) {
                    if (done || used < u) continue;
                    const uint32_t f = v[u] & OS_FLAGS;
                    if (f == 0u) continue;          // not published yet: stop here
                    excl += v[u] & OS_VALUE;
                    used = u + 1;
                    done = f == OS_INC;
                }
                if (done) break;
                j -= used;
                if (used < OS_WINDOW) {             // stopped at a word not yet published
                    if (spins++ >= spin_limit) {
                        stalled = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            // published even after a stall, so later tiles end their walks here
            __hip_atomic_store(mine, OS_INC | ((excl + tot) & OS_VALUE), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (stalled) atomicCAS(stall, 0u, pass + 1u);
        }
        goff[d] = gbase[d] + excl;
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
        const uint64_t at = (uint64_t)goff[d] + (p - tstart[d]);
        if (at < n) out[at] = key;              // bounds hold unless the pass stalled (then it is discarded)
    }
}

template <int ITEMS>
hipError_t onesweep_passes(uint64_t *keys, uint64_t n, const VKey &vk, uint32_t hi, uint32_t digit, SortScratch &sc,
                           hipStream_t s, uint64_t **out) {
    constexpr uint64_t TILE = WG * ITEMS;
    const uint32_t n_tiles = (uint32_t)((n + TILE - 1) / TILE);
    const uint32_t passes = (hi + digit - 1) / digit;
    uint32_t *ghist = sc.os, *gbase = sc.os + RADIX_OS_PASSES * 256;
    uint32_t *stall = sc.os + 2 * RADIX_OS_PASSES * 256;
    uint32_t *status[2] = {sc.hist, sc.hist + (size_t)n_tiles * 256};
    hipError_t e = launch_zero(sc.os, RADIX_OS_WORDS * 4, s);
    if (e == hipSuccess) e = launch_zero(status[0], (size_t)n_tiles * 256 * 4, s);
    if (e != hipSuccess) return e;
    const uint32_t hg = n_tiles < 1024 ? n_tiles : 1024;
    hipLaunchKernelGGL(k_os_hist, dim3(hg), dim3(WG), 0, s, keys, n, vk, hi, digit, passes, ghist);
    hipLaunchKernelGGL(k_os_bases, dim3(passes), dim3(WG), 0, s, ghist, gbase);
    uint64_t *a = keys, *b = sc.alt;
    for (uint32_t p = 0; p < passes; p++) {
        const uint32_t sh = p * digit;
        const uint32_t bits = (hi - sh) < digit ? (hi - sh) : digit;
        hipLaunchKernelGGL(k_os_scatter<ITEMS>, dim3(n_tiles), dim3(WG), 0, s, a, b, n, vk, sh, bits, p,
                           gbase + p * 256, status[p & 1], status[(p + 1) & 1], stall, sc.spin);
        uint64_t *t = a; a = b; b = t;
    }
    sc.stall = stall;
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

bool radix_onesweep(uint64_t n) { return n >= RADIX_OS_MIN_KEYS && n < (1ull << 30); }

hipError_t radix_sort(uint64_t *keys, uint64_t n, const VKey &vk, SortScratch &sc, uint32_t tile,
                      hipStream_t s, uint64_t **out, uint32_t digit) {
    if (digit < 4 || digit > 8) digit = 8;
    *out = keys;
    sc.stall = nullptr;
    if (n <= 1 || vk.vbits == 0) return hipSuccess;
    if (sc.os && radix_onesweep(n)) {
        switch (tile) {
        case 1024: return onesweep_passes<4>(keys, n, vk, vk.vbits, digit, sc, s, out);
        case 4096: return onesweep_passes<16>(keys, n, vk, vk.vbits, digit, sc, s, out);
        case 8192: return onesweep_passes<32>(keys, n, vk, vk.vbits, digit, sc, s, out);
        default: return onesweep_passes<8>(keys, n, vk, vk.vbits, digit, sc, s, out);
        }
    }
    if (n <= SMALL_N) {
        const hipError_t ea = raise_small_lds_limit();
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(k_rs_small, dim3(1), dim3(SWG), n * 8, s, keys, sc.alt, (uint32_t)n, vk, vk.vbits);
        *out = ((vk.vbits + 7) / 8) % 2 ? sc.alt : keys;
        return hipGetLastError();
    }
    return radix_sort_resume(keys, n, vk, sc, tile, s, out, digit, 0);
}

hipError_t radix_sort_resume(uint64_t *keys, uint64_t n, const VKey &vk, SortScratch &sc, uint32_t tile,
                             hipStream_t s, uint64_t **out, uint32_t digit, uint32_t pass) {
    if (digit < 4 || digit > 8) digit = 8;
    uint64_t *a = (pass & 1u) ? sc.alt : keys, *b = (pass & 1u) ? keys : sc.alt;
    const uint32_t sh0 = pass * digit;
    *out = a;
    sc.stall = nullptr;
    switch (tile) {
    case 1024: return sort_passes<4>(a, b, n, vk, sh0, vk.vbits, digit, sc, s, out);
    case 8192: return sort_passes<32>(a, b, n, vk, sh0, vk.vbits, digit, sc, s, out);
    case 4096: return sort_passes<16>(a, b, n, vk, sh0, vk.vbits, digit, sc, s, out);
    default: return sort_passes<8>(a, b, n, vk, sh0, vk.vbits, digit, sc, s, out);
    }
}

}  // namespace kc
