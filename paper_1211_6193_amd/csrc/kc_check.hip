// Conflict check over sorted access records, and the helpers of the replay.
//
// After the sort, records of one (unit, space, address, block, epoch) are
// adjacent (intra-block segment) and, for global memory, records of one
// (unit, address) are adjacent with their blocks in ascending order
// (cross-block segment).  A race (Section 3.1 of the paper: two threads, one
// location, at least one write, no synchronisation between them) exists in an
// intra-block segment iff it has a writer and two distinct threads; in a
// cross-block segment iff it has a writer and two distinct blocks.  The
// canonical tuple names the smallest writer and the smallest other thread that
// conflicts with it.
#include <algorithm>

#include "../../include/kc.h"
#include "kc_internal.h"

namespace kc {

namespace {

constexpr int WG = 256;
constexpr uint32_t NONE = 0xFFFFFFFFu;


__device__ void push_race(const CheckArgs &A, const DevRace &r) {
    uint32_t idx = atomicAdd(&A.ctr->race_count, 1u);
    if (idx < A.race_cap) A.races[idx] = r;
    else atomicOr(&A.ctr->flags, FLAG_RACE_OVERFLOW);
}

__device__ void push_edge(const CheckArgs &A, uint32_t unit, uint32_t b0, uint32_t b1) {
    uint32_t idx = atomicAdd(&A.ctr->edge_count, 1u);
    if (idx < A.edge_cap) {
        DevEdge e;
        e.unit = unit; e.b0 = b0; e.b1 = b1; e.pad = 0;
        A.edges[idx] = e;
    } else {
        atomicOr(&A.ctr->flags, FLAG_EDGE_OVERFLOW);
    }
}

constexpr int CHECK_ITEMS = 8;
constexpr int CHECK_TILE = WG * CHECK_ITEMS;
// A segment is reduced by its head thread up to this many records; a longer
// one (a location touched by many threads or blocks) goes to k_check_long,
// which reduces it with a whole workgroup.
constexpr uint32_t SEG_LIMIT = 64;
constexpr uint64_t LONG_CROSS = 1ull << 63;

__device__ void push_long(const CheckArgs &A, uint64_t entry) {
    const uint32_t idx = atomicAdd(&A.ctr->long_count, 1u);
    A.longseg[idx] = entry;     // capacity: every long segment has more than SEG_LIMIT records
}

// One workgroup per tile of sorted records, staged in LDS; thread t owns the
// records at t, t + WG, t + 2 WG, ... (conflict-free LDS reads) and reduces
// every segment that starts at one of them (reading past the tile from global
// memory when a segment continues into the next tile).
__global__ void __launch_bounds__(WG) k_check(CheckArgs A) {
    __shared__ uint64_t tk[CHECK_TILE];
    const uint64_t tile0 = (uint64_t)blockIdx.x * CHECK_TILE;
    const uint64_t tile_n = min((uint64_t)CHECK_TILE, A.n - tile0);
    for (uint32_t p = threadIdx.x; p < tile_n; p += WG) tk[p] = A.keys[tile0 + p];
    __syncthreads();
    const KeyPlan &k = A.kp;
    const uint32_t ps = k.s_ep;                  // bits below: tid and kind
    auto key_at = [&](uint64_t j) -> uint64_t {
        return (j >= tile0 && j < tile0 + tile_n) ? tk[j - tile0] : A.keys[j];
    };
    for (uint32_t q = 0; q < CHECK_ITEMS; q++) {
        const uint64_t p = (uint64_t)q * WG + threadIdx.x;
        if (p >= tile_n) break;
        const uint64_t i = tile0 + p;
        // (segments are scanned serially by their head thread)
        const uint64_t ki = tk[p];
        const uint64_t prev = i ? key_at(i - 1) : ~0ull;
        const uint64_t inner = ki >> ps;
        // representative records of locally checked epochs take part only in
        // the cross-block check
        const bool head_in = (i == 0 || (prev >> ps) != inner) && rec_field(ki, k.s_ep, k.eb) != k.ep_rep;
        const uint32_t space = rec_field(ki, k.s_sp, 1);
        const bool head_out = space == 1u && (i == 0 || (prev >> k.s_addr) != (ki >> k.s_addr));
        if (!head_in && !head_out) continue;
        const uint32_t unit = rec_field(ki, k.s_unit, k.ub);
        const uint32_t addr = rec_field(ki, k.s_addr, k.ab);
        const uint32_t block0 = rec_field(ki, k.s_blk, k.bb);
        if (head_in) {
            // intra-block segment: smallest writer and two smallest distinct tids
            uint32_t minw = NONE, t1 = NONE, t2 = NONE;
            bool is_long = false;
            for (uint64_t j = i; j < A.n; j++) {
                const uint64_t kj = key_at(j);
                if ((kj >> ps) != inner) break;
                if (j - i == SEG_LIMIT) {
                    is_long = true;
                    break;
                }
                const uint32_t tid = rec_field(kj, k.s_tid, k.tb);
                if (kj & 1ull) minw = min(minw, tid);
                if (tid < t1) { t2 = t1; t1 = tid; }
                else if (tid != t1 && tid < t2) t2 = tid;
            }
            if (is_long) {
                push_long(A, i);
            } else if (minw != NONE && t2 != NONE) {
                DevRace r;
                r.unit = unit; r.space = space; r.scope = 0; r.block = block0;
                r.epoch = rec_field(ki, k.s_ep, k.eb); r.addr = addr;
                r.w = minw; r.o = (t1 == minw) ? t2 : t1;
                push_race(A, r);
                A.blk_flags[A.units[unit].block_base + block0] = 1u;
            }
        }
        if (head_out) {
            // cross-block segment: smallest writer gtid, two smallest gtids of distinct blocks
            const uint64_t outer = ki >> k.s_addr;
            const uint32_t nt = A.units[unit].nt;
            uint32_t wg = NONE, wb = NONE, g1 = NONE, b1 = NONE, g2 = NONE;
            uint64_t end = i;
            bool is_long = false;
            for (uint64_t j = i; j < A.n; j++) {
                const uint64_t kj = key_at(j);
                if ((kj >> k.s_addr) != outer) break;
                if (j - i == SEG_LIMIT) {
                    is_long = true;
                    break;
                }
                end = j + 1;
                const uint32_t b = rec_field(kj, k.s_blk, k.bb);
                const uint32_t g = b * nt + rec_field(kj, k.s_tid, k.tb);
                if ((kj & 1ull) && g < wg) { wg = g; wb = b; }
                if (g < g1) {
                    if (b != b1) g2 = g1;    // the old minimum is in another block
                    g1 = g; b1 = b;
                } else if (b != b1 && g < g2) {
                    g2 = g;
                }
            }
            if (is_long) {
                push_long(A, i | LONG_CROSS);
            } else if (wg != NONE && g2 != NONE) {
                DevRace r;
                r.unit = unit; r.space = 1; r.scope = 1; r.block = wb; r.epoch = NONE; r.addr = addr;
                r.w = wg; r.o = (wb == b1) ? g2 : g1;
                push_race(A, r);
                // every block touching the location joins the racy component
                uint32_t prevb = NONE;
                for (uint64_t j = i; j < end; j++) {
                    const uint32_t b = rec_field(key_at(j), k.s_blk, k.bb);
                    if (b != prevb) {
                        A.blk_flags[A.units[unit].block_base + b] = 1u;
                        if (b != block0) push_edge(A, unit, block0, b);
                        prevb = b;
                    }
                }
            }
        }
    }
}

// Reduction states of a segment (merged associatively, in any order).
// Intra-block: smallest writer tid and the two smallest distinct tids.
struct IntraState { uint32_t minw, t1, t2; };
// Cross-block: smallest writer gtid (and its block), smallest gtid g1 (block b1)
// and the smallest gtid g2 of a block other than b1.
struct CrossState { uint32_t wg, wb, g1, b1, g2; };

__device__ __forceinline__ void insert2(uint32_t &a1, uint32_t &a2, uint32_t x) {
    if (x < a1) { a2 = a1; a1 = x; }
    else if (x != a1 && x < a2) a2 = x;
}
__device__ __forceinline__ IntraState merge(IntraState a, const IntraState &b) {
    a.minw = min(a.minw, b.minw);
    insert2(a.t1, a.t2, b.t1);
    insert2(a.t1, a.t2, b.t2);
    return a;
}
__device__ __forceinline__ CrossState merge(CrossState a, CrossState b) {
    if (b.wg < a.wg) { a.wg = b.wg; a.wb = b.wb; }
    if (b.g1 < a.g1) {      // b holds the overall minimum
        const uint32_t wg = a.wg, wb = a.wb;
        CrossState t = a; a = b; b = t;
        a.wg = wg; a.wb = wb;
    }
    a.g2 = min(a.g2, b.b1 != a.b1 ? b.g1 : b.g2);
    return a;
}

// One workgroup per long segment (grid-stride over the list k_check wrote):
// the threads reduce interleaved records, then a tree reduction in LDS; a
// racy cross-block segment is walked again to flag its blocks and link them.
__global__ void __launch_bounds__(WG) k_check_long(CheckArgs A) {
    __shared__ CrossState cs[WG];
    __shared__ IntraState is[WG];
    __shared__ uint32_t racy;
    const KeyPlan &k = A.kp;
    const uint32_t cnt = __hip_atomic_load(&A.ctr->long_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const uint64_t ent = A.longseg[e];
        const bool cross = (ent & LONG_CROSS) != 0;
        const uint64_t i = ent & ~LONG_CROSS;
        const uint64_t ki = A.keys[i];
        const uint32_t shift = cross ? k.s_addr : k.s_ep;
        const uint64_t tag = ki >> shift;
        const uint32_t unit = rec_field(ki, k.s_unit, k.ub);
        const uint32_t nt = A.units[unit].nt;
        IntraState a{NONE, NONE, NONE};
        CrossState c{NONE, NONE, NONE, NONE, NONE};
        for (uint64_t base = i;; base += WG) {
            const uint64_t j = base + threadIdx.x;
            const uint64_t kj = j < A.n ? A.keys[j] : 0ull;
            const bool in = j < A.n && (kj >> shift) == tag;
            if (in) {
                const uint32_t tid = rec_field(kj, k.s_tid, k.tb);
                if (cross) {
                    const uint32_t b = rec_field(kj, k.s_blk, k.bb);
                    const uint32_t g = b * nt + tid;
                    c = merge(c, CrossState{(kj & 1ull) ? g : NONE, (kj & 1ull) ? b : NONE, g, b, NONE});
                } else {
                    a = merge(a, IntraState{(kj & 1ull) ? tid : NONE, tid, NONE});
                }
            }
            if (__syncthreads_or(!in)) break;       // sorted: the segment ended in this chunk
        }
        cs[threadIdx.x] = c;
        is[threadIdx.x] = a;
        __syncthreads();
        for (uint32_t h = WG / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                cs[threadIdx.x] = merge(cs[threadIdx.x], cs[threadIdx.x + h]);
                is[threadIdx.x] = merge(is[threadIdx.x], is[threadIdx.x + h]);
            }
            __syncthreads();
        }
        const uint32_t block0 = rec_field(ki, k.s_blk, k.bb);
        if (threadIdx.x == 0) {
            racy = 0;
            DevRace r;
            r.unit = unit; r.space = rec_field(ki, k.s_sp, 1); r.addr = rec_field(ki, k.s_addr, k.ab);
            if (cross) {
                const CrossState f = cs[0];
                if (f.wg != NONE && f.g2 != NONE) {
                    r.scope = 1; r.block = f.wb; r.epoch = NONE;
                    r.w = f.wg; r.o = (f.wb == f.b1) ? f.g2 : f.g1;
                    push_race(A, r);
                    racy = 1;
                }
            } else {
                const IntraState f = is[0];
                if (f.minw != NONE && f.t2 != NONE) {
                    r.scope = 0; r.block = block0; r.epoch = rec_field(ki, k.s_ep, k.eb);
                    r.w = f.minw; r.o = (f.t1 == f.minw) ? f.t2 : f.t1;
                    push_race(A, r);
                    A.blk_flags[A.units[unit].block_base + block0] = 1u;
                }
            }
        }
        __syncthreads();
        if (racy) {             // every block touching the location joins the racy component
            for (uint64_t base = i;; base += WG) {
                const uint64_t j = base + threadIdx.x;
                const uint64_t kj = j < A.n ? A.keys[j] : 0ull;
                const bool in = j < A.n && (kj >> shift) == tag;
                if (in) {
                    const uint32_t b = rec_field(kj, k.s_blk, k.bb);
                    const bool first = j == i || rec_field(A.keys[j - 1], k.s_blk, k.bb) != b;
                    if (first) {
                        A.blk_flags[A.units[unit].block_base + b] = 1u;
                        if (b != block0) push_edge(A, unit, block0, b);
                    }
                }
                if (__syncthreads_or(!in)) break;
            }
        }
        __syncthreads();        // LDS states are reused by the next segment
    }
}

// Put back the launch-start value of every global word a flagged block wrote
// (records [0, n), or [0, min(n, *n_dev)) when the count is on the device).
__global__ void __launch_bounds__(WG) k_restore(const uint64_t *__restrict__ keys, uint64_t n, KeyPlan k,
                                                const DevUnit *__restrict__ units,
                                                const uint32_t *__restrict__ blk_flags,
                                                const unsigned long long *__restrict__ n_dev) {
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (n_dev && i >= *n_dev) return;
    if (i >= n) return;
    const uint64_t r = keys[i];
    if (!(r & 1ull) || rec_field(r, k.s_sp, 1) != 1u) return;
    const DevUnit &u = units[rec_field(r, k.s_unit, k.ub)];
    if (!blk_flags[u.block_base + rec_field(r, k.s_blk, k.bb)]) return;
    const uint32_t a = rec_field(r, k.s_addr, k.ab);
    u.mem[a] = u.snap[a];
}

// The flagged blocks in ascending global block index as (unit, block): each
// thread counts the flags of a contiguous chunk, a block-wide scan of the
// counts gives each chunk its place, and the chunk writes its blocks there.
// The same workgroup first clears the buffers `zero` lists.
// The unit of a block is found by binary search in the units' first blocks.
__global__ void __launch_bounds__(1024) k_flagged_comps(const uint32_t *__restrict__ blk_flags, uint32_t n_blocks,
                                                        const DevUnit *__restrict__ units, uint32_t n_units,
                                                        uint2 *__restrict__ comps, uint32_t *__restrict__ n_comps,
                                                        ZeroArgs zero) {
    __shared__ uint32_t part[1024];
    for (uint32_t b = 0; b < zero.n; b++)       // buffers the next kernels expect cleared
        for (size_t i = threadIdx.x; i < zero.words[b]; i += blockDim.x) zero.p[b][i] = 0u;
    const uint32_t per = (n_blocks + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = min(n_blocks, threadIdx.x * per), b1 = min(n_blocks, b0 + per);
    uint32_t mine = 0;
    for (uint32_t b = b0; b < b1; b++) mine += blk_flags[b] != 0u;
    part[threadIdx.x] = mine;
    __syncthreads();
    for (uint32_t d = 1; d < blockDim.x; d <<= 1) {      // inclusive scan of the chunk counts
        const uint32_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t at = part[threadIdx.x] - mine;
    if (mine) {
        uint32_t lo = 0, hi = n_units;      // the last unit whose first block is <= b0
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (units[mid].block_base <= b0) lo = mid; else hi = mid;
        }
        uint32_t u = lo;
        for (uint32_t b = b0; b < b1; b++) {
            while (u + 1 < n_units && units[u + 1].block_base <= b) u++;
            if (blk_flags[b]) comps[at++] = make_uint2(u, b - units[u].block_base);
        }
    }
    if (threadIdx.x == blockDim.x - 1) *n_comps = part[threadIdx.x];
}

// Exactness condition of a replay: no global location may be touched both by
// a replayed block (its canonical records `rs`, sorted) and by a block that was
// not replayed (free-run records in `log`, sorted, with blk_flags == 0) unless
// both only read it.  The first replayed record of each location looks up the
// location's records in the free-run log by binary search and scans them; a
// location with more than COV_LIMIT records on either side is listed for
// k_coverage_long instead.
constexpr uint32_t COV_LIMIT = 32;

__device__ __forceinline__ uint64_t lower_bound_loc(const uint64_t *__restrict__ log, uint64_t n_log, uint64_t target,
                                                    uint32_t shift) {
    uint64_t lo = 0, hi = n_log;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if ((log[mid] >> shift) < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(WG) k_coverage(const uint64_t *__restrict__ rs, uint64_t n_rs,
                                                 const uint64_t *__restrict__ log, uint64_t n_log, KeyPlan k,
                                                 const DevUnit *__restrict__ units,
                                                 const uint32_t *__restrict__ blk_flags, DevCounters *ctr,
                                                 uint64_t *__restrict__ list) {
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= n_rs) return;
    const uint64_t r = rs[i];
    if (rec_field(r, k.s_sp, 1) != 1u) return;
    const uint64_t target = r >> k.s_addr;
    if (i > 0 && (rs[i - 1] >> k.s_addr) == target) return;
    bool r_w = false;
    for (uint64_t j = i; j < n_rs && (rs[j] >> k.s_addr) == target; j++) {
        if (j - i == COV_LIMIT) {
            list[atomicAdd(&ctr->long_count, 1u)] = i;
            return;
        }
        r_w |= (rs[j] & 1ull) != 0;
    }
    const uint64_t lo = lower_bound_loc(log, n_log, target, k.s_addr);
    const DevUnit &u = units[rec_field(r, k.s_unit, k.ub)];
    for (uint64_t j = lo; j < n_log; j++) {
        const uint64_t x = log[j];
        if ((x >> k.s_addr) != target) break;
        if (j - lo == COV_LIMIT) {
            list[atomicAdd(&ctr->long_count, 1u)] = i;
            return;
        }
        if (blk_flags[u.block_base + rec_field(x, k.s_blk, k.bb)]) continue;    // replayed block
        if (r_w || (x & 1ull)) {
            atomicOr(&ctr->flags, FLAG_MISMATCH);
            return;
        }
    }
}

// The listed locations, one workgroup each (grid-stride over the list).
__global__ void __launch_bounds__(WG) k_coverage_long(const uint64_t *__restrict__ rs, uint64_t n_rs,
                                                      const uint64_t *__restrict__ log, uint64_t n_log, KeyPlan k,
                                                      const DevUnit *__restrict__ units,
                                                      const uint32_t *__restrict__ blk_flags, DevCounters *ctr,
                                                      const uint64_t *__restrict__ list) {
    __shared__ uint64_t lo_sh;
    const uint32_t cnt = __hip_atomic_load(&ctr->long_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const uint64_t i = list[e];
        const uint64_t r = rs[i];
        const uint64_t target = r >> k.s_addr;
        const DevUnit &u = units[rec_field(r, k.s_unit, k.ub)];
        int r_w = 0;
        for (uint64_t base = i;; base += WG) {
            const uint64_t j = base + threadIdx.x;
            const bool in = j < n_rs && (rs[j] >> k.s_addr) == target;
            const int w = __syncthreads_or(in && (rs[j] & 1ull));
            r_w |= w;
            if (__syncthreads_or(!in)) break;
        }
        if (threadIdx.x == 0) lo_sh = lower_bound_loc(log, n_log, target, k.s_addr);
        __syncthreads();
        const uint64_t lo = lo_sh;
        for (uint64_t base = lo;; base += WG) {
            const uint64_t j = base + threadIdx.x;
            const uint64_t x = j < n_log ? log[j] : 0ull;
            const bool in = j < n_log && (x >> k.s_addr) == target;
            if (in && !blk_flags[u.block_base + rec_field(x, k.s_blk, k.bb)] && (r_w || (x & 1ull)))
                atomicOr(&ctr->flags, FLAG_MISMATCH);
            if (__syncthreads_or(!in)) break;
        }
    }
}

// Records of the table's log: n_rs, or the count the producing kernel left
// on the device (n_rs is then its capacity).
__device__ __forceinline__ uint64_t n_records(const ReplayTableArgs &a) {
    if (!a.n_dev) return a.n_rs;
    const uint64_t n = __hip_atomic_load(a.n_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return n < a.n_rs ? n : a.n_rs;
}

__device__ __forceinline__ void need_sort(DevCounters *ctr) {
    if (!(__hip_atomic_load(&ctr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_NEED_SORT))
        atomicOr(&ctr->flags, FLAG_NEED_SORT);
}

// Locations of a log in a hash table (linear probing), one 64-bit word per
// slot: location + 1 (0 = empty) | first block + 1 (obits bits) | flags (bit 0
// a write, bit 1 a second block), so inserting a record is one
// compare-and-swap.
struct LocTable {
    unsigned long long *w;
    uint32_t bits, obits;
    __device__ unsigned long long loc(unsigned long long v) const { return v >> (obits + 2); }
    __device__ uint32_t owner(unsigned long long v) const { return (uint32_t)(v >> 2) & ((1u << obits) - 1u); }
    __device__ uint32_t flags(unsigned long long v) const { return (uint32_t)v & 3u; }
    __device__ unsigned long long pack(unsigned long long loc1, uint32_t own1, uint32_t f) const {
        return (loc1 << (obits + 2)) | ((unsigned long long)own1 << 2) | f;
    }
    __device__ uint32_t home(unsigned long long loc1) const {
        return (uint32_t)((loc1 * 0x9E3779B97F4A7C15ull) >> (64 - bits));
    }
};

__global__ void __launch_bounds__(WG) k_rtable_insert(ReplayTableArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= n_records(a)) return;
    const KeyPlan &k = a.kp;
    const uint64_t r = a.rs[i];
    if (rec_field(r, k.s_sp, 1) != 1u || rec_field(r, k.s_ep, k.eb) != k.ep_rep) {
        need_sort(a.ctr);    // an unreduced record
        return;
    }
    const LocTable t{(unsigned long long *)a.table, a.bits, a.obits};
    const unsigned long long loc1 = (r >> k.s_addr) + 1ull;
    const uint32_t blk = a.units[rec_field(r, k.s_unit, k.ub)].block_base + rec_field(r, k.s_blk, k.bb) + 1u;
    const uint32_t wr = (uint32_t)(r & 1ull);
    const uint32_t mask = (1u << a.bits) - 1u;
    uint32_t slot = t.home(loc1);
    for (uint32_t p = 0; p <= mask; p++) {
        unsigned long long cur = t.w[slot];
        if (cur == 0ull) {
            cur = atomicCAS(&t.w[slot], 0ull, t.pack(loc1, blk, wr));
            if (cur == 0ull) return;
        }
        if (t.loc(cur) == loc1) {
            for (;;) {
                const uint32_t own = t.owner(cur);
                const unsigned long long nw = t.pack(loc1, own, t.flags(cur) | wr | (own != blk ? 2u : 0u));
                if (nw == cur) return;
                const unsigned long long prev = atomicCAS(&t.w[slot], cur, nw);
                if (prev == cur) return;
                cur = prev;
            }
        }
        slot = (slot + 1u) & mask;
    }
    need_sort(a.ctr);        // no free slot
}

__device__ __forceinline__ int64_t ltable_find(const LocTable &t, unsigned long long loc1) {
    const uint32_t mask = (1u << t.bits) - 1u;
    uint32_t slot = t.home(loc1);
    for (uint32_t p = 0; p <= mask; p++) {
        const unsigned long long v = t.w[slot];
        if (v == 0ull) return -1;
        if (t.loc(v) == loc1) return slot;
        slot = (slot + 1u) & mask;
    }
    return -1;
}

// Direct tables, first pass: every word a record touches takes the record's
// block (one of them wins when several blocks store) and writes set its
// written flag; plain stores, no atomics.
__global__ void __launch_bounds__(WG) k_dtable_own(ReplayTableArgs a) {
    const uint64_t n = n_records(a);
    const KeyPlan &k = a.kp;
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * WG) {
        const uint64_t r = a.rs[i];
        if (rec_field(r, k.s_sp, 1) != 1u || rec_field(r, k.s_ep, k.eb) != k.ep_rep) {
            need_sort(a.ctr);
            continue;
        }
        const DevUnit &u = a.units[rec_field(r, k.s_unit, k.ub)];
        const uint64_t w = (uint64_t)(u.snap - a.snap_base) + rec_field(r, k.s_addr, k.ab);
        a.downer[w] = u.block_base + rec_field(r, k.s_blk, k.bb) + 1u;
        if (r & 1ull) a.dflags[w] = 1;
    }
}

// Second pass: a record whose block lost the word to another block marks the
// word as touched by several blocks; with a write among them that is a
// cross-block conflict.  (Every such word has a record that lost.)
__global__ void __launch_bounds__(WG) k_dtable_multi(ReplayTableArgs a) {
    const uint64_t n = n_records(a);
    const KeyPlan &k = a.kp;
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * WG) {
        const uint64_t r = a.rs[i];
        if (rec_field(r, k.s_sp, 1) != 1u || rec_field(r, k.s_ep, k.eb) != k.ep_rep) continue;
        const DevUnit &u = a.units[rec_field(r, k.s_unit, k.ub)];
        const uint64_t w = (uint64_t)(u.snap - a.snap_base) + rec_field(r, k.s_addr, k.ab);
        if (a.downer[w] == u.block_base + rec_field(r, k.s_blk, k.bb) + 1u) continue;
        const uint8_t f = a.dflags[w];
        a.dflags[w] = f | 2;        // every such store writes the same value
        if (f & 1) need_sort(a.ctr);
    }
}

// Locations written by one block and touched by another.
__global__ void __launch_bounds__(WG) k_rtable_conflicts(ReplayTableArgs a) {
    const uint32_t slot = blockIdx.x * WG + threadIdx.x;
    if (slot >= (1u << a.bits)) return;
    const unsigned long long v = ((const unsigned long long *)a.table)[slot];
    if (v != 0ull && (v & 3ull) == 3ull) need_sort(a.ctr);
}

// Per replayed location: a write shared between replayed blocks needs the
// sorted check; otherwise the location's free-run records of blocks that were
// not replayed must not conflict with it (at most COV_LIMIT of them scanned),
// or, with the free run's location table, its one block (several: sorted
// check).
__global__ void __launch_bounds__(WG) k_rtable_check(ReplayTableArgs a) {
    const uint32_t slot = blockIdx.x * WG + threadIdx.x;
    if (slot >= (1u << a.bits)) return;
    const LocTable t{(unsigned long long *)a.table, a.bits, a.obits};
    const unsigned long long v = t.w[slot];
    if (v == 0ull) return;
    const uint32_t f = t.flags(v);
    if (f == 3u) {
        need_sort(a.ctr);
        return;
    }
    const unsigned long long loc1 = t.loc(v);
    if (a.downer) {
        const KeyPlan &k = a.kp;
        const unsigned long long loc = loc1 - 1ull;     // address | space << ab | unit << (ab + 1)
        const DevUnit &u = a.units[(uint32_t)(loc >> (k.ab + 1))];
        const uint64_t w = (uint64_t)(u.snap - a.snap_base) + (uint32_t)(loc & ((1ull << k.ab) - 1ull));
        const uint32_t own = a.downer[w];
        if (own == 0u) return;                              // untouched by the free run
        const uint8_t ff = a.dflags[w];
        if (ff & 2) {
            need_sort(a.ctr);
            return;
        }
        if (a.blk_flags[own - 1u]) return;                  // its one block was replayed
        if ((f & 1u) || (ff & 1)) atomicOr(&a.ctr->flags, FLAG_MISMATCH);
        return;
    }
    if (a.ftable) {
        const LocTable ft{(unsigned long long *)const_cast<void *>(a.ftable), a.fbits, a.obits};
        const int64_t fs = ltable_find(ft, loc1);
        if (fs < 0) return;                                 // untouched by the free run
        const unsigned long long fv = ft.w[fs];
        if (ft.flags(fv) & 2u) {
            need_sort(a.ctr);
            return;
        }
        if (a.blk_flags[ft.owner(fv) - 1u]) return;        // its one block was replayed
        if ((f & 1u) || (ft.flags(fv) & 1u)) atomicOr(&a.ctr->flags, FLAG_MISMATCH);
        return;
    }
    const KeyPlan &k = a.kp;
    const uint64_t target = loc1 - 1ull;
    const uint64_t lo = lower_bound_loc(a.log, a.n_log, target, k.s_addr);
    for (uint64_t j = lo; j < a.n_log; j++) {
        const uint64_t x = a.log[j];
        if ((x >> k.s_addr) != target) break;
        if (j - lo == COV_LIMIT) {
            need_sort(a.ctr);
            return;
        }
        const DevUnit &u = a.units[rec_field(x, k.s_unit, k.ub)];
        if (a.blk_flags[u.block_base + rec_field(x, k.s_blk, k.bb)]) continue;     // replayed block
        if ((f & 1u) || (x & 1ull)) {
            atomicOr(&a.ctr->flags, FLAG_MISMATCH);
            return;
        }
    }
}

// mem <-> snapshot of each unit (blockIdx.y = unit), optionally masked.
__global__ void __launch_bounds__(WG) k_copy_units(const DevUnit *__restrict__ units, int to_snapshot,
                                                   const uint32_t *__restrict__ mask) {
    const DevUnit &u = units[blockIdx.y];
    if (mask && !mask[blockIdx.y]) return;
    const uint32_t stride = gridDim.x * WG;
    if (to_snapshot) {
        int32_t *dst = const_cast<int32_t *>(u.snap);
        for (uint32_t i = blockIdx.x * WG + threadIdx.x; i < u.n_words; i += stride) dst[i] = u.mem[i];
    } else {
        for (uint32_t i = blockIdx.x * WG + threadIdx.x; i < u.n_words; i += stride) u.mem[i] = u.snap[i];
    }
}

__global__ void __launch_bounds__(WG) k_zero(uint32_t *__restrict__ p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < words; i += (size_t)gridDim.x * WG) p[i] = 0;
}

__global__ void __launch_bounds__(WG) k_zero_many(ZeroArgs z) {
    for (uint32_t k = 0; k < z.n; k++)
        for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < z.words[k]; i += (size_t)gridDim.x * WG)
            z.p[k][i] = 0;
}

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + WG - 1) / WG); }

// Copy every item of a gather into the host-visible staging buffer: one
// kernel instead of one copy per item.
__global__ void __launch_bounds__(WG) k_gather(GatherArgs a) {
    for (uint32_t k = 0; k < a.n; k++) {
        const uint32_t *src = a.src[k];
        uint32_t *dst = a.dst + a.dst_off[k];
        for (uint32_t i = blockIdx.x * WG + threadIdx.x; i < a.words[k]; i += gridDim.x * WG) dst[i] = src[i];
    }
}

// Access summary of a launch (streams and events): per global word, the
// smallest global thread id that touched it and the smallest that wrote it,
// from the records of a log.  Every record stands for an access of its
// thread of the kind its low bit gives (representatives and unreduced
// tuples alike), so the minima over records are the minima over accesses.
__global__ void __launch_bounds__(WG) k_summary(SummaryArgs a) {
    const KeyPlan &k = a.kp;
    const uint64_t n = a.n_dev ? min((uint64_t)*a.n_dev, a.n) : a.n;
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * WG) {
        const uint64_t r = a.log[i];
        if (rec_field(r, k.s_sp, 1) != 1u) continue;
        const uint32_t unit = rec_field(r, k.s_unit, k.ub);
        uint32_t *sum = a.sums[unit];
        if (!sum || (a.skip_units && a.skip_units[unit])) continue;
        const DevUnit &u = a.units[unit];
        const uint32_t block = rec_field(r, k.s_blk, k.bb);
        if (a.skip_blocks && a.skip_blocks[u.block_base + block]) continue;
        const uint32_t addr = rec_field(r, k.s_addr, k.ab);
        const uint32_t g = block * u.nt + rec_field(r, k.s_tid, k.tb);
        atomicMin(&sum[addr], g);
        if (r & 1ull) atomicMin(&sum[u.n_words + addr], g);
    }
}

// Memory objects: records of global words outside the unit's allocations.
__global__ void __launch_bounds__(WG) k_alloc_scan(AllocScanArgs a) {
    const KeyPlan &k = a.kp;
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < a.n; i += (uint64_t)gridDim.x * WG) {
        const uint64_t r = a.log[i];
        if (rec_field(r, k.s_sp, 1) != 1u) continue;
        const uint32_t unit = rec_field(r, k.s_unit, k.ub);
        const uint32_t *bm = a.allocated[unit];
        if (!bm || (a.skip_units && a.skip_units[unit])) continue;
        if (a.skip_blocks && a.skip_blocks[a.units[unit].block_base + rec_field(r, k.s_blk, k.bb)]) continue;
        const uint32_t addr = rec_field(r, k.s_addr, k.ab);
        if ((bm[addr >> 5] >> (addr & 31u)) & 1u) continue;
        const uint32_t at = atomicAdd(a.count, 1u);
        if (at < a.cap) a.out[at] = r;
    }
}

// Offsets of the blocks' held representatives in the log: an exclusive scan
// of their counts (one workgroup) after the records counted so far.
__global__ void __launch_bounds__(1024) k_held_scan(const uint32_t *__restrict__ held, uint64_t *__restrict__ off,
                                                    uint32_t n, unsigned long long log_cap,
                                                    unsigned long long *log_count, uint32_t *flags) {
    __shared__ unsigned long long part[1024];
    __shared__ unsigned long long base_s;
    if (threadIdx.x == 0) base_s = *log_count;      // read before the last thread rewrites it
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = min(n, threadIdx.x * per), b1 = min(n, b0 + per);
    unsigned long long mine = 0;
    for (uint32_t b = b0; b < b1; b++) mine += held[b];
    part[threadIdx.x] = mine;
    __syncthreads();
    for (uint32_t d = 1; d < blockDim.x; d <<= 1) {      // inclusive scan of the chunk sums
        const unsigned long long v = threadIdx.x >= d ? part[threadIdx.x - d] : 0ull;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    const unsigned long long base = base_s;
    unsigned long long at = base + part[threadIdx.x] - mine;
    for (uint32_t b = b0; b < b1; b++) {
        off[b] = at;
        at += held[b];
    }
    if (threadIdx.x == blockDim.x - 1) {
        const unsigned long long end = base + part[threadIdx.x];
        *log_count = end;
        if (end > log_cap) atomicOr(flags, FLAG_LOG_OVERFLOW);
    }
}

__global__ void __launch_bounds__(WG) k_held_copy(const uint64_t *__restrict__ blk_log,
                                                  const uint32_t *__restrict__ held,
                                                  const uint64_t *__restrict__ off, uint32_t n, uint64_t *log,
                                                  unsigned long long log_cap) {
    for (uint32_t b = blockIdx.x; b < n; b += gridDim.x) {
        const uint32_t cnt = held[b];
        const uint64_t o = off[b];
        for (uint32_t j = threadIdx.x; j < cnt; j += WG)
            if (o + j < log_cap) log[o + j] = blk_log[(size_t)b * REP_HOLD + j];
    }
}

// Races between an earlier launch (summary si) and a later one (sj) of a job
// that may run in parallel: every word one writes and the other touches.
__global__ void __launch_bounds__(WG) k_cross_launch(const uint32_t *__restrict__ si, const uint32_t *__restrict__ sj,
                                                     uint64_t n_words, uint32_t tag, uint32_t earlier,
                                                     DevRace *__restrict__ out, uint32_t cap,
                                                     uint32_t *__restrict__ count) {
    for (uint64_t x = (uint64_t)blockIdx.x * WG + threadIdx.x; x < n_words; x += (uint64_t)gridDim.x * WG) {
        const uint32_t ai = si[x], wi = si[n_words + x], aj = sj[x], wj = sj[n_words + x];
        if (!((wi != NONE && aj != NONE) || (wj != NONE && ai != NONE))) continue;
        DevRace r;
        r.unit = tag; r.space = 1; r.scope = 2; r.block = earlier; r.epoch = NONE; r.addr = (uint32_t)x;
        r.w = wi != NONE ? aj : wj;     // the later launch's smallest conflicting thread
        r.o = wj != NONE ? ai : wi;     // the earlier launch's
        const uint32_t at = atomicAdd(count, 1u);
        if (at < cap) out[at] = r;
    }
}

// A copy (mem[dst + k] = mem[src + k]; the ranges do not overlap) or a host
// write (mem[dst + k] = value) of a job's host program.
__global__ void __launch_bounds__(WG) k_item_apply(int32_t *__restrict__ mem, uint32_t kind, uint64_t dst,
                                                   uint64_t src, uint64_t words, int32_t value) {
    for (uint64_t k = (uint64_t)blockIdx.x * WG + threadIdx.x; k < words; k += (uint64_t)gridDim.x * WG)
        mem[dst + k] = kind == KC_ITEM_COPY ? mem[src + k] : value;
}

// Access summary of a copy or host access (same layout as k_summary's):
// thread k touches the k-th word of each range it reads or writes.  The
// ranges are disjoint, so each word is written once.
__global__ void __launch_bounds__(WG) k_item_summary(uint32_t *__restrict__ sum, uint64_t n_words, uint32_t kind,
                                                     uint64_t dst, uint64_t src, uint64_t words) {
    for (uint64_t k = (uint64_t)blockIdx.x * WG + threadIdx.x; k < words; k += (uint64_t)gridDim.x * WG) {
        if (kind == KC_ITEM_COPY) sum[src + k] = (uint32_t)k;
        sum[dst + k] = (uint32_t)k;
        if (kind != KC_ITEM_HOST_READ) sum[n_words + dst + k] = (uint32_t)k;
    }
}

}  // namespace

hipError_t launch_item_apply(int32_t *mem, uint32_t kind, uint64_t dst, uint64_t src, uint64_t words, int32_t value,
                             hipStream_t s) {
    if (words == 0 || (kind != KC_ITEM_COPY && kind != KC_ITEM_HOST_WRITE)) return hipSuccess;
    hipLaunchKernelGGL(k_item_apply, dim3((uint32_t)std::min<uint64_t>(blocks_for(words), 8192)), dim3(WG), 0, s,
                       mem, kind, dst, src, words, value);
    return hipGetLastError();
}

hipError_t launch_item_summary(uint32_t *sum, uint64_t n_words, uint32_t kind, uint64_t dst, uint64_t src,
                               uint64_t words, hipStream_t s) {
    if (words == 0 || kind == KC_ITEM_LAUNCH || kind == KC_ITEM_HOST_WAIT) return hipSuccess;
    hipLaunchKernelGGL(k_item_summary, dim3((uint32_t)std::min<uint64_t>(blocks_for(words), 8192)), dim3(WG), 0, s,
                       sum, n_words, kind, dst, src, words);
    return hipGetLastError();
}

hipError_t launch_summary(const SummaryArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_summary, dim3((uint32_t)std::min<uint64_t>(blocks_for(a.n), 8192)), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_held_compact(const uint64_t *blk_log, const uint32_t *blk_held, uint64_t *blk_off,
                               uint32_t n_blocks, uint64_t *log, unsigned long long log_cap,
                               unsigned long long *log_count, uint32_t *flags, hipStream_t s) {
    if (n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_held_scan, dim3(1), dim3(1024), 0, s, blk_held, blk_off, n_blocks, log_cap, log_count, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_held_copy, dim3(std::min<uint32_t>(n_blocks, 8192)), dim3(WG), 0, s, blk_log, blk_held,
                       blk_off, n_blocks, log, log_cap);
    return hipGetLastError();
}

hipError_t launch_alloc_scan(const AllocScanArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_alloc_scan, dim3((uint32_t)std::min<uint64_t>(blocks_for(a.n), 8192)), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cross_launch(const uint32_t *si, const uint32_t *sj, uint64_t n_words, uint32_t tag,
                               uint32_t earlier, DevRace *out, uint32_t cap, uint32_t *count, hipStream_t s) {
    if (n_words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cross_launch, dim3((uint32_t)std::min<uint64_t>(blocks_for(n_words), 8192)), dim3(WG), 0, s,
                       si, sj, n_words, tag, earlier, out, cap, count);
    return hipGetLastError();
}

size_t check_long_cap(uint64_t n) { return (size_t)(2 * (n / SEG_LIMIT) + 2); }

hipError_t launch_check(const CheckArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check, dim3((uint32_t)((a.n + CHECK_TILE - 1) / CHECK_TILE)), dim3(WG), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // long segments: the list length is on the device; enough workgroups for
    // any list this check can produce, each striding over the list
    const uint32_t g = (uint32_t)std::min<uint64_t>(1024, check_long_cap(a.n));
    hipLaunchKernelGGL(k_check_long, dim3(g), dim3(WG), 0, s, a);
    return hipGetLastError();
}

// Sets *flag when a record of keys[0, n) is not a global-memory representative
// (a shared-space record, or one of an epoch that was not checked locally).
__global__ void __launch_bounds__(WG) k_log_reps_only(const uint64_t *__restrict__ keys, uint64_t n, KeyPlan k,
                                                      uint32_t *__restrict__ flag) {
    bool other = false;
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * WG) {
        const uint64_t r = keys[i];
        other |= rec_field(r, k.s_sp, 1) != 1u || rec_field(r, k.s_ep, k.eb) != k.ep_rep;
    }
    if (__ballot(other) && __lane_id() == 0) atomicOr(flag, 1u);
}

hipError_t launch_log_reps_only(const uint64_t *keys, uint64_t n, KeyPlan kp, uint32_t *flag, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint32_t g = blocks_for(n);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_log_reps_only, dim3(g), dim3(WG), 0, s, keys, n, kp, flag);
    return hipGetLastError();
}

hipError_t launch_restore(const uint64_t *keys, uint64_t n, KeyPlan kp, const DevUnit *units,
                          const uint32_t *blk_flags, hipStream_t s, const unsigned long long *n_dev) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_restore, dim3(blocks_for(n)), dim3(WG), 0, s, keys, n, kp, units, blk_flags, n_dev);
    return hipGetLastError();
}

hipError_t launch_flagged_comps(const uint32_t *blk_flags, uint32_t n_blocks, const DevUnit *units, uint32_t n_units,
                                uint2 *comps, uint32_t *n_comps, hipStream_t s, const ZeroArgs *zero) {
    const ZeroArgs none{{}, {}, 0};
    hipLaunchKernelGGL(k_flagged_comps, dim3(1), dim3(1024), 0, s, blk_flags, n_blocks, units, n_units, comps, n_comps,
                       zero ? *zero : none);
    return hipGetLastError();
}

hipError_t launch_coverage(const uint64_t *rs, uint64_t n_rs, const uint64_t *log, uint64_t n_log, KeyPlan kp,
                           const DevUnit *units, const uint32_t *blk_flags, DevCounters *ctr, uint64_t *list,
                           hipStream_t s) {
    if (n_rs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_coverage, dim3(blocks_for(n_rs)), dim3(WG), 0, s, rs, n_rs, log, n_log, kp, units, blk_flags,
                       ctr, list);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t g = (uint32_t)std::min<uint64_t>(256, n_rs);
    hipLaunchKernelGGL(k_coverage_long, dim3(g), dim3(WG), 0, s, rs, n_rs, log, n_log, kp, units, blk_flags, ctr,
                       list);
    return hipGetLastError();
}

hipError_t launch_copy_units(const DevUnit *units, uint32_t n_units, uint32_t max_words, bool to_snapshot,
                             const uint32_t *unit_mask, hipStream_t s) {
    if (n_units == 0) return hipSuccess;
    uint32_t gx = (uint32_t)std::min<uint64_t>(1024, std::max<uint64_t>(1, max_words / (WG * 16)));
    hipLaunchKernelGGL(k_copy_units, dim3(gx, n_units), dim3(WG), 0, s, units, to_snapshot ? 1 : 0, unit_mask);
    return hipGetLastError();
}

hipError_t launch_replay_table(const ReplayTableArgs &a, hipStream_t s) {
    if (a.n_rs == 0) return hipSuccess;
    ZeroArgs z{{(uint32_t *)a.table, (uint32_t *)a.ctr}, {(size_t)2 << a.bits, sizeof(DevCounters) / 4}, 2};
    hipError_t e = launch_zero_many(z, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rtable_insert, dim3(blocks_for(a.n_rs)), dim3(WG), 0, s, a);
    hipLaunchKernelGGL(k_rtable_check, dim3(blocks_for(1ull << a.bits)), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_log_table(const ReplayTableArgs &a, hipStream_t s) {
    if (a.n_rs == 0) return hipSuccess;
    ZeroArgs z{{(uint32_t *)a.table, (uint32_t *)a.ctr}, {(size_t)2 << a.bits, sizeof(DevCounters) / 4}, 2};
    hipError_t e = launch_zero_many(z, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rtable_insert, dim3(blocks_for(a.n_rs)), dim3(WG), 0, s, a);
    hipLaunchKernelGGL(k_rtable_conflicts, dim3(blocks_for(1ull << a.bits)), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_log_direct(const ReplayTableArgs &a, uint64_t words, hipStream_t s) {
    if (a.n_rs == 0) return hipSuccess;
    ZeroArgs z{{a.downer, (uint32_t *)a.dflags, (uint32_t *)a.ctr},
               {(size_t)words, (size_t)(words + 3) / 4, sizeof(DevCounters) / 4}, 3};
    hipError_t e = launch_zero_many(z, s);
    if (e != hipSuccess) return e;
    // the record count is read on the device: a strided grid sized for a
    // fraction of the capacity
    const uint32_t g = std::min<uint32_t>(blocks_for(a.n_rs), 2048);
    hipLaunchKernelGGL(k_dtable_own, dim3(g), dim3(WG), 0, s, a);
    hipLaunchKernelGGL(k_dtable_multi, dim3(g), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs &a, hipStream_t s) {
    uint32_t most = 0;
    for (uint32_t k = 0; k < a.n; k++) most = a.words[k] > most ? a.words[k] : most;
    if (most == 0) return hipSuccess;
    uint32_t g = (most + WG - 1) / WG;
    if (g > 256) g = 256;
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zero_many(const ZeroArgs &z, hipStream_t s) {
    size_t most = 0;
    for (uint32_t k = 0; k < z.n; k++) most = z.words[k] > most ? z.words[k] : most;
    if (most == 0) return hipSuccess;
    size_t g = (most + WG - 1) / WG;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_zero_many, dim3((uint32_t)g), dim3(WG), 0, s, z);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    uint32_t g = (uint32_t)((words + WG - 1) / WG);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_zero, dim3(g), dim3(WG), 0, s, (uint32_t *)p, words);
    return hipGetLastError();
}

}  // namespace kc
