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

#include "kc_internal.h"

namespace kc {

namespace {

constexpr int WG = 256;
constexpr uint32_t NONE = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t lane_prefix(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

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

__global__ void __launch_bounds__(WG) k_check(CheckArgs A) {
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= A.n) return;
    const KeyPlan &k = A.kp;
    const uint64_t *keys = A.keys;
    const uint64_t ki = keys[i];
    const uint32_t ps = k.s_ep;                  // bits below: tid and kind
    const uint64_t inner = ki >> ps;
    const uint32_t unit = rec_field(ki, k.s_unit, k.ub);
    const uint32_t space = rec_field(ki, k.s_sp, 1);
    const uint32_t addr = rec_field(ki, k.s_addr, k.ab);
    const uint32_t block0 = rec_field(ki, k.s_blk, k.bb);

    if (i == 0 || (keys[i - 1] >> ps) != inner) {
        // intra-block segment: smallest writer and two smallest distinct tids
        uint32_t minw = NONE, t1 = NONE, t2 = NONE;
        for (uint64_t j = i; j < A.n; j++) {
            const uint64_t kj = keys[j];
            if ((kj >> ps) != inner) break;
            const uint32_t tid = rec_field(kj, k.s_tid, k.tb);
            if (kj & 1ull) minw = min(minw, tid);
            if (tid < t1) { t2 = t1; t1 = tid; }
            else if (tid != t1 && tid < t2) t2 = tid;
        }
        if (minw != NONE && t2 != NONE) {
            DevRace r;
            r.unit = unit; r.space = space; r.scope = 0; r.block = block0;
            r.epoch = rec_field(ki, k.s_ep, k.eb); r.addr = addr;
            r.w = minw; r.o = (t1 == minw) ? t2 : t1;
            push_race(A, r);
            A.blk_flags[A.units[unit].block_base + block0] = 1u;
        }
    }
    if (space == 1u) {
        const uint64_t outer = ki >> k.s_addr;
        if (i == 0 || (keys[i - 1] >> k.s_addr) != outer) {
            const uint32_t nt = A.units[unit].nt;
            uint32_t wg = NONE, wb = NONE, g1 = NONE, b1 = NONE, g2 = NONE;
            uint64_t end = i;
            for (uint64_t j = i; j < A.n; j++) {
                const uint64_t kj = keys[j];
                if ((kj >> k.s_addr) != outer) break;
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
            if (wg != NONE && g2 != NONE) {
                DevRace r;
                r.unit = unit; r.space = 1; r.scope = 1; r.block = wb; r.epoch = NONE; r.addr = addr;
                r.w = wg; r.o = (wb == b1) ? g2 : g1;
                push_race(A, r);
                // every block touching the location joins the racy component
                uint32_t prev = NONE;
                for (uint64_t j = i; j < end; j++) {
                    const uint32_t b = rec_field(keys[j], k.s_blk, k.bb);
                    if (b != prev) {
                        A.blk_flags[A.units[unit].block_base + b] = 1u;
                        if (b != block0) push_edge(A, unit, block0, b);
                        prev = b;
                    }
                }
            }
        }
    }
}

// Put back the launch-start value of every global word a flagged block wrote.
__global__ void __launch_bounds__(WG) k_restore(const uint64_t *__restrict__ keys, uint64_t n, KeyPlan k,
                                                const DevUnit *__restrict__ units,
                                                const uint32_t *__restrict__ blk_flags) {
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const uint64_t r = keys[i];
    if (!(r & 1ull) || rec_field(r, k.s_sp, 1) != 1u) return;
    const DevUnit &u = units[rec_field(r, k.s_unit, k.ub)];
    if (!blk_flags[u.block_base + rec_field(r, k.s_blk, k.bb)]) return;
    const uint32_t a = rec_field(r, k.s_addr, k.ab);
    u.mem[a] = u.snap[a];
}

// Records of flagged blocks, appended in any order.
__global__ void __launch_bounds__(WG) k_extract(const uint64_t *__restrict__ keys, uint64_t n, KeyPlan k,
                                                const DevUnit *__restrict__ units,
                                                const uint32_t *__restrict__ blk_flags, uint64_t *__restrict__ out,
                                                uint64_t out_cap, unsigned long long *__restrict__ cnt) {
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    bool take = false;
    uint64_t r = 0;
    if (i < n) {
        r = keys[i];
        const DevUnit &u = units[rec_field(r, k.s_unit, k.ub)];
        take = blk_flags[u.block_base + rec_field(r, k.s_blk, k.bb)] != 0;
    }
    const uint64_t m = __ballot(take);
    if (m == 0) return;
    const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (__lane_id() == leader) base = atomicAdd(cnt, (unsigned long long)__popcll(m));
    const uint32_t lo = __shfl((uint32_t)base, (int)leader), hi = __shfl((uint32_t)(base >> 32), (int)leader);
    base = ((unsigned long long)hi << 32) | lo;
    const uint64_t idx = base + lane_prefix(m);
    if (take && idx < out_cap) out[idx] = r;
}

__global__ void __launch_bounds__(WG) k_compare(const uint64_t *__restrict__ x, const uint64_t *__restrict__ y,
                                                uint64_t n, uint32_t *__restrict__ flags) {
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    const bool diff = i < n && x[i] != y[i];
    if (__ballot(diff) && __lane_id() == 0) atomicOr(flags, FLAG_MISMATCH);
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

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + WG - 1) / WG); }

}  // namespace

hipError_t launch_check(const CheckArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check, dim3(blocks_for(a.n)), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_restore(const uint64_t *keys, uint64_t n, KeyPlan kp, const DevUnit *units,
                          const uint32_t *blk_flags, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_restore, dim3(blocks_for(n)), dim3(WG), 0, s, keys, n, kp, units, blk_flags);
    return hipGetLastError();
}

hipError_t launch_extract(const uint64_t *keys, uint64_t n, KeyPlan kp, const DevUnit *units,
                          const uint32_t *blk_flags, uint64_t *out, uint64_t out_cap,
                          unsigned long long *out_count, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_extract, dim3(blocks_for(n)), dim3(WG), 0, s, keys, n, kp, units, blk_flags, out,
                       out_cap, out_count);
    return hipGetLastError();
}

hipError_t launch_compare(const uint64_t *x, const uint64_t *y, uint64_t n, uint32_t *flags, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compare, dim3(blocks_for(n)), dim3(WG), 0, s, x, y, n, flags);
    return hipGetLastError();
}

hipError_t launch_copy_units(const DevUnit *units, uint32_t n_units, uint32_t max_words, bool to_snapshot,
                             const uint32_t *unit_mask, hipStream_t s) {
    if (n_units == 0) return hipSuccess;
    uint32_t gx = (uint32_t)std::min<uint64_t>(1024, std::max<uint64_t>(1, max_words / (WG * 16)));
    hipLaunchKernelGGL(k_copy_units, dim3(gx, n_units), dim3(WG), 0, s, units, to_snapshot ? 1 : 0, unit_mask);
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
