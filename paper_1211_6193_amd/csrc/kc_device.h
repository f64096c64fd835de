// Device code of the KC-IR interpreter on gfx950 (included by the
// interpreter kernels, and compiled at run time into the program-specialised
// kernels, which share everything but the instruction loop).
//
// SIMT interpreter of KC-IR on gfx950: one lane per simulated thread, one
// workgroup per simulated block.
//
// Free-run mode (the hot path): each wavefront executes the instruction at
// the smallest pc among its running lanes (uniform fetch/decode through the
// scalar cache), so converged lanes run together and divergent lanes
// reconverge at the smallest pc.  A lane that reaches BAR waits; when every
// wave of the block is quiescent (no running lane) the block takes one
// hardware barrier and counts arrivals with ballots: all threads waiting
// completes the barrier episode (the token-passing rules of the paper's
// Section 3 "Barrier synchronization" require all NThrds threads of the block
// and never compare barrier sites, so differing sites are reported as
// DIVERGENCE and the episode still completes); some waiting and the rest
// exited is the Section 3.1 deadlock.  Every in-bounds load/store appends a
// 64-bit access record (unit, space, address, block, epoch, tid, kind) to a
// per-wave LDS staging area that is flushed to the HBM log with one atomic
// per flush.
//
// Lockstep mode (replay of racy blocks): a workgroup runs the blocks of one
// component one after another; in every step each running thread executes
// exactly one instruction, loads see memory as of the start of the step and
// the step's stores land in ascending tid order -- the canonical execution.
#pragma once
#ifndef __HIPCC_RTC__
#include <climits>

#include "kc_internal.h"
#endif
#ifndef INT_MAX
#define INT_MAX 2147483647
#endif

namespace kc {

namespace {

constexpr int WAVE = 64;
constexpr uint32_t NONE_U32 = 0xFFFFFFFFu;
enum : int { ST_RUN = 0, ST_WAIT = 1, ST_EXIT = 2, ST_DEAD = 3 };

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lane_prefix(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniu(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// Wave-wide min/max: DPP inside each row of 16 lanes, then the four row
// results through readlane (no LDS traffic).  All 64 lanes must be active.
__device__ __forceinline__ int row_min(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // row_mirror
    return v;
}
__device__ __forceinline__ int row_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
    v = row_min(v);
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ int wave_max(int v) {
    v = row_max(v);
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ uint32_t wave_min_u(uint32_t v) {
    // order-preserving map of uint32 onto int32
    return (uint32_t)wave_min((int)(v ^ 0x80000000u)) ^ 0x80000000u;
}

__device__ __forceinline__ unsigned long long bcast_u64(unsigned long long v, uint32_t src) {
    uint32_t lo = __shfl((uint32_t)v, (int)src), hi = __shfl((uint32_t)(v >> 32), (int)src);
    return ((unsigned long long)hi << 32) | lo;
}

// int32 ALU with the library's wrap / division conventions.
__device__ __forceinline__ int32_t alu(uint32_t base, int32_t x, int32_t y, bool &arith) {
    uint32_t ux = (uint32_t)x, uy = (uint32_t)y;
    switch (base) {
    case OP_ADD: return (int32_t)(ux + uy);
    case OP_SUB: return (int32_t)(ux - uy);
    case OP_MUL: return (int32_t)(ux * uy);
    case OP_DIV:
        if (y == 0) { arith = true; return 0; }
        if (y == -1) return (int32_t)(0u - ux);          // INT_MIN / -1 wraps to INT_MIN
        return x / y;
    case OP_REM:
        if (y == 0) { arith = true; return 0; }
        if (y == -1) return 0;
        return x % y;
    case OP_AND: return x & y;
    case OP_OR: return x | y;
    case OP_XOR: return x ^ y;
    case OP_SHL: return (int32_t)(ux << (uy & 31u));
    case OP_SHRA: return x >> (int)(uy & 31u);
    case OP_SHRL: return (int32_t)(ux >> (uy & 31u));
    case OP_MIN: return min(x, y);
    case OP_MAX: return max(x, y);
    case OP_SLT: return x < y ? 1 : 0;
    case OP_SLE: return x <= y ? 1 : 0;
    case OP_SEQ: return x == y ? 1 : 0;
    case OP_SNE: return x != y ? 1 : 0;
    case OP_SLTU: return ux < uy ? 1 : 0;
    default: return 0;
    }
}

struct Shared {
    int32_t *sh;        // simulated shared memory
    uint64_t *stage;    // this wave's record staging area
    uint64_t *stage_all;// all waves' staging areas (contiguous, nwaves * stage records)
    uint64_t *alt;      // second buffer of the same size (epoch-local sort)
    uint32_t *wc;       // nwaves x 256 digit counters (epoch-local sort)
    uint32_t *tmp;      // 256 words
    unsigned long long *shadow;   // per simulated shared word: access tuple of the current epoch (replay)
    uint32_t *vmin, *vmax, *vw;   // the same region in the free run: smallest and largest accessing tid, any store
    unsigned long long *gst;      // global shadow table: per global location, its tuple of the epoch
    uint64_t *repbuf;   // with the table: representative records held until the block ends (A.rep_hold)
    uint32_t *slots;    // 16 waves x 10 words: episode reductions, lockstep rounds
    uint32_t *slots2;   // 16 x 4: divergence second round
    uint32_t *eps;      // free-run episodes: 3 sets of EPS_WORDS summary words, used in turn
    uint32_t *sinit;    // one bit per simulated shared word: stored to since the block began (option uninit)
};

typedef const __attribute__((address_space(4))) uint64_t const_word_t;   // scalar-cache reads
typedef __attribute__((address_space(1))) int32_t global_i32_t;

struct BlockCtx {
    const DevUnit *u;
    const_word_t *prog;     // program words, read through the scalar cache
    global_i32_t *mem;      // the unit's global memory
    uint32_t unit, block;
    uint32_t tid;           // linear tid of this lane
    uint32_t nt, nwaves, wave;
    uint32_t n_instr, n_words, sh_words;
    uint64_t kbase;         // record bits fixed for this lane: unit, block, tid
    uint64_t kep;           // kbase plus the current epoch
    uint32_t *gocc;         // global shadow table: occupancy and overflow words of the current epoch
    uint32_t step;          // replay: the lockstep step being executed (warp-aware model)
    uint32_t epoch;         // replay: the current epoch (warp-aware model)
};

// Wave-aggregated append of findings.
// Wave-aggregated append of findings (rare: kept out of line so the hot
// loops carry only the ballot).
__device__ __noinline__ void emit_fault_wave(uint64_t m, bool f, uint32_t *fault_count, DevFault *faults,
                                             uint32_t fault_cap, uint32_t *flags, uint32_t unit, uint32_t block,
                                             uint32_t kind, uint32_t epoch, uint32_t a, uint32_t b, uint32_t c,
                                             uint32_t d) {
    uint32_t leader = (uint32_t)__ffsll((long long)m) - 1;
    uint32_t cnt = (uint32_t)__popcll(m);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(fault_count, cnt);
    base = __shfl(base, (int)leader);
    if (f) {
        uint32_t idx = base + lane_prefix(m);
        if (idx < fault_cap) {
            DevFault F;
            F.unit = unit; F.kind = kind; F.block = block; F.epoch = epoch;
            F.a = a; F.b = b; F.c = c; F.d = d;
            faults[idx] = F;
        } else {
            atomicOr(flags, FLAG_FAULT_OVERFLOW);
        }
    }
}

__device__ __forceinline__ void emit_fault(bool f, const InterpArgs &A, const BlockCtx &B, uint32_t kind, uint32_t epoch,
                           uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    const uint64_t m = __ballot(f);
    if (m == 0) return;
    emit_fault_wave(m, f, A.fault_count, A.faults, A.fault_cap, A.flags, B.unit, B.block, kind, epoch, a, b, c, d);
}

// Warp-aware model: an in-bounds access of the replay with its step, appended
// with one reservation per wave.
// (The buffers are passed one by one: a reference to the kernel's argument
// block would make every kernel that calls this copy that block to scratch.)
__device__ __noinline__ void wlog_append_wave(WarpRec *wlog, uint32_t wlog_cap, uint32_t *wlog_count, uint32_t *flags,
                                             uint64_t m, bool on, uint32_t unit, uint32_t block, uint32_t epoch,
                                             uint32_t step, uint32_t addr, uint32_t tsk) {
    const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(wlog_count, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, (int)leader);
    if (on) {
        const uint32_t idx = base + lane_prefix(m);
        if (idx < wlog_cap) wlog[idx] = WarpRec{unit, block, epoch, step, addr, tsk};
        else atomicOr(flags, FLAG_WLOG_OVERFLOW);
    }
}
__device__ __forceinline__ void wlog_append(const InterpArgs &A, const BlockCtx &B, bool inb, uint32_t space,
                                            uint32_t addr, bool store) {
    const uint64_t m = __ballot(inb);
    if (m == 0) return;
    wlog_append_wave(A.wlog, A.wlog_cap, A.wlog_count, A.flags, m, inb, B.unit, B.block, B.epoch, B.step, addr,
                     B.tid | (store ? 1u << 16 : 0u) | (space << 17));
}

// Copy a wave's staged records to the HBM log (one atomic reservation).
__device__ __noinline__ void flush_stage_wave(uint64_t *stage, uint32_t cnt, uint64_t *log,
                                              unsigned long long log_cap, unsigned long long *log_count,
                                              uint32_t *flags) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(log_count, (unsigned long long)cnt);
    base = bcast_u64(base, 0);
    for (uint32_t i = lane_id(); i < cnt; i += WAVE) {
        unsigned long long p = base + i;
        if (p < log_cap) log[p] = stage[i];
    }
    if (lane_id() == 0 && base + cnt > log_cap) atomicOr(flags, FLAG_LOG_OVERFLOW);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ void flush_stage(const InterpArgs &A, uint64_t *stage, uint32_t cnt) {
    if (cnt == 0) return;
    flush_stage_wave(stage, cnt, A.log, A.log_cap, A.log_count, A.flags);
}

struct LogState {
    uint32_t cur;       // staged records (wave-uniform)
    uint32_t total;     // records of this wave for the block
    uint32_t gtotal;    // of which global-space
    bool spilled;       // this wave flushed records of the current epoch to HBM
};

__device__ __forceinline__ void log_rec(const InterpArgs &A, uint64_t *stage, LogState &L, bool rec,
                                        uint64_t key) {
    uint64_t m = __ballot(rec);
    if (m == 0) return;
    uint32_t cnt = (uint32_t)__popcll(m);
    if (L.cur + cnt > A.stage) {
        flush_stage(A, stage, L.cur);
        L.cur = 0;
        L.spilled = true;
    }
    if (rec) stage[L.cur + lane_prefix(m)] = key;
    L.cur += cnt;
    L.total += cnt;
}

// Per-lane thread state.  The simulated register file is a 16-wide vector so
// that reads/writes with a wave-uniform register index become indexed VGPR
// moves instead of private-memory accesses.
typedef int32_t regfile_t __attribute__((ext_vector_type(16)));
struct Lane {
    int pc;
    int st;
    uint32_t fuel;
    int bar_pc;
    int bpred;          // at a barrier with a predicate: (kind + 1) << 1 | predicate; 0 at a plain one
    int32_t bres;       // its result once the episode completes
    regfile_t r;
};

// ---- epoch-local conflict check -------------------------------------------
// At a barrier episode every record of the closing epoch is still in the
// waves' LDS staging areas unless one of them overflowed.  The block then sorts
// them in LDS by (space, address) -- block and epoch are fixed -- and reduces
// each location: an intra-block race is emitted at once, and for a global
// location only two representative records (the smallest tid, the smallest
// writer) go to the HBM log for the cross-block check, tagged with the reserved
// epoch value so the global pass does not check them again within the block.
// If a wave overflowed, all records of the epoch go to the log unreduced.

// Shadow tuple of a shared word for the current epoch (Section 3.1 keeps a
// tuple per shared location, cleared at __syncthreads()): the smallest writer
// tid and the two smallest distinct tids that accessed it, 16 bits each.
constexpr unsigned long long SHADOW_EMPTY = 0xFFFFFFFFFFFFull;
constexpr uint32_t SH_NONE = 0xFFFFu;

__device__ __forceinline__ unsigned long long shadow_add(unsigned long long s, uint32_t tid, bool write) {
    uint32_t t1 = (uint32_t)(s & 0xFFFF), t2 = (uint32_t)((s >> 16) & 0xFFFF), w = (uint32_t)((s >> 32) & 0xFFFF);
    if (tid < t1) { t2 = t1; t1 = tid; }
    else if (tid != t1 && tid < t2) t2 = tid;
    if (write && tid < w) w = tid;
    return (unsigned long long)t1 | ((unsigned long long)t2 << 16) | ((unsigned long long)w << 32);
}

__device__ __forceinline__ void shadow_update(unsigned long long *sh, uint32_t addr, uint32_t tid, bool write) {
    unsigned long long old = sh[addr];
    for (;;) {
        const unsigned long long nw = shadow_add(old, tid, write);
        if (nw == old) return;
        const unsigned long long prev = atomicCAS(&sh[addr], old, nw);
        if (prev == old) return;
        old = prev;
    }
}

// The free run needs only a verdict per shared word and epoch: a block with
// an intra-block race is replayed, and the replay computes the canonical
// tuples.  Racy means a store and two distinct threads, i.e. the smallest and
// the largest accessing tid differ and some access stored, which three
// non-returning LDS atomics maintain (no compare-and-swap loop, no wait).
__device__ __forceinline__ void shadow_mark(const Shared &S, uint32_t addr, uint32_t tid, bool write) {
    atomicMin(&S.vmin[addr], tid);
    atomicMax(&S.vmax[addr], tid);
    if (write) atomicOr(&S.vw[addr], 1u);
}

// Uninitialised shared words (option uninit): a bit per word, set by every
// store to it (in the free run at once; in the replay when the step's stores
// land, after every load of the step has tested it).
__device__ __forceinline__ bool shared_stored(const Shared &S, uint32_t addr) {
    return (S.sinit[addr >> 5] >> (addr & 31u)) & 1u;
}
__device__ __forceinline__ void mark_stored(const Shared &S, uint32_t addr) {
    atomicOr(&S.sinit[addr >> 5], 1u << (addr & 31u));
}

// Bytes of the shadow region: 8 per shared word for the replay's tuples, 12
// for the free run's three verdict words; rounded to 16.
__host__ __device__ inline size_t shadow_region_bytes(uint32_t sh_words) {
    return ((size_t)sh_words * 12 + 15) & ~(size_t)15;
}

// ---- global shadow table ------------------------------------------------------
// The same tuple for the global locations a block touches in the current
// epoch, kept in an open-addressing LDS table (linear probing).  A slot packs
// the location and its tuple in one word, so inserting a location and
// updating its tuple is one compare-and-swap:
//   t1(11) | t2(11) | w(11) | address(31),   empty slot = all ones.
// Tids are below 1024; 0x7FF is "none".  Locations need at most 31 bits.
// A location that finds no slot within GST_PROBES probes, or no free slot
// while the table is half full, is not absorbed: its access is staged as a
// record instead and the epoch is marked overflowed; at the episode the
// table's tuples then go to the log as records (at most three per location:
// t1, t2 and the smallest writer, which reduce to the same tuple) together
// with the staged ones, and the global check reduces them.
constexpr unsigned long long GST_EMPTY = ~0ull;
constexpr uint32_t GT_NONE = 0x7FFu;
constexpr uint32_t GST_PROBES = 16;

__device__ __forceinline__ unsigned long long gst_tuple(uint32_t t1, uint32_t t2, uint32_t w) {
    return (unsigned long long)t1 | ((unsigned long long)t2 << 11) | ((unsigned long long)w << 22);
}
__device__ __forceinline__ uint32_t gst_addr(unsigned long long s) { return (uint32_t)(s >> 33); }

// Merge tuple `u` (t1, t2, w fields) into slot word `s`.
__device__ __forceinline__ unsigned long long gst_merge(unsigned long long s, unsigned long long u) {
    uint32_t t1 = (uint32_t)s & GT_NONE, t2 = (uint32_t)(s >> 11) & GT_NONE, w = (uint32_t)(s >> 22) & GT_NONE;
    const uint32_t u1 = (uint32_t)u & GT_NONE, u2 = (uint32_t)(u >> 11) & GT_NONE, v = (uint32_t)(u >> 22) & GT_NONE;
    w = min(w, v);
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const uint32_t x = q ? u2 : u1;
        if (x < t1) { t2 = t1; t1 = x; }
        else if (x != t1 && x < t2) t2 = x;
    }
    return (s & ~((1ull << 33) - 1ull)) | gst_tuple(t1, t2, w);
}

// Absorb tuple `u` of location `addr`; false if the location found no slot.
__device__ __forceinline__ bool gst_insert(unsigned long long *gst, uint32_t bits, uint32_t *occupied,
                                           uint32_t addr, unsigned long long u) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t slot = (addr * 2654435761u) >> (32 - bits);
    for (uint32_t p = 0; p < GST_PROBES; p++) {
        unsigned long long cur = gst[slot];
        for (;;) {
            if (cur == GST_EMPTY) {
                if (__hip_atomic_load(occupied, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > (mask >> 1))
                    return false;                   // half full: no new locations
                const unsigned long long prev =
                    atomicCAS(&gst[slot], GST_EMPTY, ((unsigned long long)addr << 33) | u);
                if (prev == GST_EMPTY) {
                    atomicAdd(occupied, 1u);
                    return true;
                }
                cur = prev;                         // taken meanwhile: look again
                continue;
            }
            if (gst_addr(cur) != addr) break;       // another location: next slot
            const unsigned long long nw = gst_merge(cur, u);
            if (nw == cur) return true;
            const unsigned long long prev = atomicCAS(&gst[slot], cur, nw);
            if (prev == cur) return true;
            cur = prev;
        }
        slot = (slot + 1u) & mask;
    }
    return false;
}

// An in-bounds global access (lanes with `inb`) under the epoch-local check:
// absorbed into the global shadow table, else staged as record `key`.  When
// every accessing lane of the wave names one location (a broadcast read, a
// table entry), the wave's tuple -- its two lowest lanes, and the lowest as
// writer for a store -- is inserted once.
__device__ __forceinline__ void global_access(const InterpArgs &A, const BlockCtx &B, const Shared &S, LogState &L,
                                              bool inb, uint32_t addr, bool store, uint64_t key) {
    if (A.gst_bits == 0) {
        log_rec(A, S.stage, L, inb, key);
        return;
    }
    const uint64_t m = __ballot(inb);
    if (m == 0) return;
    const uint32_t first = (uint32_t)__ffsll((long long)m) - 1u;
    const uint32_t a0 = (uint32_t)__shfl((int)addr, (int)first);
    bool ok = false;
    if (__ballot(inb && addr != a0) == 0) {
        if (lane_id() == first) {
            const uint64_t m2 = m & (m - 1ull);
            const uint32_t t1 = B.tid, t2 = m2 ? B.wave * WAVE + (uint32_t)__ffsll((long long)m2) - 1u : GT_NONE;
            ok = gst_insert(S.gst, A.gst_bits, B.gocc, a0, gst_tuple(t1, t2, store ? t1 : GT_NONE));
        }
        ok = __shfl((int)ok, (int)first) != 0;
    } else if (inb) {
        ok = gst_insert(S.gst, A.gst_bits, B.gocc, addr, gst_tuple(B.tid, GT_NONE, store ? B.tid : GT_NONE));
    }
    L.total += (uint32_t)__popcll(__ballot(inb && ok));
    const bool miss = inb && !ok;
    if (__ballot(miss)) {
        if (lane_id() == 0) B.gocc[1] = 1u;         // the epoch overflowed the table
        log_rec(A, S.stage, L, miss, key);
    }
}

__device__ __forceinline__ uint32_t local_key(uint64_t r, const KeyPlan &k) {
    return (rec_field(r, k.s_sp, 1) << k.ab) | rec_field(r, k.s_addr, k.ab);
}

// One stable counting-sort pass over src[0..n) into dst by 8-bit digit.
__device__ __forceinline__ void local_sort_pass(const Shared &S, const BlockCtx &B, const KeyPlan &k,
                                                const uint64_t *src, uint64_t *dst, uint32_t n, uint32_t shift) {
    const uint32_t lane = lane_id();
    const uint32_t per = (n + B.nwaves - 1) / B.nwaves;
    const uint32_t c0 = min(n, B.wave * per), c1 = min(n, c0 + per);
    uint32_t *wc = S.wc + 256 * B.wave;
    for (uint32_t d = lane; d < 256; d += WAVE) wc[d] = 0;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint32_t base = c0; base < c1; base += WAVE) {
        const bool valid = base + lane < c1;
        const uint32_t d = valid ? (local_key(src[base + lane], k) >> shift) & 0xFFu : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(valid && bit);
            peers &= bit ? bb : ~bb;
        }
        if (valid && lane == (uint32_t)__ffsll((long long)peers) - 1) wc[d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    if (B.wave == 0) {      // exclusive offsets per (digit, wave): digit-major, wave-minor
        uint32_t sum = 0;
        for (uint32_t w = 0; w < B.nwaves; w++) {
            const uint32_t *row = S.wc + 256 * w + lane * 4;
            sum += row[0] + row[1] + row[2] + row[3];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if ((int)lane >= o) incl += y;
        }
        uint32_t run = incl - sum;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            for (uint32_t w = 0; w < B.nwaves; w++) {
                const uint32_t x = S.wc[256 * w + lane * 4 + q];
                S.wc[256 * w + lane * 4 + q] = run;
                run += x;
            }
        }
    }
    __syncthreads();
    for (uint32_t base = c0; base < c1; base += WAVE) {
        const bool valid = base + lane < c1;
        const uint64_t key = valid ? src[base + lane] : 0ull;
        const uint32_t d = valid ? (local_key(key, k) >> shift) & 0xFFu : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(valid && bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t leader = valid ? (uint32_t)__ffsll((long long)peers) - 1 : 0u;
        uint32_t old = 0;
        if (valid && lane == leader) {
            old = wc[d];
            wc[d] = old + (uint32_t)__popcll(peers);
        }
        old = __shfl(old, (int)leader);
        if (valid) dst[old + (uint32_t)__popcll(peers & lt)] = key;
    }
    __syncthreads();
}

__device__ __forceinline__ void push_local_race(const InterpArgs &A, const BlockCtx &B, uint32_t space, uint32_t epoch,
                                                uint32_t addr, uint32_t w, uint32_t o) {
    if (A.wlog) {           // warp-aware model: the host derives the block's tuples from the stepped accesses
        A.blk_flags[B.u->block_base + B.block] = 1u;
        return;
    }
    const uint32_t idx = atomicAdd(A.lrace_count, 1u);
    if (idx < A.lrace_cap) {
        DevRace r;
        r.unit = B.unit; r.space = space; r.scope = 0; r.block = B.block; r.epoch = epoch; r.addr = addr;
        r.w = w; r.o = o;
        A.lraces[idx] = r;
    } else {
        atomicOr(A.flags, FLAG_RACE_OVERFLOW);
    }
    A.blk_flags[B.u->block_base + B.block] = 1u;
}

// Reduction state of the accesses to one location in one epoch: smallest
// writer tid and the two smallest distinct tids (merged in any order).
struct SegState { uint32_t minw, t1, t2; };
constexpr uint32_t LOCAL_SEG_LIMIT = 16;

__device__ __forceinline__ void seg_insert(SegState &s, uint32_t x) {
    if (x < s.t1) { s.t2 = s.t1; s.t1 = x; }
    else if (x != s.t1 && x < s.t2) s.t2 = x;
}
__device__ __forceinline__ void seg_add(SegState &s, uint32_t tid, bool write) {
    if (write) s.minw = min(s.minw, tid);
    seg_insert(s, tid);
}
__device__ __forceinline__ void seg_merge(SegState &s, const SegState &o) {
    s.minw = min(s.minw, o.minw);
    seg_insert(s, o.t1);
    seg_insert(s, o.t2);
}

// A reduced segment whose first record is `r`: its race, and for global
// memory its representatives (the smallest tid, a write if that thread wrote,
// and the smallest writer when it is another thread) with the reserved epoch.
__device__ __forceinline__ void local_segment_done(const InterpArgs &A, const BlockCtx &B, const Shared &S,
                                                   uint64_t r, uint32_t epoch, const SegState &st, uint64_t *dst) {
    const KeyPlan &k = A.kp;
    const uint32_t space = rec_field(r, k.s_sp, 1);
    if (st.minw != NONE_U32 && st.t2 != NONE_U32)
        push_local_race(A, B, space, epoch, rec_field(r, k.s_addr, k.ab), st.minw, st.t1 == st.minw ? st.t2 : st.t1);
    if (space != 1u) return;
    const uint64_t keep = ~(((((1ull << k.tb) - 1ull) << k.s_tid)) | (((1ull << k.eb) - 1ull) << k.s_ep) | 1ull);
    const uint64_t base = (r & keep) | ((uint64_t)k.ep_rep << k.s_ep);
    const bool two = st.minw != NONE_U32 && st.minw != st.t1;
    const uint32_t at = atomicAdd(&S.tmp[32], two ? 2u : 1u);
    dst[at] = base | ((uint64_t)st.t1 << k.s_tid) | (st.minw == st.t1 ? 1ull : 0ull);
    if (two) dst[at + 1] = base | ((uint64_t)st.minw << k.s_tid) | 1ull;
}

// Empty the global shadow table at an episode.  With `reduced`, each location
// yields its intra-block race and its representatives (as from a reduced
// segment); otherwise its tuple goes to the log as up to three records of the
// epoch, for the global check.  The log space is reserved with one atomic per
// block; S.tmp[32] must be zero on entry.
__device__ __forceinline__ uint32_t gst_records(unsigned long long s, bool reduced) {
    const uint32_t t1 = (uint32_t)s & GT_NONE, t2 = (uint32_t)(s >> 11) & GT_NONE, w = (uint32_t)(s >> 22) & GT_NONE;
    if (reduced) return (w != GT_NONE && w != t1) ? 2u : 1u;
    return 1u + (t2 != GT_NONE ? 1u : 0u) + ((w != GT_NONE && w != t1 && w != t2) ? 1u : 0u);
}

__device__ __forceinline__ void gst_drain(const InterpArgs &A, const BlockCtx &B, const Shared &S, uint32_t epoch,
                                          bool reduced) {
    const KeyPlan &k = A.kp;
    const uint32_t C = 1u << A.gst_bits;
    uint32_t mine = 0;
    for (uint32_t i = threadIdx.x; i < C; i += blockDim.x) {
        const unsigned long long v = S.gst[i];
        if (v != GST_EMPTY) mine += gst_records(v, reduced);
    }
    uint32_t incl = mine;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if ((int)lane_id() >= o) incl += y;
    }
    const uint32_t wtot = (uint32_t)__shfl((int)incl, WAVE - 1);
    uint32_t woff = 0;
    if (lane_id() == WAVE - 1 && wtot) woff = atomicAdd(&S.tmp[32], wtot);
    woff = (uint32_t)__shfl((int)woff, WAVE - 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        // representatives are held in LDS while they fit (written to the log
        // at the end of the block); others are reserved in the log now
        const uint32_t total = S.tmp[32];
        const uint32_t held = S.tmp[38];
        unsigned long long base = 0;
        uint32_t hold = 0;
        if (total && reduced && held + total <= A.rep_hold) {
            base = held;
            hold = 1;
            S.tmp[38] = held + total;
        } else if (total) {
            base = atomicAdd(A.log_count, (unsigned long long)total);
            if (base + total > A.log_cap) atomicOr(A.flags, FLAG_LOG_OVERFLOW);
        }
        S.tmp[33] = (uint32_t)base;
        S.tmp[34] = (uint32_t)(base >> 32);
        S.tmp[39] = hold;
    }
    __syncthreads();
    const bool hold = S.tmp[39] != 0;
    unsigned long long pos = ((unsigned long long)S.tmp[33] | ((unsigned long long)S.tmp[34] << 32)) + woff + incl - mine;
    const uint64_t ep = reduced ? (uint64_t)k.ep_rep : (uint64_t)epoch;
    for (uint32_t i = threadIdx.x; i < C; i += blockDim.x) {
        const unsigned long long v = S.gst[i];
        if (v == GST_EMPTY) continue;
        S.gst[i] = GST_EMPTY;
        const uint32_t t1 = (uint32_t)v & GT_NONE, t2 = (uint32_t)(v >> 11) & GT_NONE, w = (uint32_t)(v >> 22) & GT_NONE;
        const uint32_t addr = gst_addr(v);
        const uint64_t base = rec_pack(k, B.unit, 1u, addr, B.block, 0u, 0u, 0u) | (ep << k.s_ep);
        uint64_t r[3];
        uint32_t n = 0;
        r[n++] = base | ((uint64_t)t1 << k.s_tid) | (w == t1 ? 1ull : 0ull);
        if (reduced) {
            if (w != GT_NONE && t2 != GT_NONE) push_local_race(A, B, 1u, epoch, addr, w, t1 == w ? t2 : t1);
            if (w != GT_NONE && w != t1) r[n++] = base | ((uint64_t)w << k.s_tid) | 1ull;
        } else {
            if (t2 != GT_NONE) r[n++] = base | ((uint64_t)t2 << k.s_tid) | (w == t2 ? 1ull : 0ull);
            if (w != GT_NONE && w != t1 && w != t2) r[n++] = base | ((uint64_t)w << k.s_tid) | 1ull;
        }
        for (uint32_t j = 0; j < n; j++, pos++) {
            if (hold) S.repbuf[pos] = r[j];
            else if (pos < A.log_cap) A.log[pos] = r[j];
        }
    }
}

// Reduce the epoch's staged global records, sorted by (space, address) in
// `src` (n records), to each location's race and representatives (compacted
// into `dst`), reserved in the log with one atomic per block.
__device__ __forceinline__ void local_reduce_sorted(const InterpArgs &A, const BlockCtx &B, const Shared &S,
                                                    uint32_t epoch, const uint64_t *src, uint64_t *dst, uint32_t n) {
    const KeyPlan &k = A.kp;
    // Segments (one location) of the sorted epoch: the head thread reduces
    // up to LOCAL_SEG_LIMIT records; longer segments (a location touched
    // by many threads) are listed and reduced by whole waves.
    // Representatives are compacted into dst (a segment yields no more
    // representatives than records, so n entries suffice) and reserved in
    // the log with one atomic per block: a single global counter serves
    // every block of the launch.
    if (threadIdx.x == 0) {
        S.tmp[32] = 0;      // representatives in dst
        S.tmp[35] = 0;      // long segments listed in wc
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint64_t r = src[i];
        const uint32_t lk = local_key(r, k);
        if (i != 0 && local_key(src[i - 1], k) == lk) continue;
        SegState st{NONE_U32, NONE_U32, NONE_U32};
        bool is_long = false;
        for (uint32_t j = i; j < n; j++) {
            const uint64_t x = src[j];
            if (local_key(x, k) != lk) break;
            if (j - i == LOCAL_SEG_LIMIT) {
                is_long = true;
                break;
            }
            seg_add(st, rec_field(x, k.s_tid, k.tb), (x & 1ull) != 0);
        }
        if (is_long) S.wc[atomicAdd(&S.tmp[35], 1u)] = i;
        else local_segment_done(A, B, S, r, epoch, st, dst);
    }
    __syncthreads();
    const uint32_t nlong = S.tmp[35];
    for (uint32_t e = B.wave; e < nlong; e += B.nwaves) {
        const uint32_t i = S.wc[e];
        const uint64_t r = src[i];
        const uint32_t lk = local_key(r, k);
        SegState st{NONE_U32, NONE_U32, NONE_U32};
        for (uint32_t base = i;; base += WAVE) {
            const uint32_t j = base + lane_id();
            const uint64_t x = j < n ? src[j] : 0ull;
            const bool in = j < n && local_key(x, k) == lk;
            if (in) seg_add(st, rec_field(x, k.s_tid, k.tb), (x & 1ull) != 0);
            if (__ballot(!in)) break;           // sorted: the segment ended in this chunk
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const SegState y{(uint32_t)__shfl_xor((int)st.minw, o), (uint32_t)__shfl_xor((int)st.t1, o),
                             (uint32_t)__shfl_xor((int)st.t2, o)};
            seg_merge(st, y);
        }
        if (lane_id() == 0) local_segment_done(A, B, S, r, epoch, st, dst);
    }
    __syncthreads();
    const uint32_t nrep = S.tmp[32];
    if (nrep) {
        if (threadIdx.x == 0) {
            const unsigned long long base = atomicAdd(A.log_count, (unsigned long long)nrep);
            S.tmp[33] = (uint32_t)base;
            S.tmp[34] = (uint32_t)(base >> 32);
            if (base + nrep > A.log_cap) atomicOr(A.flags, FLAG_LOG_OVERFLOW);
        }
        __syncthreads();
        const unsigned long long base = (unsigned long long)S.tmp[33] | ((unsigned long long)S.tmp[34] << 32);
        for (uint32_t j = threadIdx.x; j < nrep; j += blockDim.x)
            if (base + j < A.log_cap) A.log[base + j] = dst[j];
    }
}

// The replay's epoch-local check: exact tuples of the shared words, the
// global shadow table or the staged global records of the epoch.
__device__ __forceinline__ void epoch_local_check(const InterpArgs &A, const BlockCtx &B, const Shared &S,
                                                  LogState &L, uint32_t epoch) {
    const KeyPlan &k = A.kp;
    if (lane_id() == 0) {       // per-wave staged count and spill flag (tmp[w], tmp[16 + w])
        S.tmp[B.wave] = L.cur;
        S.tmp[16 + B.wave] = L.spilled ? 1u : 0u;
    }
    if (threadIdx.x == 0) S.tmp[32] = 0;
    __syncthreads();
    const uint32_t g_occupied = S.tmp[36], g_overflow = S.tmp[37];
    uint32_t n = 0, off = 0, spilled = 0;
    for (uint32_t w = 0; w < B.nwaves; w++) {
        const uint32_t c = S.tmp[w];
        if (w < B.wave) off += c;
        n += c;
        spilled |= S.tmp[16 + w];
    }
    // shared memory: reduce and clear the shadow tuples of this epoch
    for (uint32_t a = threadIdx.x; a < B.sh_words; a += blockDim.x) {
        const unsigned long long sv = S.shadow[a];
        if (sv == SHADOW_EMPTY) continue;
        const uint32_t t1 = (uint32_t)(sv & 0xFFFF), t2 = (uint32_t)((sv >> 16) & 0xFFFF),
                       w = (uint32_t)((sv >> 32) & 0xFFFF);
        if (w != SH_NONE && t2 != SH_NONE) push_local_race(A, B, 0u, epoch, a, w, t1 == w ? t2 : t1);
        S.shadow[a] = SHADOW_EMPTY;
    }
    // global memory: the table, or the staged records of the epoch
    if (A.gst_bits) {
        // Without an overflow nothing was staged and the table holds every
        // location: reduce it here.  After one, the staged records and the
        // table's tuples go to the global check unreduced.
        const bool unreduced = spilled || g_overflow;
        if (unreduced) flush_stage(A, S.stage, L.cur);
        if (g_occupied) gst_drain(A, B, S, epoch, !unreduced);
    } else if (spilled) {       // the epoch's records go to the global check unreduced
        flush_stage(A, S.stage, L.cur);
    } else if (n) {
        for (uint32_t i = lane_id(); i < L.cur; i += WAVE) S.alt[off + i] = S.stage[i];
        __syncthreads();
        uint64_t *src = S.alt, *dst = S.stage_all;
        for (uint32_t shift = 0; shift < 1 + k.ab; shift += 8) {
            local_sort_pass(S, B, k, src, dst, n, shift);
            uint64_t *t = src; src = dst; dst = t;
        }
        local_reduce_sorted(A, B, S, epoch, src, dst, n);
    }
    __syncthreads();            // the staging areas and the table are free again
    if (threadIdx.x == 0) {
        S.tmp[36] = 0;          // table occupancy
        S.tmp[37] = 0;          // table overflow
    }
    L.cur = 0;
    L.spilled = false;
}

// Result of the episode logic, uniform over the workgroup.
enum : int { EP_RELEASED = 0, EP_DONE = 1 };

// All waves are quiescent (no running lane).  Count arrivals and decide.
template <bool LOCAL>
__device__ __forceinline__ int barrier_episode(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t,
                               LogState &L, uint32_t &epoch);

// After a release: each lane released from a barrier with a predicate writes
// the result into the destination register of its barrier instruction (one
// group per barrier site, so the register index stays wave-uniform).
__device__ __forceinline__ void barrier_results(const BlockCtx &B, Lane &t) {
    uint64_t m = __ballot(t.bpred != 0);
    while (m) {
        const bool mine = (m >> lane_id()) & 1ull;
        const int pc = uni(wave_min(mine ? t.bar_pc : INT_MAX));
        const uint32_t d = uniu((uint32_t)(B.prog[(uint32_t)pc] >> 8) & 0xFFu);
        const bool here = mine && t.bar_pc == pc;
        const int32_t old = t.r[d];
        t.r[d] = here ? t.bres : old;
        m &= ~__ballot(here);
    }
    t.bpred = 0;
}

// The replay's episode (the free run's is free_episode).
template <bool LOCAL>
__device__ __forceinline__ int barrier_episode(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t,
                               LogState &L, uint32_t &epoch) {
    __syncthreads();
    if (LOCAL) epoch_local_check(A, B, S, L, epoch);
    bool is_thread = t.st != ST_DEAD;
    uint64_t wm = __ballot(t.st == ST_WAIT);
    uint64_t em = __ballot(t.st == ST_EXIT);
    int bmin = wave_min(t.st == ST_WAIT ? t.bar_pc : INT_MAX);
    int bmax = wave_max(t.st == ST_WAIT ? t.bar_pc : -1);
    const uint64_t pm = __ballot(t.st == ST_WAIT && (t.bpred & 1));
    (void)is_thread;
    if (lane_id() == 0) {
        S.slots2[4 * B.wave + 3] = (uint32_t)__popcll(pm);     // predicates that hold
        uint32_t *s = S.slots + 10 * B.wave;
        s[0] = (uint32_t)__popcll(wm);
        s[1] = (uint32_t)__popcll(em);
        s[2] = (uint32_t)bmin;
        s[3] = (uint32_t)bmax;
        s[4] = wm ? B.wave * WAVE + (uint32_t)__ffsll((long long)wm) - 1 : 0xFFFFFFFFu;
        s[5] = em ? B.wave * WAVE + (uint32_t)__ffsll((long long)em) - 1 : 0xFFFFFFFFu;
    }
    __syncthreads();
    uint32_t nw = 0, ne = 0, minw = 0xFFFFFFFFu, mine = 0xFFFFFFFFu;
    int BMIN = INT_MAX, BMAX = -1;
    for (uint32_t w = 0; w < B.nwaves; w++) {
        const uint32_t *s = S.slots + 10 * w;
        nw += s[0];
        ne += s[1];
        BMIN = min(BMIN, (int)s[2]);
        BMAX = max(BMAX, (int)s[3]);
        minw = min(minw, s[4]);
        mine = min(mine, s[5]);
    }
    if (nw == 0) return EP_DONE;                       // every thread exited
    if (ne > 0) {                                      // waiting threads can never be released
        emit_fault(threadIdx.x == 0, A, B, F_DEADLOCK, epoch, nw, minw, mine, 0);
        return EP_DONE;
    }
    if (BMIN != BMAX) {
        // sites differ: find the next larger site and the smallest tid at each
        int cw = wave_min(t.st == ST_WAIT && t.bar_pc > BMIN ? t.bar_pc : INT_MAX);
        uint64_t lo_m = __ballot(t.st == ST_WAIT && t.bar_pc == BMIN);
        uint64_t c_m = __ballot(t.st == ST_WAIT && t.bar_pc == cw && cw != INT_MAX);
        if (lane_id() == 0) {
            uint32_t *s = S.slots2 + 4 * B.wave;
            s[0] = (uint32_t)cw;
            s[1] = lo_m ? B.wave * WAVE + (uint32_t)__ffsll((long long)lo_m) - 1 : 0xFFFFFFFFu;
            s[2] = c_m ? B.wave * WAVE + (uint32_t)__ffsll((long long)c_m) - 1 : 0xFFFFFFFFu;
        }
        __syncthreads();
        int C = INT_MAX;
        uint32_t tlo = 0xFFFFFFFFu, tc = 0xFFFFFFFFu;
        for (uint32_t w = 0; w < B.nwaves; w++) C = min(C, (int)S.slots2[4 * w]);
        for (uint32_t w = 0; w < B.nwaves; w++) {
            tlo = min(tlo, S.slots2[4 * w + 1]);
            if ((int)S.slots2[4 * w] == C) tc = min(tc, S.slots2[4 * w + 2]);
        }
        emit_fault(threadIdx.x == 0, A, B, F_DIVERGENCE, epoch, (uint32_t)BMIN, tlo, (uint32_t)C, tc);
    }
    epoch++;
    if (threadIdx.x == 0 && epoch > A.kp.max_epoch) atomicOr(A.flags, FLAG_EPOCH_OVERFLOW);
    // barriers with a predicate: every thread of the block waits here, so
    // AND holds when the count reaches the thread count
    uint32_t npred = 0;
    for (uint32_t w = 0; w < B.nwaves; w++) npred += S.slots2[4 * w + 3];
    if (t.st == ST_WAIT) {
        t.st = ST_RUN;
        t.pc = t.bar_pc + 1;
        const int kind = (t.bpred >> 1) - 1;
        if (kind >= 0) t.bres = kind == 0 ? (int32_t)npred : kind == 1 ? (npred == B.nt ? 1 : 0) : (npred ? 1 : 0);
    }
    B.kep = B.kbase | ((uint64_t)epoch << A.kp.s_ep);
    return EP_RELEASED;
}

// ---- free-run barrier episode ---------------------------------------------------
// The same decisions as barrier_episode, with two workgroup barriers: every
// wave publishes its arrivals with LDS atomics into the episode's summary
// words before the first barrier (three sets used in turn, so the set the
// next episode fills was last read two episodes ago and is reset now); the
// epoch-local check (shared-word verdicts, the global shadow table) runs
// between the barriers, and the second makes its resets visible before the
// next epoch's accesses.  The global table's occupancy words alternate by
// epoch parity for the same reason.
enum : uint32_t { EPS_WAIT = 0, EPS_EXIT, EPS_BMIN, EPS_BMAX, EPS_PRED, EPS_TWAIT, EPS_TEXIT, EPS_SPILL, EPS_WORDS };

// The epoch-local check of a free-run episode, after its first barrier.
__device__ __forceinline__ void free_local_check(const InterpArgs &A, BlockCtx &B, const Shared &S, LogState &L,
                                                 uint32_t epoch, bool spilled) {
    const KeyPlan &k = A.kp;
    // shared words: verdicts; one marker per wave that found a racy word
    // flags the block for the replay (the tuple is not canonical and is
    // never reported; the count sizes the replay's race list)
    uint32_t nracy = 0, ra = 0, rmin = 0, rmax = 0;
    for (uint32_t a = threadIdx.x; a < B.sh_words; a += blockDim.x) {
        const uint32_t mn = S.vmin[a];
        if (mn == NONE_U32) continue;
        const uint32_t mx = S.vmax[a];
        if (S.vw[a] != 0u && mn != mx) {
            nracy++;
            ra = a;
            rmin = mn;
            rmax = mx;
        }
        S.vmin[a] = NONE_U32;
        S.vmax[a] = 0u;
        S.vw[a] = 0u;
    }
    const uint64_t rm = __ballot(nracy != 0);
    if (rm) {
        uint32_t tot = nracy;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tot += (uint32_t)__shfl_xor((int)tot, o);
        if (lane_id() == (uint32_t)__ffsll((long long)rm) - 1u) {
            push_local_race(A, B, 0u, epoch, ra, rmin, rmax);
            if (A.racy_words) atomicAdd(A.racy_words, tot);
        }
    }
    if (A.gst_bits) {
        const uint32_t g_occupied = B.gocc[0], g_overflow = B.gocc[1];
        const bool unreduced = spilled || g_overflow;
        if (unreduced) flush_stage(A, S.stage, L.cur);
        if (g_occupied) gst_drain(A, B, S, epoch, !unreduced);      // tmp[32] was zeroed before the barrier
    } else if (spilled) {
        flush_stage(A, S.stage, L.cur);
    } else {
        // the sorting variant: the staged records of every wave (counts in tmp[w])
        uint32_t n = 0, off = 0;
        for (uint32_t w = 0; w < B.nwaves; w++) {
            const uint32_t c = S.tmp[w];
            if (w < B.wave) off += c;
            n += c;
        }
        if (n) {
            for (uint32_t i = lane_id(); i < L.cur; i += WAVE) S.alt[off + i] = S.stage[i];
            __syncthreads();
            uint64_t *src = S.alt, *dst = S.stage_all;
            for (uint32_t shift = 0; shift < 1 + k.ab; shift += 8) {
                local_sort_pass(S, B, k, src, dst, n, shift);
                uint64_t *t = src; src = dst; dst = t;
            }
            local_reduce_sorted(A, B, S, epoch, src, dst, n);
        }
    }
    L.cur = 0;
    L.spilled = false;
}

template <bool LOCAL>
__device__ __forceinline__ int free_episode(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t, LogState &L,
                                            uint32_t &epoch) {
    uint32_t *E = S.eps + EPS_WORDS * (epoch % 3u);
    const bool waiting = t.st == ST_WAIT;
    const uint64_t wm = __ballot(waiting), em = __ballot(t.st == ST_EXIT);
    const uint64_t pm = __ballot(waiting && (t.bpred & 1));
    int bmin = INT_MAX, bmax = -1;
    if (wm) {
        const int p0 = __builtin_amdgcn_readlane(t.bar_pc, (int)((uint32_t)__ffsll((long long)wm) - 1u));
        if (__ballot(waiting && t.bar_pc != p0) == 0) {
            bmin = bmax = p0;
        } else {
            bmin = wave_min(waiting ? t.bar_pc : INT_MAX);
            bmax = wave_max(waiting ? t.bar_pc : -1);
        }
    }
    if (threadIdx.x == 0) {     // the next episode's set, and the table's reservation counter
        if (LOCAL) S.tmp[32] = 0u;
        uint32_t *F = S.eps + EPS_WORDS * ((epoch + 1u) % 3u);
        F[EPS_WAIT] = 0u;
        F[EPS_EXIT] = 0u;
        F[EPS_BMIN] = (uint32_t)INT_MAX;
        F[EPS_BMAX] = (uint32_t)-1;
        F[EPS_PRED] = 0u;
        F[EPS_TWAIT] = NONE_U32;
        F[EPS_TEXIT] = NONE_U32;
        F[EPS_SPILL] = 0u;
        if (LOCAL && A.gst_bits) {      // the next epoch's table words (last read two episodes ago)
            uint32_t *g = (epoch & 1u) ? &S.tmp[36] : &S.tmp[40];
            g[0] = 0u;
            g[1] = 0u;
        }
    }
    if (lane_id() == 0) {
        if (wm) {
            atomicAdd(&E[EPS_WAIT], (uint32_t)__popcll(wm));
            atomicMin((int *)&E[EPS_BMIN], bmin);
            atomicMax((int *)&E[EPS_BMAX], bmax);
            atomicMin(&E[EPS_TWAIT], B.wave * WAVE + (uint32_t)__ffsll((long long)wm) - 1u);
        }
        if (em) {
            atomicAdd(&E[EPS_EXIT], (uint32_t)__popcll(em));
            atomicMin(&E[EPS_TEXIT], B.wave * WAVE + (uint32_t)__ffsll((long long)em) - 1u);
        }
        if (pm) atomicAdd(&E[EPS_PRED], (uint32_t)__popcll(pm));
        if (LOCAL) {
            if (L.spilled) atomicOr(&E[EPS_SPILL], 1u);
            S.tmp[B.wave] = L.cur;      // staged records (the sorting variant)
        }
    }
    __syncthreads();
    const uint32_t nw = E[EPS_WAIT], ne = E[EPS_EXIT], npred = E[EPS_PRED];
    const int BMIN = (int)E[EPS_BMIN], BMAX = (int)E[EPS_BMAX];
    if (LOCAL) free_local_check(A, B, S, L, epoch, E[EPS_SPILL] != 0u);
    if (nw == 0) return EP_DONE;                       // every thread exited
    if (ne > 0) {                                      // waiting threads can never be released
        emit_fault(threadIdx.x == 0, A, B, F_DEADLOCK, epoch, nw, E[EPS_TWAIT], E[EPS_TEXIT], 0);
        return EP_DONE;
    }
    if (BMIN != BMAX) {
        // sites differ: find the next larger site and the smallest tid at each
        int cw = wave_min(waiting && t.bar_pc > BMIN ? t.bar_pc : INT_MAX);
        uint64_t lo_m = __ballot(waiting && t.bar_pc == BMIN);
        uint64_t c_m = __ballot(waiting && t.bar_pc == cw && cw != INT_MAX);
        if (lane_id() == 0) {
            uint32_t *q = S.slots2 + 4 * B.wave;
            q[0] = (uint32_t)cw;
            q[1] = lo_m ? B.wave * WAVE + (uint32_t)__ffsll((long long)lo_m) - 1 : 0xFFFFFFFFu;
            q[2] = c_m ? B.wave * WAVE + (uint32_t)__ffsll((long long)c_m) - 1 : 0xFFFFFFFFu;
        }
        __syncthreads();
        int C = INT_MAX;
        uint32_t tlo = 0xFFFFFFFFu, tc = 0xFFFFFFFFu;
        for (uint32_t w = 0; w < B.nwaves; w++) C = min(C, (int)S.slots2[4 * w]);
        for (uint32_t w = 0; w < B.nwaves; w++) {
            tlo = min(tlo, S.slots2[4 * w + 1]);
            if ((int)S.slots2[4 * w] == C) tc = min(tc, S.slots2[4 * w + 2]);
        }
        emit_fault(threadIdx.x == 0, A, B, F_DIVERGENCE, epoch, (uint32_t)BMIN, tlo, (uint32_t)C, tc);
    }
    epoch++;
    if (threadIdx.x == 0 && epoch > A.kp.max_epoch) atomicOr(A.flags, FLAG_EPOCH_OVERFLOW);
    if (waiting) {
        t.st = ST_RUN;
        t.pc = t.bar_pc + 1;
        const int kind = (t.bpred >> 1) - 1;
        if (kind >= 0) t.bres = kind == 0 ? (int32_t)npred : kind == 1 ? (npred == B.nt ? 1 : 0) : (npred ? 1 : 0);
    }
    B.kep = B.kbase | ((uint64_t)epoch << A.kp.s_ep);
    if (LOCAL && A.gst_bits) B.gocc = (epoch & 1u) ? &S.tmp[40] : &S.tmp[36];
    __syncthreads();            // the check's resets before the next epoch's accesses; divergence slots free
    return EP_RELEASED;
}

// After a free-run release: whether the wave's running lanes share one pc,
// and the smallest pc (the dispatch point).
__device__ __forceinline__ void free_reconverge(const Lane &t, bool &conv, int &upc) {
    const bool run = t.st == ST_RUN;
    const uint64_t rm = __ballot(run);
    if (rm == 0) {
        conv = true;
        upc = 0;
        return;
    }
    const int p0 = __builtin_amdgcn_readlane(t.pc, (int)((uint32_t)__ffsll((long long)rm) - 1u));
    if (__ballot(run && t.pc != p0) == 0) {
        conv = true;
        upc = uni(p0);
    } else {
        conv = false;
        upc = uni(wave_min(run ? t.pc : INT_MAX));
    }
}

__device__ __forceinline__ int32_t special(const BlockCtx &B, uint32_t k) {
    const DevUnit *u = B.u;
    const uint32_t bx = u->bdim[0], by = u->bdim[1], gx = u->gdim[0], gy = u->gdim[1];
    switch (k) {
    case 0: return (int32_t)(B.tid % bx);
    case 1: return (int32_t)((B.tid / bx) % by);
    case 2: return (int32_t)(B.tid / (bx * by));
    case 3: return (int32_t)(B.block % gx);
    case 4: return (int32_t)((B.block / gx) % gy);
    case 5: return (int32_t)(B.block / (gx * gy));
    case 6: return (int32_t)u->bdim[0];
    case 7: return (int32_t)u->bdim[1];
    case 8: return (int32_t)u->bdim[2];
    case 9: return (int32_t)u->gdim[0];
    case 10: return (int32_t)u->gdim[1];
    case 11: return (int32_t)u->gdim[2];
    case 12: return (int32_t)B.tid;
    case 13: return (int32_t)B.block;
    case 14: return (int32_t)B.nt;
    case 15: return 32;
    default: return u->params[k - 16];
    }
}

// Deferred store of a lockstep step.
struct Pending {
    bool on;
    bool shared;
    int32_t addr;
    int32_t val;
};


// Execute the instruction at pc `cur` (wave-uniform) for the lanes in `active`.
// ctl (wave-uniform, from the opcode alone): 0 falls through, 1 JMP,
// 2 conditional branch (cond per lane), 3 BAR/EXIT; target is the branch target.
template <bool LOCKSTEP, bool LOCAL>
__device__ __forceinline__ void exec_one(const InterpArgs &A, const BlockCtx &B, const Shared &S, Lane &t,
                                         LogState &L, Pending &P, uint32_t epoch, int cur, uint64_t w, bool active,
                                         int &ctl, int &target, bool &cond) {
    const uint32_t op = uniu((uint32_t)w & 0xFFu);
    const uint32_t d = uniu((uint32_t)(w >> 8) & 0xFFu);
    const uint32_t ra = uniu((uint32_t)(w >> 16) & 0xFFu);
    const uint32_t rb = uniu((uint32_t)(w >> 24) & 0xFFu);
    const int32_t imm = uni((int32_t)(uint32_t)(w >> 32));
    const uint32_t base = op & ~uint32_t(OP_IMM);
    const uint32_t cls = op >> 4;
    ctl = 0;
    target = cur + 1;
    cond = false;
    if (cls == 6) {                                   // control
        if (op == OP_JMP) {
            ctl = 1;
            target = imm;
        } else if (op == OP_BZ || op == OP_BNZ) {
            ctl = 2;
            target = imm;
            const int32_t x = t.r[ra];
            cond = (op == OP_BZ) ? (x == 0) : (x != 0);
        } else {
            ctl = 3;
            if (op == OP_BAR || op == OP_BARP) {
                if (active) {
                    t.st = ST_WAIT;
                    t.bar_pc = cur;
                    t.bpred = op == OP_BARP ? (int)(((uint32_t)imm + 1u) << 1) | (t.r[ra] != 0 ? 1 : 0) : 0;
                }
            } else if (active) {
                t.st = ST_EXIT;
            }
        }
        return;
    }
    int32_t v = 0;
    bool writes = true;
    if (base >= OP_ADD && base <= OP_SLTU) {         // int32 ALU
        bool arith = false;
        const int32_t x = t.r[ra];
        int32_t y;
        if (op & OP_IMM) y = imm;
        else y = t.r[rb];
        v = alu(base, x, y, arith);
        if (base == OP_DIV || base == OP_REM)
            emit_fault(active && arith, A, B, F_ARITH, epoch, 0, B.tid, (uint32_t)cur, 0);
    } else if (cls == 5) {                            // memory
        const KeyPlan &k = A.kp;
        const int32_t addr = (int32_t)((uint32_t)t.r[ra] + (uint32_t)imm);
        const bool is_sh = (op & 2u) == 0;            // LDS 0x50, STS 0x51, LDG 0x52, STG 0x53
        const bool is_st = (op & 1u) != 0;
        const bool inb = active && (uint32_t)addr < (is_sh ? B.sh_words : B.n_words);
        if (!is_st) {
            if (inb) v = is_sh ? S.sh[addr] : B.mem[addr];
            if (is_sh && A.uninit)
                emit_fault(inb && !shared_stored(S, (uint32_t)addr), A, B, F_UNINIT, epoch, 0u, B.tid, (uint32_t)addr,
                           (uint32_t)cur);
        } else {
            writes = false;
            const int32_t val = t.r[rb];
            if (LOCKSTEP) {
                if (inb) { P.on = true; P.shared = is_sh; P.addr = addr; P.val = val; }
            } else if (inb) {
                if (is_sh) S.sh[addr] = val;
                else B.mem[addr] = val;
                if (is_sh && A.uninit) mark_stored(S, (uint32_t)addr);
            }
        }
        const uint32_t space = is_sh ? 0u : 1u;
        const uint64_t key = B.kep | ((uint64_t)space << k.s_sp) | (uint64_t)(is_st ? 1u : 0u) |
                             ((uint64_t)(uint32_t)addr << k.s_addr);
        if (LOCKSTEP && A.wlog) wlog_append(A, B, inb, space, (uint32_t)addr, is_st);
        if (!is_sh) L.gtotal += (uint32_t)__popcll(__ballot(inb));
        if (LOCAL && is_sh) {       // shared accesses update the shadow tuple instead of the log
            if (inb && LOCKSTEP) shadow_update(S.shadow, (uint32_t)addr, B.tid, is_st);
            if (inb && !LOCKSTEP) shadow_mark(S, (uint32_t)addr, B.tid, is_st);
            L.total += (uint32_t)__popcll(__ballot(inb));
        } else if (LOCAL) {
            global_access(A, B, S, L, inb, (uint32_t)addr, is_st, key);
        } else {
            log_rec(A, S.stage, L, inb, key);
        }
        emit_fault(active && !inb, A, B, F_OOB, epoch, space * 2u + (is_st ? 1u : 0u), B.tid, (uint32_t)addr, 0);
    } else if (op == OP_MOV) {
        v = t.r[ra];
    } else if (op == OP_MOVI) {
        v = imm;
    } else {                                          // OP_SREG
        v = special(B, (uint32_t)imm);
    }
    if (writes) {
        const int32_t old = t.r[d];
        t.r[d] = active ? v : old;
    }
}

// `exact`: the shared words keep full tuples (replay), else verdicts (free run).
__device__ __forceinline__ void setup_block(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t, uint32_t unit,
                            uint32_t block, bool exact) {
    const DevUnit *u = &A.units[unit];
    B.u = u;
    B.prog = (const_word_t *)u->prog;
    B.mem = (global_i32_t *)u->mem;
    B.unit = unit;
    B.block = block;
    B.nt = u->nt;
    B.n_instr = u->n_instr;
    B.n_words = u->n_words;
    B.sh_words = u->sh_words;
    B.tid = threadIdx.x;
    B.kbase = rec_pack(A.kp, unit, 0u, 0u, block, 0u, B.tid, 0u);
    B.gocc = A.local ? &S.tmp[36] : nullptr;
    B.kep = B.kbase;
    for (uint32_t i = threadIdx.x; i < B.sh_words; i += blockDim.x) S.sh[i] = 0;
    if (A.uninit)
        for (uint32_t i = threadIdx.x; i < (B.sh_words + 31) / 32; i += blockDim.x) S.sinit[i] = 0u;
    if (A.local && exact)
        for (uint32_t i = threadIdx.x; i < B.sh_words; i += blockDim.x) S.shadow[i] = SHADOW_EMPTY;
    if (A.local && !exact)
        for (uint32_t i = threadIdx.x; i < B.sh_words; i += blockDim.x) {
            S.vmin[i] = NONE_U32;
            S.vmax[i] = 0u;
            S.vw[i] = 0u;
        }
    if (A.gst_bits) {
        for (uint32_t i = threadIdx.x; i < (1u << A.gst_bits); i += blockDim.x) S.gst[i] = GST_EMPTY;
        if (threadIdx.x == 0) {
            S.tmp[36] = 0;
            S.tmp[37] = 0;
            S.tmp[38] = 0;          // representatives held in LDS
            S.tmp[40] = 0;          // occupancy and overflow of odd epochs (free run)
            S.tmp[41] = 0;
        }
    }
    if (threadIdx.x == 0) {     // the first free-run episode's summary words
        S.eps[EPS_WAIT] = 0u;
        S.eps[EPS_EXIT] = 0u;
        S.eps[EPS_BMIN] = (uint32_t)INT_MAX;
        S.eps[EPS_BMAX] = (uint32_t)-1;
        S.eps[EPS_PRED] = 0u;
        S.eps[EPS_TWAIT] = NONE_U32;
        S.eps[EPS_TEXIT] = NONE_U32;
        S.eps[EPS_SPILL] = 0u;
    }
    t.pc = 0;
    t.st = (B.tid < B.nt) ? ST_RUN : ST_DEAD;
    t.fuel = u->fuel;
    t.bar_pc = 0;
    t.bpred = 0;
    t.bres = 0;
    t.r = (regfile_t)(0);
    __syncthreads();
}

// End of a block: flush the staged records, publish the block's record count,
// its last epoch (the largest it reached) and, in the free run, the
// thread-instructions it executed (every executed instruction spent one unit of
// fuel).  One global atomic per block and counter: the counters are shared by
// every block of the launch.
__device__ __forceinline__ void finish_block(const InterpArgs &A, const BlockCtx &B, const Shared &S, LogState &L,
                                             const Lane &t, uint32_t epoch) {
    flush_stage(A, S.stage, L.cur);
    L.cur = 0;
    unsigned long long spent = 0;
    if (A.blk_instr) {
        spent = (t.st != ST_DEAD) ? (unsigned long long)(B.u->fuel - t.fuel) : 0ull;
        for (int o = 32; o > 0; o >>= 1) spent += __shfl_xor(spent, o);
    }
    __syncthreads();            // the episode slots are free; held representatives are complete
    if (A.local && A.gst_bits && A.blk_log) {          // to the block's own region, appended after the kernel
        const uint32_t held = S.tmp[38];
        const size_t gb = (size_t)B.u->block_base + B.block;
        uint64_t *dst = A.blk_log + gb * REP_HOLD;
        for (uint32_t j = threadIdx.x; j < held; j += blockDim.x) dst[j] = S.repbuf[j];
        if (threadIdx.x == 0) A.blk_held[gb] = held;
    } else if (A.local && A.gst_bits) {
        const uint32_t held = S.tmp[38];
        if (held) {
            if (threadIdx.x == 0) {
                const unsigned long long base = atomicAdd(A.log_count, (unsigned long long)held);
                if (base + held > A.log_cap) atomicOr(A.flags, FLAG_LOG_OVERFLOW);
                S.tmp[33] = (uint32_t)base;
                S.tmp[34] = (uint32_t)(base >> 32);
            }
            __syncthreads();
            const unsigned long long base = (unsigned long long)S.tmp[33] | ((unsigned long long)S.tmp[34] << 32);
            for (uint32_t j = threadIdx.x; j < held; j += blockDim.x)
                if (base + j < A.log_cap) A.log[base + j] = S.repbuf[j];
            __syncthreads();
        }
    }
    if (lane_id() == 0) {
        S.slots[10 * B.wave] = L.total;
        S.slots[10 * B.wave + 1] = (uint32_t)spent;
        S.slots[10 * B.wave + 2] = (uint32_t)(spent >> 32);
        S.slots[10 * B.wave + 3] = L.gtotal;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t recs = 0, grecs = 0;
        unsigned long long instr = 0;
        for (uint32_t w = 0; w < B.nwaves; w++) {
            recs += S.slots[10 * w];
            instr += (unsigned long long)S.slots[10 * w + 1] | ((unsigned long long)S.slots[10 * w + 2] << 32);
            grecs += S.slots[10 * w + 3];
        }
        if (recs) atomicAdd(&A.blk_recs[B.u->block_base + B.block], recs);
        if (A.blk_instr) A.blk_instr[B.u->block_base + B.block] = (uint32_t)instr;
        if (A.blk_grecs) A.blk_grecs[B.u->block_base + B.block] = grecs;
        if (epoch > __hip_atomic_load(A.max_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(A.max_epoch, epoch);
    }
    L.total = 0;
    L.gtotal = 0;
    __syncthreads();
}

// ---- free-run block execution ------------------------------------------------
template <bool LOCAL>
__device__ __forceinline__ uint32_t run_block_free(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t,
                                                   LogState &L) {
    uint32_t epoch = 0;
    Pending P{false, false, 0, 0};
    bool conv = true;    // every running lane of the wave is at upc
    int upc = 0;
    uint32_t guard = B.u->fuel;     // lower bound of every live lane's fuel
    for (;;) {
        for (;;) {
            // The scheduling state is the same in every lane; reading it
            // through lane 0 lets the compiler branch on it with scalar code.
            conv = uni(conv ? 1 : 0) != 0;
            upc = uni(upc);
            guard = uniu(guard);
            uint64_t runm = __ballot(t.st == ST_RUN);
            if (runm == 0) break;
            int cur;
            bool active;
            if (conv) {
                cur = upc;
                active = (t.st == ST_RUN);
            } else {
                cur = uni(wave_min(t.st == ST_RUN ? t.pc : INT_MAX));
                active = (t.st == ST_RUN) && t.pc == cur;
                if (__ballot(active) == runm) { conv = true; upc = cur; }
            }
            if ((uint32_t)cur >= B.n_instr) {              // fell off the end
                if (active) t.st = ST_EXIT;
                continue;
            }
            // Every lane that has not exited holds at least `guard` fuel, so the
            // per-lane check is needed only when the guard runs out.
            if (guard == 0) {
                const bool nofuel = active && t.fuel == 0;
                emit_fault(nofuel, A, B, F_FUEL, epoch, 0, B.tid, 0, 0);
                if (nofuel) { t.st = ST_EXIT; active = false; }
                guard = wave_min_u((t.st == ST_RUN || t.st == ST_WAIT) ? t.fuel : 0xFFFFFFFFu);
                if (__ballot(active) == 0) continue;
            }
            if (active) t.fuel--;
            if (guard) guard--;
            int ctl, target;
            bool cond;
            exec_one<false, LOCAL>(A, B, S, t, L, P, epoch, cur, B.prog[(uint32_t)uni(cur)], active, ctl, target,
                                   cond);
            if (ctl == 3) continue;                        // BAR/EXIT: lanes left the running set
            if (ctl == 2) {
                uint64_t actm = __ballot(active);
                uint64_t taken = __ballot(active && cond);
                if (conv) {
                    if (taken == 0) upc = cur + 1;
                    else if (taken == actm) upc = target;
                    else {
                        conv = false;
                        if (t.st == ST_RUN) t.pc = cond ? target : cur + 1;
                    }
                } else if (active) {
                    t.pc = cond ? target : cur + 1;
                }
            } else {
                if (conv) upc = target;
                else if (active) t.pc = target;
            }
        }
        // wave quiescent
        if (free_episode<LOCAL>(A, B, S, t, L, epoch) == EP_DONE) break;
        barrier_results(B, t);
        free_reconverge(t, conv, upc);
    }
    return epoch;
}

// ---- lockstep (canonical) block execution ---------------------------------------
// Conflict tables of a lockstep step: the highest tid storing to a location in
// a step wins (stores land in ascending tid order).  Shared memory uses one
// owner word per simulated shared word; global memory an open-addressing hash
// table with room for twice the threads of a block.
// log2 of the global-store hash table size: at least twice the block's threads.
__host__ __device__ inline uint32_t lockstep_hash_bits(uint32_t wg_threads) {
    uint32_t b = 1;
    while ((1u << b) < 2 * wg_threads) b++;
    return b;
}

struct StoreTables {
    uint32_t *own_sh;   // sh_words_max entries, 0 = free
    uint32_t *gkey;     // hash keys (global word address), EMPTY = free
    uint32_t *gown;     // owner tid + 1
    uint32_t hbits;     // log2 of the table size
};
constexpr uint32_t EMPTY_KEY = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t ghash(uint32_t a, uint32_t hbits) { return (a * 2654435761u) >> (32 - hbits); }

// The smallest pc among the lanes of `todo` (wave-uniform).  A converged
// group -- every lane of `todo` at one pc -- needs no reduction.
__device__ __forceinline__ int group_pc(uint64_t todo, int pc) {
    const uint32_t first = (uint32_t)__ffsll((long long)todo) - 1u;
    const int p0 = __builtin_amdgcn_readlane(pc, (int)first);
    const bool mine = (todo >> lane_id()) & 1ull;
    if (__ballot(mine && pc != p0) == 0) return uni(p0);
    return uni(wave_min(mine ? pc : INT_MAX));
}

// The program word at `cur`, or 0 past the end.
__device__ __forceinline__ uint64_t fetch_word(const BlockCtx &B, int cur) {
    return (uint32_t)cur < B.n_instr ? B.prog[(uint32_t)uni(cur)] : 0ull;
}

// 1 for a load, 2 for a store at `cur`, 0 otherwise (and past the end).
__device__ __forceinline__ uint32_t prog_kind(const BlockCtx &B, int cur) {
    const uint32_t op = uniu((uint32_t)fetch_word(B, cur) & 0xFFu);
    return (op >> 4) == 5u ? 1u + (op & 1u) : 0u;
}

// One step's group: the running lanes of the wave at the smallest pc among
// `todo` execute their instruction (loads read memory now, stores are held in
// P); returns the lanes that took part.
// `exec(cur, w, active, P, epoch, ctl, target, cond)` executes the
// instruction at `cur` (program word `w`) for the lanes with `active`, as
// exec_one does in lockstep mode.
template <bool LOCAL, class Exec>
__device__ __forceinline__ uint64_t lockstep_group(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t,
                                                   LogState &L, Pending &P, uint32_t epoch, uint64_t todo, int cur,
                                                   uint64_t w, Exec &exec) {
    const bool mine = (todo >> lane_id()) & 1ull;
    bool active = mine && t.pc == cur;
    const uint64_t done = __ballot(active);
    if ((uint32_t)cur >= B.n_instr) {
        if (active) t.st = ST_EXIT;
        return done;
    }
    const bool nofuel = active && t.fuel == 0;
    if (__ballot(nofuel)) {
        emit_fault(nofuel, A, B, F_FUEL, epoch, 0, B.tid, 0, 0);
        if (nofuel) { t.st = ST_EXIT; active = false; }
        if (__ballot(active) == 0) return done;
    }
    if (active) t.fuel--;
    int ctl, target;
    bool cond;
    exec(cur, w, active, P, epoch, ctl, target, cond);
    if (active && ctl != 3) {
        if (ctl == 2) t.pc = cond ? target : cur + 1;
        else t.pc = target;
    }
    return done;
}

// Canonical lockstep execution of one block.  Within an epoch every running
// thread executes its i-th instruction at step i, and threads interact only
// through loads and stores, so a thread's memory-free instructions may run
// whenever convenient: each lane keeps the number of steps it has completed
// in the epoch, and every group of lanes at one pc runs on its own to its next
// load or store (or barrier, or exit), where it parks.  A round then takes the
// smallest step at which a running lane is parked: the lanes parked there
// execute it (loads read memory as of the start of the step, stores are held
// back), and the step's stores land with the highest tid winning per location
// -- the same order as stepping every thread through every step together,
// since all loads and stores of earlier steps have been done by then.  When
// no lane is running the block takes its barrier episode.
//
// A round costs one workgroup barrier, and one more when a store is among the
// step's accesses; the owner entries a step's stores claimed are cleared in
// the next round, behind its first barrier.
//
// `run(grp, epoch)` may execute the memory-free instructions of a converged
// group (one step each, charging fuel and leaving pc and state in `t`),
// stopping before a load or store; it returns the number of steps taken, 0
// when it took none (then the group steps through `exec` one instruction).
//
// `release()` runs after every completed episode (the results of barriers
// with a predicate).  `kind(pc)` tells a load (1) or a store (2) from other
// instructions (0; also past the end), `word(pc)` gives the program word
// `exec` takes (the specialised kernels need neither from memory).
//
// The round's smallest parked step goes through one LDS word per round (three
// used in turn: the next round's is reset before this round's barrier, after
// every read of it two rounds ago), each wave taking the minimum of
// (step << 1 | no store at it) with one atomic.
template <bool LOCAL, class Exec, class Run, class Release, class Kind, class Word>
__device__ __forceinline__ uint32_t run_block_lockstep(const InterpArgs &A, BlockCtx &B, const Shared &S,
                                                   const StoreTables &T, Lane &t, LogState &L, Exec &exec,
                                                   Run &run, Release &release, Kind &kind, Word &word) {
    constexpr uint32_t NO_STEP = 0xFFFFFFFFu;
    uint32_t epoch = 0;
    uint32_t rnd = 0;               // rounds of the block (selects the round word)
    unsigned long long *RW = (unsigned long long *)S.eps;     // three round words
    if (threadIdx.x == 0) RW[0] = ~0ull;
    __syncthreads();
    bool clear = false;             // this lane won a location in the last store round: free its owner entry
    bool clear_sh = false;
    uint32_t clear_at = 0;
    for (;;) {
        uint32_t ls = 0;            // steps this lane has completed in the epoch
        bool parked = false;        // stopped before a load or store (its step ls)
        bool pst = false;           // ... a store
        for (;;) {
            // every running lane to its next load or store
            for (;;) {
                const bool free_lane = t.st == ST_RUN && !parked;
                const uint64_t fm = __ballot(free_lane);
                if (fm == 0) break;
                const int p = uni(__builtin_amdgcn_readlane(t.pc, (int)((uint32_t)__ffsll((long long)fm) - 1u)));
                const bool mine = free_lane && t.pc == p;
                const uint64_t grp = __ballot(mine);
                const uint32_t kd = kind(p);
                if (kd != 0u) {
                    if (mine) {
                        parked = true;
                        pst = kd == 2u;
                    }
                    continue;
                }
                uint32_t k = run(grp, epoch);
                if (k == 0) {
                    Pending none{false, false, 0, 0};
                    lockstep_group<LOCAL>(A, B, S, t, L, none, epoch, grp, p, word(p), exec);
                    k = 1;
                }
                if (mine) ls += k;
            }
            // the smallest parked step of the wave, and whether a store waits there
            const bool waiting = t.st == ST_RUN && parked;
            const uint64_t wmask = __ballot(waiting);
            uint32_t m = NO_STEP;
            if (wmask) {
                const uint32_t l0 = (uint32_t)__builtin_amdgcn_readlane((int)ls, (int)((uint32_t)__ffsll((long long)wmask) - 1u));
                m = __ballot(waiting && ls != l0) ? wave_min_u(waiting ? ls : NO_STEP) : l0;
                m = uniu(m);
            }
            const bool st_m = __ballot(waiting && ls == m && pst) != 0;
            if (threadIdx.x == 0) RW[(rnd + 1u) % 3u] = ~0ull;
            if (lane_id() == 0 && wmask)
                atomicMin(&RW[rnd % 3u], ((unsigned long long)m << 1) | (st_m ? 0ull : 1ull));
            __syncthreads();
            if (clear) {            // every lane read its win before the barrier above
                if (clear_sh) {
                    T.own_sh[clear_at] = 0;
                } else {
                    T.gown[clear_at] = 0;
                    T.gkey[clear_at] = EMPTY_KEY;
                }
                clear = false;
            }
            const unsigned long long rw = RW[rnd % 3u];
            rnd++;
            if (rw == ~0ull) break;                    // no running lane anywhere: barrier episode
            const uint32_t M = (uint32_t)(rw >> 1);
            const bool any_st = (rw & 1ull) == 0;
            Pending P{false, false, 0, 0};
            B.step = M;
            B.epoch = epoch;
            if (m == M) {           // the lanes parked at step M execute it
                const bool at = waiting && ls == M;
                uint64_t todo = __ballot(at);
                while (todo) {
                    const int cur = group_pc(todo, t.pc);
                    todo &= ~lockstep_group<LOCAL>(A, B, S, t, L, P, epoch, todo, cur, word(cur), exec);
                }
                if (at) {
                    ls++;
                    parked = false;
                }
            }
            if (!any_st) continue;
            // the step's stores: the highest tid per location wins
            uint32_t slot = 0;
            if (P.on) {
                if (P.shared) {
                    atomicMax(&T.own_sh[P.addr], B.tid + 1);
                } else {
                    const uint32_t mask = (1u << T.hbits) - 1u;
                    slot = ghash((uint32_t)P.addr, T.hbits);
                    for (uint32_t probe = 0; probe <= mask; probe++) {
                        const uint32_t old = atomicCAS(&T.gkey[slot], EMPTY_KEY, (uint32_t)P.addr);
                        if (old == EMPTY_KEY || old == (uint32_t)P.addr) break;
                        slot = (slot + 1) & mask;
                    }
                    atomicMax(&T.gown[slot], B.tid + 1);
                }
            }
            __syncthreads();
            if (A.uninit && P.on && P.shared) mark_stored(S, (uint32_t)P.addr);   // every load of the step is done
            bool win = false;
            if (P.on) win = (P.shared ? T.own_sh[P.addr] : T.gown[slot]) == B.tid + 1;
            if (win && P.shared) S.sh[P.addr] = P.val;
            if (win && !P.shared) B.mem[P.addr] = P.val;
            if (win) {              // one winner per location frees its entry next round
                clear = true;
                clear_sh = P.shared;
                clear_at = P.shared ? (uint32_t)P.addr : slot;
            }
        }
        if (barrier_episode<LOCAL>(A, B, S, t, L, epoch) == EP_DONE) break;
        release();
    }
    return epoch;
}

// LDS layout: simulated shared memory | staging (nwaves x stage records) |
// [local check: second buffer of the same size | nwaves x 256 counters |
// 256 words | shared-word tuples | global shadow table] | episode slots |
// [lockstep: store-owner tables].
__device__ __forceinline__ size_t carve_lds(uint8_t *smem, const InterpArgs &A, Shared &S, uint32_t nwaves,
                                           uint32_t wave) {
    S.sh = (int32_t *)smem;
    size_t off = ((size_t)A.sh_words_max * 4 + 15) & ~(size_t)15;
    S.stage_all = (uint64_t *)(smem + off);
    S.stage = S.stage_all + (size_t)wave * A.stage;
    off += (size_t)nwaves * A.stage * 8;
    if (A.local) {
        S.alt = (uint64_t *)(smem + off);
        off += (size_t)nwaves * A.stage * 8;
        S.wc = (uint32_t *)(smem + off);
        off += (size_t)nwaves * 256 * 4;
        S.tmp = (uint32_t *)(smem + off);
        off += 256 * 4;
        S.shadow = (unsigned long long *)(smem + off);
        S.vmin = (uint32_t *)(smem + off);
        S.vmax = S.vmin + A.sh_words_max;
        S.vw = S.vmax + A.sh_words_max;
        off += shadow_region_bytes(A.sh_words_max);
        S.gst = (unsigned long long *)(smem + off);
        off += A.gst_bits ? ((size_t)8 << A.gst_bits) : 0;
        S.repbuf = (uint64_t *)(smem + off);
        off += A.gst_bits ? (size_t)A.rep_hold * 8 : 0;
    }
    S.slots = (uint32_t *)(smem + off);
    S.slots2 = S.slots + 16 * 10;
    S.eps = S.slots2 + 16 * 4;
    off += (16 * 10 + 16 * 4 + 3 * 8) * 4;
    S.sinit = (uint32_t *)(smem + off);
    off += (size_t)(A.sh_words_max + 31) / 32 * 4;
    return off;
}

// One workgroup of a free-run launch: set up the block, run it with `run`
// (the interpreter loop, or a program-specialised loop), publish its counts.
template <class Run>
__device__ __forceinline__ void free_block(const InterpArgs &A, Run run) {
    extern __shared__ __align__(16) uint8_t smem[];
    Shared S;
    const uint32_t nwaves = (blockDim.x + WAVE - 1) / WAVE;
    const uint32_t wave = threadIdx.x / WAVE;
    carve_lds(smem, A, S, nwaves, wave);

    uint32_t unit = 0, block = blockIdx.x;
    if (A.items) {
        uint2 it = A.items[blockIdx.x];
        unit = uniu(it.x);
        block = uniu(it.y);
    }
    BlockCtx B;
    B.nwaves = nwaves;
    B.wave = wave;
    Lane t;
    LogState L{0, 0, 0, false};
    setup_block(A, B, S, t, unit, block, false);
    const uint32_t epoch = run(A, B, S, t, L);
    finish_block(A, B, S, L, t, epoch);
}

template <bool LOCAL>
__device__ __forceinline__ void interp_free_body(const InterpArgs &A) {
    free_block(A, [](const InterpArgs &a, BlockCtx &b, const Shared &s, Lane &t, LogState &l) {
        return run_block_free<LOCAL>(a, b, s, t, l);
    });
}


// One workgroup of a replay launch: the blocks of one component in
// ascending order, each run with `run(A, B, S, T, t, L)` (the interpreter's
// lockstep loop, or one with program-specialised instruction bodies).
template <class Run>
__device__ __forceinline__ void lockstep_body(const InterpArgs &A, Run run) {
    extern __shared__ __align__(16) uint8_t smem[];
    Shared S;
    const uint32_t nwaves = (blockDim.x + WAVE - 1) / WAVE;
    const uint32_t wave = threadIdx.x / WAVE;
    size_t off = carve_lds(smem, A, S, nwaves, wave);

    StoreTables T;
    T.own_sh = (uint32_t *)(smem + off);
    off += (size_t)A.sh_words_max * 4;
    T.hbits = lockstep_hash_bits(blockDim.x);
    T.gkey = (uint32_t *)(smem + off);
    T.gown = T.gkey + (1u << T.hbits);
    for (uint32_t i = threadIdx.x; i < A.sh_words_max; i += blockDim.x) T.own_sh[i] = 0;
    for (uint32_t i = threadIdx.x; i < (1u << T.hbits); i += blockDim.x) {
        T.gkey[i] = EMPTY_KEY;
        T.gown[i] = 0;
    }
    // a component's blocks, or (count on the device) single-block components
    // strided over the workgroups
    const bool strided = A.n_comps_dev != nullptr;
    const uint32_t c0 = strided ? blockIdx.x : uniu(A.comp_off[blockIdx.x]);
    const uint32_t c1 = strided ? uniu(*A.n_comps_dev) : uniu(A.comp_off[blockIdx.x + 1]);
    const uint32_t dc = strided ? gridDim.x : 1u;
    BlockCtx B;
    B.nwaves = nwaves;
    B.wave = wave;
    Lane t;
    LogState L{0, 0, 0, false};
    for (uint32_t c = c0; c < c1; c += dc) {
        uint2 it = A.comp_blocks[c];
        setup_block(A, B, S, t, uniu(it.x), uniu(it.y), true);
        const uint32_t epoch = run(A, B, S, T, t, L);
        finish_block(A, B, S, L, t, epoch);
    }
}

// Source sites: a replayed access of `tid` (linear, or global for the
// cross-block key) at `pc` to a location that has a race tuple.
__device__ __forceinline__ void site_hit(const InterpArgs &A, uint32_t unit, uint32_t space, uint32_t block,
                                         uint32_t epoch, uint32_t addr, uint32_t tid, bool store, int pc) {
    const uint32_t mask = (1u << A.site_bits) - 1u;
    uint32_t h = site_hash(unit, space, block, epoch, addr) & mask;
    for (uint32_t probe = 0; probe <= mask; probe++) {
        SiteSlot &e = A.sites[h];
        if (!e.used) return;
        if (e.addr == addr && e.block == block && e.epoch == epoch && e.unit == unit && e.space == space) {
            if (store && tid == e.w) atomicMin(&e.w_pc, (uint32_t)pc);
            if (tid == e.o) atomicMin(&e.o_pc, (uint32_t)pc);
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ void site_probe(const InterpArgs &A, const BlockCtx &B, const Lane &t, int cur,
                                           uint64_t w, bool active, uint32_t epoch) {
    const uint32_t op = (uint32_t)w & 0xFFu;
    if ((op >> 4) != 5u || !active) return;
    const uint32_t ra = (uint32_t)(w >> 16) & 0xFFu;
    const uint32_t addr = (uint32_t)t.r[ra] + (uint32_t)(int32_t)(uint32_t)(w >> 32);
    const bool is_sh = (op & 2u) == 0, is_st = (op & 1u) != 0;
    if (addr >= (is_sh ? B.sh_words : B.n_words)) return;
    site_hit(A, B.unit, is_sh ? 0u : 1u, B.block, epoch, addr, B.tid, is_st, cur);
    if (!is_sh) site_hit(A, B.unit, 1u, 0xFFFFFFFFu, 0xFFFFFFFFu, addr, B.block * B.nt + B.tid, is_st, cur);
}

// The canonical replay once more, probing the source-site table at every
// access (without the epoch-local check: every access is logged).
__device__ __forceinline__ void interp_lockstep_sites_body(const InterpArgs &A) {
    lockstep_body(A, [](const InterpArgs &a, BlockCtx &b, const Shared &s, const StoreTables &tb, Lane &t,
                        LogState &l) {
        auto exec = [&](int cur, uint64_t w, bool active, Pending &P, uint32_t epoch, int &ctl, int &target,
                        bool &cond) {
            site_probe(a, b, t, cur, w, active, epoch);
            exec_one<true, false>(a, b, s, t, l, P, epoch, cur, w, active, ctl, target, cond);
        };
        auto run = [](uint64_t, uint32_t) { return 0u; };
        auto release = [&] { barrier_results(b, t); };
        auto word = [&](int p) { return fetch_word(b, p); };
        auto kind = [&](int p) { return prog_kind(b, p); };
        return run_block_lockstep<false>(a, b, s, tb, t, l, exec, run, release, kind, word);
    });
}

template <bool LOCAL>
__device__ __forceinline__ void interp_lockstep_body(const InterpArgs &A) {
    lockstep_body(A, [](const InterpArgs &a, BlockCtx &b, const Shared &s, const StoreTables &tb, Lane &t,
                        LogState &l) {
        auto exec = [&](int cur, uint64_t w, bool active, Pending &P, uint32_t epoch, int &ctl, int &target,
                        bool &cond) {
            exec_one<true, LOCAL>(a, b, s, t, l, P, epoch, cur, w, active, ctl, target, cond);
        };
        auto run = [](uint64_t, uint32_t) { return 0u; };
        auto release = [&] { barrier_results(b, t); };
        auto word = [&](int p) { return fetch_word(b, p); };
        auto kind = [&](int p) { return prog_kind(b, p); };
        return run_block_lockstep<LOCAL>(a, b, s, tb, t, l, exec, run, release, kind, word);
    });
}

}  // namespace

}  // namespace kc
