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
#include "kc_internal.h"

namespace kc {

namespace {

constexpr int WAVE = 64;
enum : int { ST_RUN = 0, ST_WAIT = 1, ST_EXIT = 2, ST_DEAD = 3 };

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lane_prefix(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniu(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
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
    uint32_t *slots;    // 16 waves x 8 words: episode reductions
    uint32_t *slots2;   // 16 x 4: divergence second round
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
};

// Wave-aggregated append of findings.
__device__ __forceinline__ void emit_fault(bool f, const InterpArgs &A, const BlockCtx &B, uint32_t kind, uint32_t epoch,
                           uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    uint64_t m = __ballot(f);
    if (m == 0) return;
    uint32_t leader = (uint32_t)__ffsll((long long)m) - 1;
    uint32_t cnt = (uint32_t)__popcll(m);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(A.fault_count, cnt);
    base = __shfl(base, (int)leader);
    if (f) {
        uint32_t idx = base + lane_prefix(m);
        if (idx < A.fault_cap) {
            DevFault F;
            F.unit = B.unit; F.kind = kind; F.block = B.block; F.epoch = epoch;
            F.a = a; F.b = b; F.c = c; F.d = d;
            A.faults[idx] = F;
        } else {
            atomicOr(A.flags, FLAG_FAULT_OVERFLOW);
        }
    }
}

__device__ __forceinline__ void flush_stage(const InterpArgs &A, uint64_t *stage, uint32_t cnt) {
    if (cnt == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(A.log_count, (unsigned long long)cnt);
    base = bcast_u64(base, 0);
    for (uint32_t i = lane_id(); i < cnt; i += WAVE) {
        unsigned long long p = base + i;
        if (p < A.log_cap) A.log[p] = stage[i];
    }
    if (lane_id() == 0 && base + cnt > A.log_cap) atomicOr(A.flags, FLAG_LOG_OVERFLOW);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

struct LogState {
    uint32_t cur;       // staged records (wave-uniform)
    uint32_t total;     // records of this wave for the block
};

__device__ __forceinline__ void log_rec(const InterpArgs &A, uint64_t *stage, LogState &L, bool rec,
                                        uint64_t key) {
    uint64_t m = __ballot(rec);
    if (m == 0) return;
    uint32_t cnt = (uint32_t)__popcll(m);
    if (L.cur + cnt > A.stage) {
        flush_stage(A, stage, L.cur);
        L.cur = 0;
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
    regfile_t r;
};

// Result of the episode logic, uniform over the workgroup.
enum : int { EP_RELEASED = 0, EP_DONE = 1 };

// All waves are quiescent (no running lane).  Count arrivals and decide.
__device__ __forceinline__ int barrier_episode(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t,
                               uint32_t &epoch) {
    __syncthreads();
    bool is_thread = t.st != ST_DEAD;
    uint64_t wm = __ballot(t.st == ST_WAIT);
    uint64_t em = __ballot(t.st == ST_EXIT);
    int bmin = wave_min(t.st == ST_WAIT ? t.bar_pc : INT_MAX);
    int bmax = wave_max(t.st == ST_WAIT ? t.bar_pc : -1);
    (void)is_thread;
    if (lane_id() == 0) {
        uint32_t *s = S.slots + 8 * B.wave;
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
        const uint32_t *s = S.slots + 8 * w;
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
    if (threadIdx.x == 0) {
        if (epoch > A.kp.max_epoch) atomicOr(A.flags, FLAG_EPOCH_OVERFLOW);
        atomicMax(A.max_epoch, epoch);
    }
    if (t.st == ST_WAIT) {
        t.st = ST_RUN;
        t.pc = t.bar_pc + 1;
    }
    B.kep = B.kbase | ((uint64_t)epoch << A.kp.s_ep);
    return EP_RELEASED;
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

// Every instruction writes at most one register.  The cases only produce the
// value; a single indexed write after the dispatch keeps the register file in
// place (one write site avoids copies of the whole 16-register vector).
struct RegWrite {
    bool writes;    // wave-uniform: the opcode writes register d
    bool on;
    int32_t v;
};
__device__ __forceinline__ void wr(RegWrite &W, bool active, int32_t v) {
    W.writes = true;
    W.on = active;
    W.v = v;
}

// Execute the instruction at pc `cur` (wave-uniform) for the lanes in `active`.
// ctl: 0 falls through, 1 JMP, 2 conditional branch (cond per lane), 3 BAR/EXIT.
template <bool LOCKSTEP>
__device__ __forceinline__ void exec_one(const InterpArgs &A, const BlockCtx &B, const Shared &S, Lane &t,
                                         LogState &L, Pending &P, uint32_t epoch, int cur, bool active,
                                         int &ctl, int &target, bool &cond) {
    ctl = 0;
    target = cur + 1;
    cond = false;
    RegWrite W{false, false, 0};
    const uint64_t w = B.prog[(uint32_t)uni(cur)];
    const uint32_t op = uniu((uint32_t)w & 0xFFu);
    const uint32_t d = uniu((uint32_t)(w >> 8) & 0xFFu);
    const uint32_t ra = uniu((uint32_t)(w >> 16) & 0xFFu);
    const uint32_t rb = uniu((uint32_t)(w >> 24) & 0xFFu);
    const int32_t imm = uni((int32_t)(uint32_t)(w >> 32));
    const uint32_t base = op & ~uint32_t(OP_IMM);
    if (base >= OP_ADD && base <= OP_SLTU) {
        bool arith = false;
        const int32_t x = t.r[ra];
        int32_t y;
        if (op & OP_IMM) y = imm;
        else y = t.r[rb];
        const int32_t v = alu(base, x, y, arith);
        if (base == OP_DIV || base == OP_REM)
            emit_fault(active && arith, A, B, F_ARITH, epoch, 0, B.tid, (uint32_t)cur, 0);
        wr(W, active, v);
    } else {
    const KeyPlan &k = A.kp;
    switch (op) {
    case OP_MOV:
        wr(W, active, t.r[ra]);
        break;
    case OP_MOVI:
        wr(W, active, imm);
        break;
    case OP_SREG:
        wr(W, active, special(B, (uint32_t)imm));
        break;
    case OP_LDS: {
        const int32_t addr = (int32_t)((uint32_t)t.r[ra] + (uint32_t)imm);
        const bool inb = active && (uint32_t)addr < B.sh_words;
        int32_t v = 0;
        if (inb) v = S.sh[addr];
        wr(W, active, v);
        log_rec(A, S.stage, L, inb, B.kep | ((uint64_t)0u << k.s_sp) | 0ull | ((uint64_t)(uint32_t)addr << k.s_addr));
        emit_fault(active && !inb, A, B, F_OOB, epoch, 0u, B.tid, (uint32_t)addr, 0);
        break;
    }
    case OP_LDG: {
        const int32_t addr = (int32_t)((uint32_t)t.r[ra] + (uint32_t)imm);
        const bool inb = active && (uint32_t)addr < B.n_words;
        int32_t v = 0;
        if (inb) v = B.mem[addr];
        wr(W, active, v);
        log_rec(A, S.stage, L, inb, B.kep | ((uint64_t)1u << k.s_sp) | 0ull | ((uint64_t)(uint32_t)addr << k.s_addr));
        emit_fault(active && !inb, A, B, F_OOB, epoch, 2u, B.tid, (uint32_t)addr, 0);
        break;
    }
    case OP_STS: {
        const int32_t addr = (int32_t)((uint32_t)t.r[ra] + (uint32_t)imm);
        const bool inb = active && (uint32_t)addr < B.sh_words;
        const int32_t v = t.r[rb];
        if (LOCKSTEP) {
            if (inb) { P.on = true; P.shared = true; P.addr = addr; P.val = v; }
        } else if (inb) {
            S.sh[addr] = v;
        }
        log_rec(A, S.stage, L, inb, B.kep | ((uint64_t)0u << k.s_sp) | 1ull | ((uint64_t)(uint32_t)addr << k.s_addr));
        emit_fault(active && !inb, A, B, F_OOB, epoch, 1u, B.tid, (uint32_t)addr, 0);
        break;
    }
    case OP_STG: {
        const int32_t addr = (int32_t)((uint32_t)t.r[ra] + (uint32_t)imm);
        const bool inb = active && (uint32_t)addr < B.n_words;
        const int32_t v = t.r[rb];
        if (LOCKSTEP) {
            if (inb) { P.on = true; P.shared = false; P.addr = addr; P.val = v; }
        } else if (inb) {
            B.mem[addr] = v;
        }
        log_rec(A, S.stage, L, inb, B.kep | ((uint64_t)1u << k.s_sp) | 1ull | ((uint64_t)(uint32_t)addr << k.s_addr));
        emit_fault(active && !inb, A, B, F_OOB, epoch, 3u, B.tid, (uint32_t)addr, 0);
        break;
    }
    case OP_JMP:
        ctl = 1;
        target = imm;
        break;
    case OP_BZ:
    case OP_BNZ: {
        const int32_t x = t.r[ra];
        cond = (op == OP_BZ) ? (x == 0) : (x != 0);
        ctl = 2;
        target = imm;
        break;
    }
    case OP_BAR:
        ctl = 3;
        if (active) { t.st = ST_WAIT; t.bar_pc = cur; }
        break;
    case OP_EXIT:
        ctl = 3;
        if (active) t.st = ST_EXIT;
        break;
    default:
        break;   // validated programs contain no other opcode
    }
    }
    if (W.writes) {
        const int32_t old = t.r[d];
        t.r[d] = W.on ? W.v : old;
    }
}

__device__ __forceinline__ void setup_block(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t, uint32_t unit,
                            uint32_t block) {
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
    B.kep = B.kbase;
    for (uint32_t i = threadIdx.x; i < B.sh_words; i += blockDim.x) S.sh[i] = 0;
    t.pc = 0;
    t.st = (B.tid < B.nt) ? ST_RUN : ST_DEAD;
    t.fuel = u->fuel;
    t.bar_pc = 0;
    t.r = (regfile_t)(0);
    __syncthreads();
}

__device__ __forceinline__ void finish_block(const InterpArgs &A, const BlockCtx &B, const Shared &S, LogState &L) {
    flush_stage(A, S.stage, L.cur);
    L.cur = 0;
    if (lane_id() == 0 && L.total) atomicAdd(&A.blk_recs[B.u->block_base + B.block], L.total);
    L.total = 0;
    __syncthreads();
}

// ---- free-run block execution ------------------------------------------------
__device__ __forceinline__ void run_block_free(const InterpArgs &A, BlockCtx &B, const Shared &S, Lane &t, LogState &L) {
    uint32_t epoch = 0;
    Pending P{false, false, 0, 0};
    bool conv = true;    // every running lane of the wave is at upc
    int upc = 0;
    uint32_t guard = B.u->fuel;     // lower bound of every live lane's fuel
    for (;;) {
        for (;;) {
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
            exec_one<false>(A, B, S, t, L, P, epoch, cur, active, ctl, target, cond);
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
        if (barrier_episode(A, B, S, t, epoch) == EP_DONE) break;
        int lo = wave_min(t.st == ST_RUN ? t.pc : INT_MAX);
        int hi = wave_max(t.st == ST_RUN ? t.pc : -1);
        conv = (lo == hi) || hi < 0;
        upc = uni(lo);
    }
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

__device__ __forceinline__ void run_block_lockstep(const InterpArgs &A, BlockCtx &B, const Shared &S,
                                                   const StoreTables &T, Lane &t, LogState &L) {
    uint32_t epoch = 0;
    uint32_t step = 0;
    bool any_run = true;
    for (;;) {
        if (!any_run) {
            if (barrier_episode(A, B, S, t, epoch) == EP_DONE) break;
            any_run = true;     // a completed episode releases every thread
        }
        // phase A: every running lane executes exactly one instruction; loads
        // read memory as of the start of the step, stores are held back
        Pending P{false, false, 0, 0};
        uint64_t todo = __ballot(t.st == ST_RUN);
        while (todo) {
            const bool mine = (todo >> lane_id()) & 1ull;
            int cur = uni(wave_min(mine ? t.pc : INT_MAX));
            bool active = mine && t.pc == cur;
            todo &= ~__ballot(active);
            if ((uint32_t)cur >= B.n_instr) {
                if (active) t.st = ST_EXIT;
                continue;
            }
            const bool nofuel = active && t.fuel == 0;
            if (__ballot(nofuel)) {
                emit_fault(nofuel, A, B, F_FUEL, epoch, 0, B.tid, 0, 0);
                if (nofuel) { t.st = ST_EXIT; active = false; }
                if (__ballot(active) == 0) continue;
            }
            if (active) t.fuel--;
            int ctl, target;
            bool cond;
            exec_one<true>(A, B, S, t, L, P, epoch, cur, active, ctl, target, cond);
            if (active && ctl != 3) {
                if (ctl == 2) t.pc = cond ? target : cur + 1;
                else t.pc = target;
            }
        }
        // publish (any lane still running, any pending store) for this step;
        // two slot words alternate by step parity so no extra barrier is needed
        const uint32_t par = step & 1u;
        const uint64_t runm = __ballot(t.st == ST_RUN);
        const uint64_t stm = __ballot(P.on);
        if (lane_id() == 0) S.slots[8 * B.wave + 6 + par] = (runm ? 1u : 0u) | (stm ? 2u : 0u);
        __syncthreads();
        uint32_t flags = 0;
        for (uint32_t w = 0; w < B.nwaves; w++) flags |= S.slots[8 * w + 6 + par];
        any_run = (flags & 1u) != 0;
        step++;
        if (!(flags & 2u)) continue;
        // phase B: the highest tid per location wins
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
        bool win = false;
        if (P.on) win = (P.shared ? T.own_sh[P.addr] : T.gown[slot]) == B.tid + 1;
        if (win && P.shared) S.sh[P.addr] = P.val;
        if (win && !P.shared) B.mem[P.addr] = P.val;
        __syncthreads();
        if (win) {      // one winner per location clears its entry for the next step
            if (P.shared) {
                T.own_sh[P.addr] = 0;
            } else {
                T.gown[slot] = 0;
                T.gkey[slot] = EMPTY_KEY;
            }
        }
    }
}

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6, 6))) k_interp_free(InterpArgs A) {
    extern __shared__ __align__(16) uint8_t smem[];
    Shared S;
    const uint32_t nwaves = (blockDim.x + WAVE - 1) / WAVE;
    const uint32_t wave = threadIdx.x / WAVE;
    S.sh = (int32_t *)smem;
    size_t off = ((size_t)A.sh_words_max * 4 + 15) & ~(size_t)15;
    S.stage = (uint64_t *)(smem + off) + (size_t)wave * A.stage;
    off += (size_t)nwaves * A.stage * 8;
    S.slots = (uint32_t *)(smem + off);
    S.slots2 = S.slots + 16 * 8;

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
    LogState L{0, 0};
    setup_block(A, B, S, t, unit, block);
    run_block_free(A, B, S, t, L);
    finish_block(A, B, S, L);
}

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6, 6))) k_interp_lockstep(InterpArgs A) {
    extern __shared__ __align__(16) uint8_t smem[];
    Shared S;
    const uint32_t nwaves = (blockDim.x + WAVE - 1) / WAVE;
    const uint32_t wave = threadIdx.x / WAVE;
    S.sh = (int32_t *)smem;
    size_t off = ((size_t)A.sh_words_max * 4 + 15) & ~(size_t)15;
    S.stage = (uint64_t *)(smem + off) + (size_t)wave * A.stage;
    off += (size_t)nwaves * A.stage * 8;
    S.slots = (uint32_t *)(smem + off);
    S.slots2 = S.slots + 16 * 8;

    off += (16 * 8 + 16 * 4) * 4;
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
    const uint32_t c0 = uniu(A.comp_off[blockIdx.x]), c1 = uniu(A.comp_off[blockIdx.x + 1]);
    BlockCtx B;
    B.nwaves = nwaves;
    B.wave = wave;
    Lane t;
    LogState L{0, 0};
    for (uint32_t c = c0; c < c1; c++) {
        uint2 it = A.comp_blocks[c];
        setup_block(A, B, S, t, uniu(it.x), uniu(it.y));
        run_block_lockstep(A, B, S, T, t, L);
        finish_block(A, B, S, L);
    }
}

}  // namespace

size_t interp_lds_bytes(uint32_t sh_words_max, uint32_t wg_threads, uint32_t stage, bool lockstep) {
    const uint32_t nwaves = (wg_threads + WAVE - 1) / WAVE;
    size_t off = ((size_t)sh_words_max * 4 + 15) & ~(size_t)15;
    off += (size_t)nwaves * stage * 8;
    off += (16 * 8 + 16 * 4) * 4;
    if (lockstep) off += (size_t)sh_words_max * 4 + ((size_t)8 << lockstep_hash_bits(wg_threads));
    return off;
}

hipError_t launch_interp(const InterpArgs &a, uint32_t n_wg, uint32_t wg_threads, bool lockstep, hipStream_t s) {
    if (n_wg == 0) return hipSuccess;
    InterpArgs args = a;
    size_t lds = interp_lds_bytes(args.sh_words_max, wg_threads, args.stage, lockstep);
    while (lds > 160 * 1024 && args.stage > 64) {   // shrink the record staging area to fit
        args.stage /= 2;
        lds = interp_lds_bytes(args.sh_words_max, wg_threads, args.stage, lockstep);
    }
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e1 = hipFuncSetAttribute((const void *)k_interp_free, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            160 * 1024);
        hipError_t e2 = hipFuncSetAttribute((const void *)k_interp_lockstep,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e1 != hipSuccess) return e1;
        if (e2 != hipSuccess) return e2;
        attr_set = true;
    }
    if (lockstep)
        hipLaunchKernelGGL(k_interp_lockstep, dim3(n_wg), dim3(wg_threads), lds, s, args);
    else
        hipLaunchKernelGGL(k_interp_free, dim3(n_wg), dim3(wg_threads), lds, s, args);
    return hipGetLastError();
}

}  // namespace kc
