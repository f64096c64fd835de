/*
 * kc_oracle.c -- plain, slow CPU oracle for the SIMT race and deadlock checker.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls this code;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no source with the HIP path: it has its own instruction decoder,
 * its own interpreter and its own conflict check.
 *
 * What it computes (Hathhorn et al., "Formal Semantics of Heterogeneous
 * CUDA-C", SSV 2012):
 *
 *   - A job is an initial global memory followed by launches executed in order,
 *     as items of one stream are executed serially (Section 2, last paragraph;
 *     Section 3 "Streams and events").  A launch whose grid does not complete
 *     (a block deadlocked) ends the job: a grid counts as complete only when
 *     all of its threads have finished (Section 3 "Threads and memory").
 *   - Streams and events (Section 3 "Streams and events"): each launch may
 *     name a stream, and a dependency (before, after) says that launch `after`
 *     waits for launch `before` to finish (an event recorded behind `before`
 *     and waited on ahead of `after`, or a host synchronisation).  Launch i
 *     happens before launch j when a chain of same-stream order (an earlier
 *     launch of the same stream) and dependencies leads from i to j.  Two
 *     launches ordered neither way may run in parallel; the job still
 *     executes them in submission order, which respects every chain.  A global
 *     word accessed by two such launches, written by at least one, is a race
 *     between them (scope 2), reported on the later launch j with
 *     block = i, epoch = 0xFFFFFFFF, w_tid = the smallest global thread id of
 *     j whose access to the word conflicts with an access of i, and o_tid the
 *     same for i: if the other launch writes the word every access conflicts,
 *     otherwise only writes do.
 *   - Memory transfers and the host (Section 3 "Streams and events": launches
 *     and memory transfers pass through the stream queues; the host
 *     synchronises with cudaStreamSynchronize, cudaEventSynchronize and
 *     cudaDeviceSynchronize).  A job may instead be a list of items in the
 *     host program's order: launches and copies (device items, each in a
 *     stream), host reads and writes of words of the memory, and host waits.
 *     A copy moves `words` words from src to dst (the ranges may not
 *     overlap); its word k is copied by "thread" k.  A host read or write of
 *     words [addr, addr + words) touches word addr + k as thread k; a write
 *     stores `value`.  A host wait blocks the host until one earlier device
 *     item (an event recorded right behind it, or the last item of a stream)
 *     or every earlier device item (the device) has finished.  Item i happens
 *     before a later item j when: both are device items of one stream; a
 *     dependency (an event) links them; i is a host item (the host issues j
 *     only after it); i is a copy the host waits for on the spot (a
 *     synchronous cudaMemcpy); or j is a host wait for i (or for every
 *     device item) -- and every chain of these.  Items ordered neither way
 *     may run in parallel and race (scope 2) as launches do, with the
 *     item indices in place of launch indices; items still execute in the
 *     host program's order.  A launch that does not complete ends the job.
 *     Copies and host accesses make no access records.
 *   - Within a launch the blocks run one after another in ascending linear
 *     block id; this is one of the interleavings the semantics admits
 *     (Section 3 "Threads and memory": scheduling is constrained only by grid
 *     completion).  Inside a block the threads run in lockstep: every running
 *     thread executes one instruction per step, loads of a step read memory as
 *     it was at the start of the step, and the step's stores are then applied
 *     in ascending thread id.  This is a legal sequentially consistent
 *     interleaving (all loads, then the stores in tid order).
 *   - Barriers: a thread at __syncthreads() waits until every thread of its
 *     block waits at a barrier; the rewrite rules of Section 3 "Barrier
 *     synchronization" pass a token through all NThrds threads of the block
 *     and never compare which barrier each thread reached.  When every thread
 *     waits, the episode completes: the block enters the next barrier epoch and
 *     all threads resume after their own barrier.  If the barrier sites differ
 *     a DIVERGENCE finding is recorded.  If some threads wait and the others
 *     have exited, no rule can fire again: that is the deadlock of Section 3.1
 *     (a thread fails to reach a barrier another thread reached); a DEADLOCK
 *     finding is recorded and the block halts.
 *   - Barriers with a predicate (Section 3 feature list: __syncthreads_count,
 *     __syncthreads_and, __syncthreads_or): BARP d, a, k waits like a plain
 *     barrier; when the episode completes, each thread that waits at a BARP
 *     receives in register d the number of threads of the block whose
 *     predicate is nonzero (k = 0), 1 if every thread's is (k = 1), or 1 if
 *     any thread's is (k = 2), else 0.  A thread's predicate is its register
 *     a while it waits (registers do not change while waiting); a thread
 *     waiting at a plain barrier counts as predicate 0.
 *   - Memory objects (Section 3 feature list: device memory allocation; the
 *     tool's checks for out-of-bounds and illegal device or host memory
 *     access): a job may list its device allocations as word ranges of its
 *     memory.  A global load or store that lands on a word of the memory
 *     outside every allocation (host memory or nothing at all, from the
 *     device's side) is an illegal access.  It still takes effect (the memory
 *     is one array); each block that made such accesses to a word gets one
 *     finding ALLOC {block, epoch 0xFFFFFFFF, a = 2 + (1 if the block stored
 *     to it), b = the smallest tid of the block that accessed it, c = the
 *     word, d = the smallest tid that stored to it or 0xFFFFFFFF}.
 *   - Uninitialised shared memory (among the checks the tool inherits from the
 *     C semantics are uninitialised memory accesses, Section 3.2; CUDA leaves
 *     shared memory undefined when a block starts), when that check is on: a
 *     load of a shared word that no thread of the block has stored to before
 *     it -- before in the block's lockstep order: an earlier step, since the
 *     loads of a step read memory as it was before the step's stores -- is a
 *     finding UNINIT {block, epoch, a = 0, b = tid, c = the word, d = pc of
 *     the load}.  The load still reads the word (zero, as shared memory starts
 *     zeroed).  For a race-free block this order is the order of every
 *     interleaving: a store by another thread to the word in the same epoch
 *     would race with the load.
 *   - Warp-aware model (the finer scheduler the paper's Section 4 proposes),
 *     when that check is on: threads form warps of 32 consecutive linear tids
 *     that execute in lock-step, so two accesses of one block and epoch by
 *     threads of one warp conflict only when they run at the same step; see
 *     warp_tuple for the tuple it reports.  Cross-block tuples are unchanged.
 *   - Every in-bounds load and store appends an access record
 *     {space, word address, block, barrier epoch, tid, read/write}, the
 *     information the race tuples of Section 3.1 keep per location.
 *   - Source sites (the tool reports a race with the source line it was
 *     detected at, Section 3.2): each race tuple carries w_pc, the smallest
 *     pc of a store by w_tid to the location, and o_pc, the smallest pc of an
 *     access by o_tid to it, within the tuple's block and epoch (intra-block)
 *     or the launch (cross-block); races between launches carry none
 *     (0xFFFFFFFF).
 *   - Races (Section 3.1): two accesses to one location by different threads,
 *     at least one a write, with no synchronization point between them.  For
 *     shared memory the synchronization point is a completed barrier episode of
 *     the block (the tuples are cleared at __syncthreads()).  The same rule is
 *     applied to global memory within a block; global accesses of different
 *     blocks are ordered only by the end of the kernel (Section 2: blocks
 *     synchronize only through the implicit barrier at kernel end), so they
 *     conflict in any epochs.
 *
 * Numeric conventions where C leaves behaviour undefined: int32 arithmetic
 * wraps; DIV/REM truncate; division by zero yields 0 and an ARITH finding;
 * INT_MIN / -1 = INT_MIN and INT_MIN % -1 = 0; shift counts use the low five
 * bits; out-of-bounds accesses yield an OOB finding, loads return 0, stores are
 * dropped and no access record is made; every thread may execute at most
 * `fuel` instructions (FUEL finding, the thread exits); falling off the end of
 * the program is an exit.  Shared memory starts zeroed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- instruction set (decoded here independently of the GPU path) ---- */
enum {
    OP_ADD = 0x01, OP_SUB, OP_MUL, OP_DIV, OP_REM, OP_AND, OP_OR, OP_XOR,
    OP_SHL, OP_SHRA, OP_SHRL, OP_MIN, OP_MAX, OP_SLT, OP_SLE, OP_SEQ, OP_SNE, OP_SLTU,
    OP_MOV = 0x40, OP_MOVI = 0x41, OP_SREG = 0x42,
    OP_LDS = 0x50, OP_STS = 0x51, OP_LDG = 0x52, OP_STG = 0x53,
    OP_JMP = 0x60, OP_BZ = 0x61, OP_BNZ = 0x62, OP_BAR = 0x63, OP_EXIT = 0x64, OP_BARP = 0x65
};

enum { ST_RUN = 0, ST_WAIT = 1, ST_EXIT = 2 };
enum { SP_SHARED = 0, SP_GLOBAL = 1 };
enum { K_READ = 0, K_WRITE = 1 };
enum { F_DEADLOCK = 1, F_DIVERGENCE = 2, F_OOB = 3, F_FUEL = 4, F_ARITH = 5, F_ALLOC = 6, F_UNINIT = 7 };
enum { CHECK_UNINIT_SHARED = 1, CHECK_WARP = 2 };
enum { WARP_SIZE = 32 };

typedef struct {
    uint32_t grid[3], block[3];
    uint32_t shmem_bytes;
    int32_t params[8];
} ora_launch;

/* An item of a job in host program order (see the header comment). */
enum { IT_LAUNCH = 0, IT_COPY = 1, IT_HOST_READ = 2, IT_HOST_WRITE = 3, IT_HOST_WAIT = 4 };
enum { IT_SYNC = 1 };           /* flags: the host waits for this copy on the spot */
#define WAIT_ALL 0xFFFFFFFFu    /* host wait target: every earlier device item */
typedef struct {
    uint32_t kind, stream;
    uint32_t ref;               /* launch index (IT_LAUNCH); item waited for (IT_HOST_WAIT) */
    uint32_t flags;
    uint64_t dst, src, words;   /* IT_COPY: dst <- src; host items: words [dst, dst + words) */
    int32_t value;              /* IT_HOST_WRITE */
    uint32_t pad;
} ora_item;

/* step: the block's lockstep step within the epoch at which the access ran */
typedef struct { uint32_t launch, space, addr, block, epoch, tid, kind, pc, step; } ora_record;
typedef struct { uint32_t launch, space, scope, block, epoch, addr, w_tid, o_tid, w_pc, o_pc; } ora_race;
typedef struct { uint32_t launch, kind, block, epoch, a, b, c, d; } ora_fault;

typedef struct {
    ora_record *recs;   uint64_t n_recs, cap_recs;     /* current launch's records */
    ora_record *kept;   uint64_t n_kept, cap_kept;     /* all records, if asked for */
    ora_race *races;    uint64_t n_races, cap_races;
    ora_fault *faults;  uint64_t n_faults, cap_faults;
    uint64_t n_records;
    uint64_t n_instructions;    /* thread-instructions executed (fuel spent) */
    uint32_t launches_completed;
    int keep_records;
    int oom;
} ora_result;

#define GROW(ptr, n, cap, T)                                                  \
    do {                                                                      \
        if ((n) == (cap)) {                                                   \
            uint64_t nc = (cap) ? 2 * (cap) : 1024;                           \
            T *np_ = (T *)realloc((ptr), nc * sizeof(T));                     \
            if (!np_) { res->oom = 1; return; }                               \
            (ptr) = np_; (cap) = nc;                                          \
        }                                                                     \
    } while (0)

static void add_record(ora_result *res, uint32_t launch, uint32_t space, uint32_t addr,
                       uint32_t block, uint32_t epoch, uint32_t tid, uint32_t kind, uint32_t pc, uint32_t step) {
    ora_record r = {launch, space, addr, block, epoch, tid, kind, pc, step};
    GROW(res->recs, res->n_recs, res->cap_recs, ora_record);
    res->recs[res->n_recs++] = r;
    res->n_records++;
    if (res->keep_records) {
        GROW(res->kept, res->n_kept, res->cap_kept, ora_record);
        res->kept[res->n_kept++] = r;
    }
}

static void add_fault(ora_result *res, uint32_t launch, uint32_t kind, uint32_t block,
                      uint32_t epoch, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    ora_fault f = {launch, kind, block, epoch, a, b, c, d};
    GROW(res->faults, res->n_faults, res->cap_faults, ora_fault);
    res->faults[res->n_faults++] = f;
}

static void add_race(ora_result *res, ora_race r) {
    GROW(res->races, res->n_races, res->cap_races, ora_race);
    res->races[res->n_races++] = r;
}

/* ---- program validation (independent of the library's validator) ---- */
static int valid_op(uint32_t op) {
    uint32_t base = op & ~0x20u;
    if (base >= OP_ADD && base <= OP_SLTU) return 1;
    return op == OP_MOV || op == OP_MOVI || op == OP_SREG || op == OP_LDS || op == OP_STS ||
           op == OP_LDG || op == OP_STG || op == OP_JMP || op == OP_BZ || op == OP_BNZ ||
           op == OP_BAR || op == OP_EXIT || op == OP_BARP;
}

int ora_validate(const uint64_t *prog, uint32_t n) {
    if (n == 0 || n > 65536) return 2;
    for (uint32_t pc = 0; pc < n; pc++) {
        uint64_t w = prog[pc];
        uint32_t op = w & 0xFF, d = (w >> 8) & 0xFF, a = (w >> 16) & 0xFF, b = (w >> 24) & 0xFF;
        int32_t imm = (int32_t)(uint32_t)(w >> 32);
        if (!valid_op(op) || d >= 16 || a >= 16 || b >= 16) return 2;
        if ((op == OP_JMP || op == OP_BZ || op == OP_BNZ) && (imm < 0 || (uint32_t)imm > n)) return 2;
        if (op == OP_SREG && (imm < 0 || imm >= 24)) return 2;
        if (op == OP_BARP && (imm < 0 || imm > 2)) return 2;
    }
    return 0;
}

/* ---- int32 ALU (wrapping two's complement; see header comment) ---- */
static int32_t alu(uint32_t base, int32_t x, int32_t y, int *arith) {
    uint32_t ux = (uint32_t)x, uy = (uint32_t)y;
    switch (base) {
    case OP_ADD: return (int32_t)(ux + uy);
    case OP_SUB: return (int32_t)(ux - uy);
    case OP_MUL: return (int32_t)(ux * uy);
    case OP_DIV:
        if (y == 0) { *arith = 1; return 0; }
        if (x == INT32_MIN && y == -1) return INT32_MIN;
        return x / y;
    case OP_REM:
        if (y == 0) { *arith = 1; return 0; }
        if (x == INT32_MIN && y == -1) return 0;
        return x % y;
    case OP_AND: return x & y;
    case OP_OR: return x | y;
    case OP_XOR: return x ^ y;
    case OP_SHL: return (int32_t)(ux << (uy & 31));
    case OP_SHRA: {
        /* arithmetic shift written without relying on implementation-defined >> */
        uint32_t s = uy & 31;
        uint32_t r = ux >> s;
        if (x < 0 && s) r |= ~(0xFFFFFFFFu >> s);
        return (int32_t)r;
    }
    case OP_SHRL: return (int32_t)(ux >> (uy & 31));
    case OP_MIN: return x < y ? x : y;
    case OP_MAX: return x > y ? x : y;
    case OP_SLT: return x < y;
    case OP_SLE: return x <= y;
    case OP_SEQ: return x == y;
    case OP_SNE: return x != y;
    case OP_SLTU: return ux < uy;
    }
    return 0;
}

typedef struct {
    uint32_t pc;
    int32_t r[16];
    int status;
    uint32_t fuel;
    uint32_t bar_pc;
} ora_thread;

typedef struct { uint32_t tid; uint32_t space; int32_t addr; int32_t val; } ora_store;

/* Special registers (Section 3 feature list: gridDim, blockDim, blockIdx, threadIdx, warpSize). */
static int32_t sreg(const ora_launch *L, uint32_t k, uint32_t tid, uint32_t bid) {
    uint32_t bx = L->block[0], by = L->block[1], gx = L->grid[0], gy = L->grid[1];
    switch (k) {
    case 0: return (int32_t)(tid % bx);
    case 1: return (int32_t)((tid / bx) % by);
    case 2: return (int32_t)(tid / (bx * by));
    case 3: return (int32_t)(bid % gx);
    case 4: return (int32_t)((bid / gx) % gy);
    case 5: return (int32_t)(bid / (gx * gy));
    case 6: return (int32_t)L->block[0];
    case 7: return (int32_t)L->block[1];
    case 8: return (int32_t)L->block[2];
    case 9: return (int32_t)L->grid[0];
    case 10: return (int32_t)L->grid[1];
    case 11: return (int32_t)L->grid[2];
    case 12: return (int32_t)tid;
    case 13: return (int32_t)bid;
    case 14: return (int32_t)(bx * by * L->block[2]);
    case 15: return 32;
    default: return L->params[k - 16];
    }
}

/* Run one block to completion or halt under lockstep steps.  Returns 1 if it deadlocked. */
static int run_block(ora_result *res, uint32_t li, const uint64_t *prog, uint32_t n,
                     const ora_launch *L, uint32_t bid, int32_t *mem, uint64_t n_words,
                     uint32_t fuel, ora_thread *th, int32_t *sh, ora_store *q, uint8_t *shinit) {
    uint32_t nt = L->block[0] * L->block[1] * L->block[2];
    uint32_t sh_words = L->shmem_bytes / 4;
    uint32_t epoch = 0, step = 0;
    memset(sh, 0, (size_t)sh_words * sizeof(int32_t));
    if (shinit) memset(shinit, 0, (size_t)sh_words);   /* no shared word stored yet */
    for (uint32_t t = 0; t < nt; t++) {
        memset(&th[t], 0, sizeof(ora_thread));
        th[t].status = ST_RUN;
        th[t].fuel = fuel;
    }
    for (;;) {
        int any_run = 0;
        for (uint32_t t = 0; t < nt; t++)
            if (th[t].status == ST_RUN) { any_run = 1; break; }
        if (any_run) {
            /* one lockstep step: phase A executes, stores are queued */
            uint32_t nq = 0;
            for (uint32_t t = 0; t < nt; t++) {
                ora_thread *T = &th[t];
                if (T->status != ST_RUN) continue;
                if (T->pc == n) { T->status = ST_EXIT; continue; }
                if (T->fuel == 0) {
                    T->status = ST_EXIT;
                    add_fault(res, li, F_FUEL, bid, epoch, 0, t, 0, 0);
                    continue;
                }
                T->fuel--;
                res->n_instructions++;
                uint64_t w = prog[T->pc];
                uint32_t op = w & 0xFF, d = (w >> 8) & 0xFF, a = (w >> 16) & 0xFF, b = (w >> 24) & 0xFF;
                int32_t imm = (int32_t)(uint32_t)(w >> 32);
                uint32_t next = T->pc + 1;
                uint32_t base = op & ~0x20u;
                if (base >= OP_ADD && base <= OP_SLTU) {
                    int arith = 0;
                    int32_t y = (op & 0x20) ? imm : T->r[b];
                    int32_t v = alu(base, T->r[a], y, &arith);
                    if (arith) add_fault(res, li, F_ARITH, bid, epoch, 0, t, T->pc, 0);
                    T->r[d] = v;
                } else {
                    switch (op) {
                    case OP_MOV: T->r[d] = T->r[a]; break;
                    case OP_MOVI: T->r[d] = imm; break;
                    case OP_SREG: T->r[d] = sreg(L, (uint32_t)imm, t, bid); break;
                    case OP_LDS: case OP_LDG: {
                        uint32_t space = (op == OP_LDS) ? SP_SHARED : SP_GLOBAL;
                        int32_t addr = (int32_t)((uint32_t)T->r[a] + (uint32_t)imm);
                        uint64_t lim = space == SP_SHARED ? sh_words : n_words;
                        if (addr < 0 || (uint64_t)addr >= lim) {
                            add_fault(res, li, F_OOB, bid, epoch, space * 2 + K_READ, t, (uint32_t)addr, 0);
                            T->r[d] = 0;
                        } else {
                            T->r[d] = space == SP_SHARED ? sh[addr] : mem[addr];
                            add_record(res, li, space, (uint32_t)addr, bid, epoch, t, K_READ, T->pc, step);
                            if (shinit && space == SP_SHARED && !shinit[addr])
                                add_fault(res, li, F_UNINIT, bid, epoch, 0, t, (uint32_t)addr, T->pc);
                        }
                        break;
                    }
                    case OP_STS: case OP_STG: {
                        uint32_t space = (op == OP_STS) ? SP_SHARED : SP_GLOBAL;
                        int32_t addr = (int32_t)((uint32_t)T->r[a] + (uint32_t)imm);
                        uint64_t lim = space == SP_SHARED ? sh_words : n_words;
                        if (addr < 0 || (uint64_t)addr >= lim) {
                            add_fault(res, li, F_OOB, bid, epoch, space * 2 + K_WRITE, t, (uint32_t)addr, 0);
                        } else {
                            q[nq].tid = t; q[nq].space = space; q[nq].addr = addr; q[nq].val = T->r[b];
                            nq++;
                            add_record(res, li, space, (uint32_t)addr, bid, epoch, t, K_WRITE, T->pc, step);
                        }
                        break;
                    }
                    case OP_JMP: next = (uint32_t)imm; break;
                    case OP_BZ: if (T->r[a] == 0) next = (uint32_t)imm; break;
                    case OP_BNZ: if (T->r[a] != 0) next = (uint32_t)imm; break;
                    case OP_BAR: case OP_BARP: T->status = ST_WAIT; T->bar_pc = T->pc; break;
                    case OP_EXIT: T->status = ST_EXIT; break;
                    }
                }
                T->pc = next;
            }
            /* phase B: stores in ascending tid order (queued in that order) */
            for (uint32_t i = 0; i < nq; i++) {
                if (q[i].space == SP_SHARED) {
                    sh[q[i].addr] = q[i].val;
                    if (shinit) shinit[q[i].addr] = 1;
                } else {
                    mem[q[i].addr] = q[i].val;
                }
            }
            step++;
            if (res->oom) return 0;
        } else {
            uint32_t nwait = 0, nexit = 0;
            for (uint32_t t = 0; t < nt; t++) {
                if (th[t].status == ST_WAIT) nwait++;
                else nexit++;
            }
            if (nwait == 0) return 0;                 /* all threads finished */
            if (nexit == 0) {
                /* every thread waits: the episode completes */
                uint32_t lo = UINT32_MAX, lo_tid = 0, hi = UINT32_MAX, hi_tid = 0;
                for (uint32_t t = 0; t < nt; t++)
                    if (th[t].bar_pc < lo) { lo = th[t].bar_pc; lo_tid = t; }
                for (uint32_t t = 0; t < nt; t++)
                    if (th[t].bar_pc > lo && th[t].bar_pc < hi) { hi = th[t].bar_pc; hi_tid = t; }
                if (hi != UINT32_MAX)
                    add_fault(res, li, F_DIVERGENCE, bid, epoch, lo, lo_tid, hi, hi_tid);
                /* predicate barriers: the block-wide count, and, or */
                uint32_t count = 0;
                for (uint32_t t = 0; t < nt; t++) {
                    uint64_t w = prog[th[t].bar_pc];
                    if ((w & 0xFF) == OP_BARP && th[t].r[(w >> 16) & 0xFF] != 0) count++;
                }
                for (uint32_t t = 0; t < nt; t++) {
                    uint64_t w = prog[th[t].bar_pc];
                    if ((w & 0xFF) != OP_BARP) continue;
                    int32_t kind = (int32_t)(uint32_t)(w >> 32);
                    int32_t v = kind == 0 ? (int32_t)count : kind == 1 ? (count == nt) : (count > 0);
                    th[t].r[(w >> 8) & 0xFF] = v;
                }
                epoch++;
                step = 0;
                for (uint32_t t = 0; t < nt; t++) {
                    th[t].status = ST_RUN;
                    th[t].pc = th[t].bar_pc + 1;
                }
            } else {
                uint32_t min_wait = UINT32_MAX, min_exit = UINT32_MAX;
                for (uint32_t t = 0; t < nt; t++) {
                    if (th[t].status == ST_WAIT && t < min_wait) min_wait = t;
                    if (th[t].status == ST_EXIT && t < min_exit) min_exit = t;
                }
                add_fault(res, li, F_DEADLOCK, bid, epoch, nwait, min_wait, min_exit, 0);
                return 1;
            }
        }
    }
}

/* ---- conflict check over one launch's records (Section 3.1) ---- */
static uint32_t g_nt;   /* threads per block of the launch being checked (qsort context) */

static int cmp_intra(const void *pa, const void *pb) {
    const ora_record *x = pa, *y = pb;
    if (x->space != y->space) return x->space < y->space ? -1 : 1;
    if (x->block != y->block) return x->block < y->block ? -1 : 1;
    if (x->epoch != y->epoch) return x->epoch < y->epoch ? -1 : 1;
    if (x->addr != y->addr) return x->addr < y->addr ? -1 : 1;
    if (x->tid != y->tid) return x->tid < y->tid ? -1 : 1;
    return (int)x->kind - (int)y->kind;
}

static int cmp_cross(const void *pa, const void *pb) {
    const ora_record *x = pa, *y = pb;
    if (x->space != y->space) return x->space < y->space ? -1 : 1;
    if (x->addr != y->addr) return x->addr < y->addr ? -1 : 1;
    uint64_t gx = (uint64_t)x->block * g_nt + x->tid, gy = (uint64_t)y->block * g_nt + y->tid;
    if (gx != gy) return gx < gy ? -1 : 1;
    return (int)x->kind - (int)y->kind;
}

/* Warp-aware model (the finer scheduler the paper's Section 4 proposes:
 * threads grouped into warps of warpSize = 32 consecutive linear tids that
 * execute in lock-step).  Two accesses of one block and epoch by threads of
 * one warp are ordered by the warp's instruction order unless they run at the
 * same lockstep step; threads of different warps stay unordered until the
 * barrier.  A write x and an access y (x != y) conflict when the threads are
 * in different warps or the two accesses share a step.  The tuple reports
 * w = the smallest thread with a write that conflicts, and o = the smallest
 * other thread with an access that conflicts with one of w's writes. */
static int warp_conflict(const ora_record *x, const ora_record *y) {
    if (x->kind != K_WRITE || x->tid == y->tid) return 0;
    return x->tid / WARP_SIZE != y->tid / WARP_SIZE || x->step == y->step;
}

/* The warp-aware tuple of one location's group r[i, j) (tids ascending): 1 and
 * (w, o) if some pair conflicts. */
static int warp_tuple(const ora_record *r, uint64_t i, uint64_t j, uint32_t *w, uint32_t *o) {
    for (uint64_t a = i; a < j; a++) {
        if (r[a].kind != K_WRITE) continue;
        /* r[a] is a write of the smallest thread not yet ruled out */
        int found = 0;
        uint32_t best = UINT32_MAX;
        for (uint64_t x = a; x < j && r[x].tid == r[a].tid; x++)
            for (uint64_t b = i; b < j; b++)
                if (warp_conflict(&r[x], &r[b]) && r[b].tid < best) { best = r[b].tid; found = 1; }
        if (found) { *w = r[a].tid; *o = best; return 1; }
    }
    return 0;
}

static void check_launch(ora_result *res, uint32_t li, uint32_t nt, int warp) {
    ora_record *r = res->recs;
    uint64_t n = res->n_recs;
    /* intra-block: records of one (space, block, epoch, addr) are unordered by barriers */
    qsort(r, n, sizeof(ora_record), cmp_intra);
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i;
        while (j < n && r[j].space == r[i].space && r[j].block == r[i].block &&
               r[j].epoch == r[i].epoch && r[j].addr == r[i].addr) j++;
        /* tids ascend inside the group: the first writer is the minimum writer */
        int has_w = 0; uint32_t w = 0, wo = 0;
        if (warp) {
            has_w = warp_tuple(r, i, j, &w, &wo);
        } else {
            for (uint64_t k = i; k < j; k++)
                if (r[k].kind == K_WRITE) { has_w = 1; w = r[k].tid; break; }
        }
        if (has_w) {
            for (uint64_t k = i; k < j; k++) {
                if (r[k].tid != w && (!warp || r[k].tid == wo)) {
                    ora_race rc = {li, r[i].space, 0, r[i].block, r[i].epoch, r[i].addr, w, r[k].tid,
                                   0xFFFFFFFFu, 0xFFFFFFFFu};
                    /* source sites: the smallest pc of w's stores to the location and of the
                     * other thread's accesses to it, in this block and epoch */
                    for (uint64_t q = i; q < j; q++) {
                        if (r[q].tid == w && r[q].kind == K_WRITE && r[q].pc < rc.w_pc) rc.w_pc = r[q].pc;
                        if (r[q].tid == rc.o_tid && r[q].pc < rc.o_pc) rc.o_pc = r[q].pc;
                    }
                    add_race(res, rc);
                    break;
                }
            }
        }
        i = j;
    }
    /* cross-block (global memory): records of different blocks are never ordered */
    g_nt = nt;
    qsort(r, n, sizeof(ora_record), cmp_cross);
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i;
        while (j < n && r[j].space == r[i].space && r[j].addr == r[i].addr) j++;
        if (r[i].space == SP_GLOBAL) {
            int has_w = 0; uint64_t wk = 0;
            for (uint64_t k = i; k < j; k++)
                if (r[k].kind == K_WRITE) { has_w = 1; wk = k; break; }
            if (has_w) {
                uint32_t wb = r[wk].block;
                for (uint64_t k = i; k < j; k++) {
                    if (r[k].block != wb) {
                        ora_race rc = {li, SP_GLOBAL, 1, wb, 0xFFFFFFFFu, r[i].addr,
                                       wb * nt + r[wk].tid, r[k].block * nt + r[k].tid, 0xFFFFFFFFu, 0xFFFFFFFFu};
                        /* source sites over the whole launch */
                        for (uint64_t q = i; q < j; q++) {
                            const uint32_t g = r[q].block * nt + r[q].tid;
                            if (g == rc.w_tid && r[q].kind == K_WRITE && r[q].pc < rc.w_pc) rc.w_pc = r[q].pc;
                            if (g == rc.o_tid && r[q].pc < rc.o_pc) rc.o_pc = r[q].pc;
                        }
                        add_race(res, rc);
                        break;
                    }
                }
            }
        }
        i = j;
    }
    res->n_recs = 0;
}

static int cmp_race(const void *pa, const void *pb) {
    const ora_race *x = pa, *y = pb;
    const uint32_t kx[6] = {x->launch, x->space, x->scope, x->block, x->epoch, x->addr};
    const uint32_t ky[6] = {y->launch, y->space, y->scope, y->block, y->epoch, y->addr};
    for (int i = 0; i < 6; i++)
        if (kx[i] != ky[i]) return kx[i] < ky[i] ? -1 : 1;
    return 0;
}

static int cmp_fault(const void *pa, const void *pb) {
    const ora_fault *x = pa, *y = pb;
    const uint32_t kx[8] = {x->launch, x->block, x->epoch, x->kind, x->a, x->b, x->c, x->d};
    const uint32_t ky[8] = {y->launch, y->block, y->epoch, y->kind, y->a, y->b, y->c, y->d};
    for (int i = 0; i < 8; i++)
        if (kx[i] != ky[i]) return kx[i] < ky[i] ? -1 : 1;
    return 0;
}

/* ---- items that may run in parallel (Section 3 "Streams and events") ---- */
static int is_device(const ora_item *it) { return it->kind == IT_LAUNCH || it->kind == IT_COPY; }

/* hb[i * n + j] = 1 when item i happens before item j: the rules of the
 * header comment, closed transitively (Warshall). */
static uint8_t *happens_before(uint32_t n, const ora_item *items, const uint32_t *deps, uint32_t n_deps) {
    uint8_t *hb = calloc((size_t)n * n + 1, 1);
    if (!hb) return NULL;
    for (uint32_t j = 0; j < n; j++)
        for (uint32_t i = 0; i < j; i++) {
            const ora_item *a = &items[i], *b = &items[j];
            int before = 0;
            if (is_device(a) && is_device(b) && a->stream == b->stream) before = 1;   /* one stream */
            if (!is_device(a)) before = 1;                                            /* host order */
            if (a->kind == IT_COPY && (a->flags & IT_SYNC)) before = 1;               /* synchronous copy */
            if (b->kind == IT_HOST_WAIT && is_device(a) && (b->ref == WAIT_ALL || b->ref == i)) before = 1;
            if (before) hb[(size_t)i * n + j] = 1;
        }
    for (uint32_t d = 0; d < n_deps; d++) hb[(size_t)deps[2 * d] * n + deps[2 * d + 1]] = 1;
    for (uint32_t k = 0; k < n; k++)
        for (uint32_t i = 0; i < n; i++)
            if (hb[(size_t)i * n + k])
                for (uint32_t j = 0; j < n; j++)
                    if (hb[(size_t)k * n + j]) hb[(size_t)i * n + j] = 1;
    return hb;
}

/* Summary of a copy or host access: thread k touches the k-th word of each
 * range it reads or writes (same layout as access_summary). */
static uint32_t *range_summary(const ora_item *it, uint64_t n_words) {
    uint32_t *sum = malloc((2 * n_words + 1) * sizeof(uint32_t));
    if (!sum) return NULL;
    for (uint64_t x = 0; x < 2 * n_words; x++) sum[x] = 0xFFFFFFFFu;
    uint32_t *acc = sum, *wr = sum + n_words;
    for (uint64_t k = 0; k < it->words; k++) {
        if (it->kind == IT_COPY) acc[it->src + k] = (uint32_t)k;
        if (it->kind != IT_HOST_WAIT) acc[it->dst + k] = (uint32_t)k;
        if (it->kind == IT_COPY || it->kind == IT_HOST_WRITE) wr[it->dst + k] = (uint32_t)k;
    }
    return sum;
}

/* Smallest global thread id accessing each global word (acc) and writing it
 * (wr) in the current launch's records; 0xFFFFFFFF where none. */
static uint32_t *access_summary(const ora_result *res, uint64_t n_words, uint32_t nt) {
    uint32_t *sum = malloc((2 * n_words + 1) * sizeof(uint32_t));
    if (!sum) return NULL;
    for (uint64_t x = 0; x < 2 * n_words; x++) sum[x] = 0xFFFFFFFFu;
    uint32_t *acc = sum, *wr = sum + n_words;
    for (uint64_t i = 0; i < res->n_recs; i++) {
        const ora_record *r = &res->recs[i];
        if (r->space != SP_GLOBAL) continue;
        const uint32_t g = r->block * nt + r->tid;
        if (g < acc[r->addr]) acc[r->addr] = g;
        if (r->kind == K_WRITE && g < wr[r->addr]) wr[r->addr] = g;
    }
    return sum;
}

/* Races between launch i (summary si) and the later launch j (sj). */
static void cross_launch_races(ora_result *res, uint32_t i, const uint32_t *si, uint32_t j, const uint32_t *sj,
                               uint64_t n_words) {
    const uint32_t NONE = 0xFFFFFFFFu;
    for (uint64_t x = 0; x < n_words; x++) {
        const uint32_t ai = si[x], wi = si[n_words + x], aj = sj[x], wj = sj[n_words + x];
        const int conflict = (wi != NONE && aj != NONE) || (wj != NONE && ai != NONE);
        if (!conflict) continue;
        const uint32_t tj = wi != NONE ? aj : wj;   /* j's smallest thread conflicting with i */
        const uint32_t ti = wj != NONE ? ai : wi;
        ora_race rc = {j, SP_GLOBAL, 2, i, 0xFFFFFFFFu, (uint32_t)x, tj, ti, 0xFFFFFFFFu, 0xFFFFFFFFu};
        add_race(res, rc);
        if (res->oom) return;
    }
}

/* ALLOC findings of the current launch's records: per block, the words it
 * accessed outside every allocation (allocated[x] = 0). */
static int cmp_block_addr(const void *pa, const void *pb) {
    const ora_record *x = pa, *y = pb;
    if (x->block != y->block) return x->block < y->block ? -1 : 1;
    if (x->addr != y->addr) return x->addr < y->addr ? -1 : 1;
    return x->tid < y->tid ? -1 : x->tid > y->tid;
}

static void illegal_accesses(ora_result *res, uint32_t li, const uint8_t *allocated) {
    uint64_t n = 0;
    ora_record *bad = malloc((res->n_recs + 1) * sizeof(ora_record));
    if (!bad) { res->oom = 1; return; }
    for (uint64_t i = 0; i < res->n_recs; i++)
        if (res->recs[i].space == SP_GLOBAL && !allocated[res->recs[i].addr]) bad[n++] = res->recs[i];
    qsort(bad, n, sizeof(ora_record), cmp_block_addr);
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i;
        uint32_t wmin = 0xFFFFFFFFu;
        while (j < n && bad[j].block == bad[i].block && bad[j].addr == bad[i].addr) {
            if (bad[j].kind == K_WRITE && bad[j].tid < wmin) wmin = bad[j].tid;
            j++;
        }
        /* tids ascend in the group: bad[i] holds the smallest */
        add_fault(res, li, F_ALLOC, bad[i].block, 0xFFFFFFFFu, 2u + (wmin != 0xFFFFFFFFu), bad[i].tid,
                  bad[i].addr, wmin);
        i = j;
    }
    free(bad);
}

/* Run a job given as items (IT_*, n_items entries, host program order).
 * progs[i]/prog_lens[i]/launches[i] describe launch i, which launch items
 * name by index; mem is updated in place.  deps (n_deps pairs before, after,
 * before < after, both device items) are event dependencies.  allocs
 * (n_allocs pairs base, words), when not NULL, lists the device allocations;
 * `checks` (CHECK_*) turns on optional checks.  launches_completed counts the
 * leading items that completed. */
int ora_run_items(uint32_t n_launches, const uint64_t *const *progs, const uint32_t *prog_lens,
                  const ora_launch *launches, const ora_item *items, uint32_t n_items, int32_t *mem,
                  uint64_t n_words, uint32_t fuel, int keep_records, const uint32_t *deps, uint32_t n_deps,
                  const uint64_t *allocs, uint32_t n_allocs, uint32_t checks, ora_result **out) {
    *out = NULL;
    for (uint32_t d = 0; d < n_deps; d++)
        if (deps[2 * d] >= deps[2 * d + 1] || deps[2 * d + 1] >= n_items || !is_device(&items[deps[2 * d]]) ||
            !is_device(&items[deps[2 * d + 1]]))
            return 1;
    for (uint32_t a = 0; allocs && a < n_allocs; a++)
        if (allocs[2 * a] > n_words || allocs[2 * a + 1] > n_words - allocs[2 * a]) return 1;
    for (uint32_t i = 0; i < n_launches; i++) {
        if (ora_validate(progs[i], prog_lens[i])) return 2;
        const ora_launch *L = &launches[i];
        uint64_t nt = (uint64_t)L->block[0] * L->block[1] * L->block[2];
        uint64_t nb = (uint64_t)L->grid[0] * L->grid[1] * L->grid[2];
        if (nt == 0 || nt > 1024 || nb == 0 || nb * nt > 0xFFFFFFFFull || (L->shmem_bytes & 3)) return 1;
    }
    for (uint32_t j = 0; j < n_items; j++) {
        const ora_item *it = &items[j];
        if (it->kind > IT_HOST_WAIT) return 1;
        if (it->kind == IT_LAUNCH && it->ref >= n_launches) return 1;
        if (it->kind == IT_HOST_WAIT && it->ref != WAIT_ALL && (it->ref >= j || !is_device(&items[it->ref])))
            return 1;
        if (it->kind == IT_COPY || it->kind == IT_HOST_READ || it->kind == IT_HOST_WRITE) {
            if (it->dst > n_words || it->words > n_words - it->dst || it->words > 0xFFFFFFFFull) return 1;
            if (it->kind == IT_COPY &&
                (it->src > n_words || it->words > n_words - it->src ||
                 (it->words && it->src < it->dst + it->words && it->dst < it->src + it->words)))
                return 1;
        }
    }
    ora_result *res = calloc(1, sizeof(ora_result));
    if (!res) return 3;
    res->keep_records = keep_records;
    uint8_t *hb = happens_before(n_items, items, deps, n_deps);
    uint32_t **sums = calloc((size_t)n_items + 1, sizeof(uint32_t *));
    uint8_t *allocated = NULL;
    if (allocs) {
        allocated = calloc(n_words + 1, 1);
        for (uint32_t a = 0; allocated && a < n_allocs; a++)
            memset(allocated + allocs[2 * a], 1, allocs[2 * a + 1]);
    }
    if (!hb || !sums || (allocs && !allocated)) res->oom = 1;
    for (uint32_t li = 0; li < n_items && !res->oom; li++) {
        const ora_item *it = &items[li];
        int deadlocked = 0;
        uint32_t nt = 1;
        if (it->kind == IT_LAUNCH) {
            const ora_launch *L = &launches[it->ref];
            nt = L->block[0] * L->block[1] * L->block[2];
            const uint32_t nb = L->grid[0] * L->grid[1] * L->grid[2];
            ora_thread *th = calloc(nt, sizeof(ora_thread));
            int32_t *sh = calloc(L->shmem_bytes / 4 + 1, sizeof(int32_t));
            ora_store *q = calloc(nt, sizeof(ora_store));
            uint8_t *shinit = (checks & CHECK_UNINIT_SHARED) ? calloc(L->shmem_bytes / 4 + 1, 1) : NULL;
            if (!th || !sh || !q || ((checks & CHECK_UNINIT_SHARED) && !shinit)) {
                free(th); free(sh); free(q); free(shinit); res->oom = 1; break;
            }
            for (uint32_t b = 0; b < nb; b++)
                deadlocked |= run_block(res, li, progs[it->ref], prog_lens[it->ref], L, b, mem, n_words, fuel, th,
                                        sh, q, shinit);
            free(th); free(sh); free(q); free(shinit);
            if (res->oom) break;
        } else if (it->kind == IT_COPY) {
            for (uint64_t k = 0; k < it->words; k++) mem[it->dst + k] = mem[it->src + k];   /* disjoint ranges */
        } else if (it->kind == IT_HOST_WRITE) {
            for (uint64_t k = 0; k < it->words; k++) mem[it->dst + k] = it->value;
        }
        int parallel = 0;   /* may this item run in parallel with another one? */
        for (uint32_t k = 0; k < n_items; k++)
            if (k != li && !hb[(size_t)k * n_items + li] && !hb[(size_t)li * n_items + k]) parallel = 1;
        if (parallel && it->kind != IT_HOST_WAIT) {
            sums[li] = it->kind == IT_LAUNCH ? access_summary(res, n_words, nt) : range_summary(it, n_words);
            if (!sums[li]) { res->oom = 1; break; }
            for (uint32_t k = 0; k < li && !res->oom; k++)
                if (sums[k] && !hb[(size_t)k * n_items + li])
                    cross_launch_races(res, k, sums[k], li, sums[li], n_words);
            if (res->oom) break;
        }
        if (it->kind == IT_LAUNCH) {
            if (allocated) illegal_accesses(res, li, allocated);
            if (res->oom) break;
            check_launch(res, li, nt, (checks & CHECK_WARP) != 0);
            if (res->oom) break;
        }
        if (deadlocked) break;
        res->launches_completed = li + 1;
    }
    if (sums)
        for (uint32_t k = 0; k < n_items; k++) free(sums[k]);
    free(sums);
    free(hb);
    free(allocated);
    if (res->oom) {
        free(res->recs); free(res->kept); free(res->races); free(res->faults); free(res);
        return 3;
    }
    qsort(res->races, res->n_races, sizeof(ora_race), cmp_race);
    qsort(res->faults, res->n_faults, sizeof(ora_fault), cmp_fault);
    uint64_t m = 0;     /* findings form a set: drop repeated identical tuples */
    for (uint64_t i = 0; i < res->n_faults; i++)
        if (m == 0 || cmp_fault(&res->faults[m - 1], &res->faults[i]) != 0) res->faults[m++] = res->faults[i];
    res->n_faults = m;
    *out = res;
    return 0;
}

/* Run a job of launches only.  streams (n_launches entries) may be NULL: one
 * stream; deps (n_deps pairs before, after with before < after) are event
 * dependencies between launches.  The launches become items in order. */
int ora_run_job_opts(uint32_t n_launches, const uint64_t *const *progs, const uint32_t *prog_lens,
                     const ora_launch *launches, int32_t *mem, uint64_t n_words, uint32_t fuel,
                     int keep_records, const uint32_t *streams, const uint32_t *deps, uint32_t n_deps,
                     const uint64_t *allocs, uint32_t n_allocs, uint32_t checks, ora_result **out) {
    ora_item *items = calloc((size_t)n_launches + 1, sizeof(ora_item));
    if (!items) return 3;
    for (uint32_t i = 0; i < n_launches; i++) {
        items[i].kind = IT_LAUNCH;
        items[i].ref = i;
        items[i].stream = streams ? streams[i] : 0;
    }
    const int rc = ora_run_items(n_launches, progs, prog_lens, launches, items, n_launches, mem, n_words, fuel,
                                 keep_records, deps, n_deps, allocs, n_allocs, checks, out);
    free(items);
    return rc;
}

int ora_run_job_ex(uint32_t n_launches, const uint64_t *const *progs, const uint32_t *prog_lens,
                   const ora_launch *launches, int32_t *mem, uint64_t n_words, uint32_t fuel,
                   int keep_records, const uint32_t *streams, const uint32_t *deps, uint32_t n_deps,
                   const uint64_t *allocs, uint32_t n_allocs, ora_result **out) {
    return ora_run_job_opts(n_launches, progs, prog_lens, launches, mem, n_words, fuel, keep_records, streams,
                            deps, n_deps, allocs, n_allocs, 0, out);
}

int ora_run_job(uint32_t n_launches, const uint64_t *const *progs, const uint32_t *prog_lens,
                const ora_launch *launches, int32_t *mem, uint64_t n_words, uint32_t fuel,
                int keep_records, ora_result **out) {
    return ora_run_job_ex(n_launches, progs, prog_lens, launches, mem, n_words, fuel, keep_records,
                          NULL, NULL, 0, NULL, 0, out);
}

uint64_t ora_records(const ora_result *r) { return r->n_records; }
uint64_t ora_instructions(const ora_result *r) { return r->n_instructions; }
uint32_t ora_launches_completed(const ora_result *r) { return r->launches_completed; }
const ora_race *ora_races(const ora_result *r, uint64_t *n) { *n = r->n_races; return r->races; }
const ora_fault *ora_faults(const ora_result *r, uint64_t *n) { *n = r->n_faults; return r->faults; }
const ora_record *ora_kept_records(const ora_result *r, uint64_t *n) { *n = r->n_kept; return r->kept; }

void ora_free(ora_result *r) {
    if (!r) return;
    free(r->recs); free(r->kept); free(r->races); free(r->faults); free(r);
}
