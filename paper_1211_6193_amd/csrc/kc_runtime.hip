// Host runtime and C ABI of libkc (see include/kc.h).
//
// A stage processes one launch of each of a set of jobs ("units"):
//   1. snapshot every unit's memory (replay needs the launch-start state);
//   2. free-run interpretation: one workgroup per simulated block, records to
//      the HBM log;
//   3. LSD radix sort of the log on the bits above (tid, kind);
//   4. conflict check: race tuples, racy blocks and cross-block links;
//   5. if there are races: the blocks linked by races form components; their
//      global writes are restored from the snapshot and the components are
//      re-executed in lockstep, blocks in ascending order (the canonical
//      schedule).  If the replayed records equal the free-run records of those
//      blocks (as multisets) the free-run verdict stands and only memory and
//      findings of the replayed blocks change; otherwise every block of the
//      affected units is re-executed canonically and checked again;
//   6. reports.
// For race-free launches every interleaving has the same per-thread traces,
// so the free run already is the canonical execution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <system_error>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/kc.h"
#include "kc_internal.h"
#include "kc_jit.h"

using namespace kc;

struct kc_program {
    std::vector<uint64_t> words;
    uint64_t *dev = nullptr;
    int device = 0;
    mutable std::mutex jit_mu;
    mutable std::shared_ptr<kc::JitEntry> jit[9];   // program-specialised kernels, by occupancy target
};

struct kc_report {
    uint64_t records = 0;
    uint32_t launches_completed = 0;
    std::vector<kc_race> races;
    std::vector<kc_race_site> sites;    // parallel to races
    std::vector<kc_fault> faults;
    uint64_t tag = 0;
    void add_race(const kc_race &r, kc_race_site site = kc_race_site{0xFFFFFFFFu, 0xFFFFFFFFu}) {
        races.push_back(r);
        sites.push_back(site);
    }
};

namespace {

struct KcError {
    kc_status st;
    std::string msg;
};

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw KcError{KC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)};    \
    } while (0)

inline uint32_t bits_for(uint64_t count) {   // bits to hold values 0 .. count-1
    uint32_t b = 0;
    while (b < 64 && (1ull << b) < count) b++;
    return b;
}

// A fixed device area from which buffers are carved while a call runs
// without allocating (kc_launch_noalloc): bump allocation from `base`,
// restarted at every such call.  Set for the calling thread only.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0, peak = 0;
};
thread_local Arena *t_arena = nullptr;

// Device bytes a context's buffers hold (the library's own HBM use, which
// its budget bounds), now and at most so far.
struct DevBytes {
    std::atomic<int64_t> live{0}, peak{0};
    void add(int64_t d) {
        const int64_t v = live.fetch_add(d) + d;
        int64_t p = peak.load();
        while (v > p && !peak.compare_exchange_weak(p, v)) {
        }
    }
};

// Grow-only device buffer.  Its contents do not survive a growth.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool carved = false;    // p lies in the calling thread's arena (never freed)
    DevBytes *acct = nullptr;   // the owning context's count of device bytes
    void reserve(size_t need) {
        if (need <= bytes) return;
        if (t_arena) {
            Arena &a = *t_arena;
            const size_t nb = (need + 255) & ~size_t(255);
            if (nb > a.cap - a.used)
                throw KcError{KC_E_BUDGET, "the launch needs more device memory than the static scratch area holds (" +
                                               std::to_string(a.cap) + " bytes)"};
            p = a.base + a.used;
            bytes = nb;
            carved = true;
            a.used += nb;
            a.peak = std::max(a.peak, a.used);
            return;
        }
        if (carved) {
            p = nullptr;
            bytes = 0;
            carved = false;
        }
        size_t nb = std::max(need, bytes + bytes / 2);
        nb = (nb + 4095) & ~size_t(4095);
        if (p) HIPCHK(hipFree(p));
        if (p && acct) acct->add(-(int64_t)bytes);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, nb) != hipSuccess) {
            (void)hipGetLastError();
            nb = (need + 4095) & ~size_t(4095);
            if (hipMalloc(&p, nb) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                throw KcError{KC_E_NOMEM, "device allocation of " + std::to_string(need) + " bytes failed"};
            }
        }
        bytes = nb;
        if (acct) acct->add((int64_t)nb);
    }
    void release() {
        if (p && !carved) {
            (void)hipFree(p);
            if (acct) acct->add(-(int64_t)bytes);
        }
        p = nullptr;
        bytes = 0;
        carved = false;
    }
    template <class T> T *as() const { return (T *)p; }
};

struct Workspace {
    DBuf units, items, comp_off, comp_blocks, mask;
    DBuf snap, log, alt, rlog, ralt, fs, hist, part;
    DBuf faults, rfaults, races, lraces, rlraces, edges, blk_recs, rblk_recs, blk_flags, rflags, ctr, rctr, wlog;
    DBuf longseg, covlist, rtable, ftable, downer, dflags, blk_instr, blk_grecs, blk_log, blk_held, blk_off;
    DBuf sctr, stctr, sncomp;   // the replay queued behind the free run: counters, table counters, components
    DevCounters *h_ctr = nullptr;   // pinned
    void *h_pin = nullptr;          // pinned staging of gathered device-to-host copies
    void *d_pin = nullptr;          // its device mapping
    size_t h_pin_bytes = 0;
    void pin_reserve(size_t need) {
        if (need <= h_pin_bytes) return;
        if (t_arena)
            throw KcError{KC_E_BUDGET, "the launch's results need more than the " + std::to_string(h_pin_bytes) +
                                           " bytes of host staging set up for calls that allocate nothing"};
        if (h_pin) HIPCHK(hipHostFree(h_pin));
        h_pin = d_pin = nullptr;
        h_pin_bytes = 0;
        const size_t nb = std::max<size_t>(need + need / 2, 1 << 16);
        // coherent: the gather kernel's stores reach host memory directly
        HIPCHK(hipHostMalloc(&h_pin, nb, hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHK(hipHostGetDevicePointer(&d_pin, h_pin, 0));
        h_pin_bytes = nb;
    }
    // Pinned staging of host-to-device uploads: a copy from pageable memory
    // returns only once the stream has reached it, which would leave the GPU
    // idle while the host queues the next work; from pinned memory it
    // returns at once.  Regions are handed out in order and reused after the
    // stream has been synchronised (uploads_done).
    void *h_up = nullptr;
    size_t h_up_bytes = 0, h_up_used = 0;
    void upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
        if (!bytes) return;
        if (h_up_used + bytes > h_up_bytes) {
            if (t_arena) {      // a call that allocates nothing: no new pinned memory
                HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
                return;
            }
            HIPCHK(hipStreamSynchronize(s));        // earlier copies from the buffer are done
            h_up_used = 0;
            if (bytes > h_up_bytes) {
                const size_t nb = std::max<size_t>(std::max<size_t>(2 * bytes, 1 << 20), 2 * h_up_bytes);
                if (h_up) HIPCHK(hipHostFree(h_up));
                h_up = nullptr;
                h_up_bytes = 0;
                HIPCHK(hipHostMalloc(&h_up, nb, hipHostMallocDefault));
                h_up_bytes = nb;
            }
        }
        char *p = (char *)h_up + h_up_used;
        std::memcpy(p, src, bytes);
        HIPCHK(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, s));
        h_up_used = std::min(h_up_bytes, (h_up_used + bytes + 255) & ~size_t(255));
    }
    void uploads_done() { h_up_used = 0; }
    hipEvent_t ev[16] = {};
    // Side streams (default priority) on which the launches of one pipeline
    // step run side by side, joined to the stage's stream by events.
    static constexpr int kSide = 4;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    bool init = false;
    void setup() {
        if (init) return;
        HIPCHK(hipHostMalloc((void **)&h_ctr, sizeof(DevCounters) * 2, hipHostMallocDefault));
        for (auto &e : ev) HIPCHK(hipEventCreate(&e));
        for (auto &q : side) HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        for (auto &e : join) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        init = true;
    }
    // Count every buffer's device bytes in `a`.
    void account(DevBytes *a) {
        DBuf *all[] = {&units, &items, &comp_off, &comp_blocks, &mask, &snap, &log, &alt, &rlog,
                       &ralt, &fs, &hist, &part, &faults, &rfaults, &races, &edges, &blk_recs,
                       &rblk_recs, &blk_flags, &rflags, &ctr, &rctr, &wlog, &lraces, &rlraces, &longseg, &covlist,
                       &rtable, &ftable, &downer, &dflags, &blk_instr, &blk_grecs, &blk_log, &blk_held, &blk_off,
                       &sctr, &stctr, &sncomp};
        for (auto *b : all) b->acct = a;
    }
    // Forget every carved buffer (the arena restarts at each call).
    void forget_carved() {
        DBuf *all[] = {&units, &items, &comp_off, &comp_blocks, &mask, &snap, &log, &alt, &rlog,
                       &ralt, &fs, &hist, &part, &faults, &rfaults, &races, &edges, &blk_recs,
                       &rblk_recs, &blk_flags, &rflags, &ctr, &rctr, &wlog, &lraces, &rlraces, &longseg, &covlist,
                       &rtable, &ftable, &downer, &dflags, &blk_instr, &blk_grecs, &blk_log, &blk_held, &blk_off,
                       &sctr, &stctr, &sncomp};
        for (auto *b : all)
            if (b->carved) b->release();
    }
    size_t device_bytes() const {
        const DBuf *all[] = {&units, &items, &comp_off, &comp_blocks, &mask, &snap, &log, &alt, &rlog,
                             &ralt, &fs, &hist, &part, &faults, &rfaults, &races, &edges, &blk_recs,
                             &rblk_recs, &blk_flags, &rflags, &ctr, &rctr, &wlog, &lraces, &rlraces, &longseg, &covlist,
                             &rtable, &ftable, &downer, &dflags, &blk_instr, &blk_grecs, &blk_log, &blk_held, &blk_off,
                       &sctr, &stctr, &sncomp};
        size_t s = 0;
        for (auto *b : all) s += b->bytes;
        return s;
    }
    ~Workspace() {
        DBuf *all[] = {&units, &items, &comp_off, &comp_blocks, &mask, &snap, &log, &alt, &rlog,
                       &ralt, &fs, &hist, &part, &faults, &rfaults, &races, &edges, &blk_recs,
                       &rblk_recs, &blk_flags, &rflags, &ctr, &rctr, &wlog, &lraces, &rlraces, &longseg, &covlist,
                       &rtable, &ftable, &downer, &dflags, &blk_instr, &blk_grecs, &blk_log, &blk_held, &blk_off,
                       &sctr, &stctr, &sncomp};
        for (auto *b : all) b->release();
        if (h_ctr) (void)hipHostFree(h_ctr);
        if (h_pin) (void)hipHostFree(h_pin);
        if (h_up) (void)hipHostFree(h_up);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &q : side)
            if (q) (void)hipStreamDestroy(q);
        if (fork) (void)hipEventDestroy(fork);
        for (auto &e : join)
            if (e) (void)hipEventDestroy(e);
    }
};

// One (job, launch) inside a stage.
struct UnitIn {
    const kc_launch_desc *desc;
    int32_t *mem;
    uint64_t n_words;
};

struct UnitOut {
    uint64_t records = 0;
    bool deadlocked = false;
    std::vector<kc_race> races;     // launch field filled by the caller
    std::vector<kc_race_site> sites;    // parallel to races (option sites), else empty
    std::vector<kc_fault> faults;
};

struct Options {
    int check = 1;
    uint32_t fuel = 1u << 20;
    int timing = 0;
    uint32_t sort_tile = 2048;
    uint32_t sort_bits = 8;         // radix digit width of the sort's passes
    uint32_t side_streams = 4;      // side streams over which a step's launches are spread
    uint64_t log_records = 1ull << 22;
    uint32_t stage = 256;           // staged records per wave in the lockstep replay
    uint32_t stage_bytes = 8192;    // LDS for staging + local sort per workgroup (free run)
    int local = 1;                  // epoch-local check in LDS
    int shadow_global = 1;          // ... with global locations in an LDS shadow table (0: stage and sort)
    int hash_check = 1;             // conflict-free logs checked through a location table, without sorting
    int jit = 0;                    // program-specialised free-run kernels (compiled at first use)
    int jit_waves = 0;              // their occupancy target, waves per SIMD (0: the compiler's choice)
    int sites = 0;                  // source sites of races (one more replay of the racy blocks)
    int uninit = 0;                 // UNINIT findings for loads of shared words not yet stored to
    int warp = 0;                   // warp-aware model: accesses of one warp conflict only at the same step
    int queue_replay = 1;           // replay of the free run's racy blocks queued behind it
    int onesweep = 0;               // large sorts: single-pass digit scatters (decoupled look-back)
    int loc_sort = 1;               // large free-run logs of representatives only: sorted by location
    uint32_t sort_spin = 1u << 16;  // bound of each look-back wait, in polls
    int arena = 0;                  // set by the library: buffers come from the static scratch area
};

}  // namespace

struct Batch;
struct ScratchDevice;

struct kc_ctx {
    int device = 0;
    ScratchDevice *scratch = nullptr;           // the device's static scratch area (kc_launch_noalloc)
    std::unique_ptr<Workspace> fixed_ws;        // its workspace: events and host staging made at creation
    uint64_t budget = 0;
    Options opt;
    std::string err;
    std::atomic<bool> poisoned{false};
    std::mutex mu;
    std::vector<std::unique_ptr<Workspace>> free_ws;
    std::unordered_map<std::string, double> stats;
    std::map<uint64_t, std::shared_ptr<Batch>> batches;
    uint64_t next_ticket = 1;
    DevBytes bytes;                             // device bytes of every workspace and summary
    std::unique_ptr<Workspace> acquire() {
        std::lock_guard<std::mutex> g(mu);
        if (!free_ws.empty()) {
            auto w = std::move(free_ws.back());
            free_ws.pop_back();
            return w;
        }
        auto w = std::make_unique<Workspace>();
        w->account(&bytes);
        return w;
    }
    // Would `extra` more device bytes exceed the budget?  Idle workspaces
    // (kept for reuse by later calls) are freed first.
    bool over_budget(uint64_t extra = 0) {
        if (!budget) return false;
        if ((uint64_t)std::max<int64_t>(bytes.live.load(), 0) + extra <= budget) return false;
        std::vector<std::unique_ptr<Workspace>> idle;
        {
            std::lock_guard<std::mutex> g(mu);
            idle.swap(free_ws);
        }
        if (!idle.empty()) stat_add("budget_trims", (double)idle.size());
        idle.clear();
        return (uint64_t)std::max<int64_t>(bytes.live.load(), 0) + extra > budget;
    }
    void release(std::unique_ptr<Workspace> w) {
        std::lock_guard<std::mutex> g(mu);
        free_ws.push_back(std::move(w));
    }
    uint64_t log_hint() {
        std::lock_guard<std::mutex> g(mu);
        return opt.log_records;
    }
    // A copy of the options for one call: kc_ctx_set_option may run while a
    // batch works.
    Options options() {
        std::lock_guard<std::mutex> g(mu);
        return opt;
    }
    void note_log_records(uint64_t n) {
        std::lock_guard<std::mutex> g(mu);
        opt.log_records = std::max(opt.log_records, n);
    }
    // Capacities of the log and race list of the replay queued behind the
    // free run, grown to what earlier stages needed.
    // and of its grid: the number of racy blocks the last such stage had
    uint64_t spec_log_hint = 1u << 14;
    uint32_t spec_race_hint = 4096, spec_grid_hint = 64;
    void spec_caps(uint64_t &log, uint32_t &races, uint32_t &grid) {
        std::lock_guard<std::mutex> g(mu);
        log = spec_log_hint;
        races = spec_race_hint;
        grid = spec_grid_hint;
    }
    // Programs whose last queued replay could not stand (its launch needed a
    // sorted check) skip it for their next stages, trying again now and then.
    std::unordered_map<const void *, uint32_t> spec_backoff;
    bool spec_skip(const void *prog) {
        std::lock_guard<std::mutex> g(mu);
        auto it = spec_backoff.find(prog);
        if (it == spec_backoff.end() || it->second == 0) return false;
        it->second--;
        return true;
    }
    void note_spec_failed(const void *prog) {
        std::lock_guard<std::mutex> g(mu);
        spec_backoff[prog] = 16;
    }
    void note_spec(uint64_t log, uint32_t races, uint32_t comps) {
        std::lock_guard<std::mutex> g(mu);
        spec_log_hint = std::max<uint64_t>(spec_log_hint, log + log / 4 + 1024);
        spec_race_hint = std::max<uint32_t>(spec_race_hint, races + races / 4 + 1024);
        spec_grid_hint = std::max<uint32_t>(64, comps + comps / 4);
    }
    // Capacities of the finding and local-race lists, grown to what earlier
    // stages needed so that a repeated workload does not interpret twice.
    uint32_t fault_hint = 4096, lrace_hint = 4096;
    void caps(uint32_t &faults, uint32_t &lraces) {
        std::lock_guard<std::mutex> g(mu);
        faults = fault_hint;
        lraces = lrace_hint;
    }
    void note_caps(uint32_t faults, uint32_t lraces) {
        std::lock_guard<std::mutex> g(mu);
        fault_hint = std::max(fault_hint, faults);
        lrace_hint = std::max(lrace_hint, lraces);
    }
    void stat_add(const char *k, double v) {
        std::lock_guard<std::mutex> g(mu);
        stats[k] += v;
    }
    void stat_max(const char *k, double v) {
        std::lock_guard<std::mutex> g(mu);
        stats[k] = std::max(stats[k], v);
    }
};

// Launches per job when streams or dependencies are given (the launch order
// is kept as one bit per pair).
constexpr uint32_t kMaxStreamLaunches = 4096;

// Steps of a job: its items when it has a host program, else its launches.
uint32_t job_steps(const kc_job &job) { return job.items ? job.n_items : job.n_launches; }
// The launch step i runs, or nullptr for a copy or host step.
const kc_launch_desc *step_launch(const kc_job &job, uint32_t i) {
    if (!job.items) return &job.launches[i];
    return job.items[i].kind == KC_ITEM_LAUNCH ? &job.launches[job.items[i].ref] : nullptr;
}
// Launches and copies run on the device, in streams; the rest on the host.
bool device_item(const kc_job &job, uint32_t i) {
    return !job.items || job.items[i].kind == KC_ITEM_LAUNCH || job.items[i].kind == KC_ITEM_COPY;
}

struct Batch {
    std::vector<kc_job> jobs;
    std::vector<std::vector<kc_launch_desc>> descs;
    std::vector<std::vector<uint32_t>> streams;
    std::vector<std::vector<kc_dep>> deps;
    std::vector<std::vector<kc_region>> allocs;
    std::vector<std::vector<kc_item>> items;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::once_flag joined;
    std::mutex mu;
    std::condition_variable cv;
    bool done = false;
    bool collected = false;         // a kc_poll took the reports (under mu)
    // Join the worker exactly once, whichever of kc_poll and kc_ctx_destroy
    // gets here first (joining a thread twice throws).
    void join() {
        std::call_once(joined, [this] {
            if (worker.joinable()) worker.join();
        });
    }
    kc_status status = KC_OK;
    std::string err;
    std::vector<kc_report *> reports;
};

namespace {

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
bool valid_opcode(uint32_t op) {
    const uint32_t base = op & ~uint32_t(OP_IMM);
    if (base >= OP_ADD && base <= OP_SLTU) return true;
    switch (op) {
    case OP_MOV: case OP_MOVI: case OP_SREG: case OP_LDS: case OP_STS: case OP_LDG: case OP_STG:
    case OP_JMP: case OP_BZ: case OP_BNZ: case OP_BAR: case OP_EXIT: case OP_BARP:
        return true;
    default:
        return false;
    }
}

std::string validate_program(const uint64_t *w, uint32_t n) {
    if (n == 0 || n > MAX_INSTR) return "program length must be in [1, 65536]";
    for (uint32_t pc = 0; pc < n; pc++) {
        const uint32_t op = w[pc] & 0xFF, d = (w[pc] >> 8) & 0xFF, a = (w[pc] >> 16) & 0xFF,
                       b = (w[pc] >> 24) & 0xFF;
        const int32_t imm = (int32_t)(uint32_t)(w[pc] >> 32);
        if (!valid_opcode(op)) return "unknown opcode at pc " + std::to_string(pc);
        if (d >= 16 || a >= 16 || b >= 16) return "register out of range at pc " + std::to_string(pc);
        if ((op == OP_JMP || op == OP_BZ || op == OP_BNZ) && (imm < 0 || (uint32_t)imm > n))
            return "branch target out of range at pc " + std::to_string(pc);
        if (op == OP_SREG && (imm < 0 || (uint32_t)imm >= N_SREGS))
            return "special register out of range at pc " + std::to_string(pc);
        if (op == OP_BARP && (imm < 0 || imm > 2))
            return "barrier predicate kind out of range at pc " + std::to_string(pc);
    }
    return "";
}

std::string validate_desc(const kc_launch_desc *d, int32_t *mem, uint64_t n_words) {
    if (!d || !d->prog) return "launch without a program";
    const uint64_t nt = (uint64_t)d->block.x * d->block.y * d->block.z;
    const uint64_t nb = (uint64_t)d->grid.x * d->grid.y * d->grid.z;
    if (nt == 0 || nt > MAX_THREADS) return "threads per block must be in [1, 1024]";
    if (nb == 0 || nb * nt > 0xFFFFFFFFull) return "grid must be non-empty and blocks*threads < 2^32";
    if (d->shmem_bytes % 4 || d->shmem_bytes / 4 > MAX_SHMEM_WORDS) return "shmem_bytes must be a multiple of 4, <= 65536";
    if (d->n_params > 8) return "at most 8 params";
    if (!mem && n_words) return "null device memory";
    if (n_words >= (1ull << 31)) return "memory must be < 2^31 words";
    return "";
}

// ---------------------------------------------------------------------------
// union-find for racy components
// ---------------------------------------------------------------------------
bool fault_less(const kc_fault &x, const kc_fault &y) {
    const uint32_t kx[8] = {x.launch, x.block, x.epoch, x.kind, x.a, x.b, x.c, x.d};
    const uint32_t ky[8] = {y.launch, y.block, y.epoch, y.kind, y.a, y.b, y.c, y.d};
    return std::lexicographical_compare(kx, kx + 8, ky, ky + 8);
}
bool fault_eq(const kc_fault &x, const kc_fault &y) { return !fault_less(x, y) && !fault_less(y, x); }
// (launch, space, scope, block, epoch, addr), compared as three 64-bit words
// (space < 2 and scope < 4): a whole step's races are sorted on the host.
bool race_less(const kc_race &x, const kc_race &y) {
    const uint64_t ax = (uint64_t)x.launch << 32 | x.space << 2 | x.scope;
    const uint64_t ay = (uint64_t)y.launch << 32 | y.space << 2 | y.scope;
    if (ax != ay) return ax < ay;
    const uint64_t bx = (uint64_t)x.block << 32 | x.epoch, by = (uint64_t)y.block << 32 | y.epoch;
    if (bx != by) return bx < by;
    return x.addr < y.addr;
}

// The races of one unit and launch into canonical order.  When space,
// scope, block, epoch and address fit one 64-bit key at their widths (the
// usual case), an LSD radix sort with 8-bit digits over that key's bits
// orders positions; otherwise (or for short lists) a comparison sort.
void sort_races(std::vector<kc_race> &v) {
    const size_t n = v.size();
    if (n < 64) {
        std::stable_sort(v.begin(), v.end(), race_less);
        return;
    }
    uint32_t mb = 0, me = 0, ma = 0, ms = 0;
    for (auto &r : v) {
        mb = std::max(mb, r.block);
        me = std::max(me, r.epoch);
        ma = std::max(ma, r.addr);
        ms = std::max(ms, (r.space << 2) | r.scope);
    }
    auto width = [](uint64_t m) {
        uint32_t b = 0;
        while (b < 64 && (m >> b)) b++;
        return b;
    };
    const uint32_t bb = width(mb), eb = width(me), ab = width(ma), sb = width(ms);
    if (v[0].launch != v[n - 1].launch || bb + eb + ab + sb > 64) {
        std::stable_sort(v.begin(), v.end(), race_less);
        return;
    }
    auto shl = [](uint64_t x, uint32_t s) { return s >= 64 ? 0ull : x << s; };
    std::vector<uint64_t> key(n), key2(n);
    std::vector<uint32_t> pos(n), pos2(n);
    for (size_t i = 0; i < n; i++) {
        const kc_race &r = v[i];
        key[i] = shl((r.space << 2) | r.scope, bb + eb + ab) | shl(r.block, eb + ab) | shl(r.epoch, ab) | r.addr;
        pos[i] = (uint32_t)i;
    }
    const uint32_t total = bb + eb + ab + sb;
    uint32_t cnt[256];
    for (uint32_t sh = 0; sh < total; sh += 8) {
        std::memset(cnt, 0, sizeof cnt);
        for (size_t i = 0; i < n; i++) cnt[(key[i] >> sh) & 255u]++;
        uint32_t at = 0;
        for (uint32_t d = 0; d < 256; d++) {
            const uint32_t c = cnt[d];
            cnt[d] = at;
            at += c;
        }
        for (size_t i = 0; i < n; i++) {
            const uint32_t to = cnt[(key[i] >> sh) & 255u]++;
            key2[to] = key[i];
            pos2[to] = pos[i];
        }
        key.swap(key2);
        pos.swap(pos2);
    }
    std::vector<kc_race> out(n);
    for (size_t i = 0; i < n; i++) out[i] = v[pos[i]];
    v.swap(out);
}

// Host time of a section, added to statistic `key` when timing is on.
struct HostTimer {
    kc_ctx *ctx;
    const char *key;
    bool on;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    ~HostTimer();
};

// Stage times from HIP events on the launch stream: level 1 times every
// stage; level 2 only the free run (marks 0 and 1), since every recorded
// event costs the stream a short pause.
struct Timer {
    kc_ctx *ctx;
    Workspace &ws;
    hipStream_t s;
    int level;
    int idx = 0;
    bool on(int i) const { return level == 1 || (level == 2 && (i == 0 || i == 1)); }
    void mark(int i) {
        if (on(i)) HIPCHK(hipEventRecord(ws.ev[i], s));
    }
    double ms(int a, int b) {
        if (!on(a) || !on(b)) return 0.0;
        float v = 0.f;
        HIPCHK(hipEventSynchronize(ws.ev[b]));
        HIPCHK(hipEventElapsedTime(&v, ws.ev[a], ws.ev[b]));
        return v;
    }
};

HostTimer::~HostTimer() {
    if (on) ctx->stat_add(key, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
}

// ---------------------------------------------------------------------------
// one stage
// ---------------------------------------------------------------------------
struct Stage {
    kc_ctx *ctx;
    Workspace &ws;
    hipStream_t s;
    const std::vector<UnitIn> &in;
    std::vector<UnitOut> &out;
    const Options &opt;     // the options as they were when the call began

    std::vector<DevUnit> hu;
    KeyPlan kp{};
    uint32_t total_blocks = 0;
    uint64_t total_words = 0;
    uint32_t max_words = 0;
    uint32_t used_epoch_bits = 0;
    uint32_t lrace_cap = 4096;
    uint32_t racy_words = 0;        // shared words the free run's verdicts found racy
    uint32_t wlog_cap = 0;          // warp-aware model: capacity of the replay's stepped accesses (0: off)

    // Sort order for the check: bits from the block field up, then the used
    // epoch bits; the full order for multiset comparison adds tid and kind.
    VKey check_key() const { return VKey{kp.s_ep, used_epoch_bits, kp.s_blk, 0, used_epoch_bits + (kp.total - kp.s_blk)}; }
    VKey full_key() const {
        return VKey{kp.s_ep, used_epoch_bits, kp.s_blk, kp.s_ep, kp.s_ep + used_epoch_bits + (kp.total - kp.s_blk)};
    }
    std::vector<uint32_t> blk_recs;
    // Queue the free run's conflict check through location tables (see
    // launch_log_table) behind the free run, for a log of up to `cap`
    // records whose count the kernels read on the device.  Memories small
    // next to the log get one table entry per memory word (two passes of
    // plain stores), others a hash table of locations.  Flags go to ws.rctr.
    bool qt_direct = false;
    uint32_t qt_bits = 0;
    bool queue_log_check(uint64_t cap, hipStream_t q) {
        // representatives exist only with the epoch-local check; a very long
        // log would spend more on its table than on the sort
        const bool direct = total_words <= 4 * cap + (1u << 16);
        if (!(opt.hash_check && opt.local && cap <= (1ull << 24) && (direct || table_obits() != 0)))
            return false;
        uint32_t bits = 10;
        while ((1ull << bits) < 2 * cap) bits++;
        ws.rctr.reserve(sizeof(DevCounters));     // zeroed by the table launch
        ReplayTableArgs ta{};
        ta.rs = ws.log.as<uint64_t>();
        ta.n_rs = cap;
        ta.n_dev = &ws.ctr.as<DevCounters>()->log_count;
        ta.kp = kp;
        ta.units = ws.units.as<DevUnit>();
        ta.ctr = ws.rctr.as<DevCounters>();
        if (direct) {
            ws.downer.reserve(std::max<uint64_t>(total_words, 1) * 4);
            ws.dflags.reserve((std::max<uint64_t>(total_words, 1) + 3) / 4 * 4);
            ta.snap_base = ws.snap.as<int32_t>();
            ta.downer = ws.downer.as<uint32_t>();
            ta.dflags = ws.dflags.as<uint8_t>();
            HIPCHK(launch_log_direct(ta, total_words, q));
        } else {
            ws.ftable.reserve((size_t)8 << bits);
            ta.table = ws.ftable.p;
            ta.bits = bits;
            ta.obits = table_obits();
            HIPCHK(launch_log_table(ta, q));
        }
        qt_direct = direct;
        qt_bits = bits;
        return true;
    }

    // Width of the block field in a location-table word (a global block index
    // + 1), or 0 when location, block and flags do not fit 64 bits.
    uint32_t table_obits() const {
        const uint32_t ob = bits_for((uint64_t)total_blocks + 1);
        return (kp.total - kp.s_addr) + ob + 2 <= 63 ? ob : 0u;
    }
    // Where the canonical accesses of the stage are once run() returns: the
    // free-run log less the blocks flagged in ws.blk_flags (replayed) or the
    // units flagged in ws.mask (replayed whole), plus the replay's records.
    const uint64_t *fin_log = nullptr;
    uint64_t fin_n = 0;
    const uint64_t *rep_log = nullptr;
    uint64_t rep_n = 0;
    bool skip_flagged = false, skip_masked = false;
    std::vector<std::vector<uint2>> replayed;   // the components the replay ran (whole units: skip_masked)
    SiteSlot *site_table = nullptr;             // set during the source-site replay
    uint32_t site_bits = 0;
    bool held_regions = false;      // free run: held representatives in per-block regions
    bool log_sorted = false;        // the free-run log was sorted for its check
    uint32_t ftable_bits = 0;       // else: log2 slots of its location table (ws.ftable),
    bool direct_tables = false;     // or its direct word tables (ws.downer, ws.dflags)

    // Device-to-host copies gathered into the pinned staging buffer and
    // completed with one synchronisation (each one costs a round trip with the
    // device idle).  Results are valid until the next fetch.
    struct Fetch {
        struct Item { const void *dev; size_t bytes, off; };
        std::vector<Item> items;
        size_t total = 0;
        size_t add(const void *dev, size_t bytes) {
            const size_t off = (total + 255) & ~size_t(255);
            items.push_back(Item{dev, bytes, off});
            total = off + bytes;
            return items.size() - 1;
        }
    };
    // One gather kernel writes every item straight into the pinned buffer
    // (its device mapping); items are whole words at 256-byte offsets.
    void run_fetch(Fetch &f) {
        ws.pin_reserve(f.total);
        GatherArgs g{};
        for (auto &it : f.items) {
            if (!it.bytes) continue;
            g.src[g.n] = (const uint32_t *)it.dev;
            g.words[g.n] = (uint32_t)(it.bytes / 4);
            g.dst_off[g.n] = (uint32_t)(it.off / 4);
            if (++g.n == GATHER_MAX) {
                g.dst = (uint32_t *)ws.d_pin;
                HIPCHK(launch_gather(g, s));
                g.n = 0;
            }
        }
        if (g.n) {
            g.dst = (uint32_t *)ws.d_pin;
            HIPCHK(launch_gather(g, s));
        }
        {
            HostTimer wt{ctx, "host_fetch_wait_ms", opt.timing != 0};
            HIPCHK(hipStreamSynchronize(s));
        }
        ws.uploads_done();
    }
    template <class T> const T *fetched(const Fetch &f, size_t i) const {
        return (const T *)((const char *)ws.h_pin + f.items[i].off);
    }
    // Entries speculatively fetched with their counts; more need a second trip.
    static constexpr uint32_t kSpec = 512;
    // the queued replay's race list holds every exact tuple: more ride along
    static constexpr uint32_t kSpecRaces = 4096;
    template <class T> void take_list(const Fetch &f, size_t item, uint32_t count, uint32_t cap, const void *dev,
                                      std::vector<T> &out, uint32_t fetched_n = kSpec) {
        const uint32_t n = std::min(count, cap);
        out.resize(n);
        const uint32_t first = std::min(n, fetched_n);
        if (first) std::memcpy(out.data(), fetched<T>(f, item), (size_t)first * sizeof(T));
        if (n > first) {
            HIPCHK(hipMemcpyAsync(out.data() + first, (const T *)dev + first, (size_t)(n - first) * sizeof(T),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
    }

    // Launches side by side: fork() makes the side streams wait for the work
    // queued on the stage's stream so far; launch i goes to side(i); join()
    // makes the stage's stream wait for every side stream used.
    uint32_t side_used = 0;
    void fork() {
        HIPCHK(hipEventRecord(ws.fork, s));
        side_used = 0;
    }
    hipStream_t side(uint32_t i) {
        const uint32_t k = i % std::max<uint32_t>(1, std::min<uint32_t>(opt.side_streams, Workspace::kSide));
        if (k >= side_used) {
            for (uint32_t q = side_used; q <= k; q++) HIPCHK(hipStreamWaitEvent(ws.side[q], ws.fork, 0));
            side_used = k + 1;
        }
        return ws.side[k];
    }
    void join() {
        for (uint32_t q = 0; q < side_used; q++) {
            HIPCHK(hipEventRecord(ws.join[q], ws.side[q]));
            HIPCHK(hipStreamWaitEvent(s, ws.join[q], 0));
        }
        side_used = 0;
    }

    // Components of the replay grouped by program (contiguous in the uploaded
    // component list): each group runs on that program's specialised replay
    // kernels, the groups side by side.
    struct CompGroup {
        uint32_t first, count, unit, wg, shmax;
    };
    std::vector<CompGroup> comp_groups;

    // The replay of the free run's racy blocks queued behind it, before the
    // host has seen any result: the blocks the free run flagged are listed
    // on the device (each its own component), their free-run writes put
    // back, and they are replayed and checked for exactness; the results come
    // back with the free run's.  They stand when the log needs no sorted
    // check and nothing overflowed (every racy block then was flagged by the
    // free run and is its own component); otherwise the stage runs again
    // from the launch start without it.  Used when every unit runs one
    // program (one replay kernel) and the replay's tables apply.
    bool spec = false, spec_off = false, spec_ok = false;
    uint32_t spec_ncomp = 0;                    // blocks the queued replay ran
    DevCounters spec_counters{};
    const uint32_t *spec_ncomps = nullptr;      // set while the queued replay is launched
    uint64_t spec_rcap = 0;
    uint32_t spec_fcap = 0, spec_rlcap = 0;
    bool spec_allowed() const {
        if (!opt.queue_replay || !opt.check || !opt.local || opt.warp || opt.sites || opt.arena || site_table)
            return false;
        if (!total_blocks || table_obits() == 0) return false;
        for (auto &u : in)
            if (u.desc->prog != in[0].desc->prog) return false;
        return !ctx->spec_skip(in[0].desc->prog);
    }
    // With `tables_aside` the free-run log's tables are being built on a side
    // stream: joined before the exactness tables, which read them.
    void queue_spec_replay(uint64_t log_cap, uint32_t fault_cap, Timer &tm, bool tables_aside) {
        tm.mark(5);
        uint32_t grid_hint = 64;
        ctx->spec_caps(spec_rcap, spec_rlcap, grid_hint);
        spec_fcap = fault_cap;
        ws.comp_blocks.reserve((size_t)total_blocks * sizeof(uint2));
        ws.sncomp.reserve(4);
        ws.sctr.reserve(sizeof(DevCounters));
        ws.stctr.reserve(sizeof(DevCounters));
        HIPCHK(launch_restore(ws.log.as<uint64_t>(), log_cap, kp, ws.units.as<DevUnit>(),
                              ws.blk_flags.as<uint32_t>(), s, &ws.ctr.as<DevCounters>()->log_count));
        ws.rblk_recs.reserve((size_t)total_blocks * 4);
        ws.rflags.reserve((size_t)total_blocks * 4);
        ws.rlog.reserve(spec_rcap * 8);
        ws.rfaults.reserve((size_t)spec_fcap * sizeof(DevFault));
        ws.rlraces.reserve((size_t)spec_rlcap * sizeof(DevRace));
        {   // the replay's counters and per-block counts are cleared by the same workgroup
            ZeroArgs z{{ws.sctr.as<uint32_t>(), ws.rblk_recs.as<uint32_t>()},
                       {sizeof(DevCounters) / 4, (size_t)total_blocks}, 2};
            HIPCHK(launch_flagged_comps(ws.blk_flags.as<uint32_t>(), total_blocks, ws.units.as<DevUnit>(),
                                        (uint32_t)hu.size(), ws.comp_blocks.as<uint2>(), ws.sncomp.as<uint32_t>(), s,
                                        &z));
        }
        uint32_t wg = 64, shmax = 0;
        for (auto &u : hu) {
            wg = std::max<uint32_t>(wg, (u.nt + 63) / 64 * 64);
            shmax = std::max(shmax, u.sh_words);
        }
        // about as many workgroups as the last such stage had racy blocks
        // (the workgroups stride over the list, so more blocks only take
        // longer; idle workgroups exit at once)
        const uint32_t grid = std::min<uint32_t>(total_blocks, std::min<uint32_t>(grid_hint, 1024));
        comp_groups.assign(1, CompGroup{0, grid, 0, wg, shmax});
        spec_ncomps = ws.sncomp.as<uint32_t>();
        wlog_cap = 0;
        interp(true, ws.rlog, spec_rcap, ws.sctr, ws.rfaults, spec_fcap, ws.rblk_recs, grid, ws.rlraces, spec_rlcap,
               ws.rflags);
        spec_ncomps = nullptr;
        uint32_t bits = 10;
        while ((1ull << bits) < 2 * spec_rcap) bits++;
        ws.rtable.reserve((size_t)8 << bits);
        ReplayTableArgs ta{ws.rlog.as<uint64_t>(), spec_rcap, ws.log.as<uint64_t>(), log_cap, kp,
                           ws.units.as<DevUnit>(), ws.blk_flags.as<uint32_t>(), ws.rtable.p, bits,
                           ws.stctr.as<DevCounters>(), qt_direct ? nullptr : ws.ftable.p, qt_direct ? 0u : qt_bits,
                           table_obits(), ws.snap.as<int32_t>(), qt_direct ? ws.downer.as<uint32_t>() : nullptr,
                           ws.dflags.as<uint8_t>(), nullptr};
        ta.n_dev = &ws.sctr.as<DevCounters>()->log_count;
        if (tables_aside) join();
        HIPCHK(launch_replay_table(ta, s));
        tm.mark(7);
    }

    DevCounters read_ctr(DBuf &c) {
        HIPCHK(hipMemcpyAsync(ws.h_ctr, c.p, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return *ws.h_ctr;
    }

    void plan() {
        const uint32_t n = (uint32_t)in.size();
        hu.resize(n);
        uint64_t max_nt = 1, max_nb = 1, max_addr = 1;
        total_blocks = 0;
        total_words = 0;
        for (uint32_t i = 0; i < n; i++) {
            const kc_launch_desc *d = in[i].desc;
            DevUnit &u = hu[i];
            std::memset(&u, 0, sizeof(u));
            u.prog = d->prog->dev;
            u.mem = in[i].mem;
            u.n_instr = (uint32_t)d->prog->words.size();
            u.n_words = (uint32_t)in[i].n_words;
            u.gdim[0] = d->grid.x; u.gdim[1] = d->grid.y; u.gdim[2] = d->grid.z;
            u.bdim[0] = d->block.x; u.bdim[1] = d->block.y; u.bdim[2] = d->block.z;
            u.nt = d->block.x * d->block.y * d->block.z;
            u.nb = d->grid.x * d->grid.y * d->grid.z;
            u.sh_words = d->shmem_bytes / 4;
            u.fuel = opt.fuel;
            for (uint32_t p = 0; p < 8; p++) u.params[p] = p < d->n_params ? d->params[p] : 0;
            u.block_base = total_blocks;
            total_blocks += u.nb;
            total_words += u.n_words;
            max_words = std::max(max_words, u.n_words);
            max_nt = std::max<uint64_t>(max_nt, u.nt);
            max_nb = std::max<uint64_t>(max_nb, u.nb);
            max_addr = std::max<uint64_t>(max_addr, std::max<uint64_t>(u.n_words, u.sh_words));
        }
        kp.tb = bits_for(max_nt);
        kp.bb = bits_for(max_nb);
        kp.ab = bits_for(max_addr);
        kp.ub = bits_for(n);
        const int used = 1 + (int)kp.tb + (int)kp.bb + (int)kp.ab + 1 + (int)kp.ub;
        int eb = std::min(63 - used, 24);   // keep every shift below 64
        if (eb < 1)
            throw KcError{KC_E_OVERFLOW, "record fields need more than 64 bits (" + std::to_string(used) + " + epoch)"};
        kp.eb = (uint32_t)eb;
        kp.s_tid = 1;
        kp.s_ep = kp.s_tid + kp.tb;
        kp.s_blk = kp.s_ep + kp.eb;
        kp.s_addr = kp.s_blk + kp.bb;
        kp.s_sp = kp.s_addr + kp.ab;
        kp.s_unit = kp.s_sp + 1;
        kp.total = kp.s_unit + kp.ub;
        kp.ep_rep = (uint32_t)((1ull << kp.eb) - 1);
        kp.max_epoch = kp.ep_rep - 1;
    }

    // Records staged per wave: the LDS budget split over the workgroup's waves
    // (staging + the epoch-local sort's second buffer), a multiple of 64;
    // workgroups of fewer than four waves count as four (a small block needs
    // no more staging per wave, and less LDS lets more of them share a CU).
    uint32_t stage_for(uint32_t wg_threads) const {
        const uint32_t nw = std::max<uint32_t>((wg_threads + 63) / 64, 4u);
        uint32_t st = (uint32_t)(opt.stage_bytes / (nw * 16u)) / 64u * 64u;
        return std::max<uint32_t>(64u, std::min<uint32_t>(st, 2048u));
    }

    // More barrier epochs than the record's epoch field holds: every unit's
    // memory goes back to the launch-start snapshot, so that the caller can
    // run the units again in smaller groups (wider epoch fields).
    [[noreturn]] void epoch_overflow() {
        HIPCHK(launch_copy_units(ws.units.as<DevUnit>(), (uint32_t)hu.size(), max_words, false, nullptr, s));
        HIPCHK(hipStreamSynchronize(s));
        throw KcError{KC_E_OVERFLOW, "barrier epochs exceed the record's epoch field"};
    }

    void upload_units() {
        ws.units.reserve(hu.size() * sizeof(DevUnit));
        ws.upload(ws.units.p, hu.data(), hu.size() * sizeof(DevUnit), s);
    }

    void reset_counters(DBuf &c) {
        c.reserve(sizeof(DevCounters));
        HIPCHK(launch_zero(c.p, sizeof(DevCounters), s));
    }

    // Interpreter launches for all units, grouped by workgroup size.
    void interp(bool lockstep, DBuf &logbuf, uint64_t log_cap, DBuf &ctr, DBuf &faults, uint32_t fault_cap,
                DBuf &recs, uint32_t n_comp, DBuf &lrace_buf, uint32_t lrace_cap_, DBuf &flags) {
        InterpArgs a{};
        a.units = ws.units.as<DevUnit>();
        a.kp = kp;
        a.log = logbuf.as<uint64_t>();
        a.log_cap = log_cap;
        a.log_count = &ctr.as<DevCounters>()->log_count;
        a.faults = faults.as<DevFault>();
        a.fault_cap = fault_cap;
        a.fault_count = &ctr.as<DevCounters>()->fault_count;
        a.blk_recs = recs.as<uint32_t>();
        a.flags = &ctr.as<DevCounters>()->flags;
        a.max_epoch = &ctr.as<DevCounters>()->max_epoch;
        a.stage = opt.stage;
        a.local = (opt.check && opt.local) ? 1u : 0u;
        a.lraces = lrace_buf.as<DevRace>();
        a.lrace_cap = lrace_cap_;
        a.lrace_count = &ctr.as<DevCounters>()->race_count;
        a.blk_flags = flags.as<uint32_t>();
        a.uninit = opt.uninit ? 1u : 0u;
        if (lockstep && wlog_cap) {
            a.wlog = ws.wlog.as<WarpRec>();
            a.wlog_cap = wlog_cap;
            a.wlog_count = &ctr.as<DevCounters>()->wlog_count;
        }
        a.racy_words = lockstep ? nullptr : &ctr.as<DevCounters>()->racy_words;
        a.blk_instr = lockstep ? nullptr : ws.blk_instr.as<uint32_t>();
        a.blk_grecs = lockstep ? nullptr : ws.blk_grecs.as<uint32_t>();
        a.blk_log = (!lockstep && held_regions) ? ws.blk_log.as<uint64_t>() : nullptr;
        a.blk_held = (!lockstep && held_regions) ? ws.blk_held.as<uint32_t>() : nullptr;
        // the global shadow table packs a location in 31 bits
        const bool gst = a.local && opt.shadow_global && kp.ab <= 31;
        if (lockstep) {
            a.stage = opt.stage;
            uint32_t wg = 64, shmax = 0;
            for (auto &u : hu) {
                wg = std::max<uint32_t>(wg, (u.nt + 63) / 64 * 64);
                shmax = std::max(shmax, u.sh_words);
            }
            a.comp_off = ws.comp_off.as<uint32_t>();
            a.comp_blocks = ws.comp_blocks.as<uint2>();
            a.n_comps_dev = spec_ncomps;
            a.sh_words_max = shmax;
            a.gst_bits = gst ? gst_bits_for(wg) : 0u;
            if (site_table) {       // the source-site replay: the interpreter with the site probe
                a.sites = site_table;
                a.site_bits = site_bits;
                HIPCHK(launch_interp(a, n_comp, wg, true, s));
                return;
            }
            // each program's components on its specialised replay kernels,
            // the programs side by side; the interpreter for the rest
            std::vector<uint32_t> interp_groups;
            bool forked = false;
            uint32_t launched = 0;
            for (uint32_t g = 0; g < comp_groups.size(); g++) {
                const CompGroup &cg = comp_groups[g];
                JitFunctions f;
                if (!jit_for(cg.unit, f)) {
                    interp_groups.push_back(g);
                    continue;
                }
                InterpArgs ga = a;
                ga.comp_off = ws.comp_off.as<uint32_t>() + cg.first;
                ga.sh_words_max = cg.shmax;
                ga.gst_bits = gst ? gst_bits_for(cg.wg) : 0u;
                if (comp_groups.size() > 1 && !forked) {
                    fork();
                    forked = true;
                }
                const hipError_t e =
                    launch_jit_lockstep(f, ga, cg.count, cg.wg, comp_groups.size() > 1 ? side(launched) : s);
                if (e == hipSuccess) {
                    launched++;
                    ctx->stat_add("jit_replays", 1);
                    continue;
                }
                if (e != hipErrorInvalidValue) HIPCHK(e);
                (void)hipGetLastError();
                interp_groups.push_back(g);
            }
            if (forked) join();
            if (interp_groups.size() == comp_groups.size()) {      // one interpreter launch for all
                HIPCHK(launch_interp(a, n_comp, wg, true, s));
                return;
            }
            for (uint32_t g : interp_groups) {
                const CompGroup &cg = comp_groups[g];
                InterpArgs ga = a;
                ga.comp_off = ws.comp_off.as<uint32_t>() + cg.first;
                ga.sh_words_max = cg.shmax;
                ga.gst_bits = gst ? gst_bits_for(cg.wg) : 0u;
                HIPCHK(launch_interp(ga, cg.count, cg.wg, true, s));
            }
            return;
        }
        // free run: one launch per (workgroup size, kernel) class; a unit whose
        // program has compiled specialised kernels runs those, the rest the
        // interpreter
        if (opt.jit) jit_prepare();
        std::vector<JitFunctions> jf(hu.size());
        std::vector<char> use_jit(hu.size(), 0);
        for (uint32_t i = 0; i < hu.size(); i++) use_jit[i] = jit_for(i, jf[i]) ? 1 : 0;
        auto launch = [&](InterpArgs args, uint32_t n_wg, uint32_t wg, bool jit, const JitFunctions &f,
                          hipStream_t q) {
            args.gst_bits = gst ? gst_bits_for(wg) : 0u;
            if (jit) {
                const hipError_t e = launch_jit(f, args, n_wg, wg, q);
                if (e == hipSuccess) {
                    ctx->stat_add("jit_launches", 1);
                    return;
                }
                if (e != hipErrorInvalidValue) HIPCHK(e);
                (void)hipGetLastError();
            }
            HIPCHK(launch_interp(args, n_wg, wg, false, q));
        };
        if (hu.size() == 1) {
            const uint32_t wg = (hu[0].nt + 63) / 64 * 64;
            a.items = nullptr;
            a.sh_words_max = hu[0].sh_words;
            a.stage = stage_for(wg);
            launch(a, hu[0].nb, wg, use_jit[0] != 0, jf[0], s);
            return;
        }
        struct Class {
            uint32_t wg;
            bool jit;
            JitFunctions f;
            std::vector<uint32_t> units;
        };
        std::map<std::pair<uint32_t, const void *>, Class> classes;
        for (uint32_t i = 0; i < hu.size(); i++) {
            const uint32_t wg = (hu[i].nt + 63) / 64 * 64;
            const void *kf = use_jit[i] ? (const void *)jf[i].local_256 : nullptr;
            Class &c = classes[{wg, kf}];
            c.wg = wg;
            c.jit = use_jit[i] != 0;
            c.f = jf[i];
            c.units.push_back(i);
        }
        std::vector<uint2> items;
        items.reserve(total_blocks);
        std::vector<std::pair<size_t, size_t>> ranges;
        for (auto &kv : classes) {
            size_t b0 = items.size();
            for (uint32_t ui : kv.second.units)
                for (uint32_t b = 0; b < hu[ui].nb; b++) items.push_back(make_uint2(ui, b));
            ranges.push_back({b0, items.size()});
        }
        ws.items.reserve(items.size() * sizeof(uint2));
        ws.upload(ws.items.p, items.data(), items.size() * sizeof(uint2), s);
        // the classes side by side: each holds few blocks of long latency
        size_t ci = 0;
        const bool par = classes.size() > 1;
        if (par) fork();
        for (auto &kv : classes) {
            uint32_t shmax = 0;
            for (uint32_t ui : kv.second.units) shmax = std::max(shmax, hu[ui].sh_words);
            a.items = ws.items.as<uint2>() + ranges[ci].first;
            a.sh_words_max = shmax;
            a.stage = stage_for(kv.second.wg);
            launch(a, (uint32_t)(ranges[ci].second - ranges[ci].first), kv.second.wg, kv.second.jit, kv.second.f,
                   par ? side((uint32_t)ci) : s);
            ci++;
        }
        if (par) join();
    }

    // Compile the stage's programs that nobody has compiled yet, in parallel;
    // every thread is joined before the launches.
    void jit_prepare() {
        std::vector<std::shared_ptr<JitEntry>> todo;
        for (uint32_t i = 0; i < hu.size(); i++) {
            std::shared_ptr<JitEntry> e = jit_entry(i);
            if (e && jit_claim(e)) todo.push_back(e);
        }
        if (todo.empty()) return;
        std::atomic<size_t> next{0};
        auto work = [&] {
            for (size_t k; (k = next.fetch_add(1)) < todo.size();) jit_compile(todo[k]);
        };
        const size_t nt = std::min<size_t>(todo.size(), std::max(1u, std::min(8u, std::thread::hardware_concurrency())));
        std::vector<std::thread> th;
        try {
            for (size_t t = 1; t < nt; t++) th.emplace_back(work);
        } catch (...) {
            // fewer helper threads: the ones started and this thread share the work
        }
        work();
        for (auto &t : th) t.join();
        ctx->stat_add("jit_compiled", (double)todo.size());
    }

    // Cache entry of unit i's program for the current occupancy target.
    std::shared_ptr<JitEntry> jit_entry(uint32_t i) {
        const kc_program *p = in[i].desc->prog;
        if (p->words.empty()) return nullptr;
        const int w = opt.jit_waves;
        std::lock_guard<std::mutex> g(p->jit_mu);
        if (!p->jit[w]) p->jit[w] = jit_request(p->words.data(), (uint32_t)p->words.size(), w);
        return p->jit[w];
    }

    // Specialised kernels of unit i's program, if enabled, compiled and the
    // launch shape fits them.
    bool jit_for(uint32_t i, JitFunctions &f) {
        if (!opt.jit) return false;
        std::shared_ptr<JitEntry> e = jit_entry(i);
        if (!e) return false;
        if (!jit_fits(hu[i].sh_words, (hu[i].nt + 63) / 64 * 64)) return false;
        double cms = 0.0;
        if (!jit_functions(e, ctx->device, true, f, &cms)) {
            if (jit_state(e) < 0) ctx->stat_add("jit_failures", 1);
            return false;
        }
        if (cms > 0.0) ctx->stat_add("jit_compile_ms", cms);
        return true;
    }

    void run() {
        HostTimer whole{ctx, "stage_host_ms", opt.timing != 0};
        std::unique_ptr<HostTimer> setup_t(new HostTimer{ctx, "host_setup_ms", opt.timing != 0});
        {
            HostTimer ht{ctx, "host_plan_ms", opt.timing != 0};
            plan();
        }
        const uint32_t n = (uint32_t)hu.size();
        out.assign(n, UnitOut{});
        const bool check = opt.check != 0;
        Timer tm{ctx, ws, s, opt.timing};

        // snapshot buffer: each unit's memory at launch start
        if (check) {
            ws.snap.reserve(std::max<uint64_t>(total_words, 1) * 4);
            uint64_t off = 0;
            for (auto &u : hu) {
                u.snap = ws.snap.as<int32_t>() + off;
                off += u.n_words;
            }
        }
        if (!opt.arena && ctx->over_budget())
            throw KcError{KC_E_BUDGET, "workspace exceeds the HBM budget"};
        upload_units();
        if (check) HIPCHK(launch_copy_units(ws.units.as<DevUnit>(), n, max_words, true, nullptr, s));

        uint64_t log_cap = check ? std::max<uint64_t>(ctx->log_hint(), 1024) : 0;
        if (opt.arena) log_cap = std::min<uint64_t>(log_cap, 1u << 20);     // grows on overflow
        if (check) ws.log.reserve(log_cap * 8);
        uint32_t fault_cap = 4096;
        ctx->caps(fault_cap, lrace_cap);
        ws.blk_recs.reserve((size_t)total_blocks * 4);
        ws.blk_flags.reserve((size_t)total_blocks * 4);
        ws.blk_instr.reserve((size_t)total_blocks * 4);
        ws.blk_grecs.reserve((size_t)total_blocks * 4);
        // held representatives go to per-block regions (no queue on the log
        // counter at the end of every block) while the regions stay small
        held_regions = check && opt.local && opt.shadow_global && kp.ab <= 31 &&
                       (uint64_t)total_blocks * REP_HOLD * 8 <= (opt.arena ? (16ull << 20) : (256ull << 20));
        if (held_regions) {
            ws.blk_log.reserve((size_t)total_blocks * REP_HOLD * 8);
            ws.blk_held.reserve((size_t)total_blocks * 4);
            ws.blk_off.reserve((size_t)total_blocks * 8);
        }
        DevCounters c{};
        size_t i_instr = 0, i_grecs = 0, i_sctr = 0, i_sncomp = 0, i_stctr = 0, i_srf = 0, i_srecs = 0, i_srl = 0;
        Fetch fetch;
        bool table_queued = false;
        setup_t.reset();
        for (;;) {
            ws.faults.reserve((size_t)fault_cap * sizeof(DevFault));
            ws.lraces.reserve((size_t)lrace_cap * sizeof(DevRace));
            ws.ctr.reserve(sizeof(DevCounters));
            // held counts start at zero: a block run without the shadow table leaves its own alone
            ZeroArgs z{{ws.ctr.as<uint32_t>(), ws.blk_recs.as<uint32_t>(), ws.blk_flags.as<uint32_t>(),
                        held_regions ? ws.blk_held.as<uint32_t>() : nullptr},
                       {sizeof(DevCounters) / 4, (size_t)total_blocks, (size_t)total_blocks,
                        held_regions ? (size_t)total_blocks : 0},
                       4};
            HIPCHK(launch_zero_many(z, s));
            tm.mark(0);
            interp(false, ws.log, log_cap, ws.ctr, ws.faults, fault_cap, ws.blk_recs, 0, ws.lraces, lrace_cap,
                   ws.blk_flags);
            tm.mark(1);
            if (held_regions)
                HIPCHK(launch_held_compact(ws.blk_log.as<uint64_t>(), ws.blk_held.as<uint32_t>(),
                                           ws.blk_off.as<uint64_t>(), total_blocks, ws.log.as<uint64_t>(), log_cap,
                                           &ws.ctr.as<DevCounters>()->log_count,
                                           &ws.ctr.as<DevCounters>()->flags, s));
            // the free-run log's location tables and the queued replay read
            // disjoint buffers until the replay's exactness check: the tables
            // go to a side stream beside the replay (not when every stage is
            // timed, whose marks need them on the stage's stream)
            const bool aside = check && !spec_off && opt.side_streams > 1 && opt.timing != 1;
            hipStream_t tq = s;
            if (aside) {
                fork();
                tq = side(0);
            }
            table_queued = check && queue_log_check(log_cap, tq);
            tm.mark(12);
            spec = table_queued && !spec_off && spec_allowed();
            if (spec) queue_spec_replay(log_cap, fault_cap, tm, aside);
            else if (aside) join();
            fetch = Fetch{};
            const size_t i_ctr = fetch.add(ws.ctr.p, sizeof(DevCounters));
            fetch.add(ws.blk_recs.p, (size_t)total_blocks * 4);
            fetch.add(ws.faults.p, (size_t)std::min(fault_cap, kSpec) * sizeof(DevFault));
            fetch.add(ws.lraces.p, (size_t)std::min(lrace_cap, kSpec) * sizeof(DevRace));
            if (table_queued) fetch.add(ws.rctr.p, sizeof(DevCounters));      // item 4
            i_instr = fetch.add(ws.blk_instr.p, (size_t)total_blocks * 4);
            i_grecs = fetch.add(ws.blk_grecs.p, (size_t)total_blocks * 4);
            if (spec) {
                i_sctr = fetch.add(ws.sctr.p, sizeof(DevCounters));
                i_sncomp = fetch.add(ws.sncomp.p, 4);
                i_stctr = fetch.add(ws.stctr.p, sizeof(DevCounters));
                i_srf = fetch.add(ws.rfaults.p, (size_t)std::min(spec_fcap, kSpec) * sizeof(DevFault));
                i_srecs = fetch.add(ws.rblk_recs.p, (size_t)total_blocks * 4);
                i_srl = fetch.add(ws.rlraces.p, (size_t)std::min(spec_rlcap, kSpecRaces) * sizeof(DevRace));
            }
            run_fetch(fetch);
            c = *fetched<DevCounters>(fetch, i_ctr);
            ctx->stat_add("interp_ms", tm.ms(0, 1));
            ctx->stat_add("interp_launches", 1);
            if (check && (c.flags & FLAG_EPOCH_OVERFLOW)) epoch_overflow();
            bool again = false;
            if (check && (c.flags & FLAG_LOG_OVERFLOW)) {
                log_cap = c.log_count + c.log_count / 8 + 1024;
                if (!opt.arena && ctx->over_budget(log_cap * 16 > ws.log.bytes + ws.alt.bytes
                                                      ? log_cap * 16 - ws.log.bytes - ws.alt.bytes : 0))
                    throw KcError{KC_E_BUDGET, "access log does not fit the HBM budget"};
                ws.log.reserve(log_cap * 8);
                again = true;
            }
            if (c.flags & FLAG_FAULT_OVERFLOW) {
                fault_cap = c.fault_count + c.fault_count / 8 + 1024;
                again = true;
            }
            if (c.flags & FLAG_RACE_OVERFLOW) {
                lrace_cap = c.race_count + c.race_count / 8 + 1024;
                again = true;
            }
            spec_ok = false;
            if (spec) {
                const DevCounters sc = *fetched<DevCounters>(fetch, i_sctr);
                const uint32_t ncomp = *fetched<uint32_t>(fetch, i_sncomp);
                ctx->note_spec(sc.log_count, sc.race_count, ncomp);
                const bool need_sort = (fetched<DevCounters>(fetch, 4)->flags & FLAG_NEED_SORT) != 0;
                const uint32_t sflags = sc.flags & (FLAG_LOG_OVERFLOW | FLAG_FAULT_OVERFLOW | FLAG_RACE_OVERFLOW |
                                                    FLAG_EPOCH_OVERFLOW | FLAG_WLOG_OVERFLOW);
                const uint32_t tflags = fetched<DevCounters>(fetch, i_stctr)->flags & (FLAG_NEED_SORT | FLAG_MISMATCH);
                spec_ok = !again && !need_sort && !sflags && !tflags;
                spec_ncomp = ncomp;
                spec_counters = sc;
                if (!spec_ok && ncomp > 0 && !again) {
                    // the queued replay changed the memory: run the stage again without it
                    spec_off = true;
                    again = true;
                    ctx->stat_add("spec_retries", 1);
                    if (need_sort) ctx->note_spec_failed(in[0].desc->prog);
                }
            }
            if (!again) break;
            if (!check) throw KcError{KC_E_OVERFLOW, "findings overflow with check disabled"};
            HIPCHK(launch_copy_units(ws.units.as<DevUnit>(), n, max_words, false, nullptr, s));   // back to launch start
            ctx->stat_add("retries", 1);
        }
        std::unique_ptr<HostTimer> parse_t(new HostTimer{ctx, "host_parse_ms", opt.timing != 0});
        {
            const uint32_t *bi = fetched<uint32_t>(fetch, i_instr);
            const uint32_t *bg = fetched<uint32_t>(fetch, i_grecs);
            uint64_t instr = 0, grecs = 0;
            for (uint32_t b = 0; b < total_blocks; b++) {
                instr += bi[b];
                grecs += bg[b];
            }
            ctx->stat_add("instructions", (double)instr);
            ctx->stat_add("global_accesses", (double)grecs);
        }
        if (check) ctx->note_log_records(c.log_count + c.log_count / 8);
        ctx->note_caps(c.fault_count + c.fault_count / 8, c.race_count + c.race_count / 8);
        used_epoch_bits = bits_for((uint64_t)c.max_epoch + 2);   // one more value: representative records

        blk_recs.resize(total_blocks);
        std::memcpy(blk_recs.data(), fetched<uint32_t>(fetch, 1), (size_t)total_blocks * 4);
        std::vector<DevFault> faults;
        std::vector<DevRace> lraces;
        take_list(fetch, 2, c.fault_count, fault_cap, ws.faults.p, faults);
        take_list(fetch, 3, c.race_count, lrace_cap, ws.lraces.p, lraces);
        {
            uint64_t total = 0;
            for (uint32_t v : blk_recs) total += v;
            ctx->stat_add("records", (double)total);
            ctx->stat_add("log_entries", (double)c.log_count);
        }

        std::vector<DevRace> races;
        std::vector<DevEdge> edges;
        uint64_t *sorted = ws.log.as<uint64_t>();
        const uint64_t nrec = c.log_count;
        log_sorted = false;
        ftable_bits = 0;
        direct_tables = false;
        if (check && nrec) {
            // Common case first: a log of representatives in which no global
            // location is written by one block and touched by another has no
            // cross-block races or links, so it needs no sort: a table of its
            // locations shows it.  Otherwise sort and check.
            bool need_sort = true;
            if (table_queued) {     // queued behind the free run: its flags came with the counters
                need_sort = (fetched<DevCounters>(fetch, 4)->flags & FLAG_NEED_SORT) != 0;
                ctx->stat_add("hash_check_ms", tm.ms(1, 12));
                if (!need_sort) {
                    ftable_bits = qt_direct ? 0 : qt_bits;
                    direct_tables = qt_direct;
                }
            }
            if (need_sort) {
                tm.mark(2);
                sorted = sort_check(ws.log, ws.alt, nrec, true);
                tm.mark(3);
                run_check(sorted, nrec, ws.blk_flags, races, edges, false);
                tm.mark(4);
                log_sorted = true;
                ctx->stat_add("sort_ms", tm.ms(2, 3));
                ctx->stat_add("check_ms", tm.ms(3, 4));
                ctx->stat_add("sort_keys", (double)nrec);
                ctx->stat_add("sorted_checks", 1);
            }
        }

        parse_t.reset();
        HostTimer post{ctx, "host_post_ms", opt.timing != 0};
        // per-unit findings of the free run
        std::vector<std::vector<kc_fault>> ufaults(n);
        for (auto &f : faults) ufaults[f.unit].push_back(kc_fault{0, f.kind, f.block, f.epoch, f.a, f.b, f.c, f.d});
        races.insert(races.end(), lraces.begin(), lraces.end());
        std::vector<std::vector<kc_race>> uraces(n);
        for (auto &r : races)
            uraces[r.unit].push_back(kc_race{0, r.space, r.scope, r.block, r.epoch, r.addr, r.w, r.o});
        std::vector<uint64_t> urecs(n, 0);
        for (uint32_t i = 0; i < n; i++)
            for (uint32_t b = 0; b < hu[i].nb; b++) urecs[i] += blk_recs[hu[i].block_base + b];

        fin_log = sorted;
        fin_n = check ? nrec : 0;
        racy_words = c.racy_words;
        if (spec_ok && spec_ncomp > 0) {
            ReplayOut ro;
            ro.recs.resize(total_blocks);
            std::memcpy(ro.recs.data(), fetched<uint32_t>(fetch, i_srecs), (size_t)total_blocks * 4);
            take_list(fetch, i_srf, spec_counters.fault_count, spec_fcap, ws.rfaults.p, ro.faults);
            take_list(fetch, i_srl, spec_counters.race_count, spec_rlcap, ws.rlraces.p, ro.lraces, kSpecRaces);
            HostTimer at{ctx, "host_replay_apply_ms", opt.timing != 0};
            spec_apply(races, ro, ufaults, uraces, urecs, tm);
        } else if (!races.empty()) {
            if (spec_ok) throw KcError{KC_E_INTERNAL, "racy blocks the free run did not flag"};
            replay(races, edges, sorted, nrec, ufaults, uraces, urecs, tm);
        }

        HostTimer ut{ctx, "host_unit_out_ms", opt.timing != 0};
        for (uint32_t i = 0; i < n; i++) {
            UnitOut &o = out[i];
            o.records = urecs[i];
            o.races = std::move(uraces[i]);
            sort_races(o.races);
            o.faults = std::move(ufaults[i]);
            std::sort(o.faults.begin(), o.faults.end(), fault_less);
            o.faults.erase(std::unique(o.faults.begin(), o.faults.end(), fault_eq), o.faults.end());
            o.deadlocked = std::any_of(o.faults.begin(), o.faults.end(),
                                       [](const kc_fault &f) { return f.kind == KC_DEADLOCK; });
        }
    }

    // Sort n records held in `keys` into check order; returns the sorted array
    // (keys itself or alt).  A large free-run log (`free_log`) made only of
    // global-memory representatives is sorted by location alone: every
    // consumer of such a log reduces a location's records in any order (the
    // intra-block segments are those of other records), and the records of
    // one block stay together, as the stable sort keeps the log's order.
    uint64_t *sort_check(DBuf &keys, DBuf &alt, uint64_t n, bool free_log = false) {
        uint64_t *res = keys.as<uint64_t>();
        if (n <= 1) return res;
        SortScratch sc;
        const bool os = opt.onesweep && !opt.arena && radix_onesweep(n);
        alt.reserve(n * 8);
        ws.hist.reserve(radix_hist_entries(n, opt.sort_tile) * (os ? 8 : 4));
        ws.part.reserve((256 + RADIX_OS_WORDS + 1) * 4);
        sc.alt = alt.as<uint64_t>();
        sc.hist = ws.hist.as<uint32_t>();
        sc.part = ws.part.as<uint32_t>();
        sc.os = os ? sc.part + 256 : nullptr;
        sc.spin = opt.sort_spin;
        VKey vk = check_key();
        if (free_log && n >= (1ull << 20) && opt.loc_sort) {
            uint32_t *flag = sc.part + 256 + RADIX_OS_WORDS;
            HIPCHK(launch_zero(flag, 4, s));
            HIPCHK(launch_log_reps_only(keys.as<uint64_t>(), n, kp, flag, s));
            Fetch f;
            const size_t i_f = f.add(flag, 4);
            run_fetch(f);
            if (*fetched<uint32_t>(f, i_f) == 0) {
                vk = VKey{0, 0, kp.s_addr, 0, kp.total - kp.s_addr};
                ctx->stat_add("loc_sorts", 1);
            }
        }
        HIPCHK(radix_sort(keys.as<uint64_t>(), n, vk, sc, opt.sort_tile, s, &res, opt.sort_bits));
        if (sc.stall) {
            // the single-pass scatter: finish with three-kernel passes if one stalled
            Fetch f;
            const size_t i_st = f.add(sc.stall, 4);
            run_fetch(f);
            const uint32_t st = *fetched<uint32_t>(f, i_st);
            ctx->stat_add("sort_onesweep", 1);
            if (st) {
                ctx->stat_add("sort_stalls", 1);
                HIPCHK(radix_sort_resume(keys.as<uint64_t>(), n, vk, sc, opt.sort_tile, s, &res, opt.sort_bits,
                                         st - 1u));
            }
        }
        return res;
    }

    // Conflict check over sorted records: races and cross-block links to the
    // host, racy blocks flagged in `flags`.  `extra` (device counters of work
    // queued before the check, or null) comes back in the same trip.
    void run_check(const uint64_t *sorted, uint64_t n, DBuf &flags, std::vector<DevRace> &races,
                   std::vector<DevEdge> &edges, bool zero_flags = true, const DevCounters *extra = nullptr,
                   DevCounters *extra_out = nullptr) {
        uint32_t race_cap = 4096, edge_cap = 4096;
        flags.reserve((size_t)std::max<uint32_t>(total_blocks, 1) * 4);
        ws.longseg.reserve(check_long_cap(n) * 8);
        for (;;) {
            ws.races.reserve((size_t)race_cap * sizeof(DevRace));
            ws.edges.reserve((size_t)edge_cap * sizeof(DevEdge));
            reset_counters(ws.rctr);
            if (zero_flags) HIPCHK(launch_zero(flags.p, (size_t)total_blocks * 4, s));
            CheckArgs ca{};
            ca.keys = sorted;
            ca.n = n;
            ca.kp = kp;
            ca.units = ws.units.as<DevUnit>();
            ca.races = ws.races.as<DevRace>();
            ca.race_cap = race_cap;
            ca.edges = ws.edges.as<DevEdge>();
            ca.edge_cap = edge_cap;
            ca.blk_flags = flags.as<uint32_t>();
            ca.ctr = ws.rctr.as<DevCounters>();
            ca.longseg = ws.longseg.as<uint64_t>();
            HIPCHK(launch_check(ca, s));
            Fetch f;
            const size_t i_ctr = f.add(ws.rctr.p, sizeof(DevCounters));
            const size_t i_r = f.add(ws.races.p, (size_t)std::min(race_cap, kSpec) * sizeof(DevRace));
            const size_t i_e = f.add(ws.edges.p, (size_t)std::min(edge_cap, kSpec) * sizeof(DevEdge));
            const size_t i_x = extra ? f.add(extra, sizeof(DevCounters)) : 0;
            run_fetch(f);
            const DevCounters rc = *fetched<DevCounters>(f, i_ctr);
            if (extra) *extra_out = *fetched<DevCounters>(f, i_x);
            if (rc.flags & (FLAG_RACE_OVERFLOW | FLAG_EDGE_OVERFLOW)) {
                race_cap = std::max(race_cap, rc.race_count + 1024);
                edge_cap = std::max(edge_cap, rc.edge_count + 1024);
                continue;
            }
            take_list(f, i_r, rc.race_count, race_cap, ws.races.p, races);
            take_list(f, i_e, rc.edge_count, edge_cap, ws.edges.p, edges);
            return;
        }
    }

    // Upload components (lists of (unit, block), each within one unit) for
    // the lockstep kernels, grouped by program (comp_groups).
    void upload_comps(const std::vector<std::vector<uint2>> &comps) {
        std::vector<uint32_t> order(comps.size());
        std::iota(order.begin(), order.end(), 0u);
        auto prog_of = [&](uint32_t c) { return in[comps[c][0].x].desc->prog; };
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t x, uint32_t y) { return std::less<const void *>()(prog_of(x), prog_of(y)); });
        comp_groups.clear();
        std::vector<uint32_t> off{0};
        std::vector<uint2> blocks;
        for (uint32_t i = 0; i < order.size(); i++) {
            const auto &c = comps[order[i]];
            if (comp_groups.empty() || prog_of(order[i]) != prog_of(order[comp_groups.back().first]))
                comp_groups.push_back(CompGroup{i, 0, c[0].x, 64, 0});
            CompGroup &g = comp_groups.back();
            g.count++;
            for (auto &ub : c) {
                g.wg = std::max<uint32_t>(g.wg, (hu[ub.x].nt + 63) / 64 * 64);
                g.shmax = std::max(g.shmax, hu[ub.x].sh_words);
            }
            blocks.insert(blocks.end(), c.begin(), c.end());
            off.push_back((uint32_t)blocks.size());
        }
        ws.comp_off.reserve(off.size() * 4);
        ws.comp_blocks.reserve(blocks.size() * sizeof(uint2));
        ws.upload(ws.comp_off.p, off.data(), off.size() * 4, s);
        ws.upload(ws.comp_blocks.p, blocks.data(), blocks.size() * sizeof(uint2), s);
    }

    // Warp-aware model (the finer scheduler the paper's Section 4 proposes:
    // warps of 32 consecutive linear tids execute in lock-step): the
    // intra-block tuples of the replayed blocks from their accesses with
    // lockstep steps.  A write x and an access y (x != y) of one location,
    // block and epoch conflict when their threads are in different warps or
    // they ran at the same step; the tuple is w = the smallest thread with a
    // conflicting write, o = the smallest thread conflicting with one of w's
    // writes.
    static void warp_races(std::vector<WarpRec> &v, std::vector<DevRace> &out) {
        auto space = [](const WarpRec &r) { return (r.tsk >> 17) & 1u; };
        auto tid = [](const WarpRec &r) { return r.tsk & 0xFFFFu; };
        auto store = [](const WarpRec &r) { return ((r.tsk >> 16) & 1u) != 0; };
        std::sort(v.begin(), v.end(), [&](const WarpRec &a, const WarpRec &b) {
            return std::make_tuple(a.unit, space(a), a.block, a.epoch, a.addr, tid(a), a.tsk, a.step) <
                   std::make_tuple(b.unit, space(b), b.block, b.epoch, b.addr, tid(b), b.tsk, b.step);
        });
        auto conflict = [&](const WarpRec &x, const WarpRec &y) {
            return store(x) && tid(x) != tid(y) && (tid(x) / 32u != tid(y) / 32u || x.step == y.step);
        };
        for (size_t i = 0; i < v.size();) {
            size_t j = i;
            while (j < v.size() && v[j].unit == v[i].unit && space(v[j]) == space(v[i]) && v[j].block == v[i].block &&
                   v[j].epoch == v[i].epoch && v[j].addr == v[i].addr)
                j++;
            for (size_t a = i; a < j;) {
                size_t ae = a;
                while (ae < j && tid(v[ae]) == tid(v[a])) ae++;
                uint32_t best = 0xFFFFFFFFu;
                for (size_t x = a; x < ae; x++)
                    for (size_t b = i; b < j; b++)
                        if (conflict(v[x], v[b])) best = std::min(best, tid(v[b]));
                if (best != 0xFFFFFFFFu) {
                    out.push_back(DevRace{v[i].unit, space(v[i]), 0u, v[i].block, v[i].epoch, v[i].addr, tid(v[a]), best});
                    break;
                }
                a = ae;
            }
            i = j;
        }
    }

    // One lockstep pass over `comps`; records go to ws.rlog (capacity rcap).
    // With `res`, its findings, per-block record counts and local races come
    // back in the same trip as the counters.
    struct ReplayOut {
        std::vector<DevFault> faults;
        std::vector<uint32_t> recs;
        std::vector<DevRace> lraces;
        std::vector<DevRace> warp;     // warp-aware model: the replayed blocks' intra-block tuples
        uint32_t table_flags = 0;      // flags of the exactness tables, if queued
    };
    DevCounters lockstep_once(const std::vector<std::vector<uint2>> &comps, uint64_t rcap, uint32_t fcap,
                              uint32_t rlcap, ReplayOut *res = nullptr, const ReplayTableArgs *table = nullptr) {
        upload_comps(comps);
        ws.rblk_recs.reserve((size_t)total_blocks * 4);
        ws.rflags.reserve((size_t)std::max<uint32_t>(total_blocks, 1) * 4);
        ws.rlog.reserve(rcap * 8);
        ws.rfaults.reserve((size_t)fcap * sizeof(DevFault));
        ws.rlraces.reserve((size_t)rlcap * sizeof(DevRace));
        ws.rctr.reserve(sizeof(DevCounters));
        {
            ZeroArgs z{{ws.rctr.as<uint32_t>(), ws.rblk_recs.as<uint32_t>()},
                       {sizeof(DevCounters) / 4, (size_t)total_blocks}, 2};
            HIPCHK(launch_zero_many(z, s));
        }
        // the warp-aware model: every replayed access with its step (not in
        // the source-site pass)
        wlog_cap = (opt.warp && opt.check && !site_table)
                       ? (uint32_t)std::min<uint64_t>(std::max<uint64_t>(rcap, 1024), 0xFFFFFFFFu) : 0u;
        if (wlog_cap) ws.wlog.reserve((size_t)wlog_cap * sizeof(WarpRec));
        interp(true, ws.rlog, rcap, ws.rctr, ws.rfaults, fcap, ws.rblk_recs, (uint32_t)comps.size(), ws.rlraces,
               rlcap, ws.rflags);
        const uint32_t used_wlog = wlog_cap;
        wlog_cap = 0;
        if (table) {            // the replay's exactness tables, queued behind it (flags in ws.ctr, zeroed there)
            ws.ctr.reserve(sizeof(DevCounters));
            HIPCHK(launch_replay_table(*table, s));
        }
        Fetch f;
        const size_t i_ctr = f.add(ws.rctr.p, sizeof(DevCounters));
        if (res) {
            f.add(ws.rfaults.p, (size_t)std::min(fcap, kSpec) * sizeof(DevFault));
            f.add(ws.rblk_recs.p, (size_t)total_blocks * 4);
            f.add(ws.rlraces.p, (size_t)std::min(rlcap, kSpec) * sizeof(DevRace));
        }
        const size_t i_tab = table ? f.add(ws.ctr.p, sizeof(DevCounters)) : 0;
        run_fetch(f);
        const DevCounters c = *fetched<DevCounters>(f, i_ctr);
        if (res && table) res->table_flags = fetched<DevCounters>(f, i_tab)->flags;
        if (c.flags & FLAG_EPOCH_OVERFLOW) epoch_overflow();
        if (res && !(c.flags & (FLAG_LOG_OVERFLOW | FLAG_FAULT_OVERFLOW | FLAG_RACE_OVERFLOW | FLAG_WLOG_OVERFLOW))) {
            res->recs.resize(total_blocks);
            std::memcpy(res->recs.data(), fetched<uint32_t>(f, 2), (size_t)total_blocks * 4);
            take_list(f, 1, c.fault_count, fcap, ws.rfaults.p, res->faults);
            take_list(f, 3, c.race_count, rlcap, ws.rlraces.p, res->lraces);
            if (used_wlog) {
                std::vector<WarpRec> wl(c.wlog_count);
                if (!wl.empty()) {
                    HIPCHK(hipMemcpyAsync(wl.data(), ws.wlog.p, wl.size() * sizeof(WarpRec), hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                }
                warp_races(wl, res->warp);
            }
        }
        return c;
    }

    // The results of an exact replay of `comps` replace the free run's for
    // their blocks: records, findings and races (`rr`: races found by a
    // sorted check of the replay's records; the replay's own intra-block
    // races are added here).
    void apply_replay(const std::vector<std::vector<uint2>> &comps, const ReplayOut &ro, std::vector<DevRace> &rr,
                      std::vector<std::vector<kc_fault>> &ufaults, std::vector<std::vector<kc_race>> &uraces,
                      std::vector<uint64_t> &urecs) {
        const std::vector<DevFault> &rf = ro.faults;
        const std::vector<uint32_t> &rrecs = ro.recs;
        rr.insert(rr.end(), ro.lraces.begin(), ro.lraces.end());
        if (opt.warp) {     // intra-block tuples of the warp-aware model replace the plain ones
            rr.erase(std::remove_if(rr.begin(), rr.end(), [](const DevRace &r) { return r.scope == 0; }), rr.end());
            rr.insert(rr.end(), ro.warp.begin(), ro.warp.end());
        }
        std::vector<char> in_s(total_blocks, 0);
        for (auto &c : comps)
            for (auto &ub : c) {
                const uint32_t gb = hu[ub.x].block_base + ub.y;
                in_s[gb] = 1;
                urecs[ub.x] += (uint64_t)rrecs[gb];
                urecs[ub.x] -= (uint64_t)blk_recs[gb];
            }
        for (uint32_t u = 0; u < hu.size(); u++) {
            auto &fv = ufaults[u];
            fv.erase(std::remove_if(fv.begin(), fv.end(),
                                    [&](const kc_fault &f) { return in_s[hu[u].block_base + f.block]; }),
                     fv.end());
            uraces[u].clear();      // every free-run race involved replayed blocks only
        }
        for (auto &f : rf) ufaults[f.unit].push_back(kc_fault{0, f.kind, f.block, f.epoch, f.a, f.b, f.c, f.d});
        for (auto &r : rr) uraces[r.unit].push_back(kc_race{0, r.space, r.scope, r.block, r.epoch, r.addr, r.w, r.o});
    }

    // The replay queued behind the free run stood (its results came with the
    // free run's): its components are the racy blocks, each alone, in
    // ascending global block index, as the device listed them.
    void spec_apply(const std::vector<DevRace> &races, const ReplayOut &ro, std::vector<std::vector<kc_fault>> &ufaults,
                    std::vector<std::vector<kc_race>> &uraces, std::vector<uint64_t> &urecs, Timer &tm) {
        std::vector<uint32_t> g;
        for (auto &r : races) g.push_back(hu[r.unit].block_base + r.block);
        std::sort(g.begin(), g.end());
        g.erase(std::unique(g.begin(), g.end()), g.end());
        if (g.size() != spec_ncomp) throw KcError{KC_E_INTERNAL, "the queued replay ran other blocks than the racy ones"};
        std::vector<std::vector<uint2>> comps;
        uint32_t unit = 0;
        for (uint32_t gb : g) {
            while (unit + 1 < hu.size() && hu[unit + 1].block_base <= gb) unit++;
            comps.push_back({make_uint2(unit, gb - hu[unit].block_base)});
        }
        ctx->stat_add("replays", (double)comps.size());
        ctx->stat_add("spec_replays", 1);
        ctx->stat_add("replay_lockstep_ms", tm.ms(5, 7));
        ctx->stat_add("replay_ms", tm.ms(5, 7));
        rep_log = ws.rlog.as<uint64_t>();
        rep_n = spec_counters.log_count;
        skip_flagged = true;
        replayed = comps;
        std::vector<DevRace> rr;
        apply_replay(comps, ro, rr, ufaults, uraces, urecs);
    }

    // Racy blocks: re-execute them canonically and take their records, findings
    // and memory from the re-execution.  This is exact when (1) no replayed
    // global access conflicts with an access of a block that was not replayed
    // and (2) the components replayed side by side do not conflict with each
    // other; then the canonical execution is the free run of the other blocks
    // plus the replay, and its races are those of the replayed records.
    // Otherwise every block of the affected units is re-executed canonically.
    void replay(const std::vector<DevRace> &races, const std::vector<DevEdge> &edges, const uint64_t *log_in,
                uint64_t nrec, std::vector<std::vector<kc_fault>> &ufaults,
                std::vector<std::vector<kc_race>> &uraces, std::vector<uint64_t> &urecs, Timer &tm) {
        tm.mark(5);
        const uint64_t *sorted = log_in;     // the free-run log; sorted if log_sorted
        // components: racy blocks (global block index) united along the
        // cross-block links; the root of a component is its smallest block
        constexpr uint32_t NOT_RACY = 0xFFFFFFFFu;
        std::vector<uint32_t> parent(total_blocks, NOT_RACY);
        auto find = [&](uint32_t x) {
            while (parent[x] != x) {
                parent[x] = parent[parent[x]];
                x = parent[x];
            }
            return x;
        };
        auto mark = [&](uint32_t g) {
            if (parent[g] == NOT_RACY) parent[g] = g;
            return g;
        };
        for (auto &r : races) mark(hu[r.unit].block_base + r.block);
        for (auto &e : edges) {
            const uint32_t a = find(mark(hu[e.unit].block_base + e.b0)), b = find(mark(hu[e.unit].block_base + e.b1));
            if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
        std::vector<std::vector<uint2>> comps;
        std::vector<uint32_t> comp_of(total_blocks, NOT_RACY);
        uint64_t s_recs = 0;
        uint32_t unit = 0;
        for (uint32_t g = 0; g < total_blocks; g++) {
            if (parent[g] == NOT_RACY) continue;
            while (unit + 1 < hu.size() && hu[unit + 1].block_base <= g) unit++;
            const uint32_t root = find(g);
            if (root == g) {
                comp_of[g] = (uint32_t)comps.size();
                comps.emplace_back();
            } else {
                comp_of[g] = comp_of[root];     // the root is smaller: already numbered
            }
            comps[comp_of[g]].push_back(make_uint2(unit, g - hu[unit].block_base));
            s_recs += blk_recs[g];
        }
        ctx->stat_add("replays", (double)comps.size());

        // put back what the racy blocks wrote, then re-execute them canonically
        HIPCHK(launch_restore(sorted, nrec, kp, ws.units.as<DevUnit>(), ws.blk_flags.as<uint32_t>(), s));
        uint64_t rcap = s_recs + s_recs / 4 + 1024;
        // the free run's verdicts report racy shared words only by count (the
        // replay computes their tuples)
        uint32_t fcap = 4096, rlcap = 4096 + (uint32_t)std::min<uint64_t>(
                                               2 * ((uint64_t)races.size() + racy_words), 1u << 30);
        ReplayOut ro;
        // Common case first: the replay's records are all representatives and
        // no replayed location is shared by replayed blocks with a write; then
        // its exactness needs no sort (a table of its locations, each looked
        // up in the free run's tables or its sorted log).  Queued behind the
        // lockstep kernel, sized for its log capacity.
        const bool use_table = table_obits() != 0;
        uint32_t bits = 10;
        while ((1ull << bits) < 2 * rcap) bits++;
        if (use_table) ws.rtable.reserve((size_t)8 << bits);
        ws.rlog.reserve(rcap * 8);
        ReplayTableArgs ta{ws.rlog.as<uint64_t>(), rcap, sorted, nrec, kp, ws.units.as<DevUnit>(),
                           ws.blk_flags.as<uint32_t>(), use_table ? ws.rtable.p : nullptr, bits,
                           ws.ctr.as<DevCounters>(), (log_sorted || direct_tables) ? nullptr : ws.ftable.p,
                           ftable_bits, table_obits(), ws.snap.as<int32_t>(),
                           (!log_sorted && direct_tables) ? ws.downer.as<uint32_t>() : nullptr,
                           ws.dflags.as<uint8_t>(), nullptr};
        ws.rctr.reserve(sizeof(DevCounters));
        ta.n_dev = &ws.rctr.as<DevCounters>()->log_count;
        replayed = comps;
        DevCounters rc = lockstep_once(comps, rcap, fcap, rlcap, &ro, use_table ? &ta : nullptr);
        tm.mark(7);
        ctx->stat_add("replay_lockstep_ms", tm.ms(5, 7));
        bool ok = !(rc.flags & (FLAG_LOG_OVERFLOW | FLAG_FAULT_OVERFLOW | FLAG_RACE_OVERFLOW | FLAG_WLOG_OVERFLOW));
        std::vector<DevRace> rr;
        std::vector<DevEdge> re;
        bool sorted_check = ok && rc.log_count > 0;
        if (sorted_check && use_table) {
            if (!(ro.table_flags & FLAG_NEED_SORT)) {
                sorted_check = false;
                ok = !(ro.table_flags & FLAG_MISMATCH);
            } else {
                ctx->stat_add("replay_sorted_checks", 1);
            }
        }
        if (sorted_check && !log_sorted) {      // the exactness scan needs the free-run log sorted
            sorted = sort_check(ws.log, ws.alt, nrec, true);
            log_sorted = true;
            fin_log = sorted;
        }
        rep_log = ws.rlog.as<uint64_t>();
        rep_n = rc.log_count;
        skip_flagged = true;
        if (sorted_check) {
            used_epoch_bits = std::max(used_epoch_bits, bits_for((uint64_t)rc.max_epoch + 2));
            uint64_t *rs = sort_check(ws.rlog, ws.ralt, rc.log_count);
            rep_log = rs;
            tm.mark(8);
            // the exactness check is queued first; its flag returns with the
            // conflict check's results
            reset_counters(ws.ctr);
            ws.covlist.reserve(std::max<uint64_t>(rc.log_count, 1) * 8);
            HIPCHK(launch_coverage(rs, rc.log_count, sorted, nrec, kp, ws.units.as<DevUnit>(),
                                   ws.blk_flags.as<uint32_t>(), ws.ctr.as<DevCounters>(),
                                   ws.covlist.as<uint64_t>(), s));
            tm.mark(10);
            DevCounters cov{};
            run_check(rs, rc.log_count, ws.rflags, rr, re, true, ws.ctr.as<DevCounters>(), &cov);
            tm.mark(9);
            ok = !(cov.flags & FLAG_MISMATCH);
            ctx->stat_add("replay_sort_ms", tm.ms(7, 8));
            ctx->stat_add("replay_coverage_ms", tm.ms(8, 10));
            ctx->stat_add("replay_check_ms", tm.ms(10, 9));
            for (auto &e : re)
                if (comp_of[hu[e.unit].block_base + e.b0] != comp_of[hu[e.unit].block_base + e.b1]) ok = false;
        }
        if (ok) {
            apply_replay(comps, ro, rr, ufaults, uraces, urecs);
            tm.mark(6);
            ctx->stat_add("replay_ms", tm.ms(5, 6));
            return;
        }

        // General case: re-run every block of the affected units canonically
        // from the launch-start snapshot and check those records.
        ctx->stat_add("fallbacks", 1);
        std::vector<uint32_t> mask(hu.size(), 0);
        for (auto &c : comps)
            for (auto &ub : c) mask[ub.x] = 1;
        ws.mask.reserve(mask.size() * 4);
        ws.upload(ws.mask.p, mask.data(), mask.size() * 4, s);
        std::vector<std::vector<uint2>> full;
        uint64_t need = 0;
        for (uint32_t u = 0; u < hu.size(); u++) {
            if (!mask[u]) continue;
            std::vector<uint2> v;
            for (uint32_t b = 0; b < hu[u].nb; b++) {
                v.push_back(make_uint2(u, b));
                need += blk_recs[hu[u].block_base + b];
            }
            full.push_back(std::move(v));
        }
        rcap = std::max<uint64_t>(rcap, need + need / 4 + 1024);
        replayed = full;
        DevCounters fc;
        ReplayOut fo;
        for (;;) {
            HIPCHK(launch_copy_units(ws.units.as<DevUnit>(), (uint32_t)hu.size(), max_words, false,
                                     ws.mask.as<uint32_t>(), s));
            fc = lockstep_once(full, rcap, fcap, rlcap, &fo);
            if (!(fc.flags & (FLAG_LOG_OVERFLOW | FLAG_FAULT_OVERFLOW | FLAG_RACE_OVERFLOW | FLAG_WLOG_OVERFLOW)))
                break;
            rcap = std::max<uint64_t>(rcap, fc.log_count + 1024);
            if (fc.flags & FLAG_WLOG_OVERFLOW) rcap = std::max<uint64_t>(rcap, (uint64_t)fc.wlog_count * 2 + 1024);
            fcap = std::max<uint32_t>(fcap, fc.fault_count + 1024);
            rlcap = std::max<uint32_t>(rlcap, fc.race_count + 1024);
        }
        const std::vector<DevFault> &ff = fo.faults;
        const std::vector<uint32_t> &rrecs = fo.recs;
        const std::vector<DevRace> &fl = fo.lraces;
        used_epoch_bits = std::max(used_epoch_bits, bits_for((uint64_t)fc.max_epoch + 2));
        uint64_t *rs = sort_check(ws.rlog, ws.ralt, fc.log_count);
        rep_log = rs;
        rep_n = fc.log_count;
        skip_flagged = false;
        skip_masked = true;
        std::vector<DevRace> nr;
        std::vector<DevEdge> ne;
        run_check(rs, fc.log_count, ws.rflags, nr, ne);
        nr.insert(nr.end(), fl.begin(), fl.end());
        if (opt.warp) {
            nr.erase(std::remove_if(nr.begin(), nr.end(), [](const DevRace &r) { return r.scope == 0; }), nr.end());
            nr.insert(nr.end(), fo.warp.begin(), fo.warp.end());
        }
        for (uint32_t u = 0; u < hu.size(); u++) {
            if (!mask[u]) continue;
            uraces[u].clear();
            ufaults[u].clear();
            urecs[u] = 0;
            for (uint32_t b = 0; b < hu[u].nb; b++) urecs[u] += rrecs[hu[u].block_base + b];
        }
        for (auto &r : nr) uraces[r.unit].push_back(kc_race{0, r.space, r.scope, r.block, r.epoch, r.addr, r.w, r.o});
        for (auto &f : ff) ufaults[f.unit].push_back(kc_fault{0, f.kind, f.block, f.epoch, f.a, f.b, f.c, f.d});
        tm.mark(6);
        ctx->stat_add("replay_ms", tm.ms(5, 6));
    }

    // Source sites of the stage's races (scope 0 and 1): put back what the
    // replay wrote, run the replayed components once more with the site
    // table (the same canonical execution, so memory ends the same), and read
    // the smallest store pc of each tuple's writer and access pc of its other
    // thread.  Fills out[i].sites parallel to out[i].races.
    void sites_pass(std::vector<UnitOut> &out) {
        constexpr uint32_t NONE = 0xFFFFFFFFu;
        uint64_t n_races = 0;
        for (auto &o : out) {
            o.sites.assign(o.races.size(), kc_race_site{NONE, NONE});
            n_races += o.races.size();
        }
        if (!n_races || replayed.empty()) return;
        uint32_t bits = 10;
        while ((1ull << bits) < 2 * n_races) bits++;
        std::vector<SiteSlot> table((size_t)1 << bits);
        std::vector<std::pair<uint32_t, size_t>> where;     // (unit, race index) per filled slot
        std::vector<uint32_t> slot_of;
        for (uint32_t u = 0; u < out.size(); u++)
            for (size_t q = 0; q < out[u].races.size(); q++) {
                const kc_race &r = out[u].races[q];
                const uint32_t mask = (1u << bits) - 1u;
                uint32_t h = site_hash(u, r.space, r.block, r.epoch, r.addr) & mask;
                if (r.scope == 1) h = site_hash(u, 1u, NONE, NONE, r.addr) & mask;
                while (table[h].used) h = (h + 1) & mask;
                SiteSlot &e = table[h];
                e.unit = u;
                e.space = r.space;
                e.block = r.scope == 1 ? NONE : r.block;
                e.epoch = r.scope == 1 ? NONE : r.epoch;
                e.addr = r.addr;
                e.w = r.w_tid;
                e.o = r.o_tid;
                e.used = 1;
                e.w_pc = e.o_pc = NONE;
                where.push_back({u, q});
                slot_of.push_back(h);
            }
        struct Scratch {
            DBuf t;
            ~Scratch() { t.release(); }
        } tmp;
        tmp.t.reserve(table.size() * sizeof(SiteSlot));
        HIPCHK(hipMemcpyAsync(tmp.t.p, table.data(), table.size() * sizeof(SiteSlot), hipMemcpyHostToDevice, s));
        // back to the memory the replay started from
        if (skip_masked)
            HIPCHK(launch_copy_units(ws.units.as<DevUnit>(), (uint32_t)hu.size(), max_words, false,
                                     ws.mask.as<uint32_t>(), s));
        else
            HIPCHK(launch_restore(rep_log, rep_n, kp, ws.units.as<DevUnit>(), ws.blk_flags.as<uint32_t>(), s));
        site_table = tmp.t.as<SiteSlot>();
        site_bits = bits;
        const uint64_t cap = std::max<uint64_t>(ws.rlog.bytes / 8, 1);
        const uint32_t fcap = (uint32_t)std::max<size_t>(ws.rfaults.bytes / sizeof(DevFault), 1);
        const uint32_t rlcap = (uint32_t)std::max<size_t>(ws.rlraces.bytes / sizeof(DevRace), 1);
        try {
            lockstep_once(replayed, cap, fcap, rlcap);      // its log may overflow: only the sites are used
        } catch (...) {
            site_table = nullptr;
            throw;
        }
        site_table = nullptr;
        HIPCHK(hipMemcpyAsync(table.data(), tmp.t.p, table.size() * sizeof(SiteSlot), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (size_t i = 0; i < where.size(); i++) {
            const SiteSlot &e = table[slot_of[i]];
            out[where[i].first].sites[where[i].second] = kc_race_site{e.w_pc, e.o_pc};
        }
        ctx->stat_add("site_replays", 1);
    }

    // Call f(log, n, skip_blocks, skip_units) for each part of the stage's
    // canonical accesses (see fin_log).
    template <class F> void canonical_logs(F f) {
        f(fin_log, fin_n, skip_flagged ? ws.blk_flags.as<uint32_t>() : nullptr,
          skip_masked ? ws.mask.as<uint32_t>() : nullptr);
        if (rep_log && rep_n) f(rep_log, rep_n, nullptr, nullptr);
    }

    // Queue the access summaries of the units with sums[u] set (device array
    // of per-unit pointers, see launch_summary) from the stage's canonical
    // accesses.
    void summarize(uint32_t *const *sums) {
        canonical_logs([&](const uint64_t *log, uint64_t n, const uint32_t *skip_b, const uint32_t *skip_u) {
            SummaryArgs a{};
            a.kp = kp;
            a.units = ws.units.as<DevUnit>();
            a.sums = sums;
            a.log = log;
            a.n = n;
            a.skip_blocks = skip_b;
            a.skip_units = skip_u;
            HIPCHK(launch_summary(a, s));
        });
    }

    // Memory objects: the canonical records of global words outside their
    // unit's allocations (allocated: device array of per-unit bitmaps), as
    // ALLOC findings per (unit, block, word) in `found`.
    void illegal_accesses(const uint32_t *const *allocated, std::vector<std::vector<kc_fault>> &found) {
        uint32_t cap = 4096;
        struct Scratch {
            DBuf list, count;
            ~Scratch() {
                list.release();
                count.release();
            }
        } tmp;
        tmp.count.reserve(4);
        std::vector<uint64_t> got;
        for (;;) {
            tmp.list.reserve((size_t)cap * 8);
            HIPCHK(launch_zero(tmp.count.p, 4, s));
            canonical_logs([&](const uint64_t *log, uint64_t n, const uint32_t *skip_b, const uint32_t *skip_u) {
                AllocScanArgs a{log, n, kp, ws.units.as<DevUnit>(), allocated, skip_b, skip_u,
                                tmp.list.as<uint64_t>(), cap, tmp.count.as<uint32_t>()};
                HIPCHK(launch_alloc_scan(a, s));
            });
            uint32_t n = 0;
            HIPCHK(hipMemcpyAsync(&n, tmp.count.p, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (n > cap) {
                cap = n;
                continue;
            }
            got.resize(n);
            if (n) {
                HIPCHK(hipMemcpyAsync(got.data(), tmp.list.p, (size_t)n * 8, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
            }
            break;
        }
        // smallest accessing and storing tid per (unit, block, word)
        constexpr uint32_t NONE_U32 = 0xFFFFFFFFu;
        std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::pair<uint32_t, uint32_t>> m;
        for (uint64_t r : got) {
            const uint32_t tid = rec_field(r, kp.s_tid, kp.tb);
            auto key = std::make_tuple(rec_field(r, kp.s_unit, kp.ub), rec_field(r, kp.s_blk, kp.bb),
                                       rec_field(r, kp.s_addr, kp.ab));
            auto it = m.emplace(key, std::make_pair(NONE_U32, NONE_U32)).first;
            it->second.first = std::min(it->second.first, tid);
            if (r & 1ull) it->second.second = std::min(it->second.second, tid);
        }
        for (auto &e : m) {
            const uint32_t w = e.second.second;
            found[std::get<0>(e.first)].push_back(kc_fault{0, F_ALLOC, std::get<1>(e.first), NONE_U32,
                                                           w != NONE_U32 ? 3u : 2u, e.second.first,
                                                           std::get<2>(e.first), w});
        }
        ctx->stat_add("alloc_findings", (double)m.size());
    }
};

kc_status fail(kc_ctx *ctx, const KcError &e) {
    if (ctx) {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->err = e.msg;
        if (e.st == KC_E_DEVICE || e.st == KC_E_INTERNAL) ctx->poisoned = true;
    }
    return e.st;
}

// The status and message of the exception being handled.  Every exception
// the library can raise maps to a status, so none reaches a C caller or ends
// a worker thread (either would end the process in std::terminate).
KcError current_error() {
    try {
        throw;
    } catch (const KcError &e) {
        return e;
    } catch (const std::bad_alloc &) {
        return KcError{KC_E_NOMEM, "host allocation failed"};
    } catch (const std::system_error &e) {
        // thread creation and mutex failures: the process is out of resources
        return KcError{KC_E_NOMEM, std::string("system resource: ") + e.what()};
    } catch (const std::exception &e) {
        return KcError{KC_E_INTERNAL, std::string("internal error: ") + e.what()};
    } catch (...) {
        return KcError{KC_E_INTERNAL, "internal error: unknown exception"};
    }
}

// Run an entry point's body; any exception becomes its status.
template <class F> kc_status guarded(kc_ctx *ctx, F &&body) {
    try {
        return body();
    } catch (...) {
        return fail(ctx, current_error());
    }
}

// Which steps (launches, or items of a host program) of a job may run in
// parallel (Section 3 "Streams and events").  before[j] holds bit i when step
// i happens before step j: the closure of same-stream order of device steps,
// dependencies, host program order (a host step, or a copy the host waits
// for on the spot, comes before every later step) and host waits (the step
// waited for, or every earlier device step, comes before the wait); every
// edge points forward, so rows are built in order.
struct LaunchOrder {
    uint32_t n = 0, words = 0;
    std::vector<uint64_t> before;       // n rows of `words` words
    std::vector<char> parallel;         // step may run in parallel with another one
    bool any = false;
    bool ordered(uint32_t i, uint32_t j) const { return (before[(size_t)j * words + i / 64] >> (i % 64)) & 1u; }

    explicit LaunchOrder(const kc_job &job) {
        if (!job.streams && !job.n_deps && !job.items) return;
        n = job_steps(job);
        words = (n + 63) / 64;
        before.assign((size_t)n * words, 0);
        std::vector<std::vector<uint32_t>> preds(n);
        std::unordered_map<uint32_t, uint32_t> last;    // stream -> its latest device step
        int64_t host_point = -1;                        // latest host step or synchronous copy
        for (uint32_t j = 0; j < n; j++) {
            const kc_item *it = job.items ? &job.items[j] : nullptr;
            if (device_item(job, j)) {
                const uint32_t sid = it ? it->stream : job.streams ? job.streams[j] : 0u;
                auto f = last.find(sid);
                if (f != last.end()) preds[j].push_back(f->second);
                last[sid] = j;
            }
            if (host_point >= 0) preds[j].push_back((uint32_t)host_point);
            if (it && it->kind == KC_ITEM_HOST_WAIT) {
                if (it->ref != KC_WAIT_ALL) preds[j].push_back(it->ref);
                else
                    for (uint32_t i = 0; i < j; i++)
                        if (device_item(job, i)) preds[j].push_back(i);
            }
            if (it && (!device_item(job, j) || (it->kind == KC_ITEM_COPY && (it->flags & KC_ITEM_SYNC))))
                host_point = j;
        }
        for (uint32_t d = 0; d < job.n_deps; d++) preds[job.deps[d].after].push_back(job.deps[d].before);
        for (uint32_t j = 0; j < n; j++) {
            uint64_t *row = &before[(size_t)j * words];
            for (uint32_t p : preds[j]) {
                const uint64_t *prow = &before[(size_t)p * words];
                for (uint32_t w = 0; w < words; w++) row[w] |= prow[w];
                row[p / 64] |= 1ull << (p % 64);
            }
        }
        parallel.assign(n, 0);
        for (uint32_t j = 0; j < n; j++)
            for (uint32_t i = 0; i < j; i++)
                if (!ordered(i, j)) parallel[i] = parallel[j] = 1, any = true;
    }
};

// Access summaries of step li for the jobs in `who` whose step may run in
// parallel with another (per job and step, kept in `sums` for the later
// steps), preset to "no access"; nullptr entries for the other jobs.
std::vector<uint32_t *> prepare_summaries(kc_ctx *ctx, Workspace &ws, hipStream_t s, uint32_t li,
                                          const kc_job *jobs, const std::vector<uint32_t> &who,
                                          const std::vector<LaunchOrder> &order,
                                          std::vector<std::vector<DBuf>> &sums) {
    (void)ws;
    std::vector<uint32_t *> ptr(who.size(), nullptr);
    for (size_t i = 0; i < who.size(); i++) {
        const uint32_t j = who[i];
        if (!order[j].any || !order[j].parallel[li]) continue;
        if (jobs[j].items && jobs[j].items[li].kind == KC_ITEM_HOST_WAIT) continue;    // touches nothing
        if (sums[j].empty()) sums[j].resize(job_steps(jobs[j]));
        DBuf &b = sums[j][li];
        b.acct = &ctx->bytes;
        if (ctx->over_budget(std::max<uint64_t>(jobs[j].n_words, 1) * 8))
            throw KcError{KC_E_BUDGET, "launch summaries exceed the HBM budget"};
        b.reserve(std::max<uint64_t>(jobs[j].n_words, 1) * 8);
        HIPCHK(hipMemsetAsync(b.p, 0xFF, jobs[j].n_words * 8, s));
        ptr[i] = b.as<uint32_t>();
    }
    return ptr;
}

// Races between step li (summaries `ptr`, per job of `who`) and every
// earlier step of the same job that may run in parallel with it.
void scan_cross(kc_ctx *ctx, hipStream_t s, uint32_t li, const kc_job *jobs, const std::vector<uint32_t> &who,
                const std::vector<uint32_t *> &ptr, const std::vector<LaunchOrder> &order,
                std::vector<std::vector<DBuf>> &sums, std::vector<kc_report *> &reports) {
    struct Scratch {
        DBuf list, count;
        ~Scratch() {
            list.release();
            count.release();
        }
    } tmp;
    DBuf &list = tmp.list, &count = tmp.count;
    uint32_t cap = 4096;
    count.reserve(4);
    std::vector<DevRace> got;
    for (;;) {
        list.reserve((size_t)cap * sizeof(DevRace));
        HIPCHK(launch_zero(count.p, 4, s));
        for (size_t i = 0; i < who.size(); i++) {
            if (!ptr[i]) continue;
            const uint32_t j = who[i];
            for (uint32_t k = 0; k < li; k++)
                if (order[j].parallel[k] && !order[j].ordered(k, li) && !sums[j].empty() && sums[j][k].p)
                    HIPCHK(launch_cross_launch(sums[j][k].as<uint32_t>(), ptr[i], jobs[j].n_words, j, k,
                                               list.as<DevRace>(), cap, count.as<uint32_t>(), s));
        }
        uint32_t n = 0;
        HIPCHK(hipMemcpyAsync(&n, count.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (n > cap) {
            cap = n;
            continue;
        }
        got.resize(n);
        if (n) {
            HIPCHK(hipMemcpyAsync(got.data(), list.p, (size_t)n * sizeof(DevRace), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        break;
    }
    std::sort(got.begin(), got.end(), [](const DevRace &a, const DevRace &b) {
        return std::tie(a.unit, a.block, a.addr) < std::tie(b.unit, b.block, b.addr);
    });
    for (auto &r : got) reports[r.unit]->add_race(kc_race{li, 1, 2, r.block, r.epoch, r.addr, r.w, r.o});
    ctx->stat_add("cross_launch_races", (double)got.size());
}

// Races between launches that may run in parallel, for the units of a stage
// (step li): the access summary of each unit whose launch may run in
// parallel with another, from the stage's log, then one scan against each
// earlier such step.
void cross_launch_check(kc_ctx *ctx, Workspace &ws, hipStream_t s, Stage &st, uint32_t li, const kc_job *jobs,
                        const std::vector<uint32_t> &who, const std::vector<LaunchOrder> &order,
                        std::vector<std::vector<DBuf>> &sums, std::vector<kc_report *> &reports) {
    std::vector<uint32_t *> ptr = prepare_summaries(ctx, ws, s, li, jobs, who, order, sums);
    if (std::all_of(ptr.begin(), ptr.end(), [](uint32_t *p) { return p == nullptr; })) return;
    DBuf dptr;
    try {
        dptr.reserve(ptr.size() * sizeof(uint32_t *));
        HIPCHK(hipMemcpyAsync(dptr.p, ptr.data(), ptr.size() * sizeof(uint32_t *), hipMemcpyHostToDevice, s));
        st.summarize(dptr.as<uint32_t *>());
        HIPCHK(hipStreamSynchronize(s));    // `ptr` is read by the copy above
    } catch (...) {
        dptr.release();
        throw;
    }
    dptr.release();
    scan_cross(ctx, s, li, jobs, who, ptr, order, sums, reports);
}

// Copy and host steps (step li of the jobs in `who`): a copy or host write
// takes effect on the job's memory; with streams, its access summary is
// written and scanned against the earlier steps.  Such steps always complete.
void run_item_steps(kc_ctx *ctx, Workspace &ws, hipStream_t s, uint32_t li, const kc_job *jobs,
                    const std::vector<uint32_t> &who, const std::vector<LaunchOrder> &order,
                    std::vector<std::vector<DBuf>> &sums, std::vector<kc_report *> &reports, bool streams) {
    for (uint32_t j : who) {
        const kc_item &it = jobs[j].items[li];
        HIPCHK(launch_item_apply(jobs[j].dev_mem, it.kind, it.dst, it.src, it.words, it.value, s));
        reports[j]->launches_completed = li + 1;
    }
    ctx->stat_add("item_steps", (double)who.size());
    if (!streams) return;
    std::vector<uint32_t *> ptr = prepare_summaries(ctx, ws, s, li, jobs, who, order, sums);
    bool any = false;
    for (size_t i = 0; i < who.size(); i++) {
        if (!ptr[i]) continue;
        const kc_item &it = jobs[who[i]].items[li];
        HIPCHK(launch_item_summary(ptr[i], jobs[who[i]].n_words, it.kind, it.dst, it.src, it.words, s));
        any = true;
    }
    if (any) scan_cross(ctx, s, li, jobs, who, ptr, order, sums, reports);
}

// Run every launch of `jobs` in order, stage by stage (launch index j of all
// jobs still running), and build one report per job.
// With `fixed` (a call that allocates nothing: the calling thread's arena is
// set) the stage buffers are carved from the arena and the interpreter runs
// (the specialised kernels would be compiled and loaded at run time).
void run_jobs(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs, hipStream_t s, std::vector<kc_report *> &reports,
              Workspace *fixed = nullptr) {
    HIPCHK(hipSetDevice(ctx->device));
    Options opt = ctx->options();
    if (fixed) {
        opt.jit = 0;
        opt.arena = 1;
    }
    std::unique_ptr<Workspace> wsp = fixed ? nullptr : ctx->acquire();
    Workspace &ws = fixed ? *fixed : *wsp;
    std::vector<std::vector<DBuf>> sums(n_jobs);
    std::vector<DBuf> allocated(n_jobs);       // memory objects: per job, one bit per allocated word
    auto free_sums = [&]() {
        for (auto &v : sums)
            for (auto &b : v) b.release();
        for (auto &b : allocated) b.release();
    };
    try {
        ws.setup();
        reports.assign(n_jobs, nullptr);
        for (uint32_t j = 0; j < n_jobs; j++) {
            reports[j] = new kc_report();
            reports[j]->tag = jobs[j].tag;
        }
        std::vector<LaunchOrder> order;
        order.reserve(n_jobs);
        bool streams = false;
        for (uint32_t j = 0; j < n_jobs; j++) {
            order.emplace_back(jobs[j]);
            streams |= order.back().any;
        }
        streams &= opt.check != 0;
        bool objects = false;
        for (uint32_t j = 0; j < n_jobs && opt.check; j++) {
            if (!jobs[j].allocs) continue;
            std::vector<uint32_t> bits((jobs[j].n_words + 31) / 32 + 1, 0u);
            for (uint32_t a = 0; a < jobs[j].n_allocs; a++) {
                uint64_t x = jobs[j].allocs[a].base;
                const uint64_t end = x + jobs[j].allocs[a].words;
                for (; x < end && (x & 31); x++) bits[x >> 5] |= 1u << (x & 31);
                for (; x + 32 <= end; x += 32) bits[x >> 5] = 0xFFFFFFFFu;
                for (; x < end; x++) bits[x >> 5] |= 1u << (x & 31);
            }
            allocated[j].acct = &ctx->bytes;
            allocated[j].reserve(bits.size() * 4);
            // on the batch's stream (the null stream would not order it with it)
            HIPCHK(hipMemcpyAsync(allocated[j].p, bits.data(), bits.size() * 4, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));    // `bits` is freed at the end of the iteration
            objects = true;
        }
        std::vector<char> alive(n_jobs, 1);
        uint32_t max_l = 0;
        for (uint32_t j = 0; j < n_jobs; j++) max_l = std::max(max_l, job_steps(jobs[j]));
        for (uint32_t li = 0; li < max_l; li++) {
            std::vector<UnitIn> in;
            std::vector<uint32_t> all_who, item_who;
            for (uint32_t j = 0; j < n_jobs; j++) {
                if (!alive[j] || li >= job_steps(jobs[j])) continue;
                const kc_launch_desc *d = step_launch(jobs[j], li);
                if (d) {
                    in.push_back(UnitIn{d, jobs[j].dev_mem, jobs[j].n_words});
                    all_who.push_back(j);
                } else {
                    item_who.push_back(j);
                }
            }
            if (in.empty() && item_who.empty()) break;
            if (!item_who.empty()) run_item_steps(ctx, ws, s, li, jobs, item_who, order, sums, reports, streams);
            // The units run as one stage unless their record key does not
            // fit (too many units for its fields next to the largest grid,
            // block and memory, or more barrier epochs than its epoch field
            // holds): then the group is halved and each half runs again, its
            // memories back at the launch start.  A single unit that does not
            // fit is KC_E_OVERFLOW.
            std::vector<std::pair<size_t, size_t>> parts;
            if (!in.empty()) parts.push_back({0, in.size()});
            for (size_t pi = 0; pi < parts.size(); pi++) {
            const size_t p0 = parts[pi].first, p1 = parts[pi].second;
            const std::vector<UnitIn> pin(in.begin() + p0, in.begin() + p1);
            const std::vector<uint32_t> who(all_who.begin() + p0, all_who.begin() + p1);
            std::vector<UnitOut> out;
            Stage st{ctx, ws, s, pin, out, opt};
            try {
                st.run();
            } catch (const KcError &e) {
                if (e.st != KC_E_OVERFLOW || p1 - p0 < 2) throw;
                const size_t mid = p0 + (p1 - p0) / 2;
                parts.push_back({p0, mid});
                parts.push_back({mid, p1});
                ctx->stat_add("stage_splits", 1);
                continue;
            }
            ctx->stat_add("launches", (double)pin.size());
            HostTimer ht{ctx, "host_reports_ms", opt.timing != 0};
            std::vector<size_t> first_race(who.size());
            for (size_t i = 0; i < who.size(); i++) {
                kc_report *r = reports[who[i]];
                UnitOut &o = out[i];
                r->records += o.records;
                first_race[i] = r->races.size();
                r->races.reserve(r->races.size() + o.races.size());
                r->sites.reserve(r->sites.size() + o.races.size());
                for (auto &x : o.races) { x.launch = li; r->add_race(x); }
                for (auto &f : o.faults) { f.launch = li; r->faults.push_back(f); }
                if (o.deadlocked) alive[who[i]] = 0;
                else r->launches_completed = li + 1;
            }
            if (streams) cross_launch_check(ctx, ws, s, st, li, jobs, who, order, sums, reports);
            if (objects) {
                std::vector<const uint32_t *> bm(who.size(), nullptr);
                bool any = false;
                for (size_t i = 0; i < who.size(); i++)
                    if (allocated[who[i]].p) bm[i] = allocated[who[i]].as<uint32_t>(), any = true;
                if (any) {
                    DBuf dbm;
                    dbm.reserve(bm.size() * sizeof(uint32_t *));
                    std::vector<std::vector<kc_fault>> found(who.size());
                    try {
                        HIPCHK(hipMemcpyAsync(dbm.p, bm.data(), bm.size() * sizeof(uint32_t *),
                                              hipMemcpyHostToDevice, s));
                        st.illegal_accesses(dbm.as<const uint32_t *>(), found);
                    } catch (...) {
                        dbm.release();
                        throw;
                    }
                    dbm.release();
                    for (size_t i = 0; i < who.size(); i++) {
                        if (found[i].empty()) continue;
                        auto &fv = reports[who[i]]->faults;
                        const size_t first = fv.size() - out[i].faults.size();     // this launch's findings
                        for (auto &f : found[i]) { f.launch = li; fv.push_back(f); }
                        std::sort(fv.begin() + first, fv.end(), fault_less);
                    }
                }
            }
            // last: it runs the replay again over the replay's log, which the
            // stream summaries and memory-object scans read
            if (opt.sites && opt.check) {
                st.sites_pass(out);
                for (size_t i = 0; i < who.size(); i++)
                    std::copy(out[i].sites.begin(), out[i].sites.end(),
                              reports[who[i]]->sites.begin() + first_race[i]);
            }
            }
        }
    } catch (...) {
        free_sums();
        for (auto *r : reports) delete r;
        reports.clear();
        if (wsp) ctx->release(std::move(wsp));
        throw;
    }
    free_sums();
    if (wsp) ctx->release(std::move(wsp));
}

// ---------------------------------------------------------------------------
// Static scratch area of kc_launch_noalloc
// ---------------------------------------------------------------------------
}  // namespace

// Device memory of the calls that allocate nothing: one area per device, part
// of the library's code object, so each device that loads the library holds
// its own copy until the process ends.  Host code never hands this name to a
// kernel or a copy (on the host it is only a stand-in): it reads the device
// address once per device with hipGetSymbolAddress and uses that.
static __device__ __align__(256) unsigned char scratch[KC_NOALLOC_SCRATCH_BYTES];

struct ScratchDevice {
    char *ptr = nullptr;    // device address of `scratch` on this device
    std::mutex mu;          // calls on the device take turns with the area
};

namespace {

std::mutex g_scratch_mu;
std::map<int, std::unique_ptr<ScratchDevice>> g_scratch;

// The scratch area of device `dev`, which must be the current device; its
// address is looked up on the first call for the device.
ScratchDevice *scratch_device(int dev) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) return it->second.get();
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        throw KcError{KC_E_DEVICE, std::string("hipGetSymbolAddress of the static scratch area: ") +
                                       hipGetErrorString(e)};
    }
    auto d = std::make_unique<ScratchDevice>();
    d->ptr = (char *)p;
    return g_scratch.emplace(dev, std::move(d)).first->second.get();
}

// Host staging of the fixed workspace: counters, per-block counts and the
// first findings and races of a launch (made at context creation).
constexpr size_t kFixedPinBytes = 1u << 20;

// Arena of the calling thread for the duration of a call.
struct ArenaUse {
    explicit ArenaUse(Arena *a) { t_arena = a; }
    ~ArenaUse() { t_arena = nullptr; }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// Option writes and statistic reads, under the context lock (batch workers
// read options and add statistics concurrently).
static kc_status set_option_locked(kc_ctx *ctx, const char *key, int64_t v) {
    const std::string k(key);
    std::lock_guard<std::mutex> g(ctx->mu);
    if (k == "check" && (v == 0 || v == 1)) ctx->opt.check = (int)v;
    else if (k == "fuel" && v >= 1 && v <= 0xFFFFFFFFll) ctx->opt.fuel = (uint32_t)v;
    else if (k == "timing" && v >= 0 && v <= 2) ctx->opt.timing = (int)v;
    else if (k == "sort_tile" && (v == 1024 || v == 2048 || v == 4096 || v == 8192)) ctx->opt.sort_tile = (uint32_t)v;
    else if (k == "sort_bits" && v >= 4 && v <= 8) ctx->opt.sort_bits = (uint32_t)v;
    else if (k == "side_streams" && v >= 1 && v <= 4) ctx->opt.side_streams = (uint32_t)v;
    else if (k == "log_records" && v >= 1024) ctx->opt.log_records = (uint64_t)v;
    else if (k == "stage" && (v == 128 || v == 256 || v == 512 || v == 1024)) ctx->opt.stage = (uint32_t)v;
    else if (k == "stage_bytes" && v >= 8192 && v <= 98304) ctx->opt.stage_bytes = (uint32_t)v;
    else if (k == "local" && (v == 0 || v == 1)) ctx->opt.local = (int)v;
    else if (k == "shadow_global" && (v == 0 || v == 1)) ctx->opt.shadow_global = (int)v;
    else if (k == "hash_check" && (v == 0 || v == 1)) ctx->opt.hash_check = (int)v;
    else if (k == "jit" && (v == 0 || v == 1)) ctx->opt.jit = (int)v;
    else if (k == "jit_waves" && (v == 0 || (v >= 2 && v <= 8))) ctx->opt.jit_waves = (int)v;
    else if (k == "sites" && (v == 0 || v == 1)) ctx->opt.sites = (int)v;
    else if (k == "uninit" && (v == 0 || v == 1)) ctx->opt.uninit = (int)v;
    else if (k == "warp" && (v == 0 || v == 1)) ctx->opt.warp = (int)v;
    else if (k == "queue_replay" && (v == 0 || v == 1)) ctx->opt.queue_replay = (int)v;
    else if (k == "onesweep" && (v == 0 || v == 1)) ctx->opt.onesweep = (int)v;
    else if (k == "loc_sort" && (v == 0 || v == 1)) ctx->opt.loc_sort = (int)v;
    else if (k == "sort_spin" && v >= 0 && v <= (1ll << 30)) ctx->opt.sort_spin = (uint32_t)v;
    else if (k == "reset" && v == 1) {
        ctx->stats.clear();
    } else {
        ctx->err = "unknown option or value: " + k;
        return KC_E_INVAL;
    }
    return KC_OK;
}

static double get_stat_locked(kc_ctx *ctx, const char *key) {
    std::lock_guard<std::mutex> g(ctx->mu);
    const std::string k(key);
    if (k == "device_bytes") return (double)ctx->bytes.live.load();
    if (k == "device_bytes_peak") return (double)ctx->bytes.peak.load();
    if (k.rfind("option.", 0) == 0) {
        const std::string o = k.substr(7);
        const Options &op = ctx->opt;
        if (o == "check") return op.check;
        if (o == "fuel") return op.fuel;
        if (o == "timing") return op.timing;
        if (o == "sort_tile") return op.sort_tile;
        if (o == "sort_bits") return op.sort_bits;
        if (o == "side_streams") return op.side_streams;
        if (o == "log_records") return (double)op.log_records;
        if (o == "stage") return op.stage;
        if (o == "stage_bytes") return op.stage_bytes;
        if (o == "local") return op.local;
        if (o == "shadow_global") return op.shadow_global;
        if (o == "hash_check") return op.hash_check;
        if (o == "jit") return op.jit;
        if (o == "jit_waves") return op.jit_waves;
        if (o == "sites") return op.sites;
        if (o == "uninit") return op.uninit;
        if (o == "warp") return op.warp;
        if (o == "queue_replay") return op.queue_replay;
        if (o == "onesweep") return op.onesweep;
        if (o == "loc_sort") return op.loc_sort;
        if (o == "sort_spin") return op.sort_spin;
        return 0.0;
    }
    auto it = ctx->stats.find(key);
    return it == ctx->stats.end() ? 0.0 : it->second;
}

// The items of a job's host program (kc_item), checked against its launches
// and memory; an empty string when they are well formed.
static std::string validate_items(const kc_job &job) {
    if (job.streams) return "streams given with items (each device item names its stream)";
    if (job.n_items > kMaxStreamLaunches) return "more than " + std::to_string(kMaxStreamLaunches) + " items";
    const uint64_t n = job.n_words;
    for (uint32_t i = 0; i < job.n_items; i++) {
        const kc_item &it = job.items[i];
        const std::string at = "item " + std::to_string(i) + ": ";
        switch (it.kind) {
        case KC_ITEM_LAUNCH:
            if (it.ref >= job.n_launches) return at + "launch index out of range";
            break;
        case KC_ITEM_COPY:
            if (it.src > n || it.words > n - it.src) return at + "copy source outside the memory";
            if (it.words && it.src < it.dst + it.words && it.dst < it.src + it.words) return at + "copy ranges overlap";
            [[fallthrough]];
        case KC_ITEM_HOST_READ:
        case KC_ITEM_HOST_WRITE:
            if (it.dst > n || it.words > n - it.dst) return at + "range outside the memory";
            if (it.words > 0xFFFFFFFFull) return at + "more than 2^32 - 1 words";
            break;
        case KC_ITEM_HOST_WAIT:
            if (it.ref != KC_WAIT_ALL && (it.ref >= i || !device_item(job, it.ref)))
                return at + "a wait must name an earlier launch or copy";
            break;
        default:
            return at + "unknown kind";
        }
    }
    return "";
}

// kc_batch_submit's argument checks.
static kc_status validate_jobs(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs) {
    for (uint32_t j = 0; j < n_jobs; j++) {
        if (jobs[j].n_launches && !jobs[j].launches) {
            ctx->err = "job without launch array";
            return KC_E_INVAL;
        }
        for (uint32_t l = 0; l < jobs[j].n_launches; l++) {
            std::string why = validate_desc(&jobs[j].launches[l], jobs[j].dev_mem, jobs[j].n_words);
            if (!why.empty()) {
                ctx->err = "job " + std::to_string(j) + " launch " + std::to_string(l) + ": " + why;
                return KC_E_INVAL;
            }
        }
        if (jobs[j].n_deps && !jobs[j].deps) {
            ctx->err = "job " + std::to_string(j) + ": n_deps without a dependency array";
            return KC_E_INVAL;
        }
        if ((jobs[j].streams || jobs[j].n_deps) && jobs[j].n_launches > kMaxStreamLaunches) {
            ctx->err = "job " + std::to_string(j) + ": more than " + std::to_string(kMaxStreamLaunches) +
                       " launches with streams";
            return KC_E_INVAL;
        }
        for (uint32_t a = 0; jobs[j].allocs && a < jobs[j].n_allocs; a++) {
            const kc_region &g = jobs[j].allocs[a];
            if (g.base > jobs[j].n_words || g.words > jobs[j].n_words - g.base) {
                ctx->err = "job " + std::to_string(j) + " allocation " + std::to_string(a) + ": outside the memory";
                return KC_E_INVAL;
            }
        }
        if (jobs[j].items) {
            std::string why = validate_items(jobs[j]);
            if (!why.empty()) {
                ctx->err = "job " + std::to_string(j) + ": " + why;
                return KC_E_INVAL;
            }
        }
        for (uint32_t d = 0; d < jobs[j].n_deps; d++) {
            const kc_dep &e = jobs[j].deps[d];
            if (e.before >= e.after || e.after >= job_steps(jobs[j]) ||
                !device_item(jobs[j], e.before) || !device_item(jobs[j], e.after)) {
                ctx->err = "job " + std::to_string(j) + " dependency " + std::to_string(d) +
                           (jobs[j].items ? ": needs before < after < n_items, both device items"
                                          : ": needs before < after < n_launches");
                return KC_E_INVAL;
            }
        }
    }
    return KC_OK;
}

// The device bytes a batch's run reserves before any growth (kc_batch_footprint):
// the access log at the context's current record hint with its sort, table
// and replay scratch (40 B per record) and the finding lists at their
// current capacities, whatever the jobs; per step, the launch-start snapshot
// and the direct location tables (9 B per word of the step's memories) and
// per-block lists (28 B per block, and 4 KiB more per block for the held
// representatives while those regions stay small) -- the most of these over
// the steps, since a workspace is reused from step to step; and, held for
// the whole run, an access summary of 8 B per word for each step that may run
// in parallel with another and the allocation bitmaps.  Every term but the
// first grows with the jobs, so the footprint of a batch is at most that of
// no jobs plus, for each job, what it adds on its own.
static uint64_t batch_footprint(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs) {
    const Options op = ctx->options();
    uint32_t fault_cap = 0, lrace_cap = 0;
    ctx->caps(fault_cap, lrace_cap);
    const uint64_t recs = std::max<uint64_t>(op.log_records, 1024);
    uint32_t steps = 0;
    for (uint32_t j = 0; j < n_jobs; j++) steps = std::max(steps, job_steps(jobs[j]));
    // what every batch reserves whatever its jobs: the log and the lists
    const uint64_t fixed = 40 * recs + (uint64_t)fault_cap * sizeof(DevFault) +
                           (uint64_t)lrace_cap * sizeof(DevRace) + (1u << 20);
    uint64_t stage_max = 0, held = 0;
    for (uint32_t li = 0; li < steps; li++) {
        uint64_t words = 0, blocks = 0;
        for (uint32_t j = 0; j < n_jobs; j++) {
            if (li >= job_steps(jobs[j])) continue;
            const kc_launch_desc *d = step_launch(jobs[j], li);
            if (!d) continue;
            words += jobs[j].n_words;
            blocks += (uint64_t)d->grid.x * d->grid.y * d->grid.z;
        }
        uint64_t b = 9 * words + 28 * blocks;
        if (blocks * REP_HOLD * 8 <= (256ull << 20)) b += blocks * (REP_HOLD * 8 + 12);
        stage_max = std::max(stage_max, b);
    }
    for (uint32_t j = 0; j < n_jobs; j++) {
        const LaunchOrder o(jobs[j]);
        if (o.any)
            for (uint32_t li = 0; li < o.n; li++)
                if (o.parallel[li]) held += std::max<uint64_t>(jobs[j].n_words, 1) * 8;
        if (jobs[j].allocs) held += (jobs[j].n_words + 31) / 32 * 4 + 4;
    }
    return fixed + stage_max + held;
}

// The part of kc_batch_submit after validation: copy the batch and start its
// worker thread.
static kc_status submit_batch(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs, void *stream, uint64_t *ticket) {
    auto b = std::make_shared<Batch>();
    b->jobs.assign(jobs, jobs + n_jobs);
    b->descs.resize(n_jobs);
    b->streams.resize(n_jobs);
    b->deps.resize(n_jobs);
    b->allocs.resize(n_jobs);
    b->items.resize(n_jobs);
    for (uint32_t j = 0; j < n_jobs; j++) {
        b->descs[j].assign(jobs[j].launches, jobs[j].launches + jobs[j].n_launches);
        b->jobs[j].launches = b->descs[j].data();
        if (jobs[j].streams) {
            b->streams[j].assign(jobs[j].streams, jobs[j].streams + jobs[j].n_launches);
            b->jobs[j].streams = b->streams[j].data();
        }
        if (jobs[j].n_deps) {
            b->deps[j].assign(jobs[j].deps, jobs[j].deps + jobs[j].n_deps);
            b->jobs[j].deps = b->deps[j].data();
        }
        if (jobs[j].allocs) {
            // one spare entry keeps the pointer non-null for an empty list
            b->allocs[j].assign(jobs[j].allocs, jobs[j].allocs + jobs[j].n_allocs);
            b->allocs[j].push_back(kc_region{0, 0});
            b->jobs[j].allocs = b->allocs[j].data();
        }
        if (jobs[j].items) {
            b->items[j].assign(jobs[j].items, jobs[j].items + jobs[j].n_items);
            b->items[j].push_back(kc_item{});     // keeps the pointer non-null for an empty list
            b->jobs[j].items = b->items[j].data();
        }
    }
    b->stream = (hipStream_t)stream;
    uint64_t t;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        t = ctx->next_ticket++;
        ctx->batches[t] = b;
    }
    Batch *bp = b.get();
    try {
        bp->worker = std::thread([ctx, bp]() {
            kc_status st = KC_OK;
            std::string err;
            std::vector<kc_report *> reps;
            try {
                run_jobs(ctx, bp->jobs.data(), (uint32_t)bp->jobs.size(), bp->stream, reps);
            } catch (...) {
                // nothing may leave the thread function: that would end the process
                const KcError e = current_error();
                st = e.st;
                err = e.msg;
            }
            std::lock_guard<std::mutex> g(bp->mu);
            bp->status = st;
            bp->err = std::move(err);
            bp->reports = std::move(reps);
            bp->done = true;
            bp->cv.notify_all();
        });
    } catch (...) {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->batches.erase(t);
        throw;
    }
    *ticket = t;
    return KC_OK;
}

// kc_poll: wait for (or test) the batch, join its worker once, hand its
// reports over once.
static kc_status poll_batch(kc_ctx *ctx, uint64_t ticket, int wait, kc_report **out, uint32_t n_out) {
    std::shared_ptr<Batch> b;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->batches.find(ticket);
        if (it == ctx->batches.end()) {
            ctx->err = "unknown ticket";
            return KC_E_INVAL;
        }
        b = it->second;
    }
    {
        std::unique_lock<std::mutex> g(b->mu);
        if (!b->done) {
            if (!wait) return KC_E_PENDING;
            b->cv.wait(g, [&] { return b->done; });
        }
    }
    b->join();
    std::vector<kc_report *> reps;
    {
        std::lock_guard<std::mutex> g(b->mu);
        if (b->collected) {
            std::lock_guard<std::mutex> gc(ctx->mu);
            ctx->err = "ticket already collected";
            return KC_E_INVAL;
        }
        if (b->status == KC_OK && (!out || n_out < b->reports.size())) {
            std::lock_guard<std::mutex> gc(ctx->mu);
            ctx->err = "output array too small";
            return KC_E_INVAL;
        }
        b->collected = true;
        reps = std::move(b->reports);
        b->reports.clear();
    }
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->batches.erase(ticket);
    if (b->status != KC_OK) {
        ctx->err = b->err;
        if (b->status == KC_E_DEVICE || b->status == KC_E_INTERNAL) ctx->poisoned = true;
        return b->status;
    }
    for (size_t i = 0; i < reps.size(); i++) out[i] = reps[i];
    return KC_OK;
}

extern "C" {

// Tuned launch parameters: a flat JSON object of integer options written by
// the autotuner, e.g. {"sort_tile": 4096, "stage_bytes": 16384, "local": 1}.
static kc_status apply_tune_cache(kc_ctx *c, const char *path) {
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        c->err = std::string("cannot open tune cache ") + path;
        return KC_E_INVAL;
    }
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    size_t i = 0;
    while ((i = text.find('"', i)) != std::string::npos) {
        const size_t j = text.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = text.substr(i + 1, j - i - 1);
        size_t k = text.find(':', j);
        if (k == std::string::npos) break;
        k++;
        while (k < text.size() && (text[k] == ' ' || text[k] == '\t' || text[k] == '\n')) k++;
        char *end = nullptr;
        const long long v = std::strtoll(text.c_str() + k, &end, 10);
        if (end == text.c_str() + k) {
            c->err = "tune cache: value of " + key + " is not an integer";
            return KC_E_INVAL;
        }
        kc_status st = kc_ctx_set_option(c, key.c_str(), (int64_t)v);
        if (st != KC_OK) return st;
        i = (size_t)(end - text.c_str());
    }
    return KC_OK;
}

kc_status kc_ctx_create(int hip_device, uint64_t hbm_budget_bytes, const char *tune_cache, kc_ctx **out) {
    if (!out) return KC_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
        (void)hipGetLastError();
        return KC_E_INVAL;
    }
    if (hipSetDevice(hip_device) != hipSuccess) return KC_E_DEVICE;
    kc_ctx *c = nullptr;
    try {
        c = new kc_ctx();
        c->device = hip_device;
        c->budget = hbm_budget_bytes;
        c->scratch = scratch_device(hip_device);
        c->fixed_ws = std::make_unique<Workspace>();
        c->fixed_ws->setup();
        c->fixed_ws->pin_reserve(kFixedPinBytes);
        if (tune_cache && *tune_cache) {
            kc_status st = apply_tune_cache(c, tune_cache);
            if (st != KC_OK) {
                delete c;
                return st;
            }
        }
    } catch (...) {
        delete c;
        return current_error().st;
    }
    *out = c;
    return KC_OK;
}

void kc_ctx_destroy(kc_ctx *ctx) {
    if (!ctx) return;
    std::vector<std::shared_ptr<Batch>> pending;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        for (auto &kv : ctx->batches) pending.push_back(kv.second);
    }
    for (auto &b : pending) {
        try {
            b->join();
        } catch (...) {
            // joining failed (the worker cannot be waited for): the reports it
            // may still write are leaked rather than freed under it
            continue;
        }
        for (auto *r : b->reports) delete r;
        b->reports.clear();
    }
    (void)hipSetDevice(ctx->device);
    ctx->free_ws.clear();
    ctx->fixed_ws.reset();
    delete ctx;
}

kc_status kc_ctx_set_option(kc_ctx *ctx, const char *key, int64_t v) {
    if (!ctx || !key) return KC_E_INVAL;
    return guarded(ctx, [&] { return set_option_locked(ctx, key, v); });
}

double kc_ctx_get_stat(kc_ctx *ctx, const char *key) {
    if (!ctx || !key) return 0.0;
    try {
        return get_stat_locked(ctx, key);
    } catch (...) {
        return 0.0;
    }
}

const char *kc_last_error(const kc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

kc_status kc_program_load(kc_ctx *ctx, const uint64_t *words, uint32_t n_words, kc_program **out) {
    if (!ctx || !out || (!words && n_words)) return KC_E_INVAL;
    *out = nullptr;
    if (ctx->poisoned) return KC_E_DEVICE;
    std::string why = validate_program(words, n_words);
    if (!why.empty()) {
        ctx->err = why;
        return KC_E_PROGRAM;
    }
    kc_program *p = nullptr;
    try {
        p = new kc_program();
        p->words.assign(words, words + n_words);
        p->device = ctx->device;
        HIPCHK(hipSetDevice(ctx->device));
        HIPCHK(hipMalloc(&p->dev, (size_t)n_words * 8));
        HIPCHK(hipMemcpy(p->dev, words, (size_t)n_words * 8, hipMemcpyHostToDevice));
    } catch (...) {
        if (p && p->dev) (void)hipFree(p->dev);
        delete p;
        return fail(ctx, current_error());
    }
    *out = p;
    return KC_OK;
}

void kc_program_free(kc_program *p) {
    if (!p) return;
    if (p->dev) {
        (void)hipSetDevice(p->device);
        (void)hipFree(p->dev);
    }
    delete p;
}

kc_status kc_launch(kc_ctx *ctx, const kc_launch_desc *desc, int32_t *dev_mem, uint64_t n_words, void *stream,
                    kc_report **out) {
    if (!ctx || !out) return KC_E_INVAL;
    *out = nullptr;
    if (ctx->poisoned) return KC_E_DEVICE;
    std::string why = validate_desc(desc, dev_mem, n_words);
    if (!why.empty()) {
        ctx->err = why;
        return KC_E_INVAL;
    }
    return guarded(ctx, [&] {
        HostTimer lt{ctx, "host_launch_ms", ctx->options().timing != 0};
        kc_job job{desc, 1, dev_mem, n_words, 0};
        std::vector<kc_report *> reps;
        run_jobs(ctx, &job, 1, (hipStream_t)stream, reps);
        *out = reps[0];
        return KC_OK;
    });
}

kc_status kc_launch_noalloc(kc_ctx *ctx, const kc_launch_desc *desc, int32_t *dev_mem, uint64_t n_words,
                            void *stream, kc_report **out) {
    if (!ctx || !out) return KC_E_INVAL;
    *out = nullptr;
    if (ctx->poisoned) return KC_E_DEVICE;
    std::string why = validate_desc(desc, dev_mem, n_words);
    if (!why.empty()) {
        ctx->err = why;
        return KC_E_INVAL;
    }
    return guarded(ctx, [&] {
        if (n_words * 4 > KC_NOALLOC_SCRATCH_BYTES)      // the launch-start snapshot alone would not fit
            throw KcError{KC_E_BUDGET, "memory of " + std::to_string(n_words) +
                                           " words exceeds the static scratch area"};
        std::lock_guard<std::mutex> g(ctx->scratch->mu);
        Arena arena;
        arena.base = ctx->scratch->ptr;
        arena.cap = KC_NOALLOC_SCRATCH_BYTES;
        ArenaUse use(&arena);
        ctx->fixed_ws->forget_carved();         // the previous call's buffers
        kc_job job{desc, 1, dev_mem, n_words, 0};
        std::vector<kc_report *> reps;
        run_jobs(ctx, &job, 1, (hipStream_t)stream, reps, ctx->fixed_ws.get());
        ctx->stat_add("noalloc_calls", 1);
        ctx->stat_max("noalloc_scratch_peak", (double)arena.peak);
        *out = reps[0];
        return KC_OK;
    });
}

kc_status kc_batch_submit(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs, void *stream, uint64_t *ticket) {
    if (!ctx || !ticket || (!jobs && n_jobs)) return KC_E_INVAL;
    if (ctx->poisoned) return KC_E_DEVICE;
    return guarded(ctx, [&] {
        const kc_status st = validate_jobs(ctx, jobs, n_jobs);
        return st != KC_OK ? st : submit_batch(ctx, jobs, n_jobs, stream, ticket);
    });
}

kc_status kc_batch_footprint(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs, uint64_t *bytes) {
    if (!ctx || !bytes || (!jobs && n_jobs)) return KC_E_INVAL;
    return guarded(ctx, [&] {
        // the memories need not exist yet: validate with a stand-in address
        std::vector<kc_job> v(jobs, jobs + n_jobs);
        for (auto &j : v)
            if (!j.dev_mem) j.dev_mem = reinterpret_cast<int32_t *>(uintptr_t{256});
        const kc_status st = validate_jobs(ctx, v.data(), n_jobs);
        if (st != KC_OK) return st;
        *bytes = batch_footprint(ctx, v.data(), n_jobs);
        return KC_OK;
    });
}

kc_status kc_poll(kc_ctx *ctx, uint64_t ticket, int wait, kc_report **out, uint32_t n_out) {
    if (!ctx) return KC_E_INVAL;
    return guarded(ctx, [&] { return poll_batch(ctx, ticket, wait, out, n_out); });
}

uint64_t kc_report_records(const kc_report *r) { return r ? r->records : 0; }
uint32_t kc_report_launches_completed(const kc_report *r) { return r ? r->launches_completed : 0; }
const kc_race *kc_report_races(const kc_report *r, uint64_t *n) {
    if (n) *n = r ? r->races.size() : 0;
    return r && !r->races.empty() ? r->races.data() : nullptr;
}
const kc_race_site *kc_report_race_sites(const kc_report *r, uint64_t *n) {
    if (n) *n = r ? r->sites.size() : 0;
    return r && !r->sites.empty() ? r->sites.data() : nullptr;
}
const kc_fault *kc_report_faults(const kc_report *r, uint64_t *n) {
    if (n) *n = r ? r->faults.size() : 0;
    return r && !r->faults.empty() ? r->faults.data() : nullptr;
}
uint64_t kc_report_tag(const kc_report *r) { return r ? r->tag : 0; }
void kc_report_free(kc_report *r) { delete r; }

kc_status kc_reports_collect(kc_report *const *reports, uint32_t n, uint64_t *records, uint32_t *launches,
                             uint64_t *tags, uint64_t *n_races, uint64_t *n_faults, kc_race *races,
                             kc_fault *faults, kc_race_site *sites) {
    if (n && !reports) return KC_E_INVAL;
    uint64_t ro = 0, fo = 0;
    for (uint32_t i = 0; i < n; i++) {
        const kc_report *r = reports[i];
        if (!r) return KC_E_INVAL;
        if (records) records[i] = r->records;
        if (launches) launches[i] = r->launches_completed;
        if (tags) tags[i] = r->tag;
        if (n_races) n_races[i] = r->races.size();
        if (n_faults) n_faults[i] = r->faults.size();
        if (races && !r->races.empty()) std::memcpy(races + ro, r->races.data(), r->races.size() * sizeof(kc_race));
        if (sites && !r->sites.empty())
            std::memcpy(sites + ro, r->sites.data(), r->sites.size() * sizeof(kc_race_site));
        if (faults && !r->faults.empty())
            std::memcpy(faults + fo, r->faults.data(), r->faults.size() * sizeof(kc_fault));
        ro += r->races.size();
        fo += r->faults.size();
    }
    return KC_OK;
}

void kc_reports_free(kc_report *const *reports, uint32_t n) {
    if (!reports) return;
    for (uint32_t i = 0; i < n; i++) delete reports[i];
}

}  // extern "C"
