// Internal structures shared by the HIP kernels and the host runtime of libkc.
// The part above the host-only section is also compiled at run time (hiprtc)
// into the program-specialised kernels, where the HIP runtime header is
// implicit.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace kc {

// ---- instruction set ------------------------------------------------------
enum : uint32_t {
    OP_ADD = 0x01, OP_SUB, OP_MUL, OP_DIV, OP_REM, OP_AND, OP_OR, OP_XOR,
    OP_SHL, OP_SHRA, OP_SHRL, OP_MIN, OP_MAX, OP_SLT, OP_SLE, OP_SEQ, OP_SNE, OP_SLTU,
    OP_IMM = 0x20,
    OP_MOV = 0x40, OP_MOVI = 0x41, OP_SREG = 0x42,
    OP_LDS = 0x50, OP_STS = 0x51, OP_LDG = 0x52, OP_STG = 0x53,
    OP_JMP = 0x60, OP_BZ = 0x61, OP_BNZ = 0x62, OP_BAR = 0x63, OP_EXIT = 0x64,
    OP_BARP = 0x65,     // barrier with a predicate: d = count / and / or (imm 0 / 1 / 2) of register a
};
constexpr uint32_t N_SREGS = 24;
constexpr uint32_t MAX_INSTR = 1u << 16;
constexpr uint32_t MAX_THREADS = 1024;
constexpr uint32_t MAX_SHMEM_WORDS = 16384;     // 64 KiB of simulated shared memory
// Representative records a block holds in LDS (with the global shadow table)
// before it reserves log space for them: one reservation per block in the
// common case instead of one per epoch, since every block of a launch
// reserves on the same counter.
constexpr uint32_t REP_HOLD = 512;
// Representatives a block of `wg_threads` threads holds in LDS (at most
// REP_HOLD): small blocks touch few locations, and a smaller buffer lets more
// of them share a CU.
__host__ __device__ inline uint32_t rep_hold_for(uint32_t wg_threads) {
    const uint32_t h = 2 * wg_threads;
    return h < 128u ? 128u : (h > REP_HOLD ? REP_HOLD : h);
}

enum : uint32_t { F_DEADLOCK = 1, F_DIVERGENCE = 2, F_OOB = 3, F_FUEL = 4, F_ARITH = 5, F_ALLOC = 6, F_UNINIT = 7 };

// ---- one (instance, launch) as the device sees it -------------------------
struct DevUnit {
    const uint64_t *prog;
    int32_t *mem;           // caller's memory (final memory lands here)
    const int32_t *snap;    // launch-start snapshot of mem
    uint32_t n_instr;
    uint32_t n_words;
    uint32_t gdim[3];
    uint32_t bdim[3];
    uint32_t nt, nb;
    uint32_t sh_words;
    uint32_t fuel;
    int32_t params[8];
    uint32_t block_base;    // index of block 0 in the per-block arrays
    uint32_t pad;
};

// Bit layout of a 64-bit access record, least significant field first:
//   kind(1) | tid(tb) | epoch(eb) | block(bb) | addr(ab) | space(1) | unit(ub)
// The sort orders records by the bits above tid; kind and tid ride along.
struct KeyPlan {
    uint32_t tb, eb, bb, ab, ub;
    uint32_t s_tid, s_ep, s_blk, s_addr, s_sp, s_unit, total;
    uint32_t max_epoch;     // largest epoch a block may reach
    uint32_t ep_rep;        // reserved epoch value of representative records
};

__host__ __device__ inline uint64_t rec_pack(const KeyPlan &k, uint32_t unit, uint32_t space, uint32_t addr,
                                             uint32_t block, uint32_t epoch, uint32_t tid, uint32_t kind) {
    return (uint64_t)kind | ((uint64_t)tid << k.s_tid) | ((uint64_t)epoch << k.s_ep) |
           ((uint64_t)block << k.s_blk) | ((uint64_t)addr << k.s_addr) | ((uint64_t)space << k.s_sp) |
           ((uint64_t)unit << k.s_unit);
}
__host__ __device__ inline uint32_t rec_field(uint64_t r, uint32_t shift, uint32_t width) {
    return width ? (uint32_t)((r >> shift) & ((1ull << width) - 1)) : 0u;
}

struct DevFault { uint32_t unit, kind, block, epoch, a, b, c, d; };
struct DevRace { uint32_t unit, space, scope, block, epoch, addr, w, o; };
// An access of the replay with its lockstep step (warp-aware model):
// tsk = tid | kind << 16 | space << 17.
struct WarpRec { uint32_t unit, block, epoch, step, addr, tsk; };
struct DevEdge { uint32_t unit, b0, b1, pad; };

// flags word bits
enum : uint32_t {
    FLAG_LOG_OVERFLOW = 1u << 0,
    FLAG_FAULT_OVERFLOW = 1u << 1,
    FLAG_EPOCH_OVERFLOW = 1u << 2,
    FLAG_RACE_OVERFLOW = 1u << 3,
    FLAG_EDGE_OVERFLOW = 1u << 4,
    FLAG_MISMATCH = 1u << 5,
    FLAG_NEED_SORT = 1u << 6,   // the replay's records need the sorted check
    FLAG_WLOG_OVERFLOW = 1u << 7,   // the replay's step-stamped accesses did not fit
};

// Counters in one small device block (zeroed before a stage).
struct DevCounters {
    unsigned long long log_count;
    unsigned long long aux_count;
    uint32_t fault_count;
    uint32_t race_count;
    uint32_t edge_count;
    uint32_t flags;
    uint32_t max_epoch;
    uint32_t pad0;
    unsigned long long instructions;   // thread-instructions of the free run
    uint32_t long_count;               // segments left to the long-segment pass of the check
    uint32_t racy_words;               // free run: shared words found racy by the verdicts (all epochs)
    uint32_t wlog_count;               // replay: step-stamped accesses (warp-aware model)
    uint32_t pad[3];
};

// Source sites of race tuples: one slot per tuple of an open-addressing
// table keyed by (unit, space, block, epoch, addr) -- block and epoch
// 0xFFFFFFFF for a cross-block tuple, whose w and o are global thread ids.
// A replay with the table (InterpArgs::sites) lowers w_pc to the smallest pc
// of w's stores to the location and o_pc to the smallest pc of o's accesses
// to it (atomicMin; both start at 0xFFFFFFFF).
struct SiteSlot {
    uint32_t unit, space, block, epoch, addr, w, o, used;
    uint32_t w_pc, o_pc, pad0, pad1;
};
__host__ __device__ inline uint32_t site_hash(uint32_t unit, uint32_t space, uint32_t block, uint32_t epoch,
                                              uint32_t addr) {
    uint32_t h = addr * 0x9E3779B1u;
    h ^= (block + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= (epoch + 0x165667B1u) * 0xC2B2AE3Du;
    h ^= (unit * 2u + space) * 0x27D4EB2Fu;
    return h ^ (h >> 15);
}

struct InterpArgs {
    const DevUnit *units;
    const uint2 *items;         // (unit, block) per workgroup; null: unit 0, block = blockIdx.x
    const uint32_t *comp_off;   // lockstep replay: blocks of component c are comp_blocks[comp_off[c] .. comp_off[c+1])
    const uint2 *comp_blocks;   // (unit, block)
    // When set, the components are single blocks comp_blocks[0 .. *n_comps_dev)
    // (a count written on the device) and workgroups stride over them.
    const uint32_t *n_comps_dev;
    uint32_t rep_hold;              // representatives a block holds in LDS (rep_hold_for its size)
    KeyPlan kp;
    uint64_t *log;
    unsigned long long log_cap;
    unsigned long long *log_count;
    DevFault *faults;
    uint32_t fault_cap;
    uint32_t *fault_count;
    uint32_t *blk_recs;         // per-block record counts (added to)
    uint32_t *flags;
    uint32_t *max_epoch;        // largest epoch reached (atomicMax)
    uint32_t sh_words_max;      // simulated shared words reserved in LDS
    uint32_t stage;             // staged records per wave (multiple of 64)
    uint32_t local;             // check each epoch's records in LDS (free run)
    DevRace *lraces;            // races found by the epoch-local check
    uint32_t lrace_cap;
    uint32_t *lrace_count;
    uint32_t *blk_flags;        // racy blocks
    uint32_t *racy_words;       // free run: count of shared words the verdicts found racy (sizes the replay's lists)
    uint32_t *blk_instr;        // free run: thread-instructions executed, per block (stored), or null
    uint32_t *blk_grecs;        // free run: in-bounds global accesses, per block (stored), or null
    uint32_t uninit;            // check loads of shared words no thread of the block stored to before
    // Warp-aware model (replay only): every access with its lockstep step goes
    // to wlog, and the replay itself reports no intra-block races.
    WarpRec *wlog;
    uint32_t wlog_cap;
    uint32_t *wlog_count;
    uint32_t gst_bits;          // local check: log2 slots of the global shadow table (0: stage and sort)
    uint32_t site_bits;         // log2 slots of `sites`
    SiteSlot *sites;            // lockstep replay for source sites, or null
    // With the shadow table: when set, each block writes its held
    // representatives to its own region (REP_HOLD records at block_base +
    // block) and their number to blk_held, instead of reserving log space on
    // the shared counter; launch_held_compact appends them to the log.
    uint64_t *blk_log;
    uint32_t *blk_held;
};

#ifndef __HIPCC_RTC__
// ---- host side ----------------------------------------------------------------
// Launchers (defined in the .hip files).
hipError_t launch_interp(const InterpArgs &a, uint32_t n_wg, uint32_t wg_threads, bool lockstep, hipStream_t s);
size_t interp_lds_bytes(uint32_t sh_words_max, uint32_t wg_threads, uint32_t stage, bool lockstep, bool local,
                        uint32_t gst_bits);
// Size (log2 slots) of the global shadow table for a workgroup: four slots per
// thread, at least 256.
uint32_t gst_bits_for(uint32_t wg_threads);

// Single-pass digit scatter: at most this many passes (64 bits, 4-bit digits),
// and its counters: per pass 256 digit counts and 256 digit bases, and the
// stall word.
constexpr uint32_t RADIX_OS_PASSES = 16;
constexpr size_t RADIX_OS_WORDS = 2 * RADIX_OS_PASSES * 256 + 1;
constexpr uint64_t RADIX_OS_MIN_KEYS = 1ull << 20;

struct SortScratch {
    uint64_t *alt = nullptr;         // ping-pong buffer, >= n keys
    uint32_t *hist = nullptr;        // 256 * n_tiles, digit-major (single-pass scatter: twice that)
    uint32_t *part = nullptr;        // 256 digit totals
    uint32_t *os = nullptr;          // RADIX_OS_WORDS, or null: no single-pass scatter
    uint32_t spin = 1u << 16;        // bound of each look-back wait (polls)
    uint32_t *stall = nullptr;       // set by radix_sort when the single-pass scatter ran
    size_t cap_keys = 0, cap_hist = 0, cap_part = 0;
};
// Virtual sort key of a record: the bits from s_blk up, then the low ueb bits
// of the epoch field, then the low pb bits (payload); vbits bits in all.
struct VKey {
    uint32_t s_ep, ueb, s_blk, pb, vbits;
};
// Sort keys[0..n) ascending by the virtual key (stable), `digit` bits (4..8)
// per pass over inputs larger than one workgroup's.  *out points at the
// sorted array: keys itself or scratch.alt.
// With scratch.os set and radix_onesweep(n), the passes are single-pass
// scatters and scratch.stall points at the device word that is 0 when they all
// ran, else the first stalled pass + 1: then radix_sort_resume(pass) finishes
// the sort (from that pass's input) and sets *out again.
hipError_t radix_sort(uint64_t *keys, uint64_t n, const VKey &vk, SortScratch &sc,
                      uint32_t tile, hipStream_t s, uint64_t **out, uint32_t digit = 8);
hipError_t radix_sort_resume(uint64_t *keys, uint64_t n, const VKey &vk, SortScratch &sc, uint32_t tile,
                             hipStream_t s, uint64_t **out, uint32_t digit, uint32_t pass);
bool radix_onesweep(uint64_t n);
size_t radix_hist_entries(uint64_t n, uint32_t tile);

struct CheckArgs {
    const uint64_t *keys;
    uint64_t n;
    KeyPlan kp;
    const DevUnit *units;
    DevRace *races;
    uint32_t race_cap;
    DevEdge *edges;
    uint32_t edge_cap;
    uint32_t *blk_flags;
    DevCounters *ctr;
    uint64_t *longseg;          // scratch: segments longer than the serial limit, check_long_cap(n) entries
};
size_t check_long_cap(uint64_t n);
hipError_t launch_check(const CheckArgs &a, hipStream_t s);
// *flag |= 1 when keys[0, n) holds a record other than a global-memory
// representative (the caller zeroes *flag).
hipError_t launch_log_reps_only(const uint64_t *keys, uint64_t n, KeyPlan kp, uint32_t *flag, hipStream_t s);
hipError_t launch_restore(const uint64_t *keys, uint64_t n, KeyPlan kp, const DevUnit *units,
                          const uint32_t *blk_flags, hipStream_t s, const unsigned long long *n_dev = nullptr);
struct ZeroArgs;
// The blocks flagged in blk_flags (n_blocks, global block indices of the
// units), in ascending order, as (unit, block) pairs into comps, and their
// number into *n_comps: one workgroup, which first clears the buffers of
// `zero` (if given).
hipError_t launch_flagged_comps(const uint32_t *blk_flags, uint32_t n_blocks, const DevUnit *units, uint32_t n_units,
                                uint2 *comps, uint32_t *n_comps, hipStream_t s, const ZeroArgs *zero = nullptr);
// Exactness of a replay; sets FLAG_MISMATCH in ctr->flags.  ctr->long_count
// must be zero; `list` holds n_rs entries.
hipError_t launch_coverage(const uint64_t *rs, uint64_t n_rs, const uint64_t *log, uint64_t n_log, KeyPlan kp,
                           const DevUnit *units, const uint32_t *blk_flags, DevCounters *ctr, uint64_t *list,
                           hipStream_t s);
// Exactness of a replay without sorting its records, for the common case:
// every replayed record is a representative (epoch ep_rep) and no global
// location is written by one replayed block and touched by another.  Sets
// FLAG_MISMATCH as launch_coverage would, or FLAG_NEED_SORT when the case does
// not hold (or a location has more free-run records than the scan takes), in
// which case the caller sorts and checks as usual.  2^bits >= 2 n_rs.
struct ReplayTableArgs {
    const uint64_t *rs;         // the replay's records (any order)
    uint64_t n_rs;
    const uint64_t *log;        // the free run's records, sorted
    uint64_t n_log;
    KeyPlan kp;
    const DevUnit *units;
    const uint32_t *blk_flags;  // replayed blocks
    void *table;                // 8 << bits bytes
    uint32_t bits;
    DevCounters *ctr;
    const void *ftable;         // when the free-run log is not sorted: its location table (launch_log_table)
    uint32_t fbits;
    uint32_t obits;             // width of the block field of a table word; location bits + obits + 2 <= 64
    // Direct tables, one entry per memory word of every unit (word index =
    // unit snapshot - snap_base + address), used instead of the hash table
    // when memories are small next to the log: the block + 1 of a record that
    // touched the word (0: untouched), and flags (bit 0 written, bit 1 several
    // blocks).  With downer set, the replay looks locations up there.
    const int32_t *snap_base;
    uint32_t *downer;
    uint8_t *dflags;
    // When set, the number of records is read here on the device (the log's
    // counter), and n_rs is only its capacity: the tables can be queued
    // behind the kernel that writes the log.
    const unsigned long long *n_dev;
};
hipError_t launch_replay_table(const ReplayTableArgs &a, hipStream_t s);
// The free run's conflict check without sorting, for the common case: every
// record is a representative and no global location is written by one block
// and touched by another.  Builds the location table of the log (rs, n_rs;
// 2^bits >= 2 n_rs) and sets FLAG_NEED_SORT in
// ctr->flags when the case does not hold; otherwise there are no cross-block
// races or links and the epoch-local races are all the races.
hipError_t launch_log_table(const ReplayTableArgs &a, hipStream_t s);
// The same check through the direct tables (rs, n_rs, kp, units, snap_base,
// downer, dflags; `words` entries, zeroed here).
hipError_t launch_log_direct(const ReplayTableArgs &a, uint64_t words, hipStream_t s);
// Access summaries of launches that may run in parallel with another launch
// of their job: for each unit u with sums[u] set, sums[u][x] becomes the
// smallest global thread id among the records of global word x and
// sums[u][n_words + x] the smallest among its writes (atomicMin: the arrays
// start at 0xFFFFFFFF).  Records of blocks flagged in skip_blocks (global
// block index) or of units flagged in skip_units are left out.
struct SummaryArgs {
    const uint64_t *log;
    uint64_t n;
    const unsigned long long *n_dev;    // when set, the record count is read here (at most n)
    KeyPlan kp;
    const DevUnit *units;
    uint32_t *const *sums;
    const uint32_t *skip_blocks;
    const uint32_t *skip_units;
};
hipError_t launch_summary(const SummaryArgs &a, hipStream_t s);
// Memory objects: the records of a log whose global word lies outside the
// unit's allocations (allocated[u]: one bit per word, bit x % 32 of word
// x / 32; null: no check) are copied to out (cap entries; *count counts them
// all).  Skips as for launch_summary.
struct AllocScanArgs {
    const uint64_t *log;
    uint64_t n;
    KeyPlan kp;
    const DevUnit *units;
    const uint32_t *const *allocated;
    const uint32_t *skip_blocks;
    const uint32_t *skip_units;
    uint64_t *out;
    uint32_t cap;
    uint32_t *count;
};
hipError_t launch_alloc_scan(const AllocScanArgs &a, hipStream_t s);
// Append the representatives the blocks of a free run held in their regions
// (blk_log, blk_held; n_blocks blocks) to the log after the records already
// counted in *log_count, and add them to it (FLAG_LOG_OVERFLOW in *flags
// beyond log_cap).  blk_off: n_blocks scratch entries.
hipError_t launch_held_compact(const uint64_t *blk_log, const uint32_t *blk_held, uint64_t *blk_off,
                               uint32_t n_blocks, uint64_t *log, unsigned long long log_cap,
                               unsigned long long *log_count, uint32_t *flags, hipStream_t s);
// Races between launch `earlier` (summary si) and a later launch (sj) over
// n_words words, appended to out (cap entries; *count counts them all) with
// unit = tag.
hipError_t launch_cross_launch(const uint32_t *si, const uint32_t *sj, uint64_t n_words, uint32_t tag,
                               uint32_t earlier, DevRace *out, uint32_t cap, uint32_t *count, hipStream_t s);
// Items of a job's host program: apply a copy or a host write (KC_ITEM_*
// kind; other kinds do nothing) to mem, and write the access summary of a
// copy or host access into sum (2 * n_words words, preset to 0xFFFFFFFF).
hipError_t launch_item_apply(int32_t *mem, uint32_t kind, uint64_t dst, uint64_t src, uint64_t words, int32_t value,
                             hipStream_t s);
hipError_t launch_item_summary(uint32_t *sum, uint64_t n_words, uint32_t kind, uint64_t dst, uint64_t src,
                               uint64_t words, hipStream_t s);
hipError_t launch_copy_units(const DevUnit *units, uint32_t n_units, uint32_t max_words, bool to_snapshot,
                             const uint32_t *unit_mask, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// Zero up to 8 buffers (whole words) with one kernel launch.
struct ZeroArgs {
    uint32_t *p[8];
    size_t words[8];
    uint32_t n;
};
hipError_t launch_zero_many(const ZeroArgs &z, hipStream_t s);
// Word copies of up to GATHER_MAX device arrays into one destination
// (host-visible pinned memory), at word offsets.
constexpr uint32_t GATHER_MAX = 16;     // buffers one gather launch copies
struct GatherArgs {
    const uint32_t *src[GATHER_MAX];
    uint32_t words[GATHER_MAX];
    uint32_t dst_off[GATHER_MAX];
    uint32_t *dst;
    uint32_t n;
};
hipError_t launch_gather(const GatherArgs &a, hipStream_t s);
#endif  // __HIPCC_RTC__

}  // namespace kc
