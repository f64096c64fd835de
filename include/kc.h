/*
 * kc.h -- C ABI of the MI355X SIMT race and deadlock checker (version 1).
 *
 * The library executes kernels written in KC-IR (see the instruction format
 * below) SIMT-style on the GPU, one lane per simulated thread, logs every
 * in-bounds memory access with its barrier epoch, and reports the canonical
 * race, barrier-divergence and deadlock findings of the execution together
 * with the final device memory.  The checked properties are those of
 * Hathhorn et al., "Formal Semantics of Heterogeneous CUDA-C" (SSV 2012),
 * Section 3.1 (race and deadlock detection), with the barrier semantics of
 * Section 3 ("Barrier synchronization") and the launch/stream model of
 * Section 2.
 *
 * Conventions
 *   - All integers are little-endian; memory sizes are in 32-bit words unless
 *     a name says bytes.  Device pointers are plain HIP device addresses
 *     (for example the data pointer of a torch int32 tensor on the GPU).
 *   - Functions return kc_status.  Races, divergence and deadlocks are
 *     findings, not errors: a run with findings returns KC_OK and a
 *     non-empty report.  On an error kc_last_error() describes it.
 *   - KC_E_DEVICE means a HIP call failed; the context is then poisoned and
 *     every later call on it returns KC_E_DEVICE.  KC_E_INTERNAL (an
 *     unexpected failure inside the library) poisons it too.  No C++
 *     exception ever leaves an entry point or a batch's worker thread.
 *   - A context is not thread-safe, except that kc_poll may be called from
 *     several threads (each ticket is handed over once), and that
 *     kc_ctx_set_option and kc_ctx_get_stat may be called while batches
 *     run: a call uses the options as they were when it started.
 *
 * Instruction format (KC-IR v1): one 64-bit word per instruction,
 *   op = bits 0..7, d = 8..15, a = 16..23, b = 24..31, imm = 32..63 (int32).
 * Opcodes: ADD 0x01 SUB 0x02 MUL 0x03 DIV 0x04 REM 0x05 AND 0x06 OR 0x07
 * XOR 0x08 SHL 0x09 SHRA 0x0A SHRL 0x0B MIN 0x0C MAX 0x0D SLT 0x0E SLE 0x0F
 * SEQ 0x10 SNE 0x11 SLTU 0x12 (d = a OP b); the same | 0x20 take imm for b;
 * MOV 0x40 (d = a), MOVI 0x41 (d = imm), SREG 0x42 (d = special imm),
 * LDS 0x50 (d = shared[a+imm]), STS 0x51 (shared[a+imm] = b),
 * LDG 0x52 (d = global[a+imm]), STG 0x53 (global[a+imm] = b),
 * JMP 0x60, BZ 0x61 (if a == 0), BNZ 0x62 (if a != 0) to absolute pc imm,
 * BAR 0x63 (__syncthreads), EXIT 0x64, BARP 0x65 (a barrier with a
 * predicate, Section 3's __syncthreads_count / _and / _or for imm 0 / 1 / 2:
 * when the episode completes, d = the number of threads of the block whose
 * register a is nonzero, 1 if all are, or 1 if any is; a thread waiting at a
 * plain BAR in the same episode counts as 0).  Special registers: 0..2 threadIdx
 * x/y/z, 3..5 blockIdx, 6..8 blockDim, 9..11 gridDim, 12 linear tid,
 * 13 linear block id, 14 threads per block, 15 warpSize (32), 16..23 the
 * launch parameters.  Registers r0..r15 are int32 and start at 0.
 *
 * Semantics of a run (the canonical execution the reports describe)
 *   - A job is one memory plus launches run in order, as in one stream
 *     (Section 2).  A launch in which some block deadlocks does not complete
 *     and ends the job.
 *   - Blocks execute in ascending linear block id; inside a block all
 *     running threads step in lockstep (loads of a step see memory as of the
 *     step's start, stores land in ascending tid order).  Race-free launches
 *     have this outcome under every interleaving; for racy launches it is the
 *     convention that reproduces the paper's printed outputs.
 *   - int32 arithmetic wraps; x/0 and x%0 give 0 and an ARITH finding;
 *     INT_MIN/-1 = INT_MIN, INT_MIN%-1 = 0; shifts use the low 5 bits of the
 *     count.  Out-of-bounds accesses give an OOB finding, load 0 / drop the
 *     store and are not logged.  Shared memory starts zeroed.  A thread may
 *     execute at most `fuel` instructions (default 2^20), then exits with a
 *     FUEL finding.  Falling off the end of the program is an exit.
 */
#ifndef KC_H
#define KC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KC_OK = 0,
    KC_E_INVAL = 1,     /* bad argument: dims, sizes, null pointers, unknown option */
    KC_E_PROGRAM = 2,   /* program failed validation at load */
    KC_E_NOMEM = 3,     /* device or host allocation failed */
    KC_E_DEVICE = 4,    /* a HIP call failed; the context is poisoned */
    KC_E_PENDING = 5,   /* kc_poll without wait: the batch is still running */
    KC_E_BUDGET = 6,    /* the job can never fit in the context's HBM budget */
    KC_E_OVERFLOW = 7,  /* one launch's ids and barrier epochs do not fit the 64-bit access record even on
                           its own (launches of a batch that do not fit together run in smaller groups) */
    KC_E_INTERNAL = 8   /* an unexpected internal failure of the library; the context is poisoned */
} kc_status;

typedef struct kc_ctx kc_ctx;
typedef struct kc_program kc_program;
typedef struct kc_report kc_report;

typedef struct { uint32_t x, y, z; } kc_dim3;

/* Finding kinds (kc_fault.kind). */
enum { KC_DEADLOCK = 1, KC_DIVERGENCE = 2, KC_OOB = 3, KC_FUEL = 4, KC_ARITH = 5, KC_ALLOC = 6, KC_UNINIT = 7 };

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` bounds the
 * library's own device memory (logs, snapshots, scratch); 0 means no bound.
 * `tune_cache` names a JSON file of autotuned launch parameters or is NULL:
 * a flat object of option names and integer values (see kc_ctx_set_option),
 * as written by the package's autotuner; each entry is applied as that
 * option.  Errors: KC_E_INVAL (bad device, unreadable cache, non-integer
 * value, unknown option or out-of-range value in the cache), KC_E_DEVICE. */
kc_status kc_ctx_create(int hip_device, uint64_t hbm_budget_bytes, const char *tune_cache, kc_ctx **out);
void kc_ctx_destroy(kc_ctx *ctx);

/* Options: "check" (1 = log and check, default; 0 = interpret only),
 * "fuel" (instructions per thread, default 1<<20), "timing" (1 = time the
 * stages with HIP events on the launch stream; 2 = time only the free run,
 * which records two events per stage instead of about six), "sort_tile" (keys per sort
 * tile: 1024, 2048 (default), 4096 or 8192), "sort_bits" (radix digit width of
 * the sort's passes, 4 to 8, default 8), "side_streams" (streams over which
 * the launches of one batch step -- one per block-size class -- are spread,
 * 1 to 4, default 4), "log_records" (initial log capacity, >= 1024),
 * "stage" (interpreter staging granule per wave: 128, 256, 512 or 1024
 * records), "stage_bytes" (LDS bytes of per-block record staging, 8192 to
 * 98304, default 8192), "local" (1 = check each barrier epoch's accesses inside
 * the interpreter, default: shared words through per-word access tuples,
 * global locations as set by "shadow_global"; 0 = log every access),
 * "shadow_global" (1 = global locations through an LDS table of per-location
 * access tuples, default; 0 = stage their records and sort them per epoch),
 * "hash_check" (1 = a log of representative records in which no global
 * location is written by one block and touched by another is checked
 * through a hash table of its locations, without sorting, default; 0 = every
 * log is sorted and checked segment by segment),
 * "jit" (1 = run free runs on program-specialised kernels: each program is
 * translated to HIP and compiled with hiprtc for gfx950 at its first launch,
 * once per process, which takes seconds; results are identical to the
 * interpreter's; 0 = interpreter only, default), "sites" (1 = fill the
 * races' source sites, kc_report_race_sites: the racy blocks are replayed
 * once more with a site table; 0 = not computed, default), "uninit" (1 =
 * report loads of uninitialised shared memory, KC_UNINIT: the tool's checks
 * inherited from the C semantics include uninitialised memory accesses,
 * Section 3.2, and CUDA leaves shared memory undefined when a block starts;
 * 0 = off, default), "warp" (1 = the warp-aware model the paper's Section 4
 * proposes: threads form warps of 32 consecutive linear tids that execute in
 * lock-step, so two accesses of one block and epoch by threads of one warp
 * race only when they run at the same lockstep step; the intra-block tuple is
 * then w = the smallest thread with a write that conflicts, o = the smallest
 * thread whose access conflicts with one of w's writes; blocks with a race in
 * the plain model are replayed to find the steps; 0 = off, default),
 * "queue_replay" (1 = default: the replay of the blocks the free run found
 * racy is queued right behind it, before the host reads any result, and
 * stands when the log needs no sorted check; 0 = the host reads the free
 * run's results first and queues the replay after; results are identical),
 * "onesweep" (1 = sorts of 2^20 to 2^30 records count every pass's digits
 * in one read and then scatter each pass in one kernel, each tile finding
 * its output offsets from the counts earlier tiles publish; 0 = default:
 * three kernels per pass (per-tile counts, their scan, the scatter), as fast
 * or faster on MI355X; results are identical), "sort_spin" (the bound, in polls, of each wait of
 * a tile for an earlier tile's counts, default 2^16, 0 to 2^30: a wait that
 * runs out leaves that pass to the three-kernel passes, counted in
 * "sort_stalls"), "loc_sort" (1 = default: a free-run log of 2^20 records or
 * more made only of global-memory representatives -- one pass over it tells
 * -- is sorted by location alone, fewer passes than the location, block and
 * epoch key, since its check reduces each location's records in any order;
 * 0 = always the whole key; results are identical),
 * "reset" (1 = clear the statistics).
 * Errors: KC_E_INVAL for an unknown key or out-of-range value. */
kc_status kc_ctx_set_option(kc_ctx *ctx, const char *key, int64_t value);

/* Accumulated statistics since the last reset ("reset" clears them):
 * "interp_ms", "sort_ms", "check_ms", "replay_ms", "launches", "records",
 * "replays", "fallbacks", "retries", "spec_replays" (stages whose replay,
 * queued behind the free run before any result was read, stood),
 * "spec_retries" (stages run again without it because it did not apply),
 * "interp_launches", "sort_keys", "sort_onesweep" and "sort_stalls" (sorts
 * that took the single-pass scatters, and those finished by three-kernel
 * passes after a wait ran out), "loc_sorts" (free-run logs sorted by
 * location alone),
 * "sorted_checks", "hash_check_ms" (free-run logs that needed the sort, and
 * the time of the location-table checks),
 * "replay_sorted_checks" (replays whose records needed the sorted check: an
 * unreduced record, or a location written by one replayed block and touched
 * by another; the others are checked through a hash table of locations),
 * "instructions" (thread-instructions executed by the parallel free run; a
 * canonical replay of racy blocks is not counted), "global_accesses"
 * (in-bounds global-memory accesses of the free run), "jit_launches", "jit_replays"
 * (replay launches on specialised kernels),
 * "jit_compiled", "jit_compile_ms", "jit_failures", "site_replays",
 * "cross_launch_races", "alloc_findings", "stage_splits" (groups of a batch's
 * launches halved because their access-record key did not fit together),
 * "item_steps" (copy and host steps of host programs run), "device_bytes"
 * and "device_bytes_peak" (see kc_batch_footprint), "budget_trims" (idle
 * workspaces freed to stay within the budget),
 * "noalloc_calls" and
 * "noalloc_scratch_peak" (calls of kc_launch_noalloc and the most bytes of
 * its static scratch area one of them used).
 * Host times ("host_launch_ms", "stage_host_ms", "host_setup_ms",
 * "host_fetch_wait_ms", "host_parse_ms", "host_post_ms",
 * "host_replay_apply_ms", "host_unit_out_ms", "host_reports_ms") and the
 * stage times are only collected with option "timing" set.  "option.<name>"
 * reads back the current value of option <name>.  Returns 0 for an unknown
 * key. */
double kc_ctx_get_stat(kc_ctx *ctx, const char *key);

/* Message of the last error on this context; valid until the next call on it. */
const char *kc_last_error(const kc_ctx *ctx);

/* ---- programs -------------------------------------------------------------- */

/* Copy and validate `n_words` instruction words (1..65536).  Validation:
 * known opcode, registers < 16, branch targets in [0, n_words], special
 * register index < 24.  The caller's buffer may be freed afterwards.
 * Errors: KC_E_PROGRAM (validation), KC_E_INVAL, KC_E_NOMEM. */
kc_status kc_program_load(kc_ctx *ctx, const uint64_t *words, uint32_t n_words, kc_program **out);
void kc_program_free(kc_program *prog);

/* ---- launches ---------------------------------------------------------------- */

typedef struct {
    const kc_program *prog;
    kc_dim3 grid, block;        /* 1 <= threads per block <= 1024; blocks*threads < 2^32 */
    uint32_t shmem_bytes;       /* dynamic shared memory per block, multiple of 4, <= 65536 */
    int32_t params[8];          /* read by SREG 16..23 */
    uint32_t n_params;          /* <= 8; unused params read as 0 */
} kc_launch_desc;

/* One launch (Section 2: a kernel launched over a grid of blocks of
 * threads), checked as Section 3.1 describes: every race of two accesses of
 * one location with no synchronisation point between them, barrier
 * divergence and the deadlock of threads waiting at a barrier others never
 * reach.  Synchronous with respect to the host.  Work is queued on
 * `stream` (a hipStream_t; NULL = the null stream).  `dev_mem` is a device
 * buffer of `n_words` int32 words (< 2^31) that the caller owns and keeps
 * untouched until the call returns; it is updated in place to the canonical
 * final memory.  On KC_OK *out is a report owned by the caller.
 * Errors: KC_E_INVAL, KC_E_NOMEM, KC_E_BUDGET, KC_E_OVERFLOW, KC_E_DEVICE. */
kc_status kc_launch(kc_ctx *ctx, const kc_launch_desc *desc, int32_t *dev_mem, uint64_t n_words,
                    void *stream, kc_report **out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: under stream capture, in tight serving loops, in harnesses that
 * forbid it): the same launch as kc_launch -- same arguments, checks, report
 * and final memory -- but the call allocates no device memory and no pinned
 * host memory.  Every device buffer of the run (snapshot, access log, sort
 * and table scratch, counters, finding lists) is carved from a static
 * scratch area of KC_NOALLOC_SCRATCH_BYTES bytes per device, which the
 * library's code object holds on every device it is loaded on until the
 * process ends; the host staging and the events it uses are made by
 * kc_ctx_create.  The interpreter runs (option "jit" is ignored: the
 * specialised kernels would be compiled and loaded at run time); the other
 * options apply.  The report itself lives on the host heap, as kc_launch's.
 * All calls on one device share its area, which keeps the last call's
 * contents (every buffer a call reads is cleared or written by that call
 * first).  The library serialises these calls per device with a lock; work
 * of two calls that overlapped on one device would race on the area.
 * Errors: those of kc_launch; KC_E_BUDGET when the run needs more than the
 * area (for example a memory of more than KC_NOALLOC_SCRATCH_BYTES / 4 words,
 * which the launch-start snapshot alone would exceed) or its results more
 * than the host staging set up at context creation. */
#define KC_NOALLOC_SCRATCH_BYTES ((uint64_t)64 << 20)
kc_status kc_launch_noalloc(kc_ctx *ctx, const kc_launch_desc *desc, int32_t *dev_mem, uint64_t n_words,
                            void *stream, kc_report **out);

/* An event dependency between two launches of a job (Section 3 "Streams
 * and events"): launch `after` starts only once launch `before` has finished,
 * as when an event recorded in before's stream right behind it is waited on
 * (cudaStreamWaitEvent) in after's stream ahead of it, or the host
 * synchronises in between.  before < after. */
typedef struct {
    uint32_t before, after;
} kc_dep;

/* A device allocation inside a job's memory: words [base, base + words). */
typedef struct {
    uint64_t base, words;
} kc_region;

/* An item of a job's host program (Section 3 "Streams and events": launches
 * and memory transfers pass through the stream queues, and the host
 * synchronises with cudaStreamSynchronize, cudaEventSynchronize and
 * cudaDeviceSynchronize).  Device items run in `stream`:
 *   KC_ITEM_LAUNCH     runs launches[ref];
 *   KC_ITEM_COPY       copies `words` words from src to dst (the two ranges
 *                      may not overlap); flags KC_ITEM_SYNC: the host waits
 *                      for it on the spot (a cudaMemcpy).  Its word k is
 *                      copied by thread k.
 * Host items (no stream):
 *   KC_ITEM_HOST_READ  the host reads words [dst, dst + words);
 *   KC_ITEM_HOST_WRITE the host stores `value` to words [dst, dst + words);
 *                      word dst + k is touched by thread k;
 *   KC_ITEM_HOST_WAIT  the host waits until device item `ref` has finished
 *                      (an event recorded right behind it, or the last
 *                      item of a stream), or every earlier device item when
 *                      ref = KC_WAIT_ALL (cudaDeviceSynchronize).
 * Item i happens before a later item j when both are device items of one
 * stream, a dependency links them (an event), i is a host item (the host
 * issues j after it), i is a synchronous copy, or j waits for i -- or a
 * chain of these leads from i to j.  Items ordered neither way race as
 * launches do (scope 2, with item indices).  Copies and host items make no
 * access records. */
enum {
    KC_ITEM_LAUNCH = 0,
    KC_ITEM_COPY = 1,
    KC_ITEM_HOST_READ = 2,
    KC_ITEM_HOST_WRITE = 3,
    KC_ITEM_HOST_WAIT = 4
};
#define KC_ITEM_SYNC 1u
#define KC_WAIT_ALL 0xFFFFFFFFu
typedef struct {
    uint32_t kind;              /* KC_ITEM_* */
    uint32_t stream;            /* device items */
    uint32_t ref;               /* launch index (LAUNCH), item waited for or KC_WAIT_ALL (HOST_WAIT) */
    uint32_t flags;             /* KC_ITEM_SYNC (COPY) */
    uint64_t dst, src, words;   /* word ranges of COPY, HOST_READ, HOST_WRITE; words < 2^32 */
    int32_t value;              /* HOST_WRITE */
    uint32_t pad;
} kc_item;

/* A job: launches on one memory (Section 2).  By default they form one
 * stream and run in order.  With `streams` (one stream id per launch) and
 * `deps`, launch i happens before launch j when a chain of same-stream order
 * (an earlier launch of the same stream) and dependencies leads from i to j;
 * two launches ordered neither way may run in parallel, and every global word
 * one of them writes and the other touches is reported as a race between
 * them (scope 2).  The launches still execute in submission order, which
 * respects every chain, so the final memory is that order's.  The report's
 * launch fields are indices into `launches`.  `streams` and `deps` are read
 * during the call (kc_batch_submit copies them). */
typedef struct {
    const kc_launch_desc *launches;
    uint32_t n_launches;
    int32_t *dev_mem;
    uint64_t n_words;
    uint64_t tag;               /* returned by kc_report_tag */
    const uint32_t *streams;    /* n_launches entries, or NULL: one stream */
    const kc_dep *deps;         /* n_deps entries (before < after < n_launches), or NULL */
    uint32_t n_deps;
    /* Memory objects: when `allocs` is not NULL it lists the job's device
     * allocations (n_allocs entries, possibly 0, each inside the memory,
     * overlaps allowed).  A global access by a kernel to a word outside every
     * allocation (host memory or nothing, from the device's side) is illegal:
     * it takes effect, and each block that made such accesses to a word gets
     * one KC_ALLOC finding.  NULL: no check. */
    const kc_region *allocs;
    uint32_t n_allocs;
    /* The host program: when `items` is not NULL the job runs its n_items
     * items in order (n_items <= 4096) instead of its launches; launch items
     * name launches by index, `deps` link device items by item index,
     * `streams` must be NULL, and every report's launch field is an item
     * index.  launches_completed then counts the leading items that
     * completed (a launch that does not complete ends the job). */
    const kc_item *items;
    uint32_t n_items;
} kc_job;

/* Submit jobs as one batch; returns at once.  All jobs of the batch execute
 * together (one interpreter launch per block-size class and launch index,
 * one sort and one check over all of them).  The descriptor, stream,
 * dependency and allocation arrays are copied; device memories stay owned by
 * the caller and must not be touched until kc_poll reports the batch done.
 * Errors: KC_E_INVAL (also for a dependency that does not point forward,
 * more than 4096 launches in a job with streams or dependencies, n_deps
 * without a dependency array, an allocation outside the job's memory, or an
 * item that is malformed: an unknown kind, a launch index out of range, a
 * range outside the memory, overlapping copy ranges, a wait for a host item
 * or a later one, a dependency on a host item, streams given with items),
 * KC_E_NOMEM (also when the batch's worker thread cannot be started),
 * KC_E_DEVICE.  Errors of the run itself come back from kc_poll. */
kc_status kc_batch_submit(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs, void *stream, uint64_t *ticket);

/* The device bytes the library would reserve to run `jobs` as one batch
 * (before any growth of its access log), for admission against the
 * context's HBM budget: the largest step's launch-start snapshot, location
 * tables, access log at the context's current record hint (which grows with
 * the logs seen so far) with its sort and replay scratch, per-block lists and
 * finding lists, plus the access summaries and allocation bitmaps held for
 * the whole run.  With n_jobs = 0 it is the part every batch reserves
 * whatever its jobs; a batch's footprint is at most that part plus, for each
 * of its jobs, what the job adds to it alone.  The jobs are checked as by
 * kc_batch_submit, except that their memories need not exist yet (dev_mem
 * may be NULL); nothing runs.
 * The context's current device bytes and their peak are the statistics
 * "device_bytes" and "device_bytes_peak"; its budget bounds all of its
 * buffers together, across concurrent batches (idle workspaces kept for reuse
 * are freed first when a call would exceed it).
 * Errors: those of kc_batch_submit's argument checks. */
kc_status kc_batch_footprint(kc_ctx *ctx, const kc_job *jobs, uint32_t n_jobs, uint64_t *bytes);

/* Collect a batch.  With wait = 0 returns KC_E_PENDING (out untouched) while
 * it runs.  On KC_OK `out` (n_out >= n_jobs pointers) receives one report per
 * job in submission order, each owned by the caller; the ticket is retired.
 * A failed batch retires its ticket with the batch's status.
 * Errors: KC_E_INVAL (unknown or already collected ticket, n_out too small:
 * the ticket stays valid), the batch's own error (KC_E_NOMEM, KC_E_BUDGET,
 * KC_E_OVERFLOW, KC_E_DEVICE, KC_E_INTERNAL). */
kc_status kc_poll(kc_ctx *ctx, uint64_t ticket, int wait, kc_report **out, uint32_t n_out);

/* ---- reports -------------------------------------------------------------------- */

/* Scope 2 (launches that may run in parallel, see kc_job): `launch` is the
 * later launch j, `block` the earlier launch i, epoch 0xFFFFFFFF, `addr` the
 * global word; w_tid is the smallest global thread id (block*threads+tid) of
 * j whose access to the word conflicts with an access of i, o_tid the same
 * for i (every access conflicts when the other launch writes the word, only
 * writes otherwise). */
typedef struct {
    uint32_t launch;
    uint32_t space;     /* 0 shared, 1 global */
    uint32_t scope;     /* 0 intra-block, 1 cross-block, 2 cross-launch */
    uint32_t block;     /* linear block id (of w_tid when cross-block); the other launch when cross-launch */
    uint32_t epoch;     /* barrier epoch; 0xFFFFFFFF when cross-block or cross-launch */
    uint32_t addr;      /* word index: shared offset or global word */
    uint32_t w_tid;     /* smallest writer; linear tid, or block*threads+tid when cross-block */
    uint32_t o_tid;     /* smallest other conflicting thread, same numbering */
} kc_race;

typedef struct {
    uint32_t launch, kind, block, epoch;
    uint32_t a, b, c, d;
    /* DEADLOCK:   a = #waiting threads, b = smallest waiting tid, c = smallest exited tid
     * DIVERGENCE: a = smallest barrier pc, b = smallest tid there, c = next barrier pc, d = its smallest tid
     * OOB:        a = space*2 + (1 if store), b = tid, c = address (int32)
     * FUEL:       b = tid
     * ARITH:      b = tid, c = pc
     * ALLOC:      epoch 0xFFFFFFFF, a = 2 + (1 if the block stored to the word), b = smallest tid of the
     *             block that accessed it, c = word, d = smallest tid that stored to it or 0xFFFFFFFF
     * UNINIT:     (option "uninit") a load of a shared word that no thread of the block stored to earlier
     *             in the canonical order (an earlier step; a step's loads come before its stores):
     *             a = 0 (shared, load), b = tid, c = word, d = pc of the load; the load reads 0 */
} kc_fault;

/* Source sites of a race (the tool names the source line a race was found
 * at, Section 3.2): w_pc is the smallest pc of a store by w_tid to the
 * location, o_pc the smallest pc of an access by o_tid to it, within the
 * tuple's block and epoch (scope 0) or its launch (scope 1); 0xFFFFFFFF when
 * not computed (option "sites" off, and always for scope 2). */
typedef struct {
    uint32_t w_pc, o_pc;
} kc_race_site;

uint64_t kc_report_records(const kc_report *r);            /* canonical access-record count */
uint32_t kc_report_launches_completed(const kc_report *r);
/* The race tuples of Section 3.1 (one per conflicting location and, within a
 * block, barrier epoch: the tuples are cleared at each __syncthreads()),
 * ascending by (launch, space, scope, block, epoch, addr); the array lives as
 * long as the report; *n receives the count. */
const kc_race *kc_report_races(const kc_report *r, uint64_t *n);
/* The findings (Section 3.1 deadlock and barrier divergence; the checks the
 * tool inherits from the C semantics, Section 3.2: out-of-bounds,
 * uninitialised and illegal memory accesses, undefined arithmetic; fuel)
 * ascending by (launch, block, epoch, kind, a, b, c, d), no repeats; the
 * array lives as long as the report. */
const kc_fault *kc_report_faults(const kc_report *r, uint64_t *n);
/* Sites of the races, one per race in the same order; lives as long as the report. */
const kc_race_site *kc_report_race_sites(const kc_report *r, uint64_t *n);
uint64_t kc_report_tag(const kc_report *r);
void kc_report_free(kc_report *r);

/* Many reports at once (a polled batch): for report i, records[i],
 * launches[i], tags[i], n_races[i] and n_faults[i] (each array n entries or
 * NULL); the races, their sites and the findings of all reports concatenated
 * in report order into `races`, `sites` and `faults` (sized by the sums of
 * n_races and n_faults, or NULL to skip).  Reports are not modified.
 * Errors: KC_E_INVAL for a null report pointer. */
kc_status kc_reports_collect(kc_report *const *reports, uint32_t n, uint64_t *records, uint32_t *launches,
                             uint64_t *tags, uint64_t *n_races, uint64_t *n_faults, kc_race *races,
                             kc_fault *faults, kc_race_site *sites);
/* Free n reports (null entries are skipped). */
void kc_reports_free(kc_report *const *reports, uint32_t n);

#ifdef __cplusplus
}
#endif
#endif /* KC_H */
