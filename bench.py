#!/usr/bin/env python3
"""Benchmark of the SIMT race and deadlock checker on one MI355X.

Workload (one step = one plain kc_launch through the whole hot path:
interpretation with access logging, radix sort, conflict check, canonical
replay of racy blocks, report): shared-memory tree reduction over 2^20 int32
inputs uniform in [0, 2^16), 4096 blocks x 256 threads, with the barrier after
a seeded level dropped in 1% of the blocks and a tid-dependent barrier in
0.1% (seed 12116193 + 2).  The memory is resident on the GPU before timing;
in the CPU-baseline leg the last step's report and memory are compared bit for
bit with the CPU oracle.

Prints one JSON line: records/s over the timed steps, per-step latency
percentiles, the dominant kernel's roofline (HIP-event timing inside the
library on the launch stream) and the oracle's CPU rate on the same workload.
The oracle is used only in the CPU-baseline leg (its timing and the bit-exact
comparison of the GPU's results with it).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "access records checked/sec (batched vs plain, bit-exact); p50/p99 check latency"
HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the workload-3 batched vs plain comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--jit", type=int, default=1, choices=(0, 1),
                    help="1: program-specialised free-run and replay kernels, compiled (hiprtc, gfx950) by the "
                         "first warm-up step (default); 0: the interpreter")
    ap.add_argument("--no-sort-path", action="store_true",
                    help="skip the comparison of the in-LDS epoch-local check with the sort-only check")
    ap.add_argument("--no-streams", action="store_true",
                    help="skip the streams-and-events measurement (two streams against one)")
    ap.add_argument("--no-workload4", action="store_true",
                    help="skip workload 4 at full size (ping-pong stencil, 2^26 elements x 16 launches)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="arrival window per served rate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB three times (the known-size kernel that scales "
                         "HBM counter readings) and exit")
    ap.add_argument("--only", choices=("none", "sort", "batched", "serve", "streams", "workload4"),
                    help="run the plain steps and this one optional leg only (no CPU baseline): for profiles")
    ap.add_argument("--option", action="append", default=[], metavar="NAME=VALUE",
                    help="set a library option on the benchmark's context before the plain steps (for profiles "
                         "of an alternative setting, e.g. onesweep=1; the line then names it in config.options)")
    args = ap.parse_args()
    if args.only:
        for leg, flag in (("sort", "no_sort_path"), ("batched", "no_batched"), ("serve", "no_serve"),
                          ("streams", "no_streams"), ("workload4", "no_workload4")):
            setattr(args, flag, args.only != leg)
        args.no_cpu_baseline = True
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (sharding the checker "
              f"over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": src.numel() * 4, "bytes_written": dst.numel() * 4}))
        return
    from paper_1211_6193_amd import kc, workloads as W

    job = W.tree256_job()
    L = job.launches[0]
    ctx = kc.Context(0)
    ctx.set_option("timing", 2)         # HIP events around the free run only, during the timed steps
    ctx.set_option("jit", args.jit)     # program-specialised free-run kernels (compiled at first use)
    extra = {}
    for kv in args.option:
        name, _, val = kv.partition("=")
        ctx.set_option(name, int(val))
        extra[name] = int(val)
    prog = ctx.program(L.program)
    mem = torch.from_numpy(job.memory.copy()).cuda()
    stream = torch.cuda.current_stream()

    launch = kc.PreparedLaunch(ctx, prog, L.grid, L.block, L.shmem_bytes, L.params)

    def step():
        return launch.run(mem, stream=stream)

    for _ in range(args.warmup):
        rep = step()
    compile_ms = ctx.stat("jit_compile_ms")
    ctx.reset_stats()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = time.perf_counter()
        rep = step()
        lat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    records = rep.records
    value = records * args.steps / elapsed

    stats = {k: ctx.stat(k) for k in ("interp_ms", "sort_ms", "check_ms", "replay_ms", "replays",
                                      "fallbacks", "retries", "sort_keys", "records", "interp_launches",
                                      "replay_lockstep_ms", "replay_sort_ms", "replay_check_ms",
                                      "replay_coverage_ms", "log_entries", "instructions", "jit_launches",
                                      "hash_check_ms", "sorted_checks", "replay_sorted_checks",
                                      "global_accesses")}
    per = {k: stats[k] / args.steps for k in ("interp_ms", "hash_check_ms", "sort_ms", "check_ms", "replay_ms")}
    # the stage breakdown: 10 more steps with every stage timed (each event
    # pauses the stream briefly, so the timed steps record only two)
    ctx.set_option("timing", 1)
    ctx.reset_stats()
    for _ in range(10):
        step()
    torch.cuda.synchronize()
    detail = {k: ctx.stat(k) / 10 for k in ("interp_ms", "hash_check_ms", "sort_ms", "check_ms", "replay_ms",
                                            "replay_lockstep_ms", "replay_sort_ms", "replay_check_ms",
                                            "replay_coverage_ms")}
    roofline = free_run_roofline(stats, args.steps, records, value, per, detail)
    roofline["copy_gbs"] = copy_bandwidth(torch)
    roofline["frac_of_copy"] = round(roofline["achieved"] / roofline["copy_gbs"], 4)

    sort_path = None if args.no_sort_path else local_vs_sort(ctx, step, rep, mem, torch, np)
    batched, sample = (None, []) if args.no_batched else batched_vs_plain(ctx, W, kc, torch, np)
    serving = None if args.no_serve else served(ctx, W, torch, np, args.serve_seconds)
    streams = None if args.no_streams else streams_leg(ctx, W, kc, torch, np)
    w4 = None if args.no_workload4 else workload4_leg(ctx, W, kc, torch, np)

    cpu, exact = None, None
    served_sample = serving.pop("sample", []) if serving else []
    if not args.no_cpu_baseline:
        cpu, exact, sample_exact = cpu_baseline_leg(job, rep, mem, args.cpu_seconds, np, sample)
        if batched is not None:
            batched["bit_exact_sample"] = sample_exact
            batched["verified_instances"] = len(sample)
            batched["oracle"] = oracle_pool_rate([j for j, _, _ in sample])
        if serving is not None:
            serving["bit_exact_sample"] = same_as_oracle(served_sample, np)
            serving["verified_requests"] = len(served_sample)
            serving["oracle"] = oracle_pool_rate([j for j, _, _ in served_sample])
        if streams is not None:
            streams["missing_event_bit_exact_vs_oracle"] = same_as_oracle(
                [(streams["job"], streams["report"], streams["memory"].cpu().numpy())], np)
    if streams is not None:
        for k in ("job", "report", "memory"):
            streams.pop(k)

    lat_ms = sorted(x * 1e3 for x in lat)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "records/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "tree256-plain: 4096 blocks x 256 threads over 2^20 int32 in [0,2^16), "
                               "1% dropped-barrier and 0.1% tid-barrier blocks, seed 12116195",
                   "form": "plain (one kc_launch per step)", "records_per_step": records,
                   "kernels": ("program-specialised (compiled once per process, before the timed steps: "
                               f"{compile_ms:.0f} ms)" if args.jit else "interpreter"),
                   "races": len(rep.races), "findings": len(rep.faults),
                   "bit_exact_vs_oracle": exact,
                   "p50_ms": round(lat_ms[len(lat_ms) // 2], 4),
                   "p99_ms": round(lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))], 4),
                   "replays_per_step": stats["replays"] / args.steps, "fallbacks": stats["fallbacks"],
                   **({"options": extra} if extra else {})},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "shadow_vs_sort": sort_path,
        "batched_vs_plain": batched,
        "served": serving,
        "streams": streams,
        "workload4": w4,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    if exact is False or (batched and batched.get("bit_exact_sample") is False) or \
            (serving and serving.get("bit_exact_sample") is False) or \
            (sort_path and not sort_path["same_reports"]) or \
            (streams and (not streams["same_otherwise"] or streams.get("missing_event_bit_exact_vs_oracle") is False)):
        sys.exit(1)


# Peak of the free run's ALU resource, reported beside the HBM roofline:
# int32 vector lane-operations.  256 CUs x 4 SIMDs x 16 lanes, one wave64
# int32 VALU instruction per SIMD every 4 cycles = 64 lane-ops per CU per
# clock, at 2.4 GHz.  (The 157.3 TFLOP/s fp32 figure counts an FMA as two
# flops and packed dual issue; int32 has neither.)
INT32_LANE_OPS_PEAK_G = 256 * 64 * 2.4       # G lane-ops/s = 39,321.6
# Algorithmic HBM bytes of the checking path: each access record written once
# and read back once (8 + 8 bytes), plus the simulated kernel's own 4-byte
# word for each global-space access.
BYTES_PER_RECORD = 16
BYTES_PER_GLOBAL_ACCESS = 4


def free_run_roofline(stats, steps, records, value, per, detail):
    """HBM roofline of the dominant kernel, the free run: its algorithmic
    bytes per launch (16 B per access record it checks + 4 B per global-space
    access of the simulated kernel) over its average duration, timed with HIP
    events inside the library on the launch stream.  The same kernel's
    instruction rate against the int32 lane-op peak is kept beside it."""
    instr = stats["instructions"] / steps
    gacc = stats["global_accesses"] / steps
    launches = max(1.0, stats["interp_launches"] / steps)
    dur_s = per["interp_ms"] / 1e3 / launches
    alg_bytes = BYTES_PER_RECORD * records + BYTES_PER_GLOBAL_ACCESS * gacc
    achieved = alg_bytes / dur_s / 1e9 if dur_s > 0 else 0.0
    lane_ops = instr / dur_s / 1e9 if dur_s > 0 else 0.0
    kernel = "kc_jit_free_local_256" if stats.get("jit_launches", 0) > 0 else "k_interp_free_local"
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(kernel),
            "algorithmic_bytes_per_launch": int(alg_bytes), "records_per_launch": records,
            "global_accesses_per_launch": int(gacc),
            "avg_ms": round(per["interp_ms"] / launches, 4),
            "alu": {"achieved": round(lane_ops, 1), "peak": INT32_LANE_OPS_PEAK_G,
                    "unit": "G thread-instructions/s (int32 lane-ops/s)",
                    "frac": round(lane_ops / INT32_LANE_OPS_PEAK_G, 5),
                    "thread_instructions_per_launch": int(instr)},
            "stage_ms": {k: round(detail[k], 4) for k in per},
            "replay_detail_ms": {k: round(detail[k], 4) for k in
                                 ("replay_lockstep_ms", "replay_sort_ms", "replay_check_ms",
                                  "replay_coverage_ms")},
            "stage_note": "avg_ms: the timed steps (events around the free run only); stage_ms and "
                          "replay_detail_ms: 10 further steps with every stage timed",
            "sorted_checks_per_step": stats["sorted_checks"] / steps,
            "replay_sorted_checks_per_step": stats["replay_sorted_checks"] / steps,
            "log_entries_per_step": stats["log_entries"] / steps,
            "path_hbm_algorithmic_gbs": round(value * BYTES_PER_RECORD / 1e9, 1),
            "path_hbm_algorithmic_frac": round(value * BYTES_PER_RECORD / (HBM_PEAK_GBS * 1e9), 4)}


def copy_bandwidth(torch, n_bytes=1 << 30, reps=5):
    """Achievable HBM bandwidth: a device-to-device copy of 1 GiB (read +
    write counted), best of ``reps``, timed with events on the current stream."""
    src = torch.ones(n_bytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del src, dst
    return round(2 * n_bytes / best / 1e9, 1)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a copy kernel's reading), or
    None when it covers another kernel or the sources changed since."""
    name = "interp" if kernel.startswith("k_interp") else "jit"
    path = os.path.join(ROOT, "profiles", f"{name}_tree256_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_1211_6193_amd.profsum import kernel_source_digest
    if t.get("kernel") != kernel or t.get("source_digest") != kernel_source_digest():
        return None
    return t.get("bytes_per_launch")


def _same(rep, got, orc, np):
    return (rep.records == orc.records and rep.race_tuples() == orc.race_tuples()
            and rep.fault_tuples() == orc.fault_tuples() and rep.launches_completed == orc.launches_completed
            and bool(np.array_equal(got, orc.memory)))


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo) and its core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def same_as_oracle(sample, np):
    """Every (job, report, final memory) of ``sample`` equals the oracle's run
    (the oracle runs on every host core)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    ok = True
    with ThreadPoolExecutor(max_workers=host_cpu()[1]) as ex:
        for (j, r, m), orc in zip(sample, ex.map(O.run_job, [j for j, _, _ in sample])):
            if not _same(r, m, orc, np):
                print(f"bench: an instance differs from the oracle: {getattr(j, 'meta', '')}", file=sys.stderr)
                ok = False
    return ok


def oracle_pool_rate(jobs, one_core_seconds=3.0):
    """The oracle over independent instances on every host core (a thread
    pool: the oracle's C code runs without the interpreter lock) and on one
    core (the instances in order until ``one_core_seconds`` have passed), in
    records/s."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    if not jobs:
        return None
    model, cores = host_cpu()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        t0 = time.perf_counter()
        recs = sum(r.records for r in ex.map(O.run_job, jobs))
        allc = time.perf_counter() - t0
    one_recs, n_one = 0, 0
    t0 = time.perf_counter()
    for j in jobs:
        one_recs += O.run_job(j).records
        n_one += 1
        if time.perf_counter() - t0 > one_core_seconds:
            break
    one = time.perf_counter() - t0
    return {"instances": len(jobs), "records": recs, "all_cores_records_per_s": round(recs / allc, 1),
            "one_core_records_per_s": round(one_recs / one, 1), "one_core_instances": n_one,
            "cores": cores, "cpu": model}


def cpu_baseline_leg(job, rep, mem, cpu_seconds, np, sample=()):
    """The oracle on the host cores: its rate on the same workload, and the
    bit-exact comparison of the GPU's last step (and of a sample of batched
    instances, (job, report, final memory)) with the oracle's runs."""
    from oracle import oracle as O
    t_o = time.perf_counter()
    orc = O.run_job(job)
    oracle_s = time.perf_counter() - t_o
    exact = _same(rep, mem.cpu().numpy(), orc, np)
    if not exact:
        print("bench: GPU result differs from the oracle", file=sys.stderr)
    sample_exact = same_as_oracle(sample, np)
    reps = max(1, int(cpu_seconds / max(oracle_s, 1e-3)))
    t_c = time.perf_counter()
    for _ in range(reps):
        O.run_job(job)
    cs = time.perf_counter() - t_c
    model, ncores = host_cpu()
    cpu = {"value": round(orc.records * reps / cs, 1), "unit": "records/s", "cores": 1, "kind": "oracle",
           "sample": f"the whole workload run {reps}x by the single-threaded C oracle ({cs:.1f} s); one "
                     f"instance, so one core", "host_cpu": model, "host_cores": ncores}
    return cpu, exact, sample_exact


def local_vs_sort(ctx, step, rep, mem, torch, np, steps=10):
    """The same step with the epoch-local check switched off (option "local" =
    0): every access goes to the log and through the sort and the segmented
    check.  Reports and final memory must equal the default path's."""
    ref = mem.clone()
    ctx.set_option("local", 0)
    try:
        for _ in range(2):
            step()
        ctx.reset_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = {k: ctx.stat(k) / steps for k in ("interp_ms", "sort_ms", "check_ms", "replay_ms", "log_entries")}
    finally:
        ctx.set_option("local", 1)
    same = (r.records == rep.records and r.race_tuples() == rep.race_tuples()
            and r.fault_tuples() == rep.fault_tuples() and bool(torch.equal(mem, ref)))
    if not same:
        print("bench: the sort-only path differs from the epoch-local path", file=sys.stderr)
    return {"sort_only_records_per_s": round(r.records * steps / el, 1), "sort_only_ms_per_step": round(el * 1e3 / steps, 4),
            "sort_only_log_entries": st["log_entries"], "sort_only_stage_ms": {k: round(st[k], 4) for k in
                                                                             ("interp_ms", "sort_ms", "check_ms", "replay_ms")},
            "same_reports": same}


TUNE_CACHE = os.path.join(ROOT, "paper_1211_6193_amd", "tune_mi355x.json")


def tune_keys():
    from paper_1211_6193_amd import tune
    return list(tune.SPACE)


def batched_vs_plain(ctx, W, kc, torch, np, reps=3, plain_sample=200, verify=400):
    """Workload 3 (10,000 mixed instances, seed 12116196): the whole set as one
    batch (kc_batch_submit + kc_poll) against one plain kc_launch per instance
    on a sample of instances; both on the same resident memories (the
    instances read their inputs and write disjoint outputs, so reruns are
    identical).  Returns the figures and a sample of (job, report, final
    memory) for the comparison with the oracle in the CPU-baseline leg."""
    jobs = W.config3_jobs(n=10000)
    mems = [torch.from_numpy(np.ascontiguousarray(j.memory)).cuda() for j in jobs]
    # the batch runs with the autotuner's setting for this GPU (written by
    # python -m paper_1211_6193_amd.tune on a 2000-instance sample)
    tuned = os.path.exists(TUNE_CACHE)
    bctx = kc.Context(ctx.device, tune_cache=TUNE_CACHE if tuned else None)
    bctx.set_option("jit", int(ctx.stat("option.jit")))
    batch = kc.Batch(bctx)
    prep = batch.prepare([(kc.job_launches(bctx, j), m, i) for i, (j, m) in enumerate(zip(jobs, mems))])
    stream = torch.cuda.current_stream()
    res = batch.poll(batch.submit(prep, stream=stream), wait=True)          # warm-up
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = batch.poll(batch.submit(prep, stream=stream), wait=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    records = res.total_records()
    best = min(times)
    idx = list(range(0, len(jobs), max(1, len(jobs) // plain_sample)))[:plain_sample]
    launches = [(ctx.program(jobs[i].launches[0].program), jobs[i].launches[0]) for i in idx]
    lat, prec = [], 0
    torch.cuda.synchronize()
    for (p, L), i in zip(launches, idx):
        t0 = time.perf_counter()
        r = kc.launch(ctx, p, L.grid, L.block, L.shmem_bytes, mems[i], L.params, stream=stream)
        lat.append(time.perf_counter() - t0)
        prec += r.records
    plain_rate = prec / sum(lat)
    vidx = list(range(0, len(jobs), max(1, len(jobs) // verify)))[:verify]
    sample = [(jobs[i], res[i], mems[i].cpu().numpy()) for i in vidx]
    lat_ms = sorted(x * 1e3 for x in lat)
    return {"workload": "workload 3: 10000 instances (tree/stencil/transpose, 1-64 blocks x 32-1024 threads, "
                        "20% seeded faults)",
            "records": records, "batched_records_per_s": round(records / best, 1),
            "batched_ms": round(best * 1e3, 3),
            "plain_records_per_s": round(plain_rate, 1),
            "plain_p50_ms": round(lat_ms[len(lat_ms) // 2], 4),
            "plain_p99_ms": round(lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))], 4),
            "speedup": round((records / best) / plain_rate, 2),
            "tune_cache": os.path.relpath(TUNE_CACHE, ROOT) if tuned else None,
            "tuned_setting": {k: int(bctx.stat("option." + k)) for k in tune_keys()},
            "bit_exact_sample": None, "verified_instances": 0}, sample


def streams_leg(ctx, W, kc, torch, np, reps=5):
    """Streams and events: two workload-2 tree reductions (4096 x 256 each,
    1% dropped-barrier blocks) in two streams, then a final reduction of both
    partial-sum arrays in the first stream that waits for the second through
    an event (seed 12116199).  Timed as one stream (no launch may overlap, no
    summaries), with the two streams and the event (the two reductions may
    run in parallel: their access summaries are built and compared; no race
    between launches), and with the event left out (the final launch races
    with the second reduction on its 4096 partial sums).  Each run starts
    from the initial memory (copied outside the timed region).  Reports must
    agree except for the races between launches."""
    variants = {"one_stream": W.streams_reduce_job(), "two_streams": W.streams_reduce_job(),
                "missing_event": W.streams_reduce_job(missing_event=True)}
    variants["one_stream"].streams, variants["one_stream"].deps = None, []
    init = torch.from_numpy(np.ascontiguousarray(variants["one_stream"].memory)).cuda()
    out, reps_of, mem_of = {}, {}, {}
    for name, job in variants.items():
        times = []
        for _ in range(reps + 1):           # the first run is a warm-up
            mem = init.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep, mem = kc.run_job(ctx, job, mem=mem)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        best = min(times[1:])
        reps_of[name], mem_of[name] = rep, mem
        out[name] = {"ms": round(best * 1e3, 3), "records_per_s": round(rep.records / best, 1),
                     "races_between_launches": sum(1 for r in rep.race_tuples() if r[2] == 2)}
    one = reps_of["one_stream"]
    same = True
    for name in ("two_streams", "missing_event"):
        r = reps_of[name]
        same &= (r.records == one.records and [x for x in r.race_tuples() if x[2] != 2] == one.race_tuples()
                 and r.fault_tuples() == one.fault_tuples() and bool(torch.equal(mem_of[name], mem_of["one_stream"])))
    if not same:
        print("bench: the stream variants differ beyond their races between launches", file=sys.stderr)
    out.update({"workload": "two workload-2 trees (4096 x 256 each, 1% dropped barriers) in two streams + a final "
                            "tree in stream 0 after an event; seed 12116199",
                "records": one.records, "same_otherwise": same,
                "job": variants["missing_event"], "report": reps_of["missing_event"],
                "memory": mem_of["missing_event"]})
    return out


def workload4_leg(ctx, W, kc, torch, np, reps=2):
    """Workload 4 at full size: the ping-pong stencil over 2^26 int32
    elements, 16 launches as one job, 0.01% in-place blocks (seed 12116197),
    from the initial memory each time (copied outside the timed region); the
    first run compiles the specialised kernels and is not timed.  Its races
    have a closed form (two boundary words of every in-place block in every
    launch), checked here."""
    job = W.stencil_pingpong_job()
    init = torch.from_numpy(np.ascontiguousarray(job.memory)).cuda()
    times, rep = [], None
    for _ in range(reps + 1):
        mem = init.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, mem = kc.run_job(ctx, job, mem=mem)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    nb = job.meta["n"] // job.meta["threads"]
    bugs = [int(b) for b in job.meta["bug_blocks"]]
    want = len(job.launches) * sum((b > 0) + (b < nb - 1) for b in bugs)
    best = min(times[1:])
    return {"workload": "workload 4: ping-pong stencil, 2^26 int32 elements x 16 launches, 256 threads per block, "
                        "0.01% in-place blocks",
            "records": rep.records, "ms": round(best * 1e3, 1), "records_per_s": round(rep.records / best, 1),
            "races": len(rep.races), "races_closed_form": want, "launches_completed": rep.launches_completed}


def served(ctx, W, torch, np, seconds, rates=(1000.0, 5000.0, 20000.0)):
    """Workload 5: Poisson arrivals at each rate for ``seconds``; 95% workload-3
    instances, 5% 4096x256 trees, drawn from a seeded pool whose initial
    memories are resident on the device (each request gets its own copy);
    continuous batching with 4 streams under a 64 GiB budget."""
    from paper_1211_6193_amd import server
    small, big = W.request_pool()
    pristine = {id(j): torch.from_numpy(np.ascontiguousarray(j.memory)).cuda() for j in small + big}
    torch.cuda.synchronize()
    out = {"workload": f"workload 5: {seconds:g} s of Poisson arrivals per rate; pool of {len(small)} workload-3 "
                       f"instances and {len(big)} 4096x256 trees (p=0.05); 4 slots, 64 GiB budget"}
    # the library enforces the same budget over all of its buffers; admission
    # charges each batch the footprint the library reports for it
    sctx = kc_budget_context(ctx, 64 << 30)
    srv = server.Server(sctx, budget_bytes=64 << 30, slots=4)
    srv.run(W.pooled_requests(1000.0, 0.3, small, big), pristine=pristine)          # warm-up
    for rate in rates:
        res = srv.run(W.pooled_requests(rate, seconds, small, big), pristine=pristine)
        out[f"{int(rate)}/s"] = {"requests": res["requests"], "records_per_s": round(res["records_per_s"], 1),
                                 "p50_ms": round(res["p50_ms"], 3), "p99_ms": round(res["p99_ms"], 3),
                                 "wall_s": round(res["wall_s"], 3), "batches": res["batches"],
                                 "mean_batch": round(res["mean_batch"], 1)}
    # an untimed run at the highest rate keeps every 25th request's report and
    # final memory for the comparison with the oracle (big trees included)
    res = srv.run(W.pooled_requests(rates[-1], 0.25, small, big, seed=W.BASE_SEED + 55), pristine=pristine,
                  keep_every=25)
    out["sample"] = res["sample"]
    out["device_bytes_peak"] = int(sctx.stat("device_bytes_peak"))
    out["budget_trims"] = int(sctx.stat("budget_trims"))
    sctx.close()
    return out


def kc_budget_context(ctx, budget):
    """A context on ctx's device with ctx's options and an HBM budget."""
    from paper_1211_6193_amd import kc
    c = kc.Context(ctx.device, hbm_budget_bytes=budget)
    for k in ("jit", "jit_waves", "sort_tile", "sort_bits", "stage_bytes", "stage", "local", "side_streams"):
        c.set_option(k, int(ctx.stat("option." + k)))
    return c


if __name__ == "__main__":
    main()
