#!/usr/bin/env python3
"""X-drop seed-and-extend benchmark on one MI355X: GCUPS and alignments/s,
batched (persistent, graph-captured) vs plain (one launch sequence per
10,000-record batch), with p50/p99 batch latency.

Workload (default, c2): 1,000,000 read pairs of uneven length shaped like a
100x long-read E. coli set (4.6 Mb random genome, reads lognormal mean 10 kb
/ sd 5 kb clipped to [1, 40] kb, 15 % CLR-like error, one exact 17-mer seed
per pair), X drawn per pair from {20, 50, 100}, match +1 / mismatch -1 /
gap -1, int32 scores, the whole batch in one captured graph.  --workload
picks another preset (c0, c1, c4, c4b).  Inputs are resident in HBM when the
timed region starts.

A step is one pass of the whole hot path over the batch: record ingest
(validation, orientation, seed score), left and right X-drop extensions,
result write-back.  GCUPS counts the candidate cells of every extension
(the oracle's definition; the GPU counting pass is verified against the
oracle on the cpu_baseline sample).

Prints one JSON line.  --gpus N > 1 exits: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SPEC_PEAK_INT32_OPS = 256 * 64 * 2.4e9      # CUs x lanes x clock: one int32 op per lane per cycle
OPS_PER_CELL = 9                            # compare, select, add, max, add gap, max, compare, select, max
KERNEL_SRC = os.path.join(ROOT, "paper_2309_07270_amd", "csrc", "xdrop_kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_valu_peak():
    """int32 lane-ops/s of independent add/max chains at full occupancy
    (libxdrop_probe.so), or None when the probe library is not built."""
    import ctypes
    path = os.path.join(ROOT, "paper_2309_07270_amd", "libxdrop_probe.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    lib.xdrop_probe_valu_ops.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
    ops, ms = ctypes.c_double(), ctypes.c_double()
    if lib.xdrop_probe_valu_ops(0, 100000, ctypes.byref(ops), ctypes.byref(ms)) != 0:
        return None
    return ops.value


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


def read_traffic(stage_name: str, workload: str):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage_name}_{workload}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*(\w+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


WORKLOAD_TEXT = {
    "c0": "read pairs, 200 kb genome at 30x, reads U[1,2] kb, 15% error, k=17, X=50, +1/-1/-1",
    "c1": "read pairs, 29x-shaped 4.6 Mb genome, reads lognormal mean 8 kb sd 4 kb [1,30] kb, 15% error "
          "(8/4/3 sub/ins/del), one planted exact 17-mer seed per pair, X=50, +1/-1/-1",
    "c2": "read pairs of uneven length, 100x-shaped 4.6 Mb genome, reads lognormal mean 10 kb sd 5 kb "
          "[1,40] kb, 15% error (8/4/3 sub/ins/del), one planted exact 17-mer seed per pair, X drawn per pair "
          "from {20,50,100}, +1/-1/-1; the whole batch in one hipGraph launch",
    "c4": "pairs: half true overlaps (100x, reads lognormal mean 20 kb sd 10 kb [1,100] kb, 15% error), "
          "half unrelated pairs against a 50,000-read decoy pool; X=100, +1/-1/-1",
    "c4b": "pairs: half true overlaps (100x, reads lognormal mean 20 kb sd 10 kb [1,100] kb, 15% error), "
           "half unrelated pairs against a 50,000-read decoy pool; X=100, +1/-2/-2",
}


def host_cpu():
    """CPU model, logical CPUs of the host and CPUs this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": allowed}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--pairs", type=int, default=None, help="shrink the workload (tests only)")
    ap.add_argument("--plain-steps", type=int, default=20, help="passes of the plain form over the batch")
    ap.add_argument("--small-batch-passes", type=int, default=5,
                    help="passes of 10,000-record batches through the persistent form")
    ap.add_argument("--tune-sample", type=int, default=200000,
                    help="records the autotuner runs on (the first ones of the batch)")
    ap.add_argument("--no-side-c1", action="store_true", help="skip the c1 side measurement")
    ap.add_argument("--cpu-sample", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="counting pass + timed persistent steps only (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="launch one device copy of 1 GiB (calibrates HBM byte counters) and exit")
    ap.add_argument("--serve", action="store_true",
                    help="serving loop: 25 producers, Poisson arrivals, swept offered load (c3 / c4)")
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--serve-min-batches", type=int, default=0,
                    help="serving: extend a load point until it has completed this many batches")
    ap.add_argument("--serve-points", default="0.1,0.3,0.5,0.7,0.9,1.0,1.1,1.2")
    ap.add_argument("--producers", type=int, default=25)
    ap.add_argument("--seeds", action="store_true",
                    help="seed discovery on a c1-shaped 1%%-error read set (k=31, stride 1, window [20, 30]), "
                         "then the X-drop batch over the seeds found (X=15)")
    ap.add_argument("--granularity", default="0",
                    help="serving hand-off granularity ablation: comma list of sub-batch sizes "
                         "(0 = whole batch); each producer batch is split into sub-batches "
                         "submitted back to back and waited together")
    ap.add_argument("--tuning-cache", default=None,
                    help="launch-parameter file: loaded if it exists (no autotune), else written by the autotuner")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU (--gpus must be 1); records are independent, so the path "
              "shards by records across GPUs with one context per GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of int32
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}))
        return

    from paper_2309_07270_amd import workload as W
    from paper_2309_07270_amd import xdrop as X

    if args.serve:
        serve_main(args)
        return
    if args.seeds:
        seeds_main(args)
        return

    t0 = time.time()
    wl = W.make_workload(args.workload, pairs=args.pairs)
    recs = wl.records
    n = len(recs)
    log(f"workload {args.workload}: {n} records, {wl.meta['reads']} reads, gen {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    d_recs = torch.from_numpy(recs.view(np.uint8).copy()).to(dev)
    d_out = torch.zeros(n * 32, dtype=torch.uint8, device=dev)
    d_cells = torch.zeros(n, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    # autotuner (untimed): launch parameters chosen on the first records of
    # the batch (every setting gives the same results), or taken from a file
    t0 = time.time()
    if args.tuning_cache and os.path.exists(args.tuning_cache):
        ctx = X.Context(wl.store, mode=X.MODE_PERSISTENT, tuning_cache=args.tuning_cache)
        tuning = ctx.tuning()
        log(f"tuning from {args.tuning_cache}: {tuning}")
    else:
        ctx = X.Context(wl.store, mode=X.MODE_PERSISTENT)
        tuning, tune_ms = ctx.autotune(recs[:args.tune_sample], cache_path=args.tuning_cache)
        log(f"autotune on {min(n, args.tune_sample)} records: {tuning} ({tune_ms:.2f} ms per sample batch, "
            f"{time.time() - t0:.1f}s)")
    # counting pass (untimed): exact candidate cells of every extension
    t = ctx.submit_device(d_recs, n, d_out, d_cells, stream=stream)
    ctx.wait(t)
    torch.cuda.synchronize()
    cells_rec = d_cells.cpu().numpy().astype(np.uint64)
    total_cells = int(cells_rec.sum())
    res_gpu = d_out.cpu().numpy().view(W.RESULT_DTYPE).copy()
    log(f"counting pass: {total_cells} cells, {total_cells / n:.0f} per record")

    def timed(c, steps, warmup):
        for _ in range(warmup):
            c.wait(c.submit_device(d_recs, n, d_out, None, stream=stream))
        torch.cuda.synchronize()
        lat, stage = [], np.zeros(X.NUM_STAGES)
        t_start = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            st = c.wait(c.submit_device(d_recs, n, d_out, None, stream=stream))
            lat.append((time.perf_counter() - s0) * 1e3)
            stage += np.asarray(st["stage_ms"])
        torch.cuda.synchronize()
        return time.perf_counter() - t_start, lat, stage / max(steps, 1)

    chunk = 10000

    def chunked(c, passes):
        """The batch as sequential 10,000-record requests: per-request
        latencies, per-pass times and the total time."""
        lat, per_pass = [], []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(passes):
            p0 = time.perf_counter()
            for off in range(0, n, chunk):
                m = min(chunk, n - off)
                s0 = time.perf_counter()
                c.wait(c.submit_device(d_recs[off * 32:(off + m) * 32], m, d_out[off * 32:(off + m) * 32], None,
                                       stream=stream))
                lat.append((time.perf_counter() - s0) * 1e3)
            per_pass.append((time.perf_counter() - p0) * 1e3)
        torch.cuda.synchronize()
        return time.perf_counter() - t_start, lat, per_pass

    # timed persistent steps: the whole batch per captured-graph launch (headline value)
    elapsed, lat, _ = timed(ctx, args.steps, args.warmup)
    ms_per_step = elapsed * 1e3 / args.steps
    gcups = total_cells * args.steps / elapsed / 1e9
    res_t = d_out.cpu().numpy().view(W.RESULT_DTYPE)
    stable = bool(np.array_equal(res_t, res_gpu))
    log(f"persistent (graph): {ms_per_step:.2f} ms/step, {gcups:.1f} GCUPS")
    host_submit = small = None
    if not args.kernel_only:   # profiling runs keep the dispatch list of the device path
        # the same batch submitted from host memory, results back to host
        # memory (PCIe both ways, pinned staging in the library): reported
        # beside the value, never as it
        h_steps = max(3, args.steps // 4)
        ctx.run(recs)
        t_h = time.perf_counter()
        for _ in range(h_steps):
            res_h, _, _ = ctx.run(recs)
        el_h = time.perf_counter() - t_h
        host_submit = {"gcups": round(total_cells * h_steps / el_h / 1e9, 2),
                       "ms_per_batch": round(el_h * 1e3 / h_steps, 3), "batches": h_steps,
                       "results_equal": bool(np.array_equal(res_h, res_gpu))}
        log(f"host-submitted batches: {host_submit['ms_per_batch']:.2f} ms/batch, {host_submit['gcups']:.1f} GCUPS")
        # the same records as 10,000-record requests through the persistent form
        chunked(ctx, 1)   # warm-up
        s_el, s_lat, _ = chunked(ctx, args.small_batch_passes)
        res_s = d_out.cpu().numpy().view(W.RESULT_DTYPE)
        small = {"gcups": round(total_cells * args.small_batch_passes / s_el / 1e9, 2),
                 "p50_ms": pct(s_lat, 50), "p99_ms": pct(s_lat, 99), "batch_records": chunk,
                 "batches": len(s_lat), "results_equal_whole": bool(np.array_equal(res_s, res_gpu))}
        log(f"persistent, 10k requests: {small['gcups']:.1f} GCUPS, p50 {small['p50_ms']:.2f} ms, "
            f"p99 {small['p99_ms']:.2f} ms")
    ctx.close()

    # the same kernel sequence launched directly with HIP events between the
    # stages (on the stream the kernels run on): per-kernel durations and the
    # cells each class completed
    pc = X.Context(wl.store, mode=X.MODE_PERSISTENT, profile=True)
    pc.set_tuning(**tuning)
    pst = pc.wait(pc.submit_device(d_recs, n, d_out, d_cells, stream=stream))
    stage_cells, stage_tasks, stage_slots = pst["stage_cells"], pst["stage_tasks"], pst["stage_slots"]
    p_elapsed, p_lat, stage_ms = timed(pc, args.steps, 1)
    pc.close()
    p_gcups = total_cells * args.steps / p_elapsed / 1e9
    log(f"persistent (profiled launches): {p_elapsed * 1e3 / args.steps:.2f} ms/step, stages "
        f"{dict(zip(X.STAGE_NAMES, np.round(stage_ms, 3).tolist()))}")

    # dominant kernel and its roofline (int32 VALU bound: no contraction, no MFMA)
    win = list(range(1, X.NUM_STAGES - 1))
    dom = max(win, key=lambda k: stage_ms[k])
    dom_name = X.STAGE_NAMES[dom]
    achieved_ops = stage_cells[dom] * OPS_PER_CELL / (stage_ms[dom] / 1e3) if stage_ms[dom] > 0 else 0.0
    traffic = read_traffic(dom_name, args.workload)
    peak_meas = measured_valu_peak()
    if peak_meas:
        log(f"measured int32 VALU peak: {peak_meas / 1e12:.1f} T ops/s (spec-derived {SPEC_PEAK_INT32_OPS / 1e12:.1f})")
    roofline = {"bound": "alu", "kernel": dom_name, "achieved": achieved_ops / 1e12,
                "peak": SPEC_PEAK_INT32_OPS / 1e12, "unit": "Tint32op/s",
                "frac": achieved_ops / SPEC_PEAK_INT32_OPS,
                "measured_peak": peak_meas / 1e12 if peak_meas else None,
                "frac_of_measured": achieved_ops / peak_meas if peak_meas else None,
                "traffic": traffic,
                "units_per_launch": int(stage_cells[dom]), "unit_name": "cells",
                "ops_per_unit": OPS_PER_CELL, "launch_ms": float(stage_ms[dom]),
                "tasks_per_launch": int(stage_tasks[dom]),
                # secondary bound: cells / window lane-steps of the kernel's extensions
                "lane_occupancy": stage_cells[dom] / stage_slots[dom] if stage_slots[dom] else None}

    text = WORKLOAD_TEXT.get(args.workload, "records")
    out = {"metric": "X-drop GCUPS + alignments/s on 1 GPU, batched vs plain; p50/p99 latency",
           "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic (seeded generator; E. coli-shaped)",
           "config": {"workload": f"{args.workload}: {n:,} {text}", "records": n,
                      "cells_per_step": total_cells, "form": "persistent+hipGraph",
                      "tuning": tuning, "parallelism": "1 GPU"},
           "alignments_per_s": round(n * args.steps / elapsed, 1),
           "batched": {"gcups": round(gcups, 2), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                       "batch_records": n, "results_stable_across_steps": stable,
                       "requests_10k": small,
                       "profiled_launches": {"gcups": round(p_gcups, 2),
                                             "stage_ms": dict(zip(X.STAGE_NAMES, np.round(stage_ms, 4).tolist())),
                                             "stage_cells": dict(zip(X.STAGE_NAMES, [int(v) for v in stage_cells])),
                                             "stage_tasks": dict(zip(X.STAGE_NAMES, [int(v) for v in stage_tasks])),
                                             "stage_slots": dict(zip(X.STAGE_NAMES, [int(v) for v in stage_slots]))},
                       "host_submit": host_submit},
           "roofline": roofline}

    if args.kernel_only:
        print(json.dumps(out))
        return

    # plain form: the same records as sequential 10,000-record launches
    # ("Method", Baseline), over --plain-steps passes of the whole batch
    pctx = X.Context(wl.store, mode=X.MODE_PLAIN)
    pctx.set_tuning(**tuning)
    chunked(pctx, 1)   # warm-up
    p_el, plat, ppass = chunked(pctx, args.plain_steps)
    plain_gcups = total_cells * args.plain_steps / p_el / 1e9
    res_p = d_out.cpu().numpy().view(W.RESULT_DTYPE)
    pctx.close()
    out["plain"] = {"gcups": round(plain_gcups, 2), "alignments_per_s": round(n * args.plain_steps / p_el, 1),
                    "requests_10k": {"p50_ms": pct(plat, 50), "p99_ms": pct(plat, 99), "batch_records": chunk,
                                     "batches": len(plat)},
                    "whole_batch": {"p50_ms": pct(ppass, 50), "p99_ms": pct(ppass, 99), "batch_records": n,
                                    "passes": args.plain_steps},
                    "results_equal_batched": bool(np.array_equal(res_p, res_gpu))}
    out["batched_over_plain"] = {
        "gcups": round(gcups / plain_gcups, 3),
        "p99_whole_batch": round(out["plain"]["whole_batch"]["p99_ms"] / pct(lat, 99), 3),
        "p99_requests_10k": round(plat and small and pct(plat, 99) / small["p99_ms"] or 0.0, 3)}
    log(f"plain: {plain_gcups:.1f} GCUPS; 10k requests p50 {pct(plat, 50):.2f} ms p99 {pct(plat, 99):.2f} ms; "
        f"whole batch p50 {pct(ppass, 50):.1f} ms p99 {pct(ppass, 99):.1f} ms")

    if not args.no_side_c1 and args.workload != "c1" and args.pairs is None:
        # side line: the 29x-shaped batch (c1) with the same launch parameters
        w1 = W.make_workload("c1")
        n1 = len(w1.records)
        r1 = torch.from_numpy(w1.records.view(np.uint8).copy()).to(dev)
        o1 = torch.zeros(n1 * 32, dtype=torch.uint8, device=dev)
        c1cells = torch.zeros(n1, dtype=torch.int64, device=dev)
        with X.Context(w1.store, mode=X.MODE_PERSISTENT) as cx:
            cx.set_tuning(**tuning)
            cx.wait(cx.submit_device(r1, n1, o1, c1cells, stream=stream))
            torch.cuda.synchronize()
            cells1 = int(c1cells.sum().item())
            for _ in range(2):
                cx.wait(cx.submit_device(r1, n1, o1, None, stream=stream))
            torch.cuda.synchronize()
            k1 = max(5, args.steps // 2)
            t1 = time.perf_counter()
            for _ in range(k1):
                cx.wait(cx.submit_device(r1, n1, o1, None, stream=stream))
            torch.cuda.synchronize()
            el1 = time.perf_counter() - t1
        out["c1"] = {"workload": f"c1: {n1:,} {WORKLOAD_TEXT['c1']}", "gcups": round(cells1 * k1 / el1 / 1e9, 2),
                     "ms_per_batch": round(el1 * 1e3 / k1, 3), "cells": cells1, "steps": k1}
        log(f"c1 side line: {out['c1']['ms_per_batch']:.2f} ms per batch, {out['c1']['gcups']:.1f} GCUPS")

    if not args.no_cpu_baseline:
        import oracle
        S = min(args.cpu_sample, n)
        threads = oracle.default_threads()
        c0 = time.perf_counter()
        ref, used = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, recs[:S], nthreads=threads)
        c_el = time.perf_counter() - c0
        ref_cells = int((ref["cells_left"] + ref["cells_right"]).sum())
        same = np.ones(S, bool)
        for fg, fr in (("score", "score"), ("left_score", "left"), ("right_score", "right"),
                       ("seed_score", "seed"), ("a_begin", "a_begin"), ("a_end", "a_end"),
                       ("b_begin", "b_begin"), ("b_end", "b_end")):
            same &= res_gpu[fg][:S].astype(np.int64) == ref[fr].astype(np.int64)
        same &= cells_rec[:S] == (ref["cells_left"] + ref["cells_right"]).astype(np.uint64)
        host = host_cpu()
        out["cpu_baseline"] = {"value": round(ref_cells / c_el / 1e9, 3), "unit": "GCUPS", "cores": int(used),
                               "kind": "oracle",
                               "sample": f"first {S} records of {args.workload} ({ref_cells} cells, {c_el:.1f} s "
                                         f"on {used} threads)",
                               "host": {**host, "threads_rule": "min(CPUs allowed, 16): the host share of one GPU"}}
        out["parity_sample"] = f"{int(same.sum())}/{S} records bit-exact (results and cells) vs oracle"
        log(f"cpu oracle: {ref_cells / c_el / 1e9:.3f} GCUPS on {used} threads ({host}); parity {int(same.sum())}/{S}")
        # the same oracle on one host thread, over a tenth of the sample
        S1 = max(1, S // 10)
        c0 = time.perf_counter()
        ref1, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, recs[:S1], nthreads=1)
        c1_el = time.perf_counter() - c0
        cells1 = int((ref1["cells_left"] + ref1["cells_right"]).sum())
        out["cpu_baseline_1core"] = {"value": round(cells1 / c1_el / 1e9, 3), "unit": "GCUPS", "cores": 1,
                                     "kind": "oracle",
                                     "sample": f"first {S1} records of {args.workload} ({cells1} cells, {c1_el:.1f} s)"}
        log(f"cpu oracle, 1 thread: {cells1 / c1_el / 1e9:.3f} GCUPS")

    print(json.dumps(out))


def seeds_main(args):
    """Seed discovery (the step before the batches) and seed-and-extend of the
    seeds it finds.  Reads: 29x of a 4.6 Mb genome, c1 length law, 1 % error
    (the paper's frequency window [20, 30] at 29x keeps only k-mers of near
    error-free reads); k = 31, stride 1, window [20, 30] and X = 15 as in the
    paper's runs ("Method")."""
    import numpy as np
    import torch

    from paper_2309_07270_amd import workload as W
    from paper_2309_07270_amd import xdrop as X

    t0 = time.time()
    st = W.make_readset("c1", error=0.01)
    log(f"read set: {st.n} reads, {int(st.length.sum())} bases, gen {time.time() - t0:.1f}s")
    ctx = X.Context(st)
    recs, s0 = ctx.find_seeds(k=31, lo=20, hi=30, x=15)          # warm-up and sizing
    ms = []
    for _ in range(max(args.steps // 4, 3)):
        r2, s1 = ctx.find_seeds(k=31, lo=20, hi=30, x=15, max_records=len(recs))
        ms.append(s1["device_ms"])
    assert len(r2) == len(recs)
    dev_ms = float(np.median(ms))
    log(f"seeds: {s0['kmers']} k-mers, {s0['distinct']} distinct, {s0['reliable']} reliable, "
        f"{len(recs)} pairs in {dev_ms:.2f} ms")
    # seed-and-extend of the pairs found, persistent form: the seed records
    # are written to HBM and handed to the batch there
    n = len(recs)
    d_recs = torch.zeros(n * 32, dtype=torch.uint8, device="cuda")
    n_dev, _ = ctx.find_seeds_device(d_recs, n, k=31, lo=20, hi=30, x=15)
    assert n_dev == n
    d_out = torch.zeros(n * 32, dtype=torch.uint8, device="cuda")
    d_cells = torch.zeros(n, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    ctx.wait(ctx.submit_device(d_recs, n, d_out, d_cells, stream=stream))
    torch.cuda.synchronize()
    cells = int(d_cells.cpu().numpy().sum())
    t1 = time.perf_counter()
    steps = args.steps
    for _ in range(steps):
        ctx.wait(ctx.submit_device(d_recs, n, d_out, None, stream=stream))
    torch.cuda.synchronize()
    ext_ms = (time.perf_counter() - t1) * 1e3 / steps
    res = d_out.cpu().numpy().view(W.RESULT_DTYPE)
    ctx.close()
    log(f"extension of the seeds: {ext_ms:.2f} ms per batch, {cells / ext_ms / 1e6:.1f} GCUPS")
    print(json.dumps({
        "metric": "seed discovery (k-mers/s, pairs/s) and seed-and-extend of the pairs found (GCUPS) on 1 GPU",
        "data": "synthetic: 29x of a 4.6 Mb genome, lognormal mean 8 kb reads, 1 % error (8:4:3 sub:ins:del)",
        "params": {"k": 31, "stride": 1, "lo": 20, "hi": 30, "x": 15, "weights": [1, -1, -1]},
        "reads": int(st.n), "bases": int(st.length.sum()),
        "seeds": {"kmers": int(s0["kmers"]), "distinct": int(s0["distinct"]), "reliable": int(s0["reliable"]),
                  "pairs": n, "device_ms": round(dev_ms, 3),
                  "kmers_per_s": round(s0["kmers"] / dev_ms * 1e3, 1), "pairs_per_s": round(n / dev_ms * 1e3, 1)},
        "extension": {"records": n, "cells": cells, "ms_per_batch": round(ext_ms, 3),
                      "gcups": round(cells / ext_ms / 1e6, 2),
                      "mean_score": round(float(res["score"].mean()), 1) if n else None}}))


def serve_main(args):
    """Continuous-batching serving loop (one context, host-submitted batches).

    Producers are threads standing in for the paper's MPI ranks sharing a GPU
    ("Method", One-to-all / One-to-one schedulers).  Batch sizes are uniform in
    [1,000, 50,000] records drawn from the workload's record pool.  Each
    producer follows its own exponential inter-arrival schedule (aggregate rate
    lambda); latency runs from the scheduled arrival to the return of wait, so
    a late submit is charged to the system.  lambda is swept as a fraction of
    the saturated batch rate measured first with every producer submitting
    back to back."""
    import threading

    import numpy as np

    from paper_2309_07270_amd import workload as W
    from paper_2309_07270_amd import xdrop as X

    name = args.workload if args.workload != "c1" else "c2"
    t0 = time.time()
    wl = W.make_workload(name, pairs=args.pairs)
    recs = wl.records
    log(f"serve workload {name}: {len(recs)} records, gen {time.time() - t0:.1f}s")
    ctx = X.Context(wl.store, max_inflight=8,
                    tuning_cache=args.tuning_cache if args.tuning_cache and os.path.exists(args.tuning_cache)
                    else None)
    # exact cells of every record (one counting pass), for GCUPS of each batch
    cells = np.zeros(len(recs), np.uint64)
    for off in range(0, len(recs), 200000):
        _, c, _ = ctx.run(recs[off:off + 200000], count_cells=True)
        cells[off:off + len(c)] = c
    ccum = np.concatenate([[0], np.cumsum(cells, dtype=np.uint64)])
    rng = np.random.default_rng(7)
    P = args.producers

    def batch_at(r):
        # batch size U[1000, 50000], clamped to the pool; start anywhere it fits
        z = min(int(r.integers(1000, 50001)), len(recs))
        s0 = int(r.integers(0, len(recs) - z + 1))
        return s0, z

    def run_phase(rate, seconds, closed, gran=0, min_batches=0):
        """One load point: open loop at `rate` batches/s (closed: back to back)
        for `seconds`, extended until `min_batches` batches have completed."""
        lat, done_recs, done_cells = [], [0], [0]
        lock = threading.Lock()
        t_begin = time.perf_counter()

        errors = []

        def producer(p):
            try:
                produce(p)
            except BaseException as e:   # re-raised in the caller after join
                errors.append(e)

        def produce(p):
            r = np.random.default_rng(1000 + p)
            t_next = t_begin
            def over(t):
                if t - t_begin <= seconds:
                    return False
                with lock:
                    return len(lat) >= min_batches

            while True:
                if not closed:
                    t_next += r.exponential(P / rate)
                    if over(t_next):
                        break
                    now = time.perf_counter()
                    if t_next > now:
                        time.sleep(t_next - now)
                else:
                    t_next = time.perf_counter()
                    if over(t_next):
                        break
                s0, z = batch_at(r)
                if gran <= 0 or z <= gran:
                    ctx.wait(ctx.submit(recs[s0:s0 + z])[0])
                else:
                    tks = [ctx.submit(recs[s0 + o:s0 + min(o + gran, z)])[0] for o in range(0, z, gran)]
                    for tk in tks:
                        ctx.wait(tk)
                t_end = time.perf_counter()
                with lock:
                    lat.append((t_end - t_next) * 1e3)
                    done_recs[0] += z
                    done_cells[0] += int(ccum[s0 + z] - ccum[s0])

        th = [threading.Thread(target=producer, args=(p,)) for p in range(P)]
        for t in th:
            t.start()
        last = time.perf_counter()
        for t in th:
            while t.is_alive():
                t.join(timeout=5.0)
                if time.perf_counter() - last > 30.0:   # a long point reports how far it got
                    last = time.perf_counter()
                    with lock:
                        log(f"  ... {len(lat)} batches after {last - t_begin:.0f} s")
        if errors:
            raise errors[0]
        el = time.perf_counter() - t_begin
        return {"offered_batches_per_s": None if closed else rate, "batches": len(lat),
                "achieved_batches_per_s": len(lat) / el, "alignments_per_s": done_recs[0] / el,
                "gcups": done_cells[0] / el / 1e9, "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)}

    def sweep(gran):
        run_phase(1.0, 1.0, True, gran)  # warm-up: slots, graphs
        sat = run_phase(1.0, args.serve_seconds, True, gran)
        log(f"sub-batch {gran}: saturated {sat['achieved_batches_per_s']:.1f} batches/s, {sat['gcups']:.1f} GCUPS")
        points = []
        for f in [float(x) for x in args.serve_points.split(",")]:
            rate = f * sat["achieved_batches_per_s"]
            r = run_phase(rate, args.serve_seconds, False, gran, args.serve_min_batches)
            r["load_fraction"] = f
            points.append(r)
            log(f"sub-batch {gran}, load {f:.1f}: {r['achieved_batches_per_s']:.1f} b/s, "
                f"p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms")
        return sat, points

    grans = [int(x) for x in args.granularity.split(",")]
    workload = (f"{name}: {len(recs)}-record pool, batches U[1000,50000], {P} producers, "
                f"Poisson arrivals, host-submitted batches")
    if grans == [0]:
        sat, points = sweep(0)
        ctx.close()
        print(json.dumps({"metric": "serving loop: throughput and p50/p99 batch latency vs offered load",
                          "workload": workload, "unit": "GCUPS", "saturated": sat, "points": points}))
        return
    runs = []
    for g in grans:
        sat, points = sweep(g)
        runs.append({"sub_batch": g, "saturated": sat, "points": points})
    ctx.close()
    print(json.dumps({"metric": "serving hand-off granularity: whole batch vs sub-batches, throughput and "
                                "p50/p99 producer-batch latency vs offered load",
                      "workload": workload, "unit": "GCUPS", "runs": runs}))


if __name__ == "__main__":
    main()
