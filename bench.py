#!/usr/bin/env python3
"""Benchmark of the planted (l, d) motif search on one MI355X.

Default: the (15,4) FM workload (n=20, t=600, seed 0), inputs resident in HBM.
One step = one whole solve through the device-level C ABI on torch's current
stream: window building (a1-a2), the persistent search (a3-a6), then the
motif count and codes copied back and sorted on the host (a7).  The steps
run twice: one at a time (each waits for its own result: `step_latency_ms`,
and the library's kernel times behind the roofline), then pipelined, two in
flight on the stream with every step's results still read back and sorted in
the timed region (whole-job throughput: `ms_per_step` and `value`).  Prints
one JSON line.  ``--mode batched`` / ``--mode serving`` / ``--mode ex`` /
``--mode intersect`` print the batched, serving, real-sequence-options
(pms_solve_ex) and neighbourhood-intersection lines instead.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# gfx950 integer VALU peak: 256 compute units x 128 lane-operations per clock
# (4 SIMDs x 32 lanes for plain 32-bit VGPR-only forms, measured with
# pms_valu_probe; the same lane rate as the published fp32 vector figure)
# x 2.4 GHz peak engine clock.
CUS, LANES_PER_CU, CLOCK_HZ = 256, 128, 2.4e9
VALU_INT32_PEAK = CUS * LANES_PER_CU * CLOCK_HZ          # lane-ops/s
# Per-lane kernel: VALU instructions per window compare in its inner loop
# (v_xor_b32, v_or_b32_sdwa, v_bcnt_u32_b32 and half of a v_min3_u32).
LANE_OPS_PER_COMPARE = 3.5
# Algorithmic operations per window compare: the method's compare without
# skipping any window, in its cheapest form here -- the 64-candidate
# kernel's shared-prefix scan, whose loop takes 147 VALU instructions per 32
# windows x 64 candidates at l = 15 in the ISA of this build (the loop with 7
# ds_bpermute and 3 ds_read_b128 per iteration).  W_skip x this / kernel time
# is the algorithmic work rate reported as the roofline's `achieved`.
ALG_OPS_PER_COMPARE = 147.0 / (32 * 64)
KERNELS = {1: ("pms_search_kernel", "pms_kernels.hip"),
           2: ("pms_search_group_kernel", "pms_group.hip"),
           3: ("pms_search_group64_kernel", "pms_group.hip")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="plain",
                    choices=["plain", "batched", "serving", "probe", "copy", "ex", "intersect"],
                    help="probe: VALU issue rates; copy: a plain device copy of known size "
                         "(calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--config", default="plain_15_4", choices=["plain_8_1", "plain_11_3", "plain_15_4"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--variant", default="auto", choices=["auto", "lane", "group16", "group64"],
                    help="search kernel variant")
    ap.add_argument("--filter", default="on", choices=["on", "off"],
                    help="window filter of the 64-candidate kernel (off: every window scanned)")
    ap.add_argument("--no-batched", action="store_true",
                    help="leave out the batched leg (256 instances in one launch) of the default line")
    ap.add_argument("--no-plain-filter-off", action="store_true",
                    help="leave out the unfiltered comparison run of the default line")
    ap.add_argument("--skip-host-level", action="store_true",
                    help="leave out the host-level pms_solve timings (profiling runs: then the "
                         "timed steps are the only search launches)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--counters", default=os.path.join(ROOT, "profiles", "counters.json"),
                    help="rocprofv3 counter results per kernel and workload")
    return ap.parse_args()


def oracle_rate(seqs, l, d, mode, threads, seconds):
    """Candidates/s of the oracle over a prefix of the candidate space sized to
    take about `seconds`; (rate, span, elapsed)."""
    import oracle
    span = 1 << 10
    while True:
        t0 = time.perf_counter()
        oracle.solve(seqs, l, d, mode=mode, threads=threads, k_range=(0, span))
        dt = time.perf_counter() - t0
        if dt >= seconds / 4 or span >= 4 ** l:
            break
        span = min(4 ** l, int(span * max(2.0, min(16.0, seconds / 4 / max(dt, 1e-3)))))
    return span / dt, span, dt


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(seqs, l, d, target_s):
    """The oracle (brute mode, unmodified) on a bounded prefix of the candidate
    space; beside it the oracle's skip mode (the paper's own CPU method,
    Section III.A) on the same instance, and skip mode on one thread for the
    (11,3) shape, the framing of the paper's speedups over one thread."""
    import oracle
    import fmgen
    threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    span = 1 << 14
    while True:
        t0 = time.perf_counter()
        oracle.solve(seqs, l, d, mode="brute", threads=threads, k_range=(0, span))
        dt = time.perf_counter() - t0
        if dt >= target_s / 4 or span >= 4 ** l:
            break
        span = min(4 ** l, int(span * max(2.0, min(16.0, target_s / 4 / max(dt, 1e-3)))))
    if dt < target_s / 2 and span < 4 ** l:
        span = min(4 ** l, int(span * target_s / dt))
        t0 = time.perf_counter()
        oracle.solve(seqs, l, d, mode="brute", threads=threads, k_range=(0, span))
        dt = time.perf_counter() - t0
    skip_rate, skip_span, skip_dt = oracle_rate(seqs, l, d, "skip", threads, 3.0)
    inst11 = fmgen.gen_fm(seed=0, **fmgen.PLAIN["plain_11_3"])
    one_rate, one_span, one_dt = oracle_rate(inst11.seqs, 11, 3, "skip", 1, 3.0)
    return {"value": span / dt, "unit": "candidates/s", "cores": threads, "kind": "oracle",
            "host_cpu": host_cpu_model(), "host_threads_online": os.cpu_count(),
            "sample": f"brute-mode oracle over candidates [0, {span}) of the same instance "
                      f"({span / 4 ** l:.2e} of 4^{l}), {dt:.1f} s on {threads} host threads",
            "skip_mode": {"value": skip_rate, "unit": "candidates/s", "cores": threads,
                          "sample": f"candidates [0, {skip_span}), {skip_dt:.1f} s"},
            "one_thread_skip_11_3": {"value": one_rate, "unit": "candidates/s", "cores": 1,
                                     "sample": f"(11,3) n=20 t=600 seed 0, candidates "
                                               f"[0, {one_span}), {one_dt:.1f} s"}}


def code_text(src):
    """Source text without // comments and blank lines: a comment edit leaves
    the counter record of a kernel valid."""
    lines = (re.sub(r"//.*", "", ln).rstrip() for ln in src.splitlines())
    return "\n".join(ln for ln in lines if ln)


def load_counters(path, key, source):
    """Counter record for `key` and whether the kernel source still matches it."""
    import hashlib
    try:
        with open(path) as f:
            rec = json.load(f).get(key)
        with open(os.path.join(ROOT, "paper_1403_1313_amd", "csrc", source)) as f:
            h = hashlib.sha256(code_text(f.read()).encode()).hexdigest()[:16]
    except (OSError, ValueError):
        return None, False
    if not rec:
        return None, False
    return rec, rec.get("kernel_source_sha256_prefix") == h


def bench_plain(args):
    import torch
    import fmgen
    from paper_1403_1313_amd import native as nat

    variant = {"auto": 0, "lane": 1, "group16": 2, "group64": 3}[args.variant]
    filt = nat.FILTER_ON if args.filter == "on" else nat.FILTER_OFF
    nat.set_config(variant=variant, filter=filt)
    shape = fmgen.PLAIN[args.config]
    inst = fmgen.gen_fm(seed=args.seed, **shape)
    l, d, n, t = inst.l, inst.d, inst.n, inst.t
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    seqs = torch.from_numpy(inst.seqs.reshape(-1).copy()).to(dev)
    cap = 1 << 20
    out = torch.zeros(cap, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    host_cnt = torch.zeros(1, dtype=torch.int64).pin_memory()
    # The count and the first codes come back in one round trip; a larger
    # motif set takes a second copy.
    head = 4096
    host_out = torch.zeros(head, dtype=torch.int32).pin_memory()

    def step():
        nat.solve_dev(seqs, n, t, l, d, out, cap, cnt, stream=stream)
        host_cnt.copy_(cnt, non_blocking=True)
        host_out.copy_(out[:head], non_blocking=True)
        stream.synchronize()
        k = min(int(host_cnt.item()), cap)
        got = host_out[:k] if k <= head else out[:k].cpu()
        codes = np.sort(got.numpy().view(np.uint32))
        return codes, nat.last_stats()

    def timed(steps, warmup):
        """(codes, stats, per-step kernel ms, windows ms, step wall s, total wall s, event ms)."""
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        kernel_ms, windows_ms, step_wall = [], [], []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        w0 = time.perf_counter()
        codes = st = None
        for _ in range(steps):
            s0 = time.perf_counter()
            codes, st = step()
            step_wall.append(time.perf_counter() - s0)
            kernel_ms.append(st["kernel_ms"])
            windows_ms.append(st["windows_ms"])
        e1.record(stream)
        torch.cuda.synchronize()
        return codes, st, kernel_ms, windows_ms, step_wall, time.perf_counter() - w0, e0.elapsed_time(e1)

    def pipelined(steps):
        """Throughput over `steps` solves with two in flight on the stream
        (outputs double buffered): step k+1 is queued before step k's count
        and codes are read back and sorted, so the device does not wait for
        the host between steps.  Every step's results still come back and
        are sorted inside the timed region.  (codes of the last step, event ms)."""
        bufs = [{"out": torch.zeros(cap, dtype=torch.int32, device=dev),
                 "cnt": torch.zeros(1, dtype=torch.int64, device=dev),
                 "hcnt": torch.zeros(1, dtype=torch.int64).pin_memory(),
                 "hout": torch.zeros(head, dtype=torch.int32).pin_memory(),
                 "ev": torch.cuda.Event()} for _ in range(2)]

        def issue(k):
            b = bufs[k % 2]
            nat.solve_dev(seqs, n, t, l, d, b["out"], cap, b["cnt"], stream=stream)
            b["hcnt"].copy_(b["cnt"], non_blocking=True)
            b["hout"].copy_(b["out"][:head], non_blocking=True)
            b["ev"].record(stream)

        def collect(k):
            b = bufs[k % 2]
            b["ev"].synchronize()
            kk = min(int(b["hcnt"].item()), cap)
            got = b["hout"][:kk] if kk <= head else b["out"][:kk].cpu()
            return np.sort(got.numpy().view(np.uint32))

        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        issue(0)
        last = None
        for k in range(steps):
            if k + 1 < steps:
                issue(k + 1)
            last = collect(k)
        e1.record(stream)
        torch.cuda.synchronize()
        return last, e0.elapsed_time(e1)

    # Per-step latency (each step waits for its own result) with the
    # library's kernel times, then the throughput of the same steps
    # pipelined, which `value` reports.
    codes, st, kernel_ms, windows_ms, step_wall, wall, ms_total = timed(args.steps, args.warmup)
    ms_latency = ms_total / args.steps
    codes_p, ms_pipe = pipelined(args.steps)
    ms_step = ms_pipe / args.steps
    cands = 4 ** l
    k_ms = float(np.mean(kernel_ms))
    wc = st["window_compares"]
    kname, ksrc = KERNELS[st["variant"]]
    rec, fresh = load_counters(args.counters, f"{kname}/{args.config}", ksrc)
    # Algorithmic work of the launch: W_skip window compares at the cost of
    # the method's compare loop with no window skipped (the per-lane kernel:
    # its own loop).
    alg_opc = LANE_OPS_PER_COMPARE if st["variant"] == 1 else ALG_OPS_PER_COMPARE
    achieved = wc * alg_opc / (k_ms * 1e-3)
    # Executed VALU work from the counter run of this kernel source.
    if rec and fresh:
        exec_opc = rec["valu_insts_per_launch"] * 64 / rec["window_compares"]
        exec_src = "SQ_INSTS_VALU x 64 / window compares (" + rec.get("profile", "profiles/") + ")"
    elif st["variant"] == 1:
        exec_opc, exec_src = LANE_OPS_PER_COMPARE, "inner-loop ISA: 56 VALU per 16 windows"
    else:
        exec_opc, exec_src = None, ("no counter run for this kernel source" if not rec
                                    else "kernel changed since the counter run")

    parity = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{args.config}.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            recs = [r for r in json.load(f)["records"] if r["seed"] == args.seed]
        if recs:
            parity = [nat.decode(int(c), l) for c in codes] == recs[0]["motifs"] and \
                st["seq_visits"] == recs[0]["skip_visits"]

    # HBM bytes follow the work-item count as well as the kernel (each claim
    # and its record are traffic), so the stored figure holds only for the
    # same table size.
    traffic = rec.get("bytes_per_launch") if (rec and fresh and
                                               rec.get("work_items") == st["work_items"]) else None
    line = {
        "metric": "candidates/s",
        "value": cands / (ms_step * 1e-3),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"FM planted ({l},{d}) motif search, n={n}, t={t}, seed {args.seed}, "
                               f"all 4^{l} candidates", "l": l, "d": d, "n": n, "t": t,
                   "seed": args.seed, "candidates": cands},
        "window_compares_per_s": wc / (ms_step * 1e-3),
        "step_latency_ms": ms_latency,
        "pipelined_same_motifs": bool(np.array_equal(codes_p, codes)),
        "kernel_ms": k_ms,
        "kernel_ms_median": float(np.median(kernel_ms)),
        "kernel_ms_min": float(np.min(kernel_ms)),
        "step_wall_ms_median": float(np.median(step_wall)) * 1e3,
        "step_wall_ms_min": float(np.min(step_wall)) * 1e3,
        "windows_kernel_ms": float(np.mean(windows_ms)),
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "seq_visits": st["seq_visits"],
        "window_compares": wc,
        "candidate_slots": st["candidate_slots"],
        "batches": st["batches"],
        "single_batches": st["single_batches"],
        "filter": args.filter,
        "filtered_batches": st["filtered_batches"],
        "filtered_dense_groups": st["filtered_groups"],
        "slot_efficiency": st["seq_visits"] / max(1, st["candidate_slots"]),
        "variant": nat.VARIANT_NAMES[st["variant"]],
        "motifs": int(codes.size),
        "parity_vs_golden": parity,
        "launch": {"grid": st["grid"], "wg_waves": st["wg_waves"], "chunk": st["chunk"],
                   "work_items": st["work_items"]},
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": VALU_INT32_PEAK / 1e12,
            "unit": "Tops/s",
            "frac": achieved / VALU_INT32_PEAK,
            "traffic": traffic,
            "kernel": kname,
            "ops_per_compare": alg_opc,
            "ops_per_compare_source": ("per-lane kernel loop ISA" if st["variant"] == 1 else
                                       "shared-prefix scan loop ISA: 147 VALU per 32 windows x 64 "
                                       "candidates, no window skipped"),
            "frac_valu_issued": (wc * exec_opc / (k_ms * 1e-3) / VALU_INT32_PEAK
                                 if exec_opc else None),
            "executed_ops_per_compare": exec_opc,
            "executed_ops_source": exec_src,
        },
        "cpu_baseline": None,
    }
    if not args.skip_host_level:
        # The host-level call on the same instance (host rows in, sorted motifs
        # out: validation, upload, both kernels, copy-back and sort).
        host_walls, host_prep, host_finish = [], [], []
        for _ in range(5):
            h0 = time.perf_counter()
            nat.solve(inst.seqs, l, d)
            host_walls.append(time.perf_counter() - h0)
            hs = nat.last_stats()
            host_prep.append(hs["host_prep_ms"])
            host_finish.append(hs["host_finish_ms"])
        line["host_level_pms_solve_ms"] = {"median": float(np.median(host_walls)) * 1e3,
                                           "min": float(np.min(host_walls)) * 1e3,
                                           "prep_median": float(np.median(host_prep)),
                                           "finish_median": float(np.median(host_finish))}
    if not args.no_plain_filter_off and filt == nat.FILTER_ON and st["variant"] == 3:
        # The same steps with every window scanned (the unfiltered sweep of the
        # method's enhanced rule), reported apart from the filtered path.
        nat.set_config(variant=variant, filter=nat.FILTER_OFF)
        codes0, st0, kms0, _, _, _, mst0 = timed(args.steps, max(1, args.warmup))
        k0 = float(np.mean(kms0))
        line["unfiltered"] = {
            "ms_per_step": mst0 / args.steps, "kernel_ms": k0,
            "candidates_per_s": cands / (mst0 / args.steps * 1e-3),
            "roofline_frac": wc * ALG_OPS_PER_COMPARE / (k0 * 1e-3) / VALU_INT32_PEAK,
            "same_motifs": bool(np.array_equal(codes0, codes)),
            "same_visits": st0["seq_visits"] == st["seq_visits"],
            "filter_speedup": k0 / k_ms}
        nat.set_config(variant=variant, filter=filt)
    if not args.no_batched:
        from paper_1403_1313_amd import benchmarks
        bl = benchmarks.bench_batched(args, emit=False)
        line["batched"] = {k: bl[k] for k in (
            "value", "unit", "ms_per_step", "instance_latency_ms_p50", "instance_latency_ms_p99",
            "speedup_vs_one_per_launch", "one_per_launch", "parity_vs_golden", "graph_ms_median",
            "eager", "autotuned", "candidates_per_s", "window_compares_per_s",
            "filtered_batches", "filtered_dense_groups", "per_ld_alone")}
        line["batched"]["workload"] = bl["config"]["workload"]
        nat.set_config(variant=variant, filter=filt)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(inst.seqs, l, d, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


def bench_probe(args):
    from paper_1403_1313_amd import native as nat
    for op in nat.PROBE_OPS:
        for wps in (2, 8):
            r = nat.valu_probe(op, waves_per_simd=wps)
            print(json.dumps({"probe": op, "waves_per_simd": wps, **r}), flush=True)
    return 0


def bench_copy(args):
    """Device-to-device copy of --copy-mib MiB, --steps times (counter calibration)."""
    import torch
    nbytes = args.copy_mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    print(json.dumps({"copy_bytes": nbytes, "ms": ms, "GB_per_s_read_plus_write": 2 * nbytes / ms / 1e6}),
          flush=True)
    return 0


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the search would "
              "shard by candidate ranges across GPUs, which this program does not launch.",
              file=sys.stderr)
        return 2
    if args.mode == "plain":
        return bench_plain(args)
    if args.mode == "probe":
        return bench_probe(args)
    if args.mode == "copy":
        return bench_copy(args)
    if args.mode == "batched":
        from paper_1403_1313_amd import benchmarks
        benchmarks.bench_batched(args)
        return 0
    if args.mode == "ex":
        from paper_1403_1313_amd import benchmarks
        return benchmarks.bench_ex(args)
    if args.mode == "intersect":
        from paper_1403_1313_amd import benchmarks
        return benchmarks.bench_intersect(args)
    from paper_1403_1313_amd import benchmarks
    return benchmarks.bench_serving(args)


if __name__ == "__main__":
    sys.exit(main())
