"""Batched and serving measurements (``bench.py --mode batched|serving``).

Both compare against the plain path run one instance per launch on the same
GPU: ``pms_solve`` called for each instance in turn.
"""
from __future__ import annotations

import gc
import hashlib
import json
import os
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def _golden(name):
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["records"]


def _sha(codes):
    return hashlib.sha256(np.ascontiguousarray(codes, dtype="<u4").tobytes()).hexdigest()


def bench_batched(args, emit=True):
    """The batched workload: 256 instances in one persistent launch replayed
    from a HIP graph, autotuned, against one pms_solve per instance.  Prints
    the line (emit) and returns it."""
    import fmgen
    from . import native as nat

    specs = fmgen.batched_specs(256)
    insts = [s.make() for s in specs]
    work = [(i.seqs, i.l, i.d) for i in insts]
    caps = [1 << 21] * len(insts)
    cache = os.environ.get("PMS_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1403_1313_amd", "autotune.json")
    try:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
    except OSError:
        import tempfile
        cache = os.path.join(tempfile.gettempdir(), "paper_1403_1313_amd_autotune.json")
    nat.set_config(variant={"auto": 0, "lane": 1, "group16": 2, "group64": 3}[args.variant],
                   filter=nat.FILTER_OFF if getattr(args, "filter", "on") == "off" else nat.FILTER_ON)
    t0 = time.perf_counter()
    tuned = nat.autotune_many(work, cache)   # tuned on the batch itself
    tune_s = time.perf_counter() - t0

    for _ in range(max(1, args.warmup)):
        st, motifs, results = nat.solve_many(work, caps)
        assert st == nat.PMS_OK, nat.last_error()
    walls, graph_ms, lat, prep_ms, finish_ms = [], [], [], [], []
    for _ in range(args.steps):
        w0 = time.perf_counter()
        st, motifs, results = nat.solve_many(work, caps)
        walls.append(time.perf_counter() - w0)
        assert st == nat.PMS_OK, nat.last_error()
        s = nat.last_stats()
        graph_ms.append(s["kernel_ms"])
        prep_ms.append(s["host_prep_ms"])
        finish_ms.append(s["host_finish_ms"])
        lat.extend(r.latency_ms for r in results)
    stats = nat.last_stats()
    # One eager launch to split the search kernel from copies and windows,
    # then each (l, d) of the mix alone: how full its candidate slots are.
    os.environ["PMS_NO_GRAPH"] = "1"
    nat.solve_many(work, caps)
    eager = nat.last_stats()
    per_ld = {}
    for ld in fmgen.BATCH_LD:
        sub = [w for w, sp in zip(work, specs) if (sp.l, sp.d) == tuple(ld)]
        nat.solve_many(sub, [1 << 21] * len(sub))
        sst = nat.last_stats()
        per_ld[f"({ld[0]},{ld[1]})"] = {
            "instances": len(sub), "search_kernel_ms": sst["kernel_ms"],
            "slot_efficiency": sst["seq_visits"] / max(1, sst["candidate_slots"]),
            "window_compares": sst["window_compares"], "filtered_batches": sst["filtered_batches"],
            "single_batches": sst["single_batches"], "batches": sst["batches"]}
    del os.environ["PMS_NO_GRAPH"]

    parity = None
    gold = _golden("batched")
    if gold:
        by_seed = {r["seed"]: r for r in gold}
        checked = 0
        parity = True
        for spec, m in zip(specs, motifs):
            r = by_seed.get(spec.seed)
            if r is None:
                continue
            checked += 1
            if not (r["count"] == m.size and r["sha256"] == _sha(m)):
                parity = False
        parity = {"ok": parity, "instances_checked": checked}

    # One instance per launch: the plain host-level path, instance by
    # instance, in the default configuration (the batch's tuning is for the
    # batch).
    tuned_cfg = nat.get_config()
    nat.set_config(variant={"auto": 0, "lane": 1, "group16": 2, "group64": 3}[args.variant],
                   filter=nat.FILTER_OFF if getattr(args, "filter", "on") == "off" else nat.FILTER_ON)
    for i in range(3):
        nat.solve_raw(work[i][0], work[i][1], work[i][2], capacity=caps[i])
    p0 = time.perf_counter()
    per_launch_ms = []
    for (seqs, l, d), cap in zip(work, caps):
        q0 = time.perf_counter()
        st1, cnt, _ = nat.solve_raw(seqs, l, d, capacity=cap)
        per_launch_ms.append((time.perf_counter() - q0) * 1e3)
        assert st1 == nat.PMS_OK
    plain_s = time.perf_counter() - p0
    nat.set_config(**tuned_cfg)

    wall = float(np.median(walls))
    cands = sum(4 ** s.l for s in specs)
    line = {
        "metric": "batched instances/s",
        "value": len(specs) / wall,
        "unit": "instances/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "256 seeded FM instances, (l,d) uniform over (9,2),(11,3),(13,4), "
                               "n in [10,30], t in [300,1000], master seed 1403, one persistent "
                               "launch replayed from a HIP graph", "instances": len(specs)},
        "candidates_per_s": cands / wall,
        "window_compares_per_s": stats["window_compares"] / wall,
        "graph_ms_median": float(np.median(graph_ms)),
        "host_ms_median": {"prep": float(np.median(prep_ms)), "finish": float(np.median(finish_ms)),
                           "binding": float(np.median(np.asarray(walls) * 1e3 - np.asarray(prep_ms)
                                                      - np.asarray(graph_ms)
                                                      - np.asarray(finish_ms)))},
        "eager": {"search_kernel_ms": eager["kernel_ms"], "windows_kernel_ms": eager["windows_ms"],
                  "variant": eager["variant"], "grid": eager["grid"], "wg_waves": eager["wg_waves"],
                  "slot_efficiency": eager["seq_visits"] / max(1, eager["candidate_slots"]),
                  "window_compares_per_s_kernel": eager["window_compares"] / (eager["kernel_ms"] * 1e-3)},
        "instance_latency_ms_p50": _pct(lat, 50),
        "instance_latency_ms_p99": _pct(lat, 99),
        "total_motifs": int(sum(m.size for m in motifs)),
        "autotuned": tuned, "autotune_s": tune_s,
        "one_per_launch": {"total_s": plain_s, "instances_per_s": len(specs) / plain_s,
                           "latency_ms_p50": _pct(per_launch_ms, 50),
                           "latency_ms_p99": _pct(per_launch_ms, 99)},
        "speedup_vs_one_per_launch": plain_s / wall,
        "parity_vs_golden": parity,
        "per_ld_alone": per_ld,
        "filtered_batches": eager["filtered_batches"],
        "filtered_dense_groups": eager["filtered_groups"],
        "batches": eager["batches"], "single_batches": eager["single_batches"],
    }
    nat.set_config(reset=True)
    if emit:
        print(json.dumps(line), flush=True)
    return line


def bench_serving(args):
    import fmgen
    from . import native as nat
    from .serve import Server

    rates = [float(r) for r in os.environ.get("PMS_SERVE_RATES", "20,200,1000,1500").split(",")]
    fixed = os.environ.get("PMS_SERVE_COUNT")
    step_ms = float(os.environ.get("PMS_SERVE_STEP_MS", "2.0"))
    oldest = float(os.environ.get("PMS_SERVE_OLDEST_SHARE", "0.5"))
    inflight = int(os.environ.get("PMS_SERVE_INFLIGHT", "2"))
    min_step = os.environ.get("PMS_SERVE_MIN_STEP_MS")
    min_step = float(min_step) if min_step else step_ms / 2
    lookahead = float(os.environ.get("PMS_SERVE_LOOKAHEAD_MS", "0.25"))
    idle_wait = float(os.environ.get("PMS_SERVE_IDLE_WAIT_MS", "1.0"))
    out = []
    for rate in rates:
        # about a second of arrivals, at least 60 and at most 300 requests
        # 15 s of arrivals at 20 req/s, 5 s at 200, 1000 requests at most:
        # enough that the 99th percentile is not one request.
        count = int(fixed) if fixed else int(min(1000, max(300, 25 * rate)))
        stream = fmgen.serving_stream(count, rate)
        reqs = [(t_arr, spec.make()) for t_arr, spec in stream]
        with Server(mem_budget=256 << 20, step_ms=step_ms, oldest_share=oldest,
                    max_inflight=inflight, min_step_ms=min_step,
                    lookahead_ms=lookahead, idle_wait_ms=idle_wait) as srv:
            # Warm up the kernels and allocator on one request of each (l,d)
            # of the stream; no garbage collection inside the timed loops.
            seen = {}
            for _, inst in reqs:
                seen.setdefault((inst.l, inst.d), inst)
            for inst in seen.values():
                srv.submit(inst.seqs, inst.l, inst.d).result()
            time.sleep(0.05)
            gc.collect()
            gc.disable()
            t0 = time.perf_counter()
            futs = []
            for t_arr, inst in reqs:
                now = time.perf_counter() - t0
                if t_arr > now:
                    time.sleep(t_arr - now)
                futs.append(srv.submit(inst.seqs, inst.l, inst.d))
            results = [f.result() for f in futs]
            gc.enable()
            span = max(r.finished for r in results) - t0
            stats = dict(srv.stats)
            stats["compares_per_s_estimate"] = srv.rate
        # Latency from each request's scheduled arrival (as for the FIFO leg
        # below), so that a client that submits late is not credited.
        lat = [(r.finished - (t0 + t_arr)) * 1e3 for (t_arr, _), r in zip(reqs, results)]
        # Where the time of the slowest requests goes (host clock, ms).
        order = sorted(range(len(results)), key=lambda i: lat[i])[-max(1, len(results) // 100):]
        worst = [results[i] for i in order]
        parts = {"submit_late": [1e3 * (results[i].arrival - (t0 + reqs[i][0])) for i in order],
                 "admit": [1e3 * (r.admitted - r.arrival) for r in worst],
                 "to_first_step": [1e3 * (r.launched - r.admitted) for r in worst],
                 "steps": [1e3 * (r.retired - r.launched) for r in worst],
                 "finish": [1e3 * (r.finished - r.retired) for r in worst],
                 "step_count": [r.steps for r in worst]}
        # the same arrivals served one instance per launch, first come first served
        t1 = time.perf_counter()
        fifo_lat, fifo_codes = [], []
        gc.collect()
        gc.disable()
        for t_arr, inst in reqs:
            now = time.perf_counter() - t1
            if t_arr > now:
                time.sleep(t_arr - now)
            st, cnt, codes = nat.solve_raw(inst.seqs, inst.l, inst.d, capacity=1 << 21)
            fifo_lat.append((time.perf_counter() - t1 - t_arr) * 1e3)
            fifo_codes.append((st, cnt, codes))
        fifo_span = time.perf_counter() - t1
        gc.enable()
        # Every served result against the same request solved alone by pms_solve.
        same = sum(1 for r, (st, cnt, codes) in zip(results, fifo_codes)
                   if st == nat.PMS_OK and r.count == cnt and np.array_equal(r.motifs, codes))
        # Latency by (l,d): the (15,4) requests set the tail.
        # Per (l,d) also the medians of the served requests' parts (host
        # clock, ms), their step counts and their motif counts.
        by_ld = {}
        for (t_arr, inst), r, srv_ms, fifo_ms in zip(reqs, results, lat, fifo_lat):
            by_ld.setdefault(f"({inst.l},{inst.d})", ([], [], []))
            by_ld[f"({inst.l},{inst.d})"][0].append(srv_ms)
            by_ld[f"({inst.l},{inst.d})"][1].append(fifo_ms)
            by_ld[f"({inst.l},{inst.d})"][2].append(r)
        by_ld = {k: {"requests": len(a), "server_ms_p50": _pct(a, 50), "server_ms_max": max(a),
                     "fifo_ms_p50": _pct(b, 50), "fifo_ms_max": max(b),
                     "server_parts_ms_p50": {
                         "admit": _pct([1e3 * (r.admitted - r.arrival) for r in c], 50),
                         "to_first_step": _pct([1e3 * (r.launched - r.admitted) for r in c], 50),
                         "steps": _pct([1e3 * (r.retired - r.launched) for r in c], 50),
                         "finish": _pct([1e3 * (r.finished - r.retired) for r in c], 50)},
                     "steps_mean": float(np.mean([r.steps for r in c])),
                     "reruns": int(sum(r.reruns for r in c)),
                     "motifs_p50": _pct([r.count for r in c], 50),
                     "motifs_max": max(r.count for r in c)}
                 for k, (a, b, c) in sorted(by_ld.items())}
        out.append({"rate": rate, "requests": count, "solves_per_s": count / span,
                    "latency_ms_p50": _pct(lat, 50), "latency_ms_p99": _pct(lat, 99),
                    "server_stats": stats,
                    "slowest_1pct_mean_ms": {k: float(np.mean(v)) for k, v in parts.items()},
                    "parity_vs_solo": {"ok": same == count, "requests_equal": same},
                    "latency_by_ld": by_ld,
                    "one_per_launch_fifo": {"solves_per_s": count / fifo_span,
                                            "latency_ms_p50": _pct(fifo_lat, 50),
                                            "latency_ms_p99": _pct(fifo_lat, 99)}})
    best = max(out, key=lambda r: r["solves_per_s"])
    line = {
        "metric": "served solves/s", "value": best["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": best["requests"], "warmup": 1, "ms_per_step": 1e3 / best["solves_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "Poisson stream of seeded FM solve requests, (l,d) over "
                               "(9,2),(11,3),(13,4),(15,4) weighted 4:3:2:1, n in [10,30], "
                               "t in [300,1000], master seed 1313", "rates": rates,
                   "requests": [r["requests"] for r in out], "step_ms": step_ms,
                   "oldest_share": oldest, "max_inflight": inflight, "min_step_ms": min_step,
                   "lookahead_ms": lookahead, "idle_wait_ms": idle_wait},
        "sweep": out,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_ex(args):
    """pms_solve_ex on the (15,4) workload with real-sequence options: both
    strands (twice the windows) and 1% N (masked), against the same rows with
    no options.  (Parity of these inputs is checked in tests/test_gpu_ex.py.)"""
    import fmgen
    from . import native as nat

    inst = fmgen.gen_fm(seed=args.seed, **fmgen.PLAIN["plain_15_4"])
    l, d = inst.l, inst.d
    rows = [bytes(r) for r in inst.seqs]
    rng = np.random.default_rng(1403)
    masked = []
    for r in rows:
        b = bytearray(r)
        for j in np.nonzero(rng.random(len(b)) < 0.01)[0]:
            b[int(j)] = ord("N")
        masked.append(bytes(b))
    cases = {"plain": (rows, False, False), "both_strands": (rows, False, True),
             "both_strands_masked_1pct": (masked, True, True)}
    out = {}
    for name, (rs, mask_n, both) in cases.items():
        for _ in range(max(1, args.warmup)):
            nat.solve_ex(rs, l, d, mask_n=mask_n, both=both)
        walls, kern = [], []
        for _ in range(args.steps):
            w0 = time.perf_counter()
            got = nat.solve_ex(rs, l, d, mask_n=mask_n, both=both)
            walls.append(time.perf_counter() - w0)
            kern.append(nat.last_stats()["kernel_ms"])
        st = nat.last_stats()
        out[name] = {"wall_ms_median": float(np.median(walls)) * 1e3,
                     "kernel_ms_median": float(np.median(kern)),
                     "candidates_per_s": 4 ** l / float(np.median(walls)),
                     "seq_visits": st["seq_visits"], "window_compares": st["window_compares"],
                     "motifs": int(got.size)}
    best = out["both_strands_masked_1pct"]
    line = {
        "metric": "candidates/s (both strands, 1% N masked)", "value": best["candidates_per_s"],
        "unit": "candidates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": best["wall_ms_median"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"FM planted ({l},{d}), n={inst.n}, t={inst.t}, seed {args.seed}, "
                               "host-level pms_solve_ex; N at 1% of positions (seed 1403)"},
        "cases": out,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_intersect(args):
    """Neighbourhood intersection (pms_solve_intersect) against the sweep
    (pms_solve) on the same FM instances: host-level solves, median wall and
    device time of each, bits set per second, and where the crossover lies."""
    import math
    import fmgen
    from . import native as nat

    shapes = [(11, 3, 20, 600), (13, 4, 20, 600), (15, 4, 20, 600), (16, 3, 20, 600),
              (16, 2, 20, 600), (14, 1, 20, 600)]
    rows = []
    for (l, d, n, t) in shapes:
        inst = fmgen.gen_fm(l, d, n, t, args.seed)
        res = {}
        for name, fn in (("sweep", nat.solve), ("intersect", nat.solve_intersect)):
            for _ in range(max(1, args.warmup)):
                got = fn(inst.seqs, l, d)
            walls, dev = [], []
            for _ in range(max(1, args.steps // 4)):
                w0 = time.perf_counter()
                got = fn(inst.seqs, l, d)
                walls.append(time.perf_counter() - w0)
                dev.append(nat.last_stats()["kernel_ms"])
            st = nat.last_stats()
            res[name] = {"wall_ms": float(np.median(walls)) * 1e3,
                         "device_ms": float(np.median(dev)),
                         "motifs": int(got.size), "codes_sha": _sha(got)}
            if name == "intersect":
                res[name]["bits_set_per_s"] = st["window_compares"] / (np.median(dev) * 1e-3)
                res[name]["sequences_processed"] = st["batches"]
        ball = sum(math.comb(l, k) * 3 ** k for k in range(d + 1))
        rows.append({"l": l, "d": d, "n": n, "t": t, "ball": ball,
                     "same_result": res["sweep"]["codes_sha"] == res["intersect"]["codes_sha"],
                     "faster": min(res, key=lambda k: res[k]["wall_ms"]), **res})
    line = {
        "metric": "intersect vs sweep wall-time ratio at (16,2)",
        "value": next(r for r in rows if (r["l"], r["d"]) == (16, 2))["sweep"]["wall_ms"]
        / next(r for r in rows if (r["l"], r["d"]) == (16, 2))["intersect"]["wall_ms"],
        "unit": "x", "n_gpus": 1, "steps": max(1, args.steps // 4), "warmup": args.warmup,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "FM planted instances, n=20, t=600, seed "
                               f"{args.seed}, both exact methods through the host-level C ABI"},
        "shapes": rows,
    }
    print(json.dumps(line), flush=True)
    return 0

