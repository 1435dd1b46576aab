"""Writes the stored expected motif sets under tests/golden/.

Every value here comes from the CPU oracle (``oracle/``) applied to the seeded
synthetic inputs of ``fmgen``; nothing is taken from the GPU library.

  python tests/golden/make_golden.py plain_8_1 plain_11_3          # brute, seeds 0-4
  python tests/golden/make_golden.py plain_15_4 --seeds 0 --mode brute
  python tests/golden/make_golden.py batched --mode skip
  python tests/golden/make_golden.py serving --mode skip

Each record holds the instance recipe, the oracle mode that produced it, the
motif count, the SHA-256 of the ascending little-endian uint32 candidate
numbers, the motifs themselves when there are at most 4096 of them, and the
enhanced method's sequence-visit count (from a skip-mode run), which times
t-l+1 is its algorithmic window-compare count.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import fmgen  # noqa: E402
import oracle  # noqa: E402

MAX_LISTED = 4096


def sha256_codes(codes: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(codes, dtype="<u4").tobytes()).hexdigest()


def record(spec: fmgen.Spec, mode: str, threads: int, max_listed: int = MAX_LISTED) -> dict:
    inst = spec.make()
    t0 = time.time()
    if mode == "skip":
        motifs, visits = oracle.solve(inst.seqs, spec.l, spec.d, mode="skip", threads=threads,
                                      cap=1 << 26, return_visits=True)
        dt = time.time() - t0
    else:
        motifs = oracle.solve(inst.seqs, spec.l, spec.d, mode=mode, threads=threads, cap=1 << 26)
        dt = time.time() - t0
        skip_motifs, visits = oracle.solve(inst.seqs, spec.l, spec.d, mode="skip",
                                           threads=threads, cap=1 << 26, return_visits=True)
        if not np.array_equal(skip_motifs, motifs):
            raise AssertionError(f"skip and {mode} disagree on {spec}")
    rec = dict(l=spec.l, d=spec.d, n=spec.n, t=spec.t, seed=spec.seed,
               generator=fmgen.GENERATOR_VERSION, mode=mode,
               count=int(motifs.size), sha256=sha256_codes(motifs),
               skip_visits=int(visits), consensus=inst.consensus,
               oracle_seconds=round(dt, 2), oracle_threads=threads)
    if motifs.size <= max_listed:
        rec["motifs"] = [oracle.number_to_lmer(int(k), spec.l) for k in motifs]
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--seeds", type=int, nargs="*", default=[0, 1, 2, 3, 4])
    ap.add_argument("--mode", default="brute", choices=["brute", "skip"])
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--count", type=int, default=256, help="batched: number of instances")
    ap.add_argument("--max-listed", type=int, default=None,
                    help="list motifs only up to this count (default 4096, batched 64)")
    args = ap.parse_args()
    for cfg in args.configs:
        path = os.path.join(HERE, f"{cfg}.json")
        old = {}
        if os.path.exists(path):
            with open(path) as f:
                old = {(r["seed"], r["l"], r["d"], r["n"], r["t"]): r for r in json.load(f)["records"]}
        if cfg == "batched":
            specs = fmgen.batched_specs(args.count)
            recipe = "fmgen.batched_specs(256, master_seed=1403)"
        elif cfg == "serving":
            specs = fmgen.serving_check_specs()
            recipe = "fmgen.serving_check_specs()"
        else:
            shape = fmgen.PLAIN[cfg]
            specs = [fmgen.Spec(seed=s, **shape) for s in args.seeds]
            recipe = f"fmgen.gen_fm(seed=s, **fmgen.PLAIN[{cfg!r}])"
        for q, spec in enumerate(specs):
            key = (spec.seed, spec.l, spec.d, spec.n, spec.t)
            if key in old and (old[key]["mode"] == "brute" or args.mode == "skip"):
                continue
            listed = args.max_listed if args.max_listed is not None else (
                64 if cfg in ("batched", "serving") else MAX_LISTED)
            rec = record(spec, args.mode, args.threads, listed)
            old[key] = rec
            print(f"{cfg} #{q} l={spec.l} d={spec.d} n={spec.n} t={spec.t} "
                  f"count={rec['count']} {rec['oracle_seconds']}s", flush=True)
            recs = sorted(old.values(), key=lambda r: (r["seed"], r["l"], r["n"], r["t"]))
            with open(path + ".tmp", "w") as f:
                json.dump({"config": cfg, "recipe": recipe, "records": recs}, f, indent=1)
            os.replace(path + ".tmp", path)


if __name__ == "__main__":
    main()
