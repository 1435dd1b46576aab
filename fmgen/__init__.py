"""Seeded synthetic inputs for the planted (l, d) motif problem.

This module only draws inputs.  It holds none of the search arithmetic and is
shared by the oracle's tests and by the GPU path's tests and benchmarks.

The Fixed number of Mutations (FM) model (Section I.B, Section IV.B): n i.i.d.
uniform ACGT background sequences of length t (25% per base), one uniformly
drawn consensus l-mer, and in every sequence exactly one planted instance in
which exactly d distinct positions of the consensus are replaced by one of the
three other bases, planted at a uniform offset in [0, t - l].

The paper generated its data with RmotifGen, which is not available; these
draws stand in for those datasets with the same shapes and composition.

Draw order per instance (numpy PCG64 via ``default_rng(seed)``):
  1. background  = integers(0, 4, (n, t))
  2. consensus   = integers(0, 4, l)
  3. for each sequence i in order:
       pos   = choice(l, d, replace=False)
       shift = integers(1, 4, d)          # 1..3, so the base always changes
       inst  = consensus; inst[pos] = (consensus[pos] + shift) mod 4
       off   = integers(0, t - l + 1)
       background[i, off:off + l] = inst
  4. codes 0..3 map to the bytes A, C, G, T.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

GENERATOR_VERSION = "fm-pcg64-v1"
ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclasses.dataclass
class Instance:
    """One planted (l, d) instance: n rows of t ACGT bytes plus the planting truth."""

    seqs: np.ndarray          # (n, t) uint8, bytes from b"ACGT"
    l: int
    d: int
    consensus: str            # the planted consensus l-mer
    offsets: np.ndarray       # (n,) planting offsets
    mutated: np.ndarray       # (n, d) mutated positions of each planted instance
    seed: int

    @property
    def n(self) -> int:
        return int(self.seqs.shape[0])

    @property
    def t(self) -> int:
        return int(self.seqs.shape[1])

    def rows(self) -> List[bytes]:
        return [bytes(r) for r in self.seqs]

    def planted(self, i: int) -> str:
        o = int(self.offsets[i])
        return bytes(self.seqs[i, o:o + self.l]).decode()


def gen_fm(l: int, d: int, n: int, t: int, seed: int) -> Instance:
    """Draw one FM instance in the documented order."""
    if not (1 <= l <= t and 0 <= d <= l and n >= 1):
        raise ValueError(f"bad FM shape l={l} d={d} n={n} t={t}")
    rng = np.random.default_rng(seed)
    bg = rng.integers(0, 4, (n, t))
    cons = rng.integers(0, 4, l)
    offsets = np.empty(n, dtype=np.int64)
    mutated = np.empty((n, d), dtype=np.int64)
    for i in range(n):
        pos = rng.choice(l, d, replace=False)
        shift = rng.integers(1, 4, d)
        inst = cons.copy()
        inst[pos] = (cons[pos] + shift) % 4
        off = int(rng.integers(0, t - l + 1))
        bg[i, off:off + l] = inst
        offsets[i] = off
        mutated[i] = np.sort(pos)
    seqs = ALPHABET[bg].astype(np.uint8)
    consensus = bytes(ALPHABET[cons]).decode()
    return Instance(seqs=seqs, l=l, d=d, consensus=consensus, offsets=offsets,
                    mutated=mutated, seed=seed)


def random_seqs(n: int, t: int, seed: int) -> np.ndarray:
    """Plain uniform ACGT rows with nothing planted (edge-case inputs)."""
    rng = np.random.default_rng(seed)
    return ALPHABET[rng.integers(0, 4, (n, t))].astype(np.uint8)


# Named workloads: the small case, the two full plain cases and the mixes.
PLAIN = {
    "plain_8_1": dict(l=8, d=1, n=10, t=200),
    "plain_11_3": dict(l=11, d=3, n=20, t=600),
    "plain_15_4": dict(l=15, d=4, n=20, t=600),
}

BATCH_LD = [(9, 2), (11, 3), (13, 4)]
SERVE_LD = [(9, 2), (11, 3), (13, 4), (15, 4)]
SERVE_WEIGHTS = [4, 3, 2, 1]


@dataclasses.dataclass
class Spec:
    l: int
    d: int
    n: int
    t: int
    seed: int

    def make(self) -> Instance:
        return gen_fm(self.l, self.d, self.n, self.t, self.seed)


def batched_specs(count: int = 256, master_seed: int = 1403,
                  ld: Sequence = BATCH_LD) -> List[Spec]:
    """The batched mix: (l, d) uniform over ``ld``, n in [10, 30], t in [300, 1000]."""
    rng = np.random.default_rng(master_seed)
    out = []
    for _ in range(count):
        l, d = ld[int(rng.integers(0, len(ld)))]
        n = int(rng.integers(10, 31))
        t = int(rng.integers(300, 1001))
        seed = int(rng.integers(2 ** 63))
        out.append(Spec(l, d, n, t, seed))
    return out


def serving_stream(count: int, rate: float, master_seed: int = 1313):
    """Poisson arrivals at ``rate`` requests/s; (l, d) weighted 4:3:2:1 over SERVE_LD.

    Returns a list of (arrival_time_s, Spec), arrival times ascending from 0.
    """
    rng = np.random.default_rng(master_seed)
    w = np.asarray(SERVE_WEIGHTS, dtype=np.float64)
    w = w / w.sum()
    t_now = 0.0
    out = []
    for _ in range(count):
        t_now += float(rng.exponential(1.0 / rate))
        l, d = SERVE_LD[int(rng.choice(len(SERVE_LD), p=w))]
        n = int(rng.integers(10, 31))
        t = int(rng.integers(300, 1001))
        seed = int(rng.integers(2 ** 63))
        out.append((t_now, Spec(l, d, n, t, seed)))
    return out


def serving_check_specs() -> List[Spec]:
    """Requests of the serving workload with stored oracle results: the first
    13 requests of ``serving_stream(64, 100.0)`` ((9,2), (11,3) and four
    (13,4)), its two (15,4) requests at positions 19 and 31, and one (13,4)
    request at n = 10, t = 1000, the largest output the workload draws
    (about 6e5 motifs; seed 1313)."""
    stream = [spec for _, spec in serving_stream(64, 100.0)]
    return stream[:13] + [stream[19], stream[31], Spec(13, 4, 10, 1000, 1313)]
