"""Pins for the CPU oracle: facts fixed by the paper's definitions and by
mathematics, computed without the oracle's code.

Each ``pin_*`` takes an object with the oracle's ``solve`` /
``candidate_distances`` interface and raises AssertionError on a mismatch.
The same battery pins the real oracle and must catch planted mistakes in
copies of it.

Definitions pinned (Section I.A; Section III.A): windows are the t-l+1
length-l substrings of a sequence; the distance is the number of differing
positions; an l-mer matches a window at distance <= d; the motif set keeps the
l-mers that match a window of every sequence.
"""
from __future__ import annotations

import itertools
import math
from typing import Iterable, List, Sequence

import numpy as np

import fmgen

BASES = "ACGT"


# ---------------------------------------------------------------------------
# Independent computations
# ---------------------------------------------------------------------------
def definition_motifs(rows: Sequence[str], l: int, d: int) -> List[int]:
    """The motif set by the definition, enumerating strings (tiny inputs only).

    ``itertools.product`` yields l-mers in dictionary order, so the running
    index is the candidate number (first base most significant, A<C<G<T).
    """
    rows = [r.upper() for r in rows]
    out = []
    for k, x in enumerate(itertools.product(BASES, repeat=l)):
        ok = True
        for row in rows:
            if not any(sum(a != b for a, b in zip(x, row[j:j + l])) <= d
                       for j in range(len(row) - l + 1)):
                ok = False
                break
        if ok:
            out.append(k)
    return out


def definition_visits(rows: Sequence[str], l: int, d: int) -> int:
    """Sequence scans of the enhanced method: each candidate is checked against
    sequences in order until the first one with no matching window."""
    total = 0
    for x in itertools.product(BASES, repeat=l):
        for row in rows:
            total += 1
            if not any(sum(a != b for a, b in zip(x, row[j:j + l])) <= d
                       for j in range(len(row) - l + 1)):
                break
    return total


def ball_size(l: int, d: int) -> int:
    """|{x : d_H(x, w) <= d}| over a 4-letter alphabet: sum_k C(l,k) 3^k."""
    return sum(math.comb(l, k) * 3 ** k for k in range(d + 1))


def _codes(mat: np.ndarray) -> np.ndarray:
    lut = np.zeros(256, dtype=np.uint32)
    for v, ch in enumerate(BASES):
        lut[ord(ch)] = v
        lut[ord(ch.lower())] = v
    return lut[mat]


def window_numbers(row_codes: np.ndarray, l: int) -> np.ndarray:
    """Candidate number of every window of one sequence (first base most significant)."""
    win = np.lib.stride_tricks.sliding_window_view(row_codes, l)
    weights = (np.uint64(4) ** np.arange(l - 1, -1, -1, dtype=np.uint64))
    return (win.astype(np.uint64) * weights).sum(axis=1).astype(np.uint64)


def ball_deltas(l: int, d: int) -> np.ndarray:
    """XOR masks that change between 0 and d of the l base-4 digits (each digit
    change is a nonzero 2-bit XOR, i.e. a move to one of the other 3 bases)."""
    out = [np.zeros(1, dtype=np.uint64)]
    for k in range(1, d + 1):
        for pos in itertools.combinations(range(l), k):
            for digs in itertools.product((1, 2, 3), repeat=k):
                m = 0
                for p, g in zip(pos, digs):
                    m |= g << (2 * (l - 1 - p))
                out.append(np.array([m], dtype=np.uint64))
    return np.concatenate(out)


def ball_intersection(mat: np.ndarray, l: int, d: int) -> np.ndarray:
    """Second algorithm: M = intersection over sequences of the union of the
    distance-d balls around that sequence's windows (the sample-driven form
    named among the exact algorithms in Section I.A)."""
    codes = _codes(mat)
    deltas = ball_deltas(l, d)
    assert deltas.size == ball_size(l, d)
    cur = None
    for i in range(codes.shape[0]):
        w = np.unique(window_numbers(codes[i], l))
        if cur is not None and cur.size * w.size < 40_000_000:
            # Few candidates left: test them directly against this sequence.
            keep = min_dist_numbers(cur, codes[i], l) <= d
            cur = cur[keep]
        else:
            u = np.unique((w[:, None] ^ deltas[None, :]).ravel())
            cur = u if cur is None else np.intersect1d(cur, u, assume_unique=True)
        if cur.size == 0:
            break
    return cur.astype(np.uint32)


def min_dist_numbers(numbers: np.ndarray, row_codes: np.ndarray, l: int) -> np.ndarray:
    """For each candidate number, the smallest distance to a window of one sequence."""
    numbers = np.asarray(numbers, dtype=np.uint64)
    shifts = np.uint64(2) * np.arange(l - 1, -1, -1, dtype=np.uint64)
    digits = ((numbers[:, None] >> shifts[None, :]) & np.uint64(3)).astype(np.uint8)
    win = np.lib.stride_tricks.sliding_window_view(row_codes.astype(np.uint8), l)
    best = np.full(numbers.size, l + 1, dtype=np.int64)
    for c0 in range(0, numbers.size, 4096):
        blk = digits[c0:c0 + 4096]
        dist = (blk[:, None, :] != win[None, :, :]).sum(axis=2)
        best[c0:c0 + 4096] = dist.min(axis=1)
    return best


def verify_sound(mat: np.ndarray, l: int, d: int, numbers: Iterable[int]) -> None:
    """Every reported number is within d of some window of every sequence."""
    numbers = np.asarray(list(numbers), dtype=np.uint64)
    if numbers.size == 0:
        return
    codes = _codes(mat)
    for i in range(codes.shape[0]):
        md = min_dist_numbers(numbers, codes[i], l)
        assert (md <= d).all(), f"reported motif fails sequence {i}"


def relabel(mat: np.ndarray, perm: Sequence[int]) -> np.ndarray:
    lut = np.arange(256, dtype=np.uint8)
    for v, ch in enumerate(BASES):
        lut[ord(ch)] = ord(BASES[perm[v]])
    return lut[mat]


def relabel_number(k: int, l: int, perm: Sequence[int]) -> int:
    out = 0
    for p in range(l):
        dgt = (k >> (2 * (l - 1 - p))) & 3
        out = 4 * out + perm[dgt]
    return out


def reverse_number(k: int, l: int) -> int:
    out = 0
    for p in range(l):
        out = 4 * out + ((k >> (2 * p)) & 3)
    return out


def rows_of(mat: np.ndarray) -> List[str]:
    return [bytes(r).decode() for r in mat]


# ---------------------------------------------------------------------------
# Pins
# ---------------------------------------------------------------------------
def pin_definition_tiny(orc, cases: int = 120, seed: int = 7) -> None:
    """Exhaustive string enumeration on tiny random inputs, every d in [0, l]."""
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        l = int(rng.integers(1, 6))
        n = int(rng.integers(1, 5))
        t = int(rng.integers(l, l + 8))
        mat = fmgen.random_seqs(n, t, int(rng.integers(2 ** 31)))
        rows = rows_of(mat)
        for d in range(0, l + 1):
            want = definition_motifs(rows, l, d)
            for mode in ("brute", "skip"):
                got = orc.solve(mat, l, d, mode=mode, threads=int(rng.integers(1, 4)))
                assert list(got) == want, (mode, l, d, rows)


def pin_skip_visits(orc, cases: int = 40, seed: int = 11) -> None:
    """The enhanced method's sequence-visit count equals a direct count."""
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        l = int(rng.integers(1, 5))
        n = int(rng.integers(1, 5))
        t = int(rng.integers(l, l + 7))
        d = int(rng.integers(0, l + 1))
        mat = fmgen.random_seqs(n, t, int(rng.integers(2 ** 31)))
        _, visits = orc.solve(mat, l, d, mode="skip", threads=2, return_visits=True)
        assert visits == definition_visits(rows_of(mat), l, d)
        _, vb = orc.solve(mat, l, d, mode="brute", threads=2, return_visits=True)
        assert vb == n * 4 ** l


def pin_closed_forms(orc) -> None:
    """d = l keeps every l-mer; one sequence of length l keeps exactly the ball;
    d = 0 keeps the l-mers occurring in every sequence."""
    for l in (1, 2, 4, 6):
        mat = fmgen.random_seqs(3, l + 5, 100 + l)
        got = orc.solve(mat, l, l)
        assert got.size == 4 ** l and (got == np.arange(4 ** l)).all()
    for l in (1, 3, 5, 7, 9):
        mat = fmgen.random_seqs(1, l, 200 + l)
        for d in range(0, l + 1):
            assert orc.solve(mat, l, d).size == ball_size(l, d), (l, d)
    for l in (2, 3, 4):
        mat = fmgen.random_seqs(3, 30, 300 + l)
        rows = rows_of(mat)
        sets = [{r[j:j + l] for j in range(len(r) - l + 1)} for r in rows]
        common = sorted(set.intersection(*sets))
        want = [int("".join(str("ACGT".index(c)) for c in s), 4) for s in common]
        assert list(orc.solve(mat, l, 0)) == want


def pin_edges(orc) -> None:
    """Windows at both ends count, lower case is the same base, and a single
    planted copy at the last offset is found with d = 0."""
    l = 6
    rng = np.random.default_rng(5)
    for off_kind in ("first", "last"):
        mat = fmgen.random_seqs(4, 20, int(rng.integers(2 ** 31)))
        motif = b"GATTCA"
        off = 0 if off_kind == "first" else 20 - l
        mat[:, off:off + l] = np.frombuffer(motif, dtype=np.uint8)
        got = orc.solve(mat, l, 0)
        k = int("".join(str("ACGT".index(c)) for c in motif.decode()), 4)
        assert k in set(got.tolist()), off_kind
        dist = orc.candidate_distances(mat, l, k)
        assert (dist == 0).all()
    mat = fmgen.random_seqs(3, 25, 9)
    lower = np.char.lower(mat.view("S1")).view(np.uint8).reshape(mat.shape)
    assert np.array_equal(orc.solve(mat, 5, 1), orc.solve(lower, 5, 1))


def pin_ball_intersection(orc, shapes=((5, 1, 4, 40), (6, 2, 5, 60), (8, 1, 10, 200),
                                        (7, 2, 6, 80)), seeds=(0, 1)) -> None:
    """The oracle equals an independent second algorithm (intersection of
    Hamming-ball unions) on planted instances."""
    for (l, d, n, t) in shapes:
        for s in seeds:
            inst = fmgen.gen_fm(l, d, n, t, s)
            got = orc.solve(inst.seqs, l, d)
            want = ball_intersection(inst.seqs, l, d)
            assert np.array_equal(got, want), (l, d, n, t, s)


def pin_invariants(orc, seed: int = 3) -> None:
    """Planted consensus reported; soundness; order; monotone in d; reorder,
    duplicate and drop of sequences; base relabelling and reversal."""
    l, d, n, t = 7, 2, 6, 50
    inst = fmgen.gen_fm(l, d, n, t, seed)
    mat = inst.seqs
    got = orc.solve(mat, l, d)
    cons = int("".join(str("ACGT".index(c)) for c in inst.consensus), 4)
    assert cons in set(got.tolist())
    assert (np.diff(got.astype(np.int64)) > 0).all() and (got < 4 ** l).all()
    verify_sound(mat, l, d, got)
    lower = set(orc.solve(mat, l, d - 1).tolist())
    upper = set(orc.solve(mat, l, d + 1).tolist())
    assert lower <= set(got.tolist()) <= upper
    perm_rows = mat[np.random.default_rng(seed).permutation(n)]
    assert np.array_equal(orc.solve(perm_rows, l, d), got)
    dup = np.concatenate([mat, mat[2:3]], axis=0)
    assert np.array_equal(orc.solve(dup, l, d), got)
    drop = orc.solve(mat[:-1], l, d)
    assert set(got.tolist()) <= set(drop.tolist())
    perm = [2, 0, 3, 1]
    rel = orc.solve(relabel(mat, perm), l, d)
    assert sorted(relabel_number(int(k), l, perm) for k in got) == rel.tolist()
    rev = orc.solve(np.ascontiguousarray(mat[:, ::-1]), l, d)
    assert sorted(reverse_number(int(k), l) for k in got) == rev.tolist()


def pin_ranges_and_distances(orc, seed: int = 13) -> None:
    """Index ranges partition the candidate space; per-candidate distances agree
    with a direct numpy computation."""
    inst = fmgen.gen_fm(8, 2, 5, 40, seed)
    whole = orc.solve(inst.seqs, 8, 2, threads=3)
    cuts = [0, 1, 999, 30000, 4 ** 8]
    parts = [orc.solve(inst.seqs, 8, 2, k_range=(a, b), threads=2)
             for a, b in zip(cuts[:-1], cuts[1:])]
    assert np.array_equal(np.concatenate(parts), whole)
    rng = np.random.default_rng(seed)
    codes = _codes(inst.seqs)
    ks = rng.integers(0, 4 ** 8, 64)
    for k in ks:
        dist = orc.candidate_distances(inst.seqs, 8, int(k))
        want = [int(min_dist_numbers(np.array([k]), codes[i], 8)[0]) for i in range(5)]
        assert dist.tolist() == want


ALL_PINS = [pin_definition_tiny, pin_skip_visits, pin_closed_forms, pin_edges,
            pin_ball_intersection, pin_invariants, pin_ranges_and_distances]


# ---------------------------------------------------------------------------
# Rows of their own lengths, N masking and both strands (the oracle's
# ``solve_ex``; the reading of Section VI's real-sequence future work)
# ---------------------------------------------------------------------------
RC = {"A": "T", "C": "G", "G": "C", "T": "A"}


def revcomp(s: str) -> str:
    return "".join(RC[c] for c in reversed(s.upper()))


def definition_window_set(row: str, l: int, mask_n: bool, both: bool) -> List[str]:
    """W_i spelled out: every length-l substring (none holding N when masking),
    plus, for both strands, the reverse complement of each."""
    row = row.upper()
    fwd = [row[j:j + l] for j in range(len(row) - l + 1)]
    if mask_n:
        fwd = [w for w in fwd if "N" not in w]
    return fwd + ([revcomp(w) for w in fwd] if both else [])


def definition_motifs_ex(rows: Sequence[str], l: int, d: int, mask_n: bool, both: bool) -> List[int]:
    sets = [definition_window_set(r, l, mask_n, both) for r in rows]
    out = []
    for k, x in enumerate(itertools.product(BASES, repeat=l)):
        if all(any(sum(a != b for a, b in zip(x, w)) <= d for w in ws) for ws in sets):
            out.append(k)
    return out


def random_rows_ex(rng, n: int, l: int, t_max: int, n_rate: float) -> List[str]:
    """Rows of lengths in [l, t_max] over ACGT (either case) with N at n_rate."""
    rows = []
    for _ in range(n):
        t = int(rng.integers(l, t_max + 1))
        codes = rng.integers(0, 4, t)
        row = "".join("ACGT"[c] if rng.random() > 0.3 else "acgt"[c] for c in codes)
        row = "".join("N" if rng.random() < n_rate else ch for ch in row)
        rows.append(row)
    return rows


def number_of(s: str) -> int:
    return int("".join(str("ACGT".index(c)) for c in s.upper()), 4) if s else 0


def pin_ex_definition_tiny(orc, cases: int = 80, seed: int = 17) -> None:
    """Exhaustive enumeration against the spelled-out window sets: ragged
    lengths, N masking and both strands, every d."""
    rng = np.random.default_rng(seed)
    for case in range(cases):
        l = int(rng.integers(1, 5))
        n = int(rng.integers(1, 5))
        mask_n, both = bool(case & 1), bool(case & 2)
        rows = random_rows_ex(rng, n, l, l + 9, 0.12 if mask_n else 0.0)
        for d in range(0, l + 1):
            want = definition_motifs_ex(rows, l, d, mask_n, both)
            for mode in ("brute", "skip"):
                got = orc.solve_ex(rows, l, d, mask_n=mask_n, both=both, mode=mode,
                                   threads=int(rng.integers(1, 4)))
                assert list(got) == want, (mode, l, d, mask_n, both, rows)


def pin_ex_identities(orc, seed: int = 19) -> None:
    """Identities between the options, each side computed by a different route.

    * both strands on S = N masking on s + "N" + revcomp(s) (a window across
      the junction holds the N);
    * ragged lengths = N masking on rows padded with N to one length;
    * no options, equal lengths = the plain oracle;
    * with both strands M is closed under reverse complement.
    """
    rng = np.random.default_rng(seed)
    for _ in range(12):
        l = int(rng.integers(3, 7))
        d = int(rng.integers(0, 3))
        rows = random_rows_ex(rng, int(rng.integers(2, 5)), l, 40, 0.0)
        both = orc.solve_ex(rows, l, d, both=True)
        glued = [r + "N" + revcomp(r) for r in rows]
        assert list(both) == list(orc.solve_ex(glued, l, d, mask_n=True)), (l, d, rows)
        rc_of = {number_of(revcomp(number_to_string(int(k), l))) for k in both}
        assert rc_of == {int(k) for k in both}, (l, d, rows)
        t_max = max(len(r) for r in rows)
        padded = [r + "N" * (t_max - len(r)) for r in rows]
        assert list(orc.solve_ex(rows, l, d)) == list(orc.solve_ex(padded, l, d, mask_n=True))
        eq = [r[:l + 20].ljust(l + 20, "A") for r in rows]
        mat = np.frombuffer("".join(eq).encode(), dtype=np.uint8).reshape(len(eq), -1)
        assert list(orc.solve_ex(eq, l, d)) == list(orc.solve(mat, l, d))


def number_to_string(k: int, l: int) -> str:
    return "".join(BASES[(k >> (2 * (l - 1 - p))) & 3] for p in range(l))


def pin_ex_closed_forms(orc) -> None:
    """A sequence whose only N-free window is w keeps exactly the ball around
    w (and around revcomp(w) as well, with both strands); a sequence with no
    N-free window empties M; N itself is refused without masking."""
    rng = np.random.default_rng(23)
    for l in (2, 4, 6):
        w = "".join(rng.choice(list(BASES), l))
        row = "NN" + w + "N" + "ACGT"[: max(0, l - 2)]
        for d in range(0, l + 1):
            assert orc.solve_ex([row], l, d, mask_n=True).size == ball_size(l, d), (l, d)
        if w != revcomp(w):
            ball_w = set(definition_motifs_ex([w], l, 1, False, False))
            ball_rc = set(definition_motifs_ex([revcomp(w)], l, 1, False, False))
            got = set(int(k) for k in orc.solve_ex([row], l, 1, mask_n=True, both=True))
            assert got == ball_w | ball_rc, (l, w)
    assert orc.solve_ex(["ACGTACGT", "ACNNNNGT"], 3, 3, mask_n=True).size == 0
    try:
        orc.solve_ex(["ACGTNACG"], 3, 1)
    except ValueError:
        pass
    else:
        raise AssertionError("N accepted without masking")
