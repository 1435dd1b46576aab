"""The 64-candidate kernel's single-candidate scans on the GPU against the
oracle, exactly (motif sets and the enhanced rule's visit counts).

A group whose live members drop to one or two is scanned one candidate per
lane from then on.  The inputs here make that happen in bulk: the first
sequence holds every 5-base prefix at the start of exactly two distinct
8-mer windows (two different de Bruijn sequences of order 5 one after the
other), so after it almost every 64-candidate group of (8, 0) keeps exactly
two members and a single wavefront's queue of singles overflows (those
groups then stay groups).  Other cases reach l = 16 (the widest count) and
64 sequences (deep stages).
"""
import numpy as np
import pytest

import fmgen
import oracle


@pytest.fixture(scope="module")
def nat():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1403_1313_amd import native
    native.set_config(reset=True)
    yield native
    native.set_config(reset=True)


def announce(msg):
    print(f"[case] {msg}", flush=True)


def de_bruijn(k, n):
    """The lexicographically least de Bruijn sequence B(k, n) (the standard
    construction from Lyndon words of length dividing n)."""
    a = [0] * (k * n)
    seq = []

    def db(t, p):
        if t > n:
            if n % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, k):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    return seq


def two_per_prefix_rows():
    b1 = de_bruijn(4, 5)
    b2 = b1[::-1]
    s0 = b1 + b1[:7] + b2 + b2[:7]
    s1 = b2 + b2[:7] + b1 + b1[:7]
    rows = np.array([s0, s1, s0], dtype=np.uint8)
    return np.frombuffer(b"ACGT", dtype=np.uint8)[rows]


def test_two_per_prefix_construction():
    """Most prefixes of the first row start exactly two distinct 8-mers."""
    s0 = two_per_prefix_rows()[0].tobytes().decode()
    per = {}
    for j in range(len(s0) - 7):
        per.setdefault(s0[j:j + 5], set()).add(s0[j:j + 8])
    counts = np.bincount([len(v) for v in per.values()])
    assert len(per) == 4 ** 5 and counts[2] > 900


@pytest.mark.gpu
@pytest.mark.parametrize("d", [0, 1])
def test_singles_queue_overflow(nat, d):
    seqs = two_per_prefix_rows()
    nat.set_config(variant=nat.VARIANT_GROUP64, chunk=16384)
    announce(f"singles overflow (8,{d}) t={seqs.shape[1]}")
    want, visits = oracle.solve(seqs, 8, d, mode="skip", return_visits=True, cap=4 ** 8)
    got = nat.solve(seqs, 8, d)
    st = nat.last_stats()
    nat.set_config(reset=True)
    assert np.array_equal(got, want)
    assert st["seq_visits"] == visits
    if d == 0:
        # Single-candidate scans ran: fewer slots than 64 x 64 per batch.
        # (At d = 1 every group keeps many live members after the first
        # sequence: no group turns sparse.)
        assert st["candidate_slots"] < st["batches"] * 64 * 64
        assert got.size > 1900


@pytest.mark.gpu
@pytest.mark.parametrize("variant", ["group64", "group16", "lane"])
def test_singles_agree_with_other_kernels(nat, variant):
    seqs = two_per_prefix_rows()
    nat.set_config(variant={"lane": nat.VARIANT_LANE, "group16": nat.VARIANT_GROUP,
                            "group64": nat.VARIANT_GROUP64}[variant])
    announce(f"singles cross-check {variant}")
    got = nat.solve(seqs, 8, 1)
    visits = nat.last_stats()["seq_visits"]
    nat.set_config(reset=True)
    ref = oracle.solve(seqs, 8, 1, cap=4 ** 8)
    assert np.array_equal(got, ref)
    _, want_visits = oracle.solve(seqs, 8, 1, mode="skip", return_visits=True, cap=4 ** 8)
    assert visits == want_visits


@pytest.mark.gpu
@pytest.mark.parametrize("d", [1, 2, 3])
def test_singles_l16(nat, d):
    """l = 16: sixteen counted positions per single; exact on an oracle
    sub-range around the planted consensus."""
    inst = fmgen.gen_fm(16, d, 3, 40, 900 + d)
    nat.set_config(variant=nat.VARIANT_GROUP64)
    announce(f"singles l=16 d={d}")
    cons = oracle.lmer_to_number(inst.consensus)
    lo = max(0, cons - (1 << 17))
    hi = lo + (1 << 18)
    want = oracle.solve(inst.seqs, 16, d, k_range=(lo, hi), cap=1 << 18)
    got = nat.solve(inst.seqs, 16, d)
    st = nat.last_stats()
    nat.set_config(reset=True)
    assert cons in set(got.tolist())
    assert np.array_equal(got[(got >= lo) & (got < hi)], want)
    assert st["candidate_slots"] < st["batches"] * 64 * 64


@pytest.mark.gpu
def test_singles_deep_stages(nat):
    """64 sequences of (9, 2): groups and singles reach stages far past the
    ones kept in LDS; whole set and visit count."""
    inst = fmgen.gen_fm(9, 2, 64, 90, 31)
    nat.set_config(variant=nat.VARIANT_GROUP64)
    announce("singles deep stages n=64")
    got = nat.solve(inst.seqs, 9, 2)
    visits = nat.last_stats()["seq_visits"]
    nat.set_config(reset=True)
    want, want_visits = oracle.solve(inst.seqs, 9, 2, mode="skip", return_visits=True, cap=4 ** 9)
    assert np.array_equal(got, want)
    assert visits == want_visits
