"""The 64-candidate kernel's shared-prefix group scans on the GPU against the
oracle, exactly (motif sets and the enhanced rule's visit counts).

A group batch whose live lanes fall into at most 64 / G blocks of 64
consecutive groups (G = groups of 32 windows per row) is scanned with each
block's count over its shared bases done once per window group, and with the
suffix mismatch vectors read from a per-wavefront LDS table of 12 words per
window group; rows of more than 42 window groups take the general scan.
The cases sit on both sides of each boundary of G (21/22: at most three
blocks, then two; 32/33: two, then one; 42/43: the table's limit), reach
stage-1 and deeper batches, and cover l = 6 (no shared base) up to l = 16 and
d = 0 up to d = l.  (Measured once with a device count of these scans, kept
out of the kernel since: at G = 1 every group batch took the path; at
G = 19, 21, 22, 32, 33 and 42, 362, 396, 342, 482, 454 and 512 batches did,
against 64 stage-0 batches; at G = 43 none.)
"""
import numpy as np
import pytest

import fmgen
import oracle

pytestmark = pytest.mark.gpu


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


def stage0_batches(l):
    """Fresh stage-0 batches of one instance: 64 groups of 64 candidates."""
    return max(1, 4 ** l // 4096)


@pytest.mark.parametrize("G,ragged", [(1, 0), (19, 3), (21, 0), (22, 0), (32, 7), (33, 0),
                                      (42, 0), (43, 0)])
def test_shared_window_group_boundaries(nat, G, ragged):
    l, d, n = 9, 2, 8
    t = 32 * G + l - 1 - ragged
    inst = fmgen.gen_fm(l, d, n, t, 100 + G)
    announce(f"shared scan G={G} ({l},{d}) n={n} t={t}")
    want, visits = oracle.solve(inst.seqs, l, d, mode="skip", return_visits=True, cap=4 ** l)
    got = nat.solve(inst.seqs, l, d)
    st = nat.last_stats()
    assert np.array_equal(got, want)
    assert st["seq_visits"] == visits
    assert st["variant"] == nat.VARIANT_GROUP64
    # Deeper stages ran: more batches than the 64 of stage 0.
    assert st["batches"] - st["single_batches"] > stage0_batches(l)


@pytest.mark.parametrize("l,d", [(6, 0), (6, 1), (6, 6), (7, 3), (8, 0), (8, 8), (10, 1)])
def test_shared_small_l_every_d(nat, l, d):
    """l = 6 has no shared base (P - 3 = 0); d = l accepts every candidate."""
    inst = fmgen.gen_fm(l, min(d, l), 6, 300, 7 * l + d)
    announce(f"shared scan ({l},{d}) n=6 t=300")
    want, visits = oracle.solve(inst.seqs, l, d, mode="skip", return_visits=True, cap=4 ** l)
    got = nat.solve(inst.seqs, l, d)
    st = nat.last_stats()
    assert np.array_equal(got, want)
    assert st["seq_visits"] == visits
    if d == l:
        assert got.size == 4 ** l


@pytest.mark.parametrize("d", [0, 3, 5])
def test_shared_l16(nat, d):
    """l = 16 (13 prefix positions, 10 of them shared): exact on oracle
    sub-ranges around the planted consensus and at the two ends of the
    candidate space."""
    l, n, t = 16, 6, 420
    inst = fmgen.gen_fm(l, d, n, t, 500 + d)
    announce(f"shared scan l=16 d={d}")
    got = nat.solve(inst.seqs, l, d)
    assert nat.last_stats()["variant"] == nat.VARIANT_GROUP64
    cons = oracle.lmer_to_number(inst.consensus)
    assert cons in set(got.tolist())
    for lo in (max(0, cons - (1 << 15)), 0, 4 ** l - (1 << 16)):
        hi = lo + (1 << 16)
        want = oracle.solve(inst.seqs, l, d, k_range=(lo, hi), cap=1 << 16)
        assert np.array_equal(got[(got >= lo) & (got < hi)], want), (d, lo)
