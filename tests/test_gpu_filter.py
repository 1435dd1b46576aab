"""The 64-candidate kernel's window filter on the GPU against the oracle,
exactly (motif sets and the enhanced rule's visit counts), with the filter on
and off.

A group batch whose live lanes lie in at most four blocks of 64 consecutive
groups (every fresh stage-0 batch is one block; deeper batches often span
two or three) keeps only the windows within d of some block's shared first
l-6 bases, re-sliced into dense 32-window groups of 12 + 8 x blocks LDS
words each beside a 64-entry list of the windows that pass (at most 22
dense groups for one block); rows of more than 64 window groups, batches
over more blocks, and batches that would need more dense groups than fit
scan every window.  The cases straddle those limits (G = 1, 2, 19, 22/23,
31, 63/64/65 window groups per row), include shapes where most windows pass
(l = 6: no shared base, so every window passes and the table overflows from
23 window groups on) and where almost none pass ((16,2)), and reach deeper
stages.  The filtered batches and dense groups the kernel counts show which
path ran.
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


def solve_both(nat, inst, l, d):
    """(codes, stats) with the filter on, then off."""
    out = []
    for f in (nat.FILTER_ON, nat.FILTER_OFF):
        nat.set_config(filter=f)
        try:
            got = nat.solve(inst.seqs, l, d)
            out.append((got, nat.last_stats()))
        finally:
            nat.set_config(reset=True)
    return out


@pytest.mark.parametrize("l,d,G,ragged", [(10, 1, 1, 0), (10, 1, 2, 5), (11, 3, 19, 3),
                                          (10, 2, 22, 0), (10, 2, 23, 0), (10, 2, 31, 1),
                                          (10, 2, 63, 0), (10, 2, 64, 0), (10, 2, 65, 0)])
def test_filter_window_group_counts(nat, l, d, G, ragged):
    n = 8
    t = 32 * G + l - 1 - ragged
    inst = fmgen.gen_fm(l, d, n, t, 300 + G)
    announce(f"filter ({l},{d}) n={n} t={t} G={G}")
    want, visits = oracle.solve(inst.seqs, l, d, mode="skip", return_visits=True, cap=4 ** l)
    (on, s_on), (off, s_off) = solve_both(nat, inst, l, d)
    for got, st in ((on, s_on), (off, s_off)):
        assert np.array_equal(got, want)
        assert st["seq_visits"] == visits
        assert st["variant"] == nat.VARIANT_GROUP64
    assert s_off["filtered_batches"] == 0
    stage0 = 4 ** l // 4096
    if G <= 64:
        assert s_on["filtered_batches"] >= stage0
        assert s_on["filtered_groups"] <= s_on["filtered_batches"] * G
        if G >= 19:   # most windows fail the shared bases here
            assert s_on["filtered_groups"] < s_on["filtered_batches"] * G // 2
    else:
        assert s_on["filtered_batches"] == 0


@pytest.mark.parametrize("G", [22, 23, 40])
def test_filter_every_window_passes(nat, G):
    """l = 6: no shared base, so every window would pass the filter; it is
    never tried (it only pays when it is expected to drop at least half of
    the windows) and the sets are exact with the filter on and off."""
    l, d, n = 6, 1, 5
    t = 32 * G + l - 1
    inst = fmgen.gen_fm(l, d, n, t, 600 + G)
    announce(f"filter all-pass l=6 G={G}")
    want, visits = oracle.solve(inst.seqs, l, d, mode="skip", return_visits=True, cap=4 ** l)
    (on, s_on), (off, _) = solve_both(nat, inst, l, d)
    assert np.array_equal(on, want) and np.array_equal(off, want)
    assert s_on["seq_visits"] == visits
    assert s_on["filtered_batches"] == 0


@pytest.mark.parametrize("l,d", [(7, 0), (7, 7), (8, 2), (10, 0), (10, 5), (12, 6), (13, 1)])
def test_filter_every_d(nat, l, d):
    """Every d from 0 to l: where the filter is expected to drop most windows
    (small d for the shared bases) it runs, elsewhere it is not tried."""
    inst = fmgen.gen_fm(l, d, 10, 400, 40 * l + d)
    announce(f"filter ({l},{d}) n=10 t=400")
    want, visits = oracle.solve(inst.seqs, l, d, mode="skip", return_visits=True, cap=4 ** l)
    (on, s_on), (off, _) = solve_both(nat, inst, l, d)
    assert np.array_equal(on, want) and np.array_equal(off, want)
    assert s_on["seq_visits"] == visits
    if d == l:
        assert on.size == 4 ** l


@pytest.mark.parametrize("l,d,t", [(16, 2, 600), (16, 3, 600), (15, 4, 600), (14, 4, 600),
                                   (13, 4, 1000), (12, 3, 2000), (13, 4, 1611)])
def test_filter_long_motifs_on_subranges(nat, l, d, t):
    """l = 12..16 at n = 20: filter on equals filter off as whole sets (with
    equal visit counts), and both equal the oracle on sub-ranges around the
    planted consensus and at the ends of the candidate space."""
    inst = fmgen.gen_fm(l, d, 20, t, 900 + l + d)
    announce(f"filter long ({l},{d}) n=20 t={t}")
    (on, s_on), (off, s_off) = solve_both(nat, inst, l, d)
    assert np.array_equal(on, off)
    assert s_on["seq_visits"] == s_off["seq_visits"]
    assert s_on["filtered_batches"] >= 4 ** l // 4096
    cons = oracle.lmer_to_number(inst.consensus)
    assert cons in set(on.tolist())
    for lo in (max(0, cons - (1 << 15)), 0, 4 ** l - (1 << 16)):
        hi = lo + (1 << 16)
        want = oracle.solve(inst.seqs, l, d, k_range=(lo, hi), cap=1 << 16)
        assert np.array_equal(on[(on >= lo) & (on < hi)], want), (l, d, lo)
