"""pms_solve_ex (rows of their own lengths, N masking, both strands) on the
GPU against the oracle's solve_ex, exactly, for every search kernel variant.

The options are the reading of the real-sequence future work of Section VI;
the oracle spells out each sequence's window set and is pinned in
test_oracle_ex.py.
"""
import numpy as np
import pytest

import fmgen
import oracle
import _pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1403_1313_amd import native
    native.set_config(reset=True)
    return native


@pytest.fixture(params=["lane", "group16", "group64"])
def variant(request, nat):
    v = {"lane": nat.VARIANT_LANE, "group16": nat.VARIANT_GROUP,
         "group64": nat.VARIANT_GROUP64}[request.param]
    nat.set_config(variant=v)
    yield v
    nat.set_config(reset=True)


def announce(msg):
    print(f"[case] {msg}", flush=True)


def fm_rows(rng, n, l, d, t_lo, t_hi, n_rate):
    """A planted FM instance with rows of their own lengths and scattered N
    outside the planted copy (so the consensus stays a motif)."""
    cons = rng.integers(0, 4, l)
    rows = []
    for _ in range(n):
        t = int(rng.integers(t_lo, t_hi + 1))
        row = rng.integers(0, 4, t)
        inst = cons.copy()
        pos = rng.choice(l, d, replace=False)
        inst[pos] = (inst[pos] + rng.integers(1, 4, d)) % 4
        off = int(rng.integers(0, t - l + 1))
        row[off:off + l] = inst
        s = ["ACGT"[c] for c in row]
        for j in range(t):
            if not (off <= j < off + l) and rng.random() < n_rate:
                s[j] = "N"
        rows.append("".join(s))
    return rows, "".join("ACGT"[c] for c in cons)


@pytest.mark.parametrize("mask_n,both", [(False, False), (True, False), (False, True), (True, True)])
def test_ex_random_small(nat, variant, mask_n, both):
    """l <= 8: whole sets, every option, ragged lengths around the 16- and
    32-window groups."""
    rng = np.random.default_rng(41 + 2 * mask_n + both)
    for case in range(12):
        l = int(rng.integers(1, 9))
        d = int(rng.integers(0, min(l, 3) + 1))
        n = int(rng.integers(1, 9))
        rows = _pins.random_rows_ex(rng, n, l, l + int(rng.integers(1, 90)), 0.05 if mask_n else 0.0)
        announce(f"ex small v={variant} mask={mask_n} both={both} l={l} d={d} n={n} "
                 f"lens={[len(r) for r in rows]}")
        want = oracle.solve_ex(rows, l, d, mask_n=mask_n, both=both)
        got = nat.solve_ex(rows, l, d, mask_n=mask_n, both=both)
        assert np.array_equal(got, want), (l, d, rows)


@pytest.mark.parametrize("mask_n,both", [(True, False), (False, True), (True, True)])
def test_ex_planted_larger(nat, variant, mask_n, both):
    """(11,3) planted, n = 12, lengths 300-700 with N: the whole set against a
    sub-range swept by the oracle plus the planted consensus, and every
    reported motif re-checked by the oracle's window sets."""
    rng = np.random.default_rng(97 + 2 * mask_n + both)
    l, d = 11, 3
    rows, cons = fm_rows(rng, 12, l, d, 300, 700, 0.02 if mask_n else 0.0)
    announce(f"ex planted v={variant} mask={mask_n} both={both} lens={[len(r) for r in rows]}")
    got = nat.solve_ex(rows, l, d, mask_n=mask_n, both=both)
    assert _pins.number_of(cons) in set(int(k) for k in got)
    lo, hi = 0x1A0000, 0x1A0000 + (1 << 15)
    want = oracle.solve_ex(rows, l, d, mask_n=mask_n, both=both, k_range=(lo, hi))
    sub = got[(got >= lo) & (got < hi)]
    assert np.array_equal(sub, want)
    sets = [_pins.definition_window_set(r, l, mask_n, both) for r in rows]
    for k in got[:200]:
        x = _pins.number_to_string(int(k), l)
        assert all(any(sum(a != b for a, b in zip(x, w)) <= d for w in ws) for ws in sets), x


def test_ex_long_rows_both_strands(nat, variant):
    """Rows up to 3000 bases on both strands (up to 188 window groups of 32)
    and one short row: whole set at l = 7."""
    rng = np.random.default_rng(5)
    rows = _pins.random_rows_ex(rng, 5, 7, 3000, 0.01)
    rows.append("ACGTTGCA")
    announce(f"ex long v={variant} lens={[len(r) for r in rows]}")
    want = oracle.solve_ex(rows, 7, 2, mask_n=True, both=True)
    got = nat.solve_ex(rows, 7, 2, mask_n=True, both=True)
    assert np.array_equal(got, want)


def test_ex_without_options_equals_plain(nat, variant):
    """Equal lengths and no options: pms_solve_ex == pms_solve."""
    inst = fmgen.gen_fm(10, 2, 12, 400, 3)
    rows = [bytes(r) for r in inst.seqs]
    announce(f"ex plain v={variant}")
    assert np.array_equal(nat.solve_ex(rows, 10, 2), nat.solve(inst.seqs, 10, 2))


def test_ex_both_strands_closed_under_revcomp(nat):
    """With both strands the GPU's set is closed under reverse complement."""
    rng = np.random.default_rng(8)
    rows = _pins.random_rows_ex(rng, 6, 9, 300, 0.0)
    announce("ex revcomp closure")
    got = set(int(k) for k in nat.solve_ex(rows, 9, 2, both=True))
    rc = {_pins.number_of(_pins.revcomp(_pins.number_to_string(k, 9))) for k in got}
    assert got == rc and got
