"""The API's limits on the GPU: rows of PMS_MAX_T bases, and l = 16 with
d = l, where |M| = 4^16 = 2^32 does not fit 32 bits (a size query)."""
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


@pytest.fixture(scope="module")
def longest():
    """(9,1) planted in 3 rows of PMS_MAX_T bases, and the oracle's answer on
    the 4096 candidates starting at the consensus's block."""
    inst = fmgen.gen_fm(9, 1, 3, 1 << 17, 21)
    cons = oracle.lmer_to_number(inst.consensus)
    lo = cons // 4096 * 4096
    want = oracle.solve(inst.seqs, 9, 1, k_range=(lo, lo + 4096))
    return inst, lo, want


def test_rows_of_max_length(nat, variant, longest):
    inst, lo, want = longest
    assert inst.t == nat.PMS_MAX_T
    announce(f"max t v={variant}")
    got = nat.solve(inst.seqs, 9, 1)
    assert np.array_equal(got[(got >= lo) & (got < lo + 4096)], want)
    assert oracle.lmer_to_number(inst.consensus) in set(got.tolist())
    for k in got[:40]:
        assert oracle.is_motif(inst.seqs, 9, 1, int(k))


def test_ex_rows_of_max_length_both_strands(nat):
    """pms_solve_ex with a PMS_MAX_T row on both strands (twice the window
    slots of any plain row) and N masking."""
    rng = np.random.default_rng(33)
    rows = _pins.random_rows_ex(rng, 2, 9, 200, 0.0)
    long = "".join("ACGT"[c] for c in rng.integers(0, 4, 1 << 17))
    long = long[:5000] + "N" * 30 + long[5030:]
    rows.append(long)
    announce("max t ex both strands")
    got = nat.solve_ex(rows, 9, 1, mask_n=True, both=True)
    lo = 0x1B000
    want = oracle.solve_ex(rows, 9, 1, mask_n=True, both=True, k_range=(lo, lo + 4096))
    assert np.array_equal(got[(got >= lo) & (got < lo + 4096)], want)


def test_size_query_l16_d16(nat):
    """d = l keeps all 4^16 l-mers: a size query (capacity 0) returns the
    exact count 2^32 and writes nothing."""
    seqs = fmgen.random_seqs(2, 20, 77)
    announce("size query (16,16)")
    st, cnt, res = nat.solve_raw(seqs, 16, 16, capacity=0)
    assert st == nat.PMS_ERR_OVERFLOW and cnt == 4 ** 16 and res.size == 0
    assert nat.last_stats()["seq_visits"] == 2 * 4 ** 16


def test_size_query_matches_full_count(nat):
    """Capacity 0 and a full solve agree on |M| (the size query skips the
    codes, not the search)."""
    inst = fmgen.gen_fm(11, 3, 20, 600, 4)
    full = nat.solve(inst.seqs, 11, 3)
    st, cnt, _ = nat.solve_raw(inst.seqs, 11, 3, capacity=0)
    assert cnt == full.size and st == (nat.PMS_ERR_OVERFLOW if full.size else nat.PMS_OK)
