"""GPU path (through the C ABI) against the CPU oracle, element by element.

Integer work, so the bar is exact equality of the sorted motif sets and of
the enhanced rule's sequence-visit count.  Stored sets come from the oracle
(tests/golden/); everything else is recomputed by the oracle here.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import fmgen
import oracle
import _pins

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def nat():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1403_1313_amd import native
    native.set_config(reset=True)
    return native


def gpu_solve(nat, seqs, l, d):
    """Motif codes from the GPU (sorted by the library) and the launch stats."""
    res = nat.solve(seqs, l, d)
    return res, nat.last_stats()


@pytest.fixture(params=["lane", "group16", "group64"])
def variant(request, nat):
    """Runs a test once per search kernel variant."""
    v = {"lane": nat.VARIANT_LANE, "group16": nat.VARIANT_GROUP,
         "group64": nat.VARIANT_GROUP64}[request.param]
    nat.set_config(variant=v)
    yield v
    nat.set_config(reset=True)


def records(cfg):
    path = os.path.join(GOLDEN, f"{cfg}.json")
    if not os.path.exists(path):
        pytest.skip(f"missing {path}")
    with open(path) as f:
        return json.load(f)["records"]


def announce(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.parametrize("cfg", ["plain_8_1", "plain_11_3", "plain_15_4"])
def test_plain_configs_match_golden(nat, variant, cfg):
    for r in records(cfg):
        announce(f"{cfg} seed={r['seed']}")
        inst = fmgen.gen_fm(r["l"], r["d"], r["n"], r["t"], r["seed"])
        got, st = gpu_solve(nat, inst.seqs, r["l"], r["d"])
        assert got.size == r["count"]
        assert hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == r["sha256"]
        assert [nat.decode(int(k), r["l"]) for k in got] == r["motifs"]
        assert st["seq_visits"] == r["skip_visits"]
        assert st["window_compares"] == r["skip_visits"] * (r["t"] - r["l"] + 1)
        assert st["variant"] == variant


def test_plain_15_4_sampled_candidates(nat):
    """Full (15,4) launch; 512 sampled candidates checked one by one by the oracle."""
    inst = fmgen.gen_fm(15, 4, 20, 600, 0)
    got, _ = gpu_solve(nat, inst.seqs, 15, 4)
    members = set(got.tolist())
    rng = np.random.default_rng(1513)
    cons = oracle.lmer_to_number(inst.consensus)
    # random candidates plus near neighbours of the consensus (likely to go deep)
    picks = list(rng.integers(0, 4 ** 15, 256))
    for _ in range(256):
        k = cons
        for p in rng.choice(15, 3, replace=False):
            k ^= int(rng.integers(1, 4)) << (2 * int(p))
        picks.append(k)
    for k in picks:
        want = oracle.is_motif(inst.seqs, 15, 4, int(k))
        assert (int(k) in members) == want, k
    for k in got:
        assert oracle.is_motif(inst.seqs, 15, 4, int(k))


def test_random_small_instances(nat, variant):
    """l <= 8 over every d regime, ragged window counts, n up to 30."""
    rng = np.random.default_rng(2024)
    for case in range(60):
        l = int(rng.integers(1, 9))
        d = int(rng.integers(0, min(l, 4) + 1)) if rng.random() < 0.8 else l
        n = int(rng.integers(1, 31))
        t = int(rng.integers(l, 140))
        seed = int(rng.integers(2 ** 31))
        announce(f"small #{case} l={l} d={d} n={n} t={t} seed={seed}")
        if rng.random() < 0.5 and d <= l:
            seqs = fmgen.gen_fm(l, d, n, t, seed).seqs
        else:
            seqs = fmgen.random_seqs(n, t, seed)
        want, visits = oracle.solve(seqs, l, d, mode="skip", return_visits=True, cap=4 ** l)
        got, st = gpu_solve(nat, seqs, l, d)
        assert np.array_equal(got, want), (l, d, n, t, seed)
        assert st["seq_visits"] == visits


def test_random_large_l_sampled(nat, variant):
    """l in [10, 16]: exact comparison on an oracle sub-range of candidates,
    soundness of every motif, and the planted consensus."""
    rng = np.random.default_rng(77)
    for case in range(10):
        l = int(rng.integers(10, 17))
        d = int(rng.integers(max(0, l // 4 - 1), l // 4 + 2))
        n = int(rng.integers(2, 12))
        t = int(rng.integers(l, 160))
        seed = int(rng.integers(2 ** 31))
        announce(f"large #{case} l={l} d={d} n={n} t={t} seed={seed}")
        inst = fmgen.gen_fm(l, d, n, t, seed)
        got, _ = gpu_solve(nat, inst.seqs, l, d)
        assert oracle.lmer_to_number(inst.consensus) in set(got.tolist())
        assert (np.diff(got.astype(np.int64)) > 0).all()
        for k in got[:200]:
            assert oracle.is_motif(inst.seqs, l, d, int(k))
        lo = int(rng.integers(0, 4 ** l - (1 << 18)))
        want = oracle.solve(inst.seqs, l, d, k_range=(lo, lo + (1 << 18)))
        inside = got[(got >= lo) & (got < lo + (1 << 18))]
        assert np.array_equal(inside, want)


@pytest.mark.parametrize("l,d,n,t", [(1, 0, 3, 5), (1, 1, 2, 1), (4, 0, 1, 4), (6, 2, 1, 6),
                                     (16, 0, 2, 16), (16, 2, 1, 16), (5, 5, 3, 9), (7, 7, 2, 7),
                                     (8, 1, 64, 60), (9, 2, 64, 17), (12, 3, 3, 12)])
def test_edge_shapes(nat, variant, l, d, n, t):
    announce(f"edge l={l} d={d} n={n} t={t}")
    seqs = fmgen.random_seqs(n, t, 1000 * l + 10 * d + n)
    got, _ = gpu_solve(nat, seqs, l, d)
    if l <= 12:
        want = oracle.solve(seqs, l, d, cap=4 ** l)
        assert np.array_equal(got, want)
    if n == 1 and t == l:
        assert got.size == _pins.ball_size(l, d)
    if d == l:
        assert got.size == 4 ** l
    for k in got[:100]:
        assert oracle.is_motif(seqs, l, d, int(k))


def test_window_count_ragged_tail(nat, variant):
    """Window counts around the 16- and 32-window scan groups: nw = 1..70."""
    for nw in range(1, 71):
        l, d, n = 7, 1, 4
        t = l + nw - 1
        seqs = fmgen.random_seqs(n, t, 500 + nw)
        # plant the same 7-mer at the last window of every row
        seqs[:, t - l:] = np.frombuffer(b"GATTACA", dtype=np.uint8)
        got, _ = gpu_solve(nat, seqs, l, d)
        want = oracle.solve(seqs, l, d)
        assert np.array_equal(got, want), nw
        assert oracle.lmer_to_number("GATTACA") in set(got.tolist())


def test_lower_case_is_the_same(nat):
    inst = fmgen.gen_fm(8, 1, 10, 200, 3)
    lower = np.char.lower(inst.seqs.view("S1")).view(np.uint8).reshape(inst.seqs.shape)
    a, _ = gpu_solve(nat, inst.seqs, 8, 1)
    b, _ = gpu_solve(nat, lower, 8, 1)
    assert np.array_equal(a, b)


def test_capacity_overflow_semantics(nat):
    seqs = fmgen.random_seqs(3, 40, 11)
    want = oracle.solve(seqs, 6, 2)
    assert want.size > 20
    st, cnt, res = nat.solve_raw(seqs, 6, 2, capacity=20)
    assert st == nat.PMS_ERR_OVERFLOW and cnt == want.size
    assert np.array_equal(res, want[:20])
    st, cnt, res = nat.solve_raw(seqs, 6, 2, capacity=0)
    assert st == nat.PMS_ERR_OVERFLOW and cnt == want.size and res.size == 0
    st, cnt, res = nat.solve_raw(seqs, 6, 2, capacity=want.size)
    assert st == nat.PMS_OK and np.array_equal(res, want)


def test_device_output_rerun(nat, monkeypatch):
    """A device reservation smaller than |M| triggers one exact rerun."""
    monkeypatch.setenv("PMS_TEST_DEVICE_CAP", "5")
    seqs = fmgen.random_seqs(3, 60, 12)
    want = oracle.solve(seqs, 7, 2)
    assert want.size > 5
    got, st = gpu_solve(nat, seqs, 7, 2)
    assert np.array_equal(got, want)
    assert st["reruns"] == 1


def test_launch_configurations_agree(nat):
    """Every chunk / workgroup shape / tail split gives the same set and visits."""
    inst = fmgen.gen_fm(11, 3, 20, 600, 0)
    want = oracle.solve(inst.seqs, 11, 3, mode="skip", return_visits=True)
    try:
        for var in (nat.VARIANT_LANE, nat.VARIANT_GROUP, nat.VARIANT_GROUP64):
            for chunk in (64, 1024, 16384, 1 << 16):
                for waves in (1, 2, 4, 8, 16):
                    for tail in (0, 8, 64):
                        announce(f"config variant={var} chunk={chunk} waves={waves} tail={tail}")
                        nat.set_config(chunk=chunk, wg_waves=waves, tail_split=tail, variant=var)
                        got, st = gpu_solve(nat, inst.seqs, 11, 3)
                        assert np.array_equal(got, want[0])
                        assert st["seq_visits"] == want[1]
                        assert st["variant"] == var
    finally:
        nat.set_config(reset=True)


def test_solve_dev_through_torch(nat):
    import torch
    inst = fmgen.gen_fm(11, 3, 20, 600, 1)
    want, visits = oracle.solve(inst.seqs, 11, 3, mode="skip", return_visits=True)
    dev_seqs = torch.from_numpy(inst.seqs.reshape(-1).copy()).cuda()
    out = torch.zeros(1024, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        nat.solve_dev(dev_seqs, 20, 600, 11, 3, out, 1024, cnt, stream=stream)
    stream.synchronize()
    k = int(cnt.item())
    codes = np.sort(out[:k].cpu().numpy().view(np.uint32))
    assert np.array_equal(codes, want)
    st = nat.last_stats()
    assert st["seq_visits"] == visits and st["kernel_ms"] > 0
    # One instance is cut into about 8 items per resident wavefront, never
    # under 4096 candidates: 4^11 candidates fill only 1024 such items.
    assert st["work_items"] == 4 ** 11 // 4096


def _reference_windows(seqs, l, layout):
    """The documented window-table layouts, written out in Python."""
    codes = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}
    n, t = seqs.shape
    nw = t - l + 1
    rows = []
    for i in range(n):
        base = [codes[int(x)] for x in seqs[i]]
        if layout == 0:
            stride = (nw + 15) // 16 * 16
            row = []
            for j in range(stride):
                jj = j if j < nw else 0
                hi = lo = 0
                for p in range(l):
                    b = base[jj + p]
                    hi |= (b >> 1) << (l - 1 - p)
                    lo |= (b & 1) << (l - 1 - p)
                row.append((hi << 16) | lo)
        else:
            groups = (nw + 31) // 32
            row = []
            for g in range(groups):
                words = [0] * (2 * l)
                for j in range(32):
                    w = 32 * g + j
                    w = w if w < nw else 0
                    for p in range(l):
                        b = base[w + p]
                        words[p] |= (b >> 1) << j
                        words[l + p] |= (b & 1) << j
                row.extend(words)
        rows.append(row)
    return np.array(rows, dtype=np.uint64).astype(np.uint32)


@pytest.mark.parametrize("layout", [0, 1])
def test_build_windows_layout(nat, layout):
    """Windows written by the device equal the documented layouts."""
    import torch
    seqs = fmgen.random_seqs(3, 77, 5)
    l = 9
    stride = nat.window_stride(77, l, layout)
    dev = torch.from_numpy(seqs.reshape(-1).copy()).cuda()
    win = torch.zeros(3 * stride, dtype=torch.int32, device="cuda")
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    nat.build_windows(dev, 3, 77, l, win, bad, layout=layout)
    torch.cuda.synchronize()
    got = win.cpu().numpy().view(np.uint32).reshape(3, stride)
    assert np.array_equal(got, _reference_windows(seqs, l, layout))
    assert int(bad.item()) == 0
    seqs[1, 4] = ord("N")
    dev = torch.from_numpy(seqs.reshape(-1).copy()).cuda()
    nat.build_windows(dev, 3, 77, l, win, bad, layout=layout)
    torch.cuda.synchronize()
    assert int(bad.item()) == 1
