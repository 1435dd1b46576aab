"""Batched solves and the continuous-batching server against the oracle.

Integer results: every comparison is exact equality of sorted motif sets.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import fmgen
import oracle

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


def mixed_batch():
    rng = np.random.default_rng(99)
    batch = []
    for q in range(14):
        l = int(rng.integers(5, 10))
        d = int(rng.integers(0, min(3, l) + 1))
        n = int(rng.integers(2, 25))
        t = int(rng.integers(l, 300))
        batch.append((fmgen.gen_fm(l, d, n, t, 500 + q).seqs, l, d))
    batch.append((fmgen.gen_fm(11, 3, 10, 300, 7).seqs, 11, 3))
    batch.append((fmgen.random_seqs(2, 9, 8), 5, 5))        # d = l: every 5-mer
    batch.append((fmgen.random_seqs(1, 12, 9), 12, 2))      # one window: a ball
    return batch


def oracle_sets(batch):
    return [oracle.solve(s, l, d, mode="skip", cap=4 ** l) for s, l, d in batch]


def test_solve_many_matches_oracle_and_solo(nat):
    batch = mixed_batch()
    want = oracle_sets(batch)
    bad = (np.frombuffer(b"ACGTN" * 4, dtype=np.uint8).reshape(1, 20), 4, 1)
    st, got, res = nat.solve_many(batch[:5] + [bad] + batch[5:], capacities=[1 << 16] * (len(batch) + 1))
    assert st == nat.PMS_ERR_INVALID
    assert res[5].status == nat.PMS_ERR_INVALID
    got = got[:5] + got[6:]
    res = res[:5] + res[6:]
    for i, (g, w) in enumerate(zip(got, want)):
        assert res[i].status == nat.PMS_OK and res[i].count == w.size
        assert np.array_equal(g, w), i
        assert np.array_equal(nat.solve(*batch[i]), w)
        assert res[i].latency_ms >= 0


def test_graph_replays_and_eager_agree(nat, monkeypatch):
    batch = mixed_batch()
    st, first, _ = nat.solve_many(batch)
    assert st == nat.PMS_OK
    for _ in range(10):
        st, again, _ = nat.solve_many(batch)
        assert st == nat.PMS_OK
        assert all(np.array_equal(a, b) for a, b in zip(first, again))
    monkeypatch.setenv("PMS_NO_GRAPH", "1")
    st, eager, _ = nat.solve_many(batch)
    assert st == nat.PMS_OK and all(np.array_equal(a, b) for a, b in zip(first, eager))


def test_solve_many_per_instance_overflow(nat):
    batch = mixed_batch()
    want = oracle_sets(batch)
    caps = [1 << 16] * len(batch)
    big = max(range(len(batch)), key=lambda i: want[i].size)
    caps[big] = 3
    st, got, res = nat.solve_many(batch, capacities=caps)
    assert st == nat.PMS_ERR_OVERFLOW
    for i, (g, w) in enumerate(zip(got, want)):
        assert res[i].count == w.size
        if i == big:
            assert res[i].status == nat.PMS_ERR_OVERFLOW and np.array_equal(g, w[:3])
        else:
            assert res[i].status == nat.PMS_OK and np.array_equal(g, w)


def test_solve_many_gather_with_size_queries_and_small_batches(nat):
    """The batch copy-back: more than four instances go through one device
    gather, the others through a copy each; size queries (capacity 0) and
    an overflowing instance sit between instances that return codes, and
    both ways give the oracle's sets."""
    batch = mixed_batch()
    want = oracle_sets(batch)
    caps = [1 << 16] * len(batch)
    caps[1] = caps[6] = 0
    big = max(range(len(batch)), key=lambda i: want[i].size)
    caps[big] = 2
    for sub in (list(range(len(batch))), [0, 1, 2], [big, 6, 3, 4]):
        st, got, res = nat.solve_many([batch[i] for i in sub], capacities=[caps[i] for i in sub])
        for j, i in enumerate(sub):
            assert res[j].count == want[i].size, (sub, i)
            k = min(caps[i], want[i].size)
            assert np.array_equal(got[j], want[i][:k]), (sub, i)
            assert res[j].status == (nat.PMS_ERR_OVERFLOW if want[i].size > caps[i] else nat.PMS_OK)


def test_autotune_cache_and_results(nat, tmp_path):
    path = str(tmp_path / "tune.json")
    inst = fmgen.gen_fm(9, 2, 12, 300, 4)
    want = oracle.solve(inst.seqs, 9, 2)
    try:
        cfg = nat.autotune(12, 300, 9, 2, path)
        assert os.path.exists(path)
        text = open(path).read()
        assert "/l9/d2/n12/" in text and json.loads(text)
        assert nat.get_config() == cfg
        assert np.array_equal(nat.solve(inst.seqs, 9, 2), want)
        nat.set_config(reset=True)
        assert nat.autotune(12, 300, 9, 2, path) == cfg      # served from the cache
    finally:
        nat.set_config(reset=True)


def test_autotune_many_on_the_batch(nat, tmp_path):
    """Tuning on the batch itself: the cache gets the batch's key, the tuned
    configuration gives the oracle's sets, and a second call is served from
    the cache."""
    path = str(tmp_path / "tune_many.json")
    batch = mixed_batch()[:8]
    want = oracle_sets(batch)
    try:
        cfg = nat.autotune_many(batch, path)
        text = open(path).read()
        assert "/batch8/" in text and json.loads(text)
        assert nat.get_config() == cfg
        assert cfg["variant"] in (0, nat.VARIANT_GROUP, nat.VARIANT_GROUP64)
        st, got, _ = nat.solve_many(batch)
        assert st == nat.PMS_OK and all(np.array_equal(g, w) for g, w in zip(got, want))
        nat.set_config(reset=True)
        assert nat.autotune_many(batch, path) == cfg
    finally:
        nat.set_config(reset=True)


def test_batched_workload_matches_golden(nat):
    """The 256-instance batched workload in the benchmark's configuration."""
    path = os.path.join(GOLDEN, "batched.json")
    if not os.path.exists(path):
        pytest.skip("no batched golden yet")
    gold = {r["seed"]: r for r in json.load(open(path))["records"]}
    specs = fmgen.batched_specs(256)
    specs = [s for s in specs if s.seed in gold]
    if not specs:
        pytest.skip("batched golden has no records")
    batch = [(s.make().seqs, s.l, s.d) for s in specs]
    st, got, res = nat.solve_many(batch, capacities=[1 << 21] * len(batch))
    assert st == nat.PMS_OK
    for s, g, r in zip(specs, got, res):
        rec = gold[s.seed]
        assert r.count == rec["count"], s
        assert hashlib.sha256(g.astype("<u4").tobytes()).hexdigest() == rec["sha256"], s


# --------------------------------------------------------------------------
# Serving
# --------------------------------------------------------------------------
def test_serving_results_alone_and_in_the_mix(nat):
    from paper_1403_1313_amd.serve import Server
    batch = mixed_batch()
    want = oracle_sets(batch)
    with Server(mem_budget=64 << 20, step_ms=0.5) as srv:
        alone = [srv.submit(*b).result(timeout=120) for b in batch]
        futs = [srv.submit(*b) for b in batch]
        mixed = [f.result(timeout=120) for f in futs]
        assert srv.stats["steps"] >= 1
    for a, m, w in zip(alone, mixed, want):
        assert np.array_equal(a.motifs, w)
        assert np.array_equal(m.motifs, w)
        assert a.count == m.count == w.size
        assert m.latency_s > 0


def test_serving_tiny_budget_queues_but_completes(nat):
    from paper_1403_1313_amd.serve import Server
    batch = mixed_batch()[:6]
    want = oracle_sets(batch)
    with Server(mem_budget=1, step_ms=0.5) as srv:
        futs = [srv.submit(*b) for b in batch]
        got = [f.result(timeout=120) for f in futs]
        assert srv.stats["admission_waits"] >= 1
    for g, w in zip(got, want):
        assert np.array_equal(g.motifs, w)


def test_serving_overflow_reruns(nat):
    from paper_1403_1313_amd.serve import Server
    batch = mixed_batch()[-3:]
    want = oracle_sets(batch)
    with Server(mem_budget=64 << 20, reserve=1) as srv:
        got = [srv.submit(*b).result(timeout=120) for b in batch]
        assert srv.stats["reruns"] >= 1
    for g, w in zip(got, want):
        assert np.array_equal(g.motifs, w)


def test_serving_rejects_invalid_requests(nat):
    from paper_1403_1313_amd.serve import Server
    with Server() as srv:
        f = srv.submit(np.frombuffer(b"ACGTNACGT", dtype=np.uint8).reshape(1, 9), 4, 1)
        with pytest.raises(nat.PmsError):
            f.result(timeout=10)
        f = srv.submit(fmgen.random_seqs(2, 10, 1), 12, 1)
        with pytest.raises(nat.PmsError):
            f.result(timeout=10)
        ok = srv.submit(fmgen.random_seqs(3, 40, 2), 5, 1).result(timeout=60)
        assert np.array_equal(ok.motifs, oracle.solve(fmgen.random_seqs(3, 40, 2), 5, 1))
        one = srv.submit(fmgen.random_seqs(3, 40, 3), 1, 0).result(timeout=60)
        assert np.array_equal(one.motifs, oracle.solve(fmgen.random_seqs(3, 40, 3), 1, 0))


def test_serving_large_outputs_and_their_order(nat):
    """Outputs larger than the codes copied back with a request's last step
    (d = l at l = 9 and 10: every l-mer; a radius-5 ball of 12-mers) come
    back on the side stream; small requests submitted after them still
    complete, each with its own set."""
    from paper_1403_1313_amd.serve import EAGER_CODES, Server
    big = [(fmgen.random_seqs(2, 12, 70), 9, 9), (fmgen.random_seqs(3, 15, 71), 10, 10),
           (fmgen.random_seqs(1, 12, 72), 12, 5)]
    small = mixed_batch()[:8]
    want_small = oracle_sets(small)
    want_ball = oracle.solve(big[2][0], 12, 5, mode="skip", cap=4 ** 12)
    assert want_ball.size > EAGER_CODES
    with Server(mem_budget=256 << 20, step_ms=0.5) as srv:
        futs = [srv.submit(*b) for b in big] + [srv.submit(*b) for b in small]
        got = [f.result(timeout=120) for f in futs]
    assert np.array_equal(got[0].motifs, np.arange(4 ** 9, dtype=np.uint32))
    assert np.array_equal(got[1].motifs, np.arange(4 ** 10, dtype=np.uint32))
    assert np.array_equal(got[2].motifs, want_ball)
    for g, w in zip(got[3:], want_small):
        assert np.array_equal(g.motifs, w)


def test_serving_burst_of_small_requests(nat):
    """120 requests submitted at once: many share each step, each is exact."""
    from paper_1403_1313_amd.serve import Server
    rng = np.random.default_rng(123)
    batch = []
    for q in range(120):
        l = int(rng.integers(4, 10))
        d = int(rng.integers(0, min(2, l) + 1))
        n = int(rng.integers(2, 9))
        t = int(rng.integers(l, 120))
        batch.append((fmgen.gen_fm(l, d, n, t, 4000 + q).seqs, l, d))
    want = oracle_sets(batch)
    with Server(mem_budget=256 << 20) as srv:
        futs = [srv.submit(*b) for b in batch]
        got = [f.result(timeout=120) for f in futs]
        steps = srv.stats["steps"]
    assert steps < len(batch)
    for i, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g.motifs, w), i
