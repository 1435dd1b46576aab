"""The continuous-batching server at the serving workload's own shapes, against
the oracle's stored results, and its failure handling.

Requests: ``fmgen.serving_check_specs()`` -- the first 13 requests of the
serving stream ((9,2), (11,3), four (13,4)), its two (15,4) requests and a
(13,4) request at n = 10, t = 1000 whose output is about 6e5 motifs.  Each is
compared with ``tests/golden/serving.json`` (oracle, skip mode): motif count,
SHA-256 of the ascending codes and the enhanced rule's visit count, exactly.
They are served one at a time, all at once, at the stream's own arrival
times, and with a small first output reservation (so that the large outputs
take the rerun path); the server's work items are checked to start blocks
of 4096 candidates and to cover each request once, and items moved off
those boundaries still give the oracle's results.  Failure handling is forced from the host: an injected
launch failure, an injected window-build failure, a step whose kernel
reports an instance it could not run (the server is told a too small n
bound), and a step timeout; every kernel still runs to its normal end.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import fmgen
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "serving.json")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1403_1313_amd import native
    from paper_1403_1313_amd import serve
    native.set_config(reset=True)
    return native, serve


@pytest.fixture(scope="module")
def cases():
    if not os.path.exists(GOLDEN):
        pytest.skip("no serving golden")
    gold = {(r["seed"], r["l"], r["d"], r["n"], r["t"]): r
            for r in json.load(open(GOLDEN))["records"]}
    out = []
    for spec in fmgen.serving_check_specs():
        rec = gold[(spec.seed, spec.l, spec.d, spec.n, spec.t)]
        out.append((spec, spec.make(), rec))
    return out


def sha(codes):
    return hashlib.sha256(np.ascontiguousarray(codes, dtype="<u4").tobytes()).hexdigest()


def check(res, rec, what):
    assert res.count == rec["count"], what
    assert res.motifs.size == rec["count"], what
    assert sha(res.motifs) == rec["sha256"], what
    assert res.visits == rec["skip_visits"], what


def announce(msg):
    print(f"[case] {msg}", flush=True)


def test_serving_shapes_one_at_a_time(env, cases):
    nat, serve = env
    with serve.Server() as srv:
        for spec, inst, rec in cases:
            announce(f"alone ({spec.l},{spec.d}) n={spec.n} t={spec.t} count={rec['count']}")
            check(srv.submit(inst.seqs, spec.l, spec.d).result(timeout=120), rec, spec)


def test_serving_shapes_all_at_once(env, cases):
    nat, serve = env
    announce(f"all {len(cases)} at once")
    with serve.Server() as srv:
        futs = [srv.submit(inst.seqs, spec.l, spec.d) for spec, inst, _ in cases]
        for (spec, _, rec), f in zip(cases, futs):
            check(f.result(timeout=300), rec, spec)
        assert srv.stats["steps"] >= 2


def test_serving_shapes_at_stream_arrivals(env, cases):
    """The stream's own inter-arrival gaps (rate 100 req/s), one pass."""
    nat, serve = env
    arrivals = [t for t, _ in fmgen.serving_stream(64, 100.0)]
    times = arrivals[:13] + [arrivals[19], arrivals[31], arrivals[31] + 0.01]
    announce("stream arrivals")
    with serve.Server() as srv:
        t0 = time.perf_counter()
        futs = []
        for (spec, inst, _), ta in zip(cases, times):
            wait = ta - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            futs.append(srv.submit(inst.seqs, spec.l, spec.d))
        for (spec, _, rec), f in zip(cases, futs):
            check(f.result(timeout=300), rec, spec)


def test_serving_shapes_rerun_path(env, cases):
    """First reservation of 1000 codes: every request with more motifs is
    re-run with its exact count (the 6e5-motif request among them)."""
    nat, serve = env
    announce("reserve 1000")
    with serve.Server(reserve=1000) as srv:
        futs = [srv.submit(inst.seqs, spec.l, spec.d) for spec, inst, _ in cases]
        for (spec, _, rec), f in zip(cases, futs):
            res = f.result(timeout=300)
            check(res, rec, spec)
            assert res.reruns == (1 if rec["count"] > 1000 else 0)
        assert srv.stats["reruns"] == sum(rec["count"] > 1000 for _, _, rec in cases)


def test_work_items_start_blocks_and_cover_each_request_once(env, cases, monkeypatch):
    """Every work item the server writes starts a block of 4096 candidates
    and holds whole blocks (the window filter's single-block batches depend
    on it; the last item of a request may end at 4^l), and each request's
    items, over all its steps, cover [0, 4^l) exactly once; the requests are
    submitted together, so steps hold several of them, and each result equals
    the oracle's."""
    nat, serve = env
    calls = []
    real = serve.nat.fill_work_items

    def record(begin, count, item_len, inst, out, max_items):
        k = real(begin, count, item_len, inst, out, max_items)
        if k > 0:
            calls.append((inst, begin, min(count, k * item_len), item_len))
        return k

    monkeypatch.setattr(serve.nat, "fill_work_items", record)
    announce("work item layout, all requests at once")
    with serve.Server() as srv:
        futs = [srv.submit(inst.seqs, spec.l, spec.d) for spec, inst, _ in cases]
        for (spec, _, rec), f in zip(cases, futs):
            check(f.result(timeout=300), rec, spec)
        assert srv.stats["reruns"] == 0
    # A request's items come in ascending order on its slot; a slot taken
    # over by a later request starts again at 0.
    at, ends = {}, []
    for slot, begin, covered, item_len in calls:
        assert begin % 4096 == 0 and item_len % 4096 == 0, (slot, begin, item_len)
        if begin == 0 and at.get(slot, 0) != 0:
            ends.append(at[slot])
        assert begin == at.get(slot, 0) or begin == 0, (slot, begin, at.get(slot))   # no gap, no overlap
        at[slot] = begin + covered
    ends += list(at.values())
    assert sorted(ends) == sorted(4 ** spec.l for spec, _, _ in cases)


def test_unaligned_work_items_match_oracle(env, cases, monkeypatch):
    """Work items that do not start on blocks of 4096 candidates: each call's
    interior item boundaries are moved by 17 groups of 64 candidates (the
    items still cover the same range, once), so stage-0 batches straddle
    two blocks and take the window filter's block count instead of its
    single-block path; every result still equals the oracle's."""
    import ctypes
    nat, serve = env
    real = serve.nat.fill_work_items
    shift = 17 * 64
    moved = []

    def unaligned(begin, count, item_len, inst, out, max_items):
        k = real(begin, count, item_len, inst, out, max_items)
        if k >= 2:
            recs = (nat.WorkItem * k).from_address(out)
            end = recs[k - 1].begin + recs[k - 1].len
            if recs[k - 1].len > shift:
                for i in range(1, k):
                    recs[i].begin += shift
                for i in range(k - 1):
                    recs[i].len = recs[i + 1].begin - recs[i].begin
                recs[k - 1].len = end - recs[k - 1].begin
                assert recs[0].begin == begin and recs[k - 1].begin + recs[k - 1].len == end
                moved.append(k)
        return k

    monkeypatch.setattr(serve.nat, "fill_work_items", unaligned)
    announce("unaligned work items, all requests at once")
    with serve.Server() as srv:
        futs = [srv.submit(inst.seqs, spec.l, spec.d) for spec, inst, _ in cases]
        for (spec, _, rec), f in zip(cases, futs):
            check(f.result(timeout=300), rec, spec)
    assert moved


def small_cases():
    """A few quick requests with oracle results computed here."""
    out = []
    for q, (l, d, n, t) in enumerate([(9, 2, 12, 300), (8, 1, 10, 200), (10, 2, 15, 400)]):
        inst = fmgen.gen_fm(l, d, n, t, 2000 + q)
        want, visits = oracle.solve(inst.seqs, l, d, mode="skip", return_visits=True, cap=4 ** l)
        out.append((inst, l, d, want, visits))
    return out


def test_injected_step_failure_fails_only_its_requests(env, monkeypatch):
    nat, serve = env
    quick = small_cases()
    with serve.Server() as srv:
        inst, l, d, want, visits = quick[0]
        assert np.array_equal(srv.submit(inst.seqs, l, d).result(timeout=60).motifs, want)
        announce("step launch fails once")
        monkeypatch.setenv("PMS_TEST_FAIL_NEXT", f"{nat.PMS_ERR_DEVICE}:pms_step_launch")
        inst, l, d, _, _ = quick[1]
        f = srv.submit(inst.seqs, l, d)
        with pytest.raises(nat.PmsError) as e:
            f.result(timeout=60)
        assert e.value.status == nat.PMS_ERR_DEVICE
        assert srv.stats["failed_steps"] == 1
        monkeypatch.delenv("PMS_TEST_FAIL_NEXT")
        for inst, l, d, want, visits in quick:
            res = srv.submit(inst.seqs, l, d).result(timeout=60)
            assert np.array_equal(res.motifs, want) and res.visits == visits
        assert srv.error is None


def test_injected_window_build_failure(env, monkeypatch):
    nat, serve = env
    quick = small_cases()
    with serve.Server() as srv:
        announce("window build fails once")
        monkeypatch.setenv("PMS_TEST_FAIL_NEXT", f"{nat.PMS_ERR_NOMEM}:pms_build_windows")
        inst, l, d, _, _ = quick[0]
        with pytest.raises(nat.PmsError) as e:
            srv.submit(inst.seqs, l, d).result(timeout=60)
        assert e.value.status == nat.PMS_ERR_NOMEM
        monkeypatch.delenv("PMS_TEST_FAIL_NEXT")
        futs = [srv.submit(inst.seqs, l, d) for inst, l, d, _, _ in quick]
        for f, (_, _, _, want, _) in zip(futs, quick):
            assert np.array_equal(f.result(timeout=60).motifs, want)
        assert srv.stats["failed_admissions"] == 1 and srv.mem_used == 0


def test_kernel_error_flag_fails_the_step(env):
    """The first step is launched with an n bound of 1, so the kernel skips
    its instances and raises the counters' error flag; those requests fail,
    the server goes on and later requests are exact."""
    nat, serve = env
    quick = small_cases()

    class Once(serve.Server):
        bad = True

        def _launch_max_n(self, reqs):
            if self.bad:
                self.bad = False
                return 1
            return super()._launch_max_n(reqs)

    with Once() as srv:
        announce("error flag")
        inst, l, d, _, _ = quick[2]
        with pytest.raises(nat.PmsError) as e:
            srv.submit(inst.seqs, l, d).result(timeout=60)
        assert e.value.status == nat.PMS_ERR_DEVICE
        for inst, l, d, want, visits in quick:
            res = srv.submit(inst.seqs, l, d).result(timeout=60)
            assert np.array_equal(res.motifs, want) and res.visits == visits
        assert srv.stats["failed_steps"] == 1 and srv.mem_used == 0


def test_step_timeout_stops_the_server(env, cases):
    """A step timeout of zero: the first wait for a (15,4) step expires
    (the kernel itself runs to its end); every pending request fails with
    StepTimeout and the server refuses new work."""
    nat, serve = env
    spec, inst, _ = next(c for c in cases if c[0].l == 15)
    announce("step timeout")
    srv = serve.Server(step_timeout_s=0.0)
    try:
        f = srv.submit(inst.seqs, spec.l, spec.d)
        with pytest.raises(serve.StepTimeout):
            f.result(timeout=60)
        srv.thread.join(timeout=60)
        assert not srv.thread.is_alive()
        with pytest.raises(RuntimeError):
            srv.submit(inst.seqs, spec.l, spec.d)
    finally:
        srv.close()
        import torch
        torch.cuda.synchronize()


def test_variant_config(env):
    """AUTO with an l = 2 request runs the 16-candidate kernel on the
    bit-sliced tables; the per-lane kernel cannot read them and is refused."""
    nat, serve = env
    inst = fmgen.gen_fm(2, 1, 4, 30, 77)
    want = oracle.solve(inst.seqs, 2, 1, mode="skip", cap=16)
    with serve.Server(config={"variant": nat.VARIANT_AUTO}) as srv:
        assert np.array_equal(srv.submit(inst.seqs, 2, 1).result(timeout=60).motifs, want)
    with serve.Server(config={"variant": nat.VARIANT_GROUP64}) as srv:
        assert np.array_equal(srv.submit(inst.seqs, 2, 1).result(timeout=60).motifs, want)
    with pytest.raises(ValueError):
        serve.Server(config={"variant": nat.VARIANT_LANE})
