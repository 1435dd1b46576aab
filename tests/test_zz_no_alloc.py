"""pms_solve_dev_noalloc (the entry point for callers that cannot allocate)
against pms_solve_dev on the same device inputs, through the C ABI.

Integer work: counts and sorted motif sets must be equal.  Two calls in a
row share the library's fixed scratch, the second with a smaller instance, so
whatever the first left there must not leak into the second.  The stored
oracle sets of the plain configs are checked as well.
"""
import json
import os

import numpy as np
import pytest

import fmgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1403_1313_amd import native
    native.set_config(reset=True)
    return native, torch


def golden_motifs(cfg, seed):
    with open(os.path.join(GOLDEN, f"{cfg}.json")) as f:
        for r in json.load(f)["records"]:
            if r["seed"] == seed:
                return r["motifs"]
    raise KeyError((cfg, seed))


def run(env, fn, inst, cap=1 << 16):
    """(count, sorted codes) of one device-level call on torch's stream."""
    nat, torch = env
    dev = torch.device("cuda:0")
    seqs = torch.from_numpy(inst.seqs.reshape(-1).copy()).to(dev)
    out = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    cnt = torch.full((1,), -1, dtype=torch.int64, device=dev)
    print(f"[case] {fn.__name__} l={inst.l} d={inst.d} n={inst.n} t={inst.t} seed={inst.seed}",
          flush=True)
    fn(seqs, inst.n, inst.t, inst.l, inst.d, out, cap, cnt)
    torch.cuda.synchronize()
    k = int(cnt.item())
    codes = np.sort(out[:min(k, cap)].cpu().numpy().view(np.uint32))
    return k, codes


def check_pair(env, inst, cfg=None):
    nat = env[0]
    k_ref, ref = run(env, nat.solve_dev, inst)
    k_na, got = run(env, nat.solve_dev_noalloc, inst)
    assert k_na == k_ref
    assert np.array_equal(got, ref)
    if cfg:
        assert [nat.decode(int(c), inst.l) for c in got] == golden_motifs(cfg, inst.seed)
    return got


def test_noalloc_equals_solve_dev_two_calls(env):
    """A larger instance, then a smaller one, each against pms_solve_dev."""
    big = fmgen.gen_fm(seed=0, **fmgen.PLAIN["plain_11_3"])
    small = fmgen.gen_fm(seed=1, **fmgen.PLAIN["plain_8_1"])
    check_pair(env, big, "plain_11_3")
    check_pair(env, small, "plain_8_1")
    # and back up again, after the small call
    check_pair(env, fmgen.gen_fm(seed=2, **fmgen.PLAIN["plain_11_3"]), "plain_11_3")


def test_noalloc_headline_shape(env):
    inst = fmgen.gen_fm(seed=0, **fmgen.PLAIN["plain_15_4"])
    got = check_pair(env, inst, "plain_15_4")
    assert inst.consensus in [env[0].decode(int(c), 15) for c in got]


@pytest.mark.parametrize("l,d,n,t,seed", [(2, 1, 3, 9, 5), (3, 3, 2, 3, 6), (5, 1, 40, 70, 7),
                                          (9, 2, 30, 1000, 8), (12, 4, 64, 37, 9)])
def test_noalloc_edge_shapes(env, l, d, n, t, seed):
    """Per-lane and 16-per-lane kernels (l < 3), d = l, many rows, one window
    group, more rows than the LDS stage queues hold."""
    inst = fmgen.gen_fm(l, d, n, t, seed)
    check_pair(env, inst)


def test_noalloc_reduced_grid_and_size_error(env, monkeypatch):
    """A smaller usable scratch launches fewer workgroups with the same result;
    one too small for the tables is refused before any device work."""
    nat = env[0]
    inst = fmgen.gen_fm(seed=3, **fmgen.PLAIN["plain_11_3"])
    full = check_pair(env, inst, "plain_11_3")
    grid_full = nat.last_stats()["grid"]
    # room for the tables (about 100 KB here) and a few workgroups' queues
    monkeypatch.setenv("PMS_TEST_NOALLOC_CAP", str(1 << 20))
    k, got = run(env, nat.solve_dev_noalloc, inst)
    grid_small = nat.last_stats()["grid"]
    assert 1 <= grid_small < grid_full
    assert k == full.size and np.array_equal(got, full)
    monkeypatch.setenv("PMS_TEST_NOALLOC_CAP", "4096")
    with pytest.raises(nat.PmsError) as e:
        run(env, nat.solve_dev_noalloc, inst)
    assert e.value.status == nat.PMS_ERR_INVALID
    monkeypatch.delenv("PMS_TEST_NOALLOC_CAP")
    k, got = run(env, nat.solve_dev_noalloc, inst)
    assert nat.last_stats()["grid"] == grid_full
    assert k == full.size and np.array_equal(got, full)
