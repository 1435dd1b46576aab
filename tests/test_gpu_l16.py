"""l = 16, whole motif sets, every search kernel variant.

The brute-force oracle cannot sweep 4^16 candidates in test time, so the
whole sets are compared with the second exact algorithm of tests/_pins.py
(intersection over sequences of the unions of the windows' Hamming balls),
which the CPU suite pins against the oracle on every plain configuration.
(16,2) and (16,3) at n = 20, t = 600, two seeds each; the 64-candidate
kernel with its window filter on and off, the 16-candidate and per-lane
kernels; all must also agree on the enhanced rule's visit count.
"""
import numpy as np
import pytest

import fmgen
import _pins

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


CONFIGS = {"group64": dict(variant=3), "group64_nofilter": dict(variant=3, filter=2),
           "group16": dict(variant=2), "lane": dict(variant=1)}


@pytest.mark.parametrize("l,d,seed", [(16, 2, 0), (16, 2, 1), (16, 3, 0), (16, 3, 1)])
def test_l16_whole_sets(nat, l, d, seed):
    inst = fmgen.gen_fm(l, d, 20, 600, seed)
    want = _pins.ball_intersection(inst.seqs, l, d)
    visits = {}
    for name, cfg in CONFIGS.items():
        print(f"[case] l=16 ({l},{d}) seed={seed} {name}", flush=True)
        nat.set_config(**cfg)
        try:
            got = nat.solve(inst.seqs, l, d)
            st = nat.last_stats()
        finally:
            nat.set_config(reset=True)
        assert np.array_equal(got, want), name
        assert st["variant"] == cfg["variant"]
        visits[name] = st["seq_visits"]
    assert len(set(visits.values())) == 1, visits
