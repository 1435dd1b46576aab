"""The FM-model input generator (Section I.B; Section IV.B)."""
import numpy as np

import fmgen


def test_fm_instances_are_planted_at_exactly_d():
    for (l, d, n, t) in [(8, 1, 10, 200), (11, 3, 20, 600), (15, 4, 20, 600), (5, 5, 3, 9), (4, 0, 2, 4)]:
        for seed in range(3):
            inst = fmgen.gen_fm(l, d, n, t, seed)
            assert inst.seqs.shape == (n, t) and inst.seqs.dtype == np.uint8
            assert set(np.unique(inst.seqs).tolist()) <= set(b"ACGT")
            for i in range(n):
                o = int(inst.offsets[i])
                assert 0 <= o <= t - l
                planted = inst.planted(i)
                diff = [p for p in range(l) if planted[p] != inst.consensus[p]]
                assert len(diff) == d
                assert diff == sorted(inst.mutated[i].tolist())


def test_fm_is_deterministic_per_seed():
    a = fmgen.gen_fm(11, 3, 20, 600, 42)
    b = fmgen.gen_fm(11, 3, 20, 600, 42)
    c = fmgen.gen_fm(11, 3, 20, 600, 43)
    assert np.array_equal(a.seqs, b.seqs) and a.consensus == b.consensus
    assert not np.array_equal(a.seqs, c.seqs)


def test_fm_background_is_uniform():
    inst = fmgen.gen_fm(15, 4, 200, 600, 1)
    counts = np.array([(inst.seqs == b).sum() for b in b"ACGT"], dtype=np.float64)
    expected = inst.seqs.size / 4
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 30.0


def test_batched_and_serving_recipes():
    specs = fmgen.batched_specs()
    assert len(specs) == 256
    assert {(s.l, s.d) for s in specs} == set(fmgen.BATCH_LD)
    assert all(10 <= s.n <= 30 and 300 <= s.t <= 1000 for s in specs)
    assert specs[0] == fmgen.batched_specs()[0]
    stream = fmgen.serving_stream(400, rate=20.0)
    times = [a for a, _ in stream]
    assert times == sorted(times) and times[0] > 0
    mix = np.array([fmgen.SERVE_LD.index((s.l, s.d)) for _, s in stream])
    frac = np.bincount(mix, minlength=4) / len(mix)
    assert np.allclose(frac, [0.4, 0.3, 0.2, 0.1], atol=0.07)
    gaps = np.diff([0.0] + times)
    assert 0.03 < gaps.mean() < 0.07
