"""The oracle against facts that do not come from its own code."""
import hashlib
import json
import os

import numpy as np
import pytest

import fmgen
import oracle
import _pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("pin", _pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


@pytest.mark.parametrize("cfg", ["plain_8_1", "plain_11_3"])
def test_ball_intersection_plain(orc, cfg):
    """Whole configurations: oracle == second algorithm, seeds 0-4."""
    shape = fmgen.PLAIN[cfg]
    for s in range(5):
        inst = fmgen.gen_fm(seed=s, **shape)
        got = orc.solve(inst.seqs, inst.l, inst.d)
        want = _pins.ball_intersection(inst.seqs, inst.l, inst.d)
        assert np.array_equal(got, want), (cfg, s)


def _records(cfg):
    path = os.path.join(GOLDEN, f"{cfg}.json")
    if not os.path.exists(path):
        pytest.skip(f"no golden file {path}")
    with open(path) as f:
        return json.load(f)["records"]


@pytest.mark.parametrize("cfg", ["plain_8_1", "plain_11_3"])
def test_golden_reproduces(orc, cfg):
    """Stored expected sets are what the oracle computes from the recipe."""
    for r in _records(cfg):
        inst = fmgen.gen_fm(r["l"], r["d"], r["n"], r["t"], r["seed"])
        got, visits = orc.solve(inst.seqs, r["l"], r["d"], mode="skip", return_visits=True)
        assert got.size == r["count"] and hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == r["sha256"]
        assert visits == r["skip_visits"]


@pytest.mark.parametrize("cfg", ["plain_8_1", "plain_11_3", "plain_15_4"])
def test_golden_invariants(cfg):
    """Every stored set holds the planted consensus and is sound, checked with
    numpy distances (not the oracle)."""
    for r in _records(cfg):
        assert r["generator"] == fmgen.GENERATOR_VERSION
        inst = fmgen.gen_fm(r["l"], r["d"], r["n"], r["t"], r["seed"])
        assert r["consensus"] == inst.consensus
        motifs = r["motifs"]
        assert len(motifs) == r["count"] and motifs == sorted(motifs)
        assert inst.consensus in motifs
        nums = [oracle.lmer_to_number(m) for m in motifs]
        _pins.verify_sound(inst.seqs, r["l"], r["d"], nums)


def _ball_15_4(seeds):
    for r in _records("plain_15_4"):
        if r["seed"] not in seeds:
            continue
        inst = fmgen.gen_fm(r["l"], r["d"], r["n"], r["t"], r["seed"])
        want = _pins.ball_intersection(inst.seqs, r["l"], r["d"])
        assert [oracle.number_to_lmer(int(k), r["l"]) for k in want] == r["motifs"]


def test_ball_intersection_15_4_seed0():
    """(15,4), the benchmark's seed: the second algorithm reproduces the
    stored set (the one record made in brute mode), about 15 s."""
    _ball_15_4({0})


@pytest.mark.slow
def test_ball_intersection_15_4_golden():
    """(15,4), the other seeds (skip-mode records): about 15 s each."""
    _ball_15_4({1, 2, 3, 4})
