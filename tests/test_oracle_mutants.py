"""Planted mistakes in copies of the oracle must each fail some pin.

Each mutant is a textual edit of ``oracle/pms_oracle.c`` compiled into a
temporary library on the CPU; the real source is untouched.
"""
import os
import shutil
import subprocess

import pytest

import oracle
from oracle import build as obuild
import _pins

MUTANTS = {
    "drops_last_window": ("const int nw = t - l + 1;", "const int nw = t - l;"),
    "strict_threshold": ("if (m > d) {", "if (m >= d) {"),
    "drops_last_position": ("for (int p = 0; p < l; ++p) {\n        const char xp",
                            "for (int p = 0; p < l - 1; ++p) {\n        const char xp"),
    "reversed_numbering": ("(k >> (2 * (l - 1 - p))) & 3u", "(k >> (2 * p)) & 3u"),
    "never_rejects": ("accepted = 0;\n", "\n"),
    "min_starts_at_zero": ("int best = l + 1;", "int best = 0;"),
    "swapped_bases": ("{'A', 'C', 'G', 'T'}", "{'A', 'C', 'T', 'G'}"),
    "overlapping_ranges": ("span * (uint64_t)(w + 1) / (uint64_t)threads",
                           "span * (uint64_t)(w + 1) / (uint64_t)threads + (w + 1 < threads)"),
    "counts_matches": ("(sp[j] != xp)", "(sp[j] == xp)"),
    "wrong_row_stride": ("job->seqs + (size_t)i * t", "job->seqs + (size_t)i * (t - 1)"),
    "skip_breaks_on_pass": ("if (job->mode == ORACLE_SKIP) break; /* the enhanced rule */",
                            "}\n            if (m <= d && job->mode == ORACLE_SKIP) { break;"),
}

# Mistakes in the extended-input path (oracle_solve_ex).
EX_MUTANTS = {
    "ex_mask_keeps_n": ("if (has_n) continue;", ""),
    "ex_no_complement": ("= complement(w[(size_t)q * l + l - 1 - p]);",
                         "= w[(size_t)q * l + l - 1 - p];"),
    "ex_rc_not_reversed": ("complement(w[(size_t)q * l + l - 1 - p])",
                           "complement(w[(size_t)q * l + p])"),
    "ex_drops_last_start": ("const int nstarts = t - l + 1;", "const int nstarts = t - l;"),
    "ex_mask_misses_last_base": ("for (int p = 0; p < l; ++p) has_n |= up[j + p] == 'N';",
                                 "for (int p = 0; p < l - 1; ++p) has_n |= up[j + p] == 'N';"),
    "ex_strict_threshold": ("if (d < m) {", "if (d <= m) {"),
    "ex_bad_complement": ("case 'C': return 'G';", "case 'C': return 'C';"),
    "ex_rc_skips_first": ("for (int q = 0; q < fwd; ++q) {", "for (int q = 1; q < fwd; ++q) {"),
}

EX_PINS = [
    lambda o: _pins.pin_ex_definition_tiny(o, cases=40),
    _pins.pin_ex_identities,
    _pins.pin_ex_closed_forms,
]

QUICK_PINS = [
    lambda o: _pins.pin_definition_tiny(o, cases=40),
    lambda o: _pins.pin_skip_visits(o, cases=15),
    _pins.pin_closed_forms,
    _pins.pin_edges,
    lambda o: _pins.pin_ball_intersection(o, shapes=((5, 1, 4, 40), (6, 2, 5, 60)), seeds=(0,)),
    _pins.pin_invariants,
    _pins.pin_ranges_and_distances,
]


@pytest.fixture(scope="module")
def src():
    with open(obuild.SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, src, name):
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / f"lib_{name}.so")
    obuild.build(str(path), lib)
    orc = oracle.OracleLib(lib)
    caught = []
    for pin in QUICK_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError, OverflowError) as e:  # noqa: PERF203
            caught.append(repr(e)[:80])
            break
    assert caught, f"mutant {name} passed every pin"


def test_unmutated_copy_passes(tmp_path, src):
    path = tmp_path / "copy.c"
    path.write_text(src)
    lib = str(tmp_path / "lib_copy.so")
    obuild.build(str(path), lib)
    orc = oracle.OracleLib(lib)
    for pin in QUICK_PINS:
        pin(orc)


@pytest.mark.parametrize("name", sorted(EX_MUTANTS))
def test_ex_mutant_is_caught(tmp_path, src, name):
    old, new = EX_MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / f"lib_{name}.so")
    obuild.build(str(path), lib)
    orc = oracle.OracleLib(lib)
    caught = []
    for pin in EX_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError, OverflowError) as e:  # noqa: PERF203
            caught.append(repr(e)[:80])
            break
    assert caught, f"mutant {name} passed every pin"
