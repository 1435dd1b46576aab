"""Pins of the oracle's extended inputs (rows of their own lengths, N masking,
both strands): the reading of the real-sequence future work of Section VI."""
import oracle
import _pins


def test_ex_definition_tiny():
    _pins.pin_ex_definition_tiny(oracle.default())


def test_ex_identities():
    _pins.pin_ex_identities(oracle.default())


def test_ex_closed_forms():
    _pins.pin_ex_closed_forms(oracle.default())


def test_ex_skip_visits_stop_at_first_failure():
    """Skip mode counts one scan per sequence up to the first without a window
    within d, over the spelled-out window sets."""
    import itertools
    import numpy as np
    rng = np.random.default_rng(29)
    for case in range(20):
        l = int(rng.integers(1, 4))
        d = int(rng.integers(0, l + 1))
        mask_n, both = bool(case & 1), bool(case & 2)
        rows = _pins.random_rows_ex(rng, int(rng.integers(1, 4)), l, l + 6, 0.1 if mask_n else 0.0)
        sets = [_pins.definition_window_set(r, l, mask_n, both) for r in rows]
        if any(not s for s in sets):
            continue
        want = 0
        for x in itertools.product(_pins.BASES, repeat=l):
            for ws in sets:
                want += 1
                if not any(sum(a != b for a, b in zip(x, w)) <= d for w in ws):
                    break
        _, got = oracle.solve_ex(rows, l, d, mask_n=mask_n, both=both, mode="skip",
                                 return_visits=True)
        assert got == want, (l, d, rows)
