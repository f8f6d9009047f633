"""The oracle reproduces its committed results exactly
(tests/golden/oracle_sequences.json, written by
tests/golden/make_oracle_sequences.py from the oracle alone).  The inputs are
bitwise reproducible (problems/exact.py) and the oracle's arithmetic does not
depend on its thread count (row-parallel products, inner products summed in a
fixed order), so every value must match to the last bit: iteration counts,
ranks, residuals and the SHA-256 of each solution.  A change to the oracle's
arithmetic must be justified by a passage of the paper and regenerate the
fixture."""

import json
import os

from tests.golden.make_oracle_sequences import records

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_committed_sequences_exactly():
    with open(os.path.join(HERE, "golden", "oracle_sequences.json")) as f:
        ref = json.load(f)
    now = records()
    assert set(now) == set(ref)
    for name in ref:
        assert len(now[name]) == len(ref[name])
        for a, b in zip(now[name], ref[name]):
            assert a == b, (name, a["j"])
