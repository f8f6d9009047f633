"""The oracle still reproduces its committed results on the 2-D diffusion
sequences (tests/golden/oracle_sequences.json, written by
tests/golden/make_oracle_sequences.py from the oracle alone): integer results
exactly, residuals to 1e-6 relative (the oracle's OpenMP dot products are not
bitwise reproducible, and a residual near 1e-8 ||b|| carries cancellation).  A change to the oracle's arithmetic
must be justified by a passage of the paper and regenerate the fixture."""

import json
import os

from tests.golden.make_oracle_sequences import records

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_committed_sequences():
    with open(os.path.join(HERE, "golden", "oracle_sequences.json")) as f:
        ref = json.load(f)
    now = records()
    assert set(now) == set(ref)
    for name in ref:
        for a, b in zip(now[name], ref[name]):
            assert (a["j"], a["iters"], a["rank"], a["rank_next"]) == (b["j"], b["iters"], b["rank"], b["rank_next"])
            for key in ("stage1_relres", "true_relres"):
                assert abs(a[key] - b[key]) <= 1e-6 * abs(b[key]) + 1e-15, (name, a["j"], key)
