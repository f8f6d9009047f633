"""Writes oracle_sequences.json: per-system results of the oracle on two
small 2-D diffusion sequences whose inputs are bitwise reproducible on any
machine (problems/exact.py: integer hashing and + - * / only).  The first
solves every system from zero and snapshots the solutions; the second starts
each system from the previous solution and snapshots the increments.  Both
have a snapshot memory of 3 over 8 systems, so the ring evicts.

Calls only the oracle and the input generator.  Floating-point results are
stored as hex strings and the solutions as SHA-256 digests of their bytes, so
the comparison is exact.  Rerun it only when a change to the oracle's
arithmetic is justified by the paper (and say which passage in the commit)."""

import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from problems.exact import exact2d  # noqa: E402

SEQUENCES = {
    "exact2d_24_solutions": dict(aug_xbar="zero"),
    "exact2d_24_increments": dict(aug_xbar="prev"),
}


def records():
    out = {}
    for name, kw in SEQUENCES.items():
        cfg = exact2d(N=24, steps=8, omega=3, rank=2, tol=1e-10)
        rows = oracle.run_sequence(cfg, "aug", keep_x=True, **kw)
        out[name] = [{"j": r["j"], "iters": r["iters"], "rank": r["rank"], "rank_next": r["rank_next"],
                      "stage1_relres": float(r["stage1_relres"]).hex(),
                      "relres": float(r["relres"]).hex(),
                      "true_relres": float(r["true_relres"]).hex(),
                      "x_sha256": hashlib.sha256(r["x"].tobytes()).hexdigest()} for r in rows]
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_sequences.json"), "w") as f:
        json.dump(records(), f, indent=1)
    print("written")
