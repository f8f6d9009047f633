"""Writes oracle_sequences.json: per-system results of the oracle on the 2-D
diffusion sequence (32 x 32, 10 systems, rotating load) and its two-field
variant.  Calls only the oracle and the input generators; rerun it only when
a change to the oracle's arithmetic is justified by the paper (and say which
passage in the commit)."""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from problems import config1  # noqa: E402


def records():
    out = {}
    for name, cfg in (("diffusion2d_32_rotate", config1()), ("diffusion2d_32_two_fields", config1(variant="r2"))):
        rows = oracle.run_sequence(cfg, "aug")
        out[name] = [{"j": r["j"], "iters": r["iters"], "rank": r["rank"], "rank_next": r["rank_next"],
                      "stage1_relres": r["stage1_relres"], "true_relres": r["true_relres"]} for r in rows]
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_sequences.json"), "w") as f:
        json.dump(records(), f, indent=1)
    print("written")
