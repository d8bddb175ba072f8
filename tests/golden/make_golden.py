"""Writes tests/golden/datagen_sha256.json: SHA-256 of every array the seeded
generators produce for the named workloads, so any change to the generators
shows up as a test failure.  Calls the generators only."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1406_5161_amd import datagen as g  # noqa: E402


def hashes():
    out = {}
    for name, fn in [("config1", g.config1), ("config2", g.config2), ("config4", g.config4)]:
        c = fn()
        out[name] = {"train": c.data.sha256(), "heldout": c.queries.sha256(), "n": c.data.n, "d": c.data.d,
                     "nnz": c.data.nnz}
    reqs = g.config5(num=6)
    out["config5_first6"] = [{"sha": r.config.data.sha256(), "arrival_s": r.arrival_s, "n": r.config.data.n,
                              "d": r.config.data.d, "C": r.config.C, "gamma": r.config.gamma} for r in reqs]
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "datagen_sha256.json"), "w") as fh:
        json.dump(hashes(), fh, indent=1, sort_keys=True)
