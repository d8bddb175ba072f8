"""Writes the oracle's trained models for the parity tests at sizes the oracle cannot solve
inside a test: tests/golden/oracle_<case>.npz.

Each file holds, for one seeded workload, what the FP64 CPU oracle computes (and nothing
else: this script calls only oracle/ and the seeded generators):
  sha256           SHA-256 of the generated training set (the tests regenerate it and compare)
  alpha            the trained alpha (float64, n)
  i_up, i_low      the selected pair of every iteration (int32)
  scalars          beta, b_up, b_low, dual from the maintained f, dual from a fresh
                   O(n_sv^2) recompute, iterations, n_sv, n_bsv, n_recon, shrink_passes
  q_rows, q_dec    held-out query rows (the first n_q of the workload's held-out set) and the
                   oracle's decision values on them (eq:classi before the sign)

Run: python tests/golden/make_oracle_artifacts.py [case ...]   (all cases by default; the
oracle uses every core; ORACLE_THREADS=k limits it, without changing any value).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1406_5161_amd import datagen as g  # noqa: E402

SCALARS = ["beta", "b_up", "b_low", "dual_obj", "dual_fresh", "iterations", "n_sv", "n_bsv", "n_recon",
           "shrink_passes"]

# case name -> (config factory, held-out queries)
CASES = {
    # the sparse-binary workload at full size: n = 50,000, d = 300, lazy shrinking, multi
    "cfg2_full": (lambda: g.config2(), 2000),
    # the text-like generator at n = 20,000 (d = 47,000, CSR with values), earliest shrinking, multi
    "cfg3_n20000": (lambda: g.config3(n=20_000), 1000),
    # the dense mixture generator at n = 50,000 (d = 28), lazy shrinking, multi
    "cfg4_n50000": (lambda: g.config4(n=50_000), 1000),
}


def path_for(case):
    return os.path.join(HERE, "oracle_%s.npz" % case)


def make(case):
    factory, nq = CASES[case]
    cfg = factory()
    t0 = time.perf_counter()
    r = O.train_config(cfg, trace_cap=4_000_000)
    t1 = time.perf_counter()
    assert r.rc == O.OK, r.rc
    dual_fresh = O.dual(cfg.data, r.alpha, cfg.gamma)
    q = cfg.queries.subset(np.arange(nq))
    dec = O.decision(cfg.data, r.alpha, r.beta, cfg.gamma, q)
    t2 = time.perf_counter()
    sc = np.array([r.beta, r.b_up, r.b_low, r.dual_obj, dual_fresh, r.iterations, r.n_sv, r.n_bsv, r.n_recon,
                   r.shrink_passes], np.float64)
    np.savez_compressed(path_for(case), sha256=np.array(cfg.data.sha256()), workload=np.array(cfg.name),
                        alpha=r.alpha, i_up=r.trace["i_up"].astype(np.int32),
                        i_low=r.trace["i_low"].astype(np.int32), scalars=sc,
                        scalar_names=np.array(SCALARS), q_rows=np.arange(nq, dtype=np.int32), q_dec=dec)
    info = {"case": case, "workload": cfg.name, "n": cfg.data.n, "iterations": r.iterations, "n_sv": r.n_sv,
            "dual": r.dual_obj, "dual_fresh": dual_fresh, "train_s": round(t1 - t0, 1),
            "extras_s": round(t2 - t1, 1), "threads": O.get_threads()}
    print(json.dumps(info), flush=True)


def load(case):
    """The stored record as a dict (scalars by name); no pickled objects are read."""
    z = np.load(path_for(case), allow_pickle=False)
    out = {k: z[k] for k in z.files}
    for name, v in zip(out["scalar_names"], out["scalars"]):
        out[str(name)] = float(v)
    out["sha256"] = str(out["sha256"])
    out["workload"] = str(out["workload"])
    return out


if __name__ == "__main__":
    for c in sys.argv[1:] or list(CASES):
        make(c)
