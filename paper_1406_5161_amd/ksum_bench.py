"""Kernel sums on the matrix cores, measured alone: decision values (eq:classi) of `nq`
queries against `nsv` support vectors, the same kernels the gradient reconstruction runs.
Family "dense": dense-mixture rows (d = 28 by default), `kernel_sum_mfma_kernel`.  Family
"text": text-like CSR rows (d = 47,000, about 75 nonzeros), `kernel_sum_ht_kernel` (the 128
most frequent columns as dense rows on the matrix cores, the rest as a sparse tail).

    python -m paper_1406_5161_amd.ksum_bench [--family dense|text] [--nq N] [--nsv N] [--d D] [--reps 5]

Prints one JSON line: pairs per call, executed matrix-core flops per call (2 dpad per pair,
dpad = d rounded up to 4; 2 H per pair for the text family), the average time of `reps` calls after one untimed call (HIP
events on the calling stream; each call also validates the queries and lists the support
vectors), TFLOP/s and its fraction of the FP32 matrix peak (157.3 TFLOP/s).  Inputs: seeded
mixture rows; coefficients uniform in [0, 1] on every training row.
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import datagen as g

FP32_MATRIX_PEAK_TFLOPS = 157.3
HEAD_COLS = 128   # the library's default head width of wide CSR kernel sums


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", choices=["dense", "text"], default="dense")
    ap.add_argument("--nq", type=int, default=100_000)
    ap.add_argument("--nsv", type=int, default=150_000)
    ap.add_argument("--d", type=int, default=0, help="features (default 28 dense, 47,000 text)")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    import torch
    from . import svmhip as S
    S.lib()
    text = a.family == "text"
    a.d = a.d or (47_000 if text else 28)
    rng = g.rng_for(6, a.d)
    if text:
        train = g.gen_text_like(a.nsv, a.d, 75.0, rng, name="ksum_train")
        queries = g.gen_text_like(a.nq, a.d, 75.0, rng, name="ksum_queries")
    else:
        train = g.gen_mixture(a.nsv, a.d, rng, name="ksum_train")
        queries = g.gen_mixture(a.nq, a.d, rng, name="ksum_queries")
    tp = S.to_device(train)
    qp = S.to_device(queries, with_labels=False)
    alpha = torch.from_numpy(rng.uniform(0.0, 1.0, a.nsv)).to("cuda")
    out = torch.zeros(a.nq, dtype=torch.float64, device="cuda")
    gamma = 1.0 if text else 0.1
    rc = S.svm_decision(tp, alpha, 0.0, gamma, qp, out)
    assert rc == S.SVM_OK, S.strerror(rc)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.reps):
        rc = S.svm_decision(tp, alpha, 0.0, gamma, qp, out)
        assert rc == S.SVM_OK, S.strerror(rc)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.reps
    dpad = HEAD_COLS if text else (a.d + 3) & ~3
    pairs = float(a.nq) * float(a.nsv)
    flops = 2.0 * dpad * pairs
    tflops = flops / (ms * 1e-3) / 1e12
    print(json.dumps({"kernel": "kernel_sum_ht_kernel" if text else "kernel_sum_mfma_kernel", "family": a.family,
                      "nq": a.nq, "nsv": a.nsv, "d": a.d, "k_per_pair": dpad,
                      "pairs_per_call": pairs, "mfma_flops_per_call": flops, "ms_per_call": ms,
                      "tflops": tflops, "peak_tflops": FP32_MATRIX_PEAK_TFLOPS,
                      "frac": tflops / FP32_MATRIX_PEAK_TFLOPS, "pairs_per_s": pairs / (ms * 1e-3),
                      "finite": bool(np.isfinite(out.cpu().numpy()).all())}), flush=True)


if __name__ == "__main__":
    main()
