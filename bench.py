"""Benchmark of the SMO trainer on one MI355X.

A step is one full training solve (every part of the hot path: pair updates,
f updates, two-threshold selection, shrinking with compaction, gradient
reconstruction, closing recompute) of the sparse-binary workload:
n = 50,000, d = 300, CSR at 12% density, values 1.0, Zipf(1.1) columns, labels
from a sparse linear teacher with 10% flips; RBF gamma = 1/300, C = 1,
eps = 1e-3, lazy shrinking (numsamples 50%) with multi reconstruction.  The
inputs are resident in HBM before the timed region starts.

Prints ONE JSON line.  ``value`` is SMO iterations per second over the timed
solves; ``train_s`` is seconds to KKT at eps = 1e-3.  ``roofline`` is the SMO
loop kernel's algorithmic bytes (rows and nonzeros it actually streamed, times
the per-row / per-nonzero byte counts below) over its HIP-event-timed duration.
``cpu_baseline`` is the FP64 oracle on the host cores on a bounded sample of the
same solve.  ``--serve`` adds the batched / serving comparison.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# committed HBM-counter summaries of the loop kernel, by workload
PROFILE_COUNTERS = {
    "cfg2_sparse_binary_n50000_d300": os.path.join(ROOT, "profiles", "smo_loop_cfg2_traffic.json"),
    "cfg4_mixture_n500000_d28": os.path.join(ROOT, "profiles", "smo_loop_cfg4_traffic.json"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(res, data):
    """Bytes one streaming pass must move per active row: CSR 4 B per nonzero (column id;
    values skipped when all are 1.0, else 8 B with the value) + f read and write 16 + status 1
    + active id 4 + row pointer 4 + norm 4 = 29 per row.  Dense: 4 B per feature + 25 per row."""
    if data.layout == "csr":
        per_nnz = 4 if res.pattern_only else 8
        return per_nnz * res.nnz_streamed + 29 * res.rows_streamed
    return (4 * data.d + 25) * res.rows_streamed


# sources of the SMO loop kernel, hashed in this order by the counter summary
LOOP_SOURCES = [os.path.join("paper_1406_5161_amd", "csrc", f)
                for f in ("svm_step.hip", "svm_device.h", "svm_internal.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in LOOP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload):
    """HBM bytes per loop launch from the committed counter summary, if it was taken on this
    workload and the loop kernel's sources have not changed since."""
    try:
        prof = json.load(open(PROFILE_COUNTERS.get(workload, "")))
    except Exception:
        return None
    if prof.get("kernel_source_sha256_16") != kernel_source_hash() or prof.get("workload") != workload:
        return None
    return prof.get("hbm_bytes_per_launch")


FP32_MFMA_PEAK_TFLOPS = 157.3


def recon_summary(results, data):
    """Reconstruction / closing-recompute kernel sums over the timed solves: (row, support
    vector) pairs, their time, and for dense rows on the matrix cores the dot-product flops
    (2 * dpad per pair) against the FP32 matrix peak."""
    ms = sum(r.ms_ksum for r in results)
    pairs = sum(r.recon_pairs for r in results)
    kern = ("kernel_sum_mfma_kernel" if results[-1].ksum_mfma
            else "kernel_sum_bits_kernel" if data.layout == "csr" and results[-1].pattern_only and data.d <= 1024
            else "kernel_sum_slot_kernel" if data.layout == "csr" and data.d > 12288 else "kernel_sum_kernel")
    rec = {"kernel": kern,
           "ms_per_solve": ms / len(results), "pairs_per_solve": pairs / len(results),
           "pairs_per_s": pairs / (ms * 1e-3) if ms > 0 else None}
    if results[-1].ksum_mfma:
        dpad = (data.d + 3) // 4 * 4
        tflops = 2.0 * dpad * pairs / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        rec.update({"bound": "mfma", "achieved": tflops, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops / FP32_MFMA_PEAK_TFLOPS})
    return rec


def decision_summary(S, torch, dp, alpha, res, cfg, reps=3):
    """svm_decision over the workload's held-out queries with the trained alpha: queries/s and
    kernel values (query x support vector) per second, from the average of `reps` timed calls
    on the current stream after one untimed call."""
    q = S.to_device(cfg.queries, with_labels=False)
    out = torch.zeros(cfg.queries.n, dtype=torch.float64, device="cuda")
    rc = S.svm_decision(dp, alpha, res.beta, cfg.gamma, q, out)
    assert rc == S.SVM_OK, S.strerror(rc)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rc = S.svm_decision(dp, alpha, res.beta, cfg.gamma, q, out)
        assert rc == S.SVM_OK, S.strerror(rc)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"queries": cfg.queries.n, "n_sv": res.n_sv, "ms_per_call": ms,
            "queries_per_s": cfg.queries.n / (ms * 1e-3),
            "kernel_values_per_s": cfg.queries.n * res.n_sv / (ms * 1e-3)}


def cpu_baseline(cfg, iters):
    import numpy as np  # noqa: F401
    from oracle import oracle as O
    t0 = time.perf_counter()
    r = O.train_config(cfg, max_iter=iters)
    dt = time.perf_counter() - t0
    return {"value": r.iterations / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": "first %d SMO iterations of the same solve (full active set: the lazy schedule first "
                      "shrinks after n/2 iterations), FP64, single thread, %.1f s" % (r.iterations, dt)}


def run_serve(args):
    from paper_1406_5161_amd import serve_bench
    return serve_bench.run(num=args.serve_problems, rate_hz=200.0, log=log)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, help="workload: 2 (default), 1, 3 or 4")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-iters", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true", help="also run the batched / serving comparison")
    ap.add_argument("--serve-problems", type=int, default=256)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the method shards by samples; "
              "see the design notes), so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1406_5161_amd import datagen as g
    from paper_1406_5161_amd import svmhip as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    S.lib()
    cfg = g.CONFIGS[args.config]()
    data = cfg.data
    prec = S.SVM_KERNEL_FP32 if args.precision == "fp32" else S.SVM_KERNEL_FP64
    log("workload %s n=%d d=%d nnz=%d" % (cfg.name, data.n, data.d, data.nnz))
    dp = S.to_device(data)
    params = S.params_for(cfg, kernel_precision=prec)
    alpha = torch.zeros(data.n, dtype=torch.float64, device="cuda")
    f = torch.zeros(data.n, dtype=torch.float64, device="cuda")
    ws = torch.empty(S.svm_train_workspace_size(dp, params), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    for w in range(args.warmup):
        rc, res = S.svm_train(dp, params, alpha, f, workspace=ws)
        assert rc == S.SVM_OK, S.strerror(rc)
        log("warmup %d: %d iterations, %.1f ms" % (w, res.iterations, res.ms_total))

    # per-iteration cost at the full active set (first 200 iterations, before any shrinking); run
    # after the warm-up and before the timed solves, whose loop launches are the last in a trace
    p200 = S.params_for(cfg, kernel_precision=prec, max_iter=200, flags=S.SVM_FLAG_NO_FINAL_RECOMPUTE)
    rc, r200 = S.svm_train(dp, p200, alpha, f, workspace=ws)
    assert rc in (S.SVM_OK, S.SVM_NOT_CONVERGED), S.strerror(rc)
    full_us = r200.ms_step * 1e3 / max(1, r200.iterations)
    full_gbs = algorithmic_bytes(r200, data) / (r200.ms_step * 1e-3) / 1e9

    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rc, res = S.svm_train(dp, params, alpha, f, workspace=ws)
        assert rc == S.SVM_OK, S.strerror(rc)
        results.append(res)
        log("step %d: %d iterations, %.1f ms (loop %.1f ms, recon %.1f ms)"
            % (k, res.iterations, res.ms_total, res.ms_step, res.ms_recon))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    iters = sum(r.iterations for r in results)
    loop_ms = sum(r.ms_step for r in results)
    launches = sum(r.n_launches for r in results)
    byts = sum(algorithmic_bytes(r, data) for r in results)
    achieved = byts / (loop_ms * 1e-3) / 1e9
    per_launch_bytes = byts / max(1, launches)
    # the committed counter summaries were taken on the FP32-kernel-value loop
    traffic = traffic_from_profile(cfg.name) if args.precision == "fp32" else None

    last = results[-1]
    out = {
        "metric": "train s to KKT eps=1e-3 + iters/s; batched solves/s & p99 vs plain loop",
        "value": iters / elapsed,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n": data.n, "d": data.d, "nnz": data.nnz, "layout": data.layout,
                   "C": cfg.C, "gamma": cfg.gamma, "eps": cfg.eps, "shrink_mode": cfg.shrink_mode,
                   "shrink_kind": cfg.shrink_kind, "shrink_param": cfg.shrink_param,
                   "kernel_precision": args.precision, "f_dtype": "f64", "grid_blocks": last.grid_blocks,
                   "lanes_per_row": last.lanes_per_row},
        "train_s": elapsed / args.steps,
        "iterations_per_solve": last.iterations,
        "n_sv": last.n_sv, "n_bsv": last.n_bsv, "n_recon": last.n_recon, "dual_obj": last.dual_obj,
        "loop_ms_per_solve": loop_ms / args.steps,
        "recon_ms_per_solve": sum(r.ms_recon for r in results) / args.steps,
        "us_per_iter_full_active": full_us,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "smo_loop_kernel", "algorithmic_bytes_per_launch": per_launch_bytes,
                     "launches": launches, "avg_launch_us": loop_ms * 1e3 / max(1, launches),
                     "full_active_set_GBs": full_gbs},
    }
    out["reconstruction"] = recon_summary(results, data)
    if cfg.queries is not None:
        out["decision"] = decision_summary(S, torch, dp, alpha, last, cfg)
    if args.serve:
        out["serving"] = run_serve(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
