"""Benchmark of the SMO trainer on one MI355X.

A step is one full training solve to the KKT tolerance, with every part of the hot path:
pair updates, f updates, two-threshold selection, shrinking with compaction, gradient
reconstruction (on the matrix cores) and the closing recompute.  The default workload is the
largest single-GPU configuration by bytes per SMO step, the text-like one: n = 200,000,
d = 47,000 CSR with about 75 nonzeros per row (Zipf(1.1) columns, lognormal values, unit
rows), labels from a sparse linear teacher with 5% flips; RBF gamma = 1, C = 4, eps = 1e-3,
earliest shrinking (random:2) with multi reconstruction.  The inputs are resident in HBM
before the timed region starts.  With ``--tune``, svm_autotune measures a few grid sizes of
the SMO loop on the workload's first iterations before the clock starts and the timed solves
use its choice; by default the built-in rule sets the grid (one workgroup per CU on the
text-like workload).

Prints ONE JSON line.  ``value`` is SMO iterations per second over the timed solves;
``train_s`` is seconds to KKT at eps = 1e-3.  ``roofline`` is the SMO loop kernel's
algorithmic bytes (rows and nonzeros it actually streamed, times the per-row / per-nonzero
byte counts below, plus the kernel-row cache values it read or wrote) over its HIP-event-timed
duration; the loop's CSR stream moves 6 of the 8 bytes per nonzero counted there (u16 column
ids), which ``traffic`` (HBM counters) shows.  ``reconstruction`` gives the kernel sums'
matrix-core rate.  The text-like workload runs with a 160 GiB kernel-row cache by default
(``--cache-mb 0`` turns it off); ``kernel_matrix`` is one more solve with the whole kernel matrix
computed into that cache before the loop (SVM_FLAG_KERNEL_MATRIX), reported beside the headline.
``serving`` is the batched / serving comparison on the 256-problem
Poisson stream (``--no-serve`` skips it).  ``cpu_baseline`` is the FP64 oracle on the host
cores (all of them, and one) on a bounded sample of the same solve.
"""
import argparse
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
    "cfg3_text_n200000_d47000": os.path.join(ROOT, "profiles", "smo_loop_cfg3_traffic.json"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(res, data, kbytes=4):
    """Bytes the streaming passes must move: per active row visited, f read and write 16 +
    status 1 + active id 4 + norm 4 = 25; per row whose data is read, CSR 4 B per nonzero
    (column id; values skipped when all are 1.0, else 8 B with the value) + row pointer 4, or
    dense 4 B per feature; per kernel value read from or written to the row cache, its size."""
    payload = (4 if res.pattern_only else 8) * res.nnz_streamed + 4 * res.rows_read if data.layout == "csr" \
        else 4 * data.d * res.rows_read
    return payload + 25 * res.rows_streamed + kbytes * res.cache_values


# sources of the SMO loop kernel, hashed in this order by the counter summary
LOOP_SOURCES = [os.path.join("paper_1406_5161_amd", "csrc", f)
                for f in ("svm_step.hip", "svm_device.h", "svm_internal.h")]


def kernel_source_hash():
    """Hash of the loop kernel's code, comments removed (as the counter summary takes it)."""
    from paper_1406_5161_amd.profsum import source_hash
    return source_hash([os.path.join(ROOT, f) for f in LOOP_SOURCES])


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
# kernel-row cache of the SMO loop per workload (MiB of the workspace), where rows stream from HBM
# (the text-like workload: 160 GiB holds all 200,000 rows of 800 KB; 11.9 s against 14.6 s per
# solve without it, measured)
DEFAULT_CACHE_MB = {3: 163840}


def recon_summary(results, data):
    """Reconstruction / closing-recompute kernel sums over the timed solves: (row, support
    vector) pairs and their time; on the matrix cores, the dot-product flops per pair (2 * dpad
    for dense rows, 2 * H for the dense head of wide CSR rows) against the FP32 matrix peak."""
    ms = sum(r.ms_ksum for r in results)
    pairs = sum(r.recon_pairs for r in results)
    last = results[-1]
    kern = ("kernel_sum_mfma_kernel" if last.ksum_mfma == 1
            else "kernel_sum_ht_kernel" if last.ksum_mfma == 2
            else "kernel_sum_bits_kernel" if data.layout == "csr" and last.pattern_only and data.d <= 1024
            else "kernel_sum_slot_kernel" if data.layout == "csr" and data.d > 12288 else "kernel_sum_kernel")
    rec = {"kernel": kern,
           "ms_per_solve": ms / len(results), "pairs_per_solve": pairs / len(results),
           "pairs_per_s": pairs / (ms * 1e-3) if ms > 0 else None}
    if last.ksum_mfma:
        k = (data.d + 3) // 4 * 4 if last.ksum_mfma == 1 else last.head_cols
        tflops = 2.0 * k * pairs / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        rec.update({"bound": "mfma", "achieved": tflops, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops / FP32_MFMA_PEAK_TFLOPS, "k_per_pair": k})
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


def kernel_matrix_summary(S, torch, cfg, dp, cache_mb, alpha, f, ws, head):
    """One more solve of the same problem with SVM_FLAG_KERNEL_MATRIX (after one untimed one):
    the whole kernel matrix computed into the row cache on the matrix cores before the loop, so
    the loop stages no pair rows and computes no kernel rows.  Not the headline, which runs every
    step of the loop; reported beside it."""
    params = S.params_for(cfg, cache_mb=cache_mb, flags=S.SVM_FLAG_KERNEL_MATRIX)
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = S.svm_train(dp, params, alpha, f, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        assert rc == S.SVM_OK, S.strerror(rc)
        if r.kernel_matrix != 1:
            return {"flag": "SVM_FLAG_KERNEL_MATRIX", "kernel_matrix": 0,
                    "note": "not filled: a tile of rows has more tail nonzeros than the kernel's LDS table"}
        log("kernel matrix %d: %d iterations, %.1f ms (fill %.1f ms, loop %.1f ms, recon %.1f ms)"
            % (k, r.iterations, t * 1e3, r.ms_kmatrix, r.ms_step, r.ms_recon))
    loop_gbs = algorithmic_bytes(r, cfg.data) / (r.ms_step * 1e-3) / 1e9 if r.ms_step > 0 else None
    return {"flag": "SVM_FLAG_KERNEL_MATRIX", "train_s": t, "iters_per_s": r.iterations / t,
            "iterations": r.iterations, "n_recon": r.n_recon, "n_sv": r.n_sv, "fill_ms": r.ms_kmatrix,
            "loop_ms": r.ms_step, "recon_ms": r.ms_recon, "us_per_iter": r.ms_step * 1e3 / max(1, r.iterations),
            "loop_algorithmic_GBs": loop_gbs,
            "dual_obj": r.dual_obj, "dual_rel_vs_headline": abs(r.dual_obj - head.dual_obj) / abs(head.dual_obj)}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(cfg, seconds):
    """The oracle (FP64, as it stands) on the first iterations of the same solve, once on every
    core this process may use and once on one thread: a short calibration run, then about
    `seconds` of work per leg; iterations per second."""
    from oracle import oracle as O
    model, cores = host_cpu()
    legs = {}
    old = O.get_threads()
    try:
        for label, threads in (("all_cores", cores), ("single_thread", 1)):
            O.set_threads(threads)
            t0 = time.perf_counter()
            r = O.train_config(cfg, max_iter=8)
            dt = time.perf_counter() - t0
            k = int(max(8, min(50_000, 8 * seconds / max(dt, 1e-3))))
            t0 = time.perf_counter()
            r = O.train_config(cfg, max_iter=k)
            dt = time.perf_counter() - t0
            legs[label] = {"value": r.iterations / dt, "unit": "iters/s", "cores": threads,
                           "iterations": r.iterations, "seconds": dt}
            log("cpu baseline %s: %d iterations in %.1f s on %d threads" % (label, r.iterations, dt, threads))
    finally:
        O.set_threads(old)
    main = legs["all_cores"]
    return {"value": main["value"], "unit": "iters/s", "cores": main["cores"], "kind": "oracle",
            "sample": "first %d SMO iterations of the same solve (FP64 oracle, %d threads, %.1f s; a capped "
                      "exit reconstructs any shrunk samples)" % (main["iterations"], main["cores"], main["seconds"]),
            "single_thread": legs["single_thread"], "host_cpu": model, "nproc": cores}


def run_serve(args):
    from paper_1406_5161_amd import serve_bench
    return serve_bench.run(num=args.serve_problems, rate_hz=200.0, log=log)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3, help="workload: 3 (default), 1, 2 or 4")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle work per CPU-baseline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the batched / serving comparison")
    ap.add_argument("--cache-mb", type=int, default=-1,
                    help="kernel-row cache of the SMO loop in MiB (-1: the workload's default, 0: none)")
    ap.add_argument("--serve-problems", type=int, default=256)
    ap.add_argument("--tune", action="store_true", help="take the loop's grid from svm_autotune (before the clock)")
    ap.add_argument("--no-kernel-matrix", action="store_true",
                    help="skip the extra solve with the whole kernel matrix in the row cache")
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
    cache_mb = args.cache_mb if args.cache_mb >= 0 else DEFAULT_CACHE_MB.get(args.config, 0)
    params = S.params_for(cfg, kernel_precision=prec, cache_mb=cache_mb)
    tuned = None
    if args.tune:
        # the loop's grid for this problem class, measured on the device before the clock starts
        # (trial solves of the first iterations); automatic solves of the class then use it
        S.svm_autotune_reset()
        rc, tuned = S.svm_autotune(dp, params, S.SVM_TUNE_GRID)
        assert rc == S.SVM_OK, S.strerror(rc)
        log("autotune: grid %d (candidates %s)" % (tuned["chosen"], ", ".join(
            "%d: %.2f us" % (c["shape"], c["us_per_iter"]) for c in tuned["candidates"])))
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
    full_gbs = algorithmic_bytes(r200, data, 8 if args.precision == 'fp64' else 4) / (r200.ms_step * 1e-3) / 1e9

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
    byts = sum(algorithmic_bytes(r, data, 8 if args.precision == 'fp64' else 4) for r in results)
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
                   "lanes_per_row": last.lanes_per_row, "head_cols": last.head_cols, "cache_mb": cache_mb,
                   "cache_rows": last.cache_rows, "grid_from": "rule" if tuned is None else "svm_autotune"},
        "train_s": elapsed / args.steps,
        "iterations_per_solve": last.iterations,
        "n_sv": last.n_sv, "n_bsv": last.n_bsv, "n_recon": last.n_recon, "dual_obj": last.dual_obj,
        "loop_ms_per_solve": loop_ms / args.steps,
        "cache_both_per_solve": last.cache_both, "rows_read_frac": last.rows_read / max(1, last.rows_streamed),
        "recon_ms_per_solve": sum(r.ms_recon for r in results) / args.steps,
        "us_per_iter_full_active": full_us,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "smo_loop_kernel", "algorithmic_bytes_per_launch": per_launch_bytes,
                     "launches": launches, "avg_launch_us": loop_ms * 1e3 / max(1, launches),
                     "full_active_set_GBs": full_gbs},
    }
    if tuned is not None:
        out["autotune"] = tuned
    out["reconstruction"] = recon_summary(results, data)
    if cfg.queries is not None:
        out["decision"] = decision_summary(S, torch, dp, alpha, last, cfg)
    if not args.no_kernel_matrix and args.precision == "fp32" and last.cache_rows == data.n and last.head_cols:
        out["kernel_matrix"] = kernel_matrix_summary(S, torch, cfg, dp, cache_mb, alpha, f, ws, last)
    del ws   # the training workspace (with its row cache) is not needed past this point
    torch.cuda.empty_cache()
    if not args.no_serve:
        out["serving"] = run_serve(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
