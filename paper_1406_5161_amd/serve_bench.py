"""Serving comparison on the Poisson stream of mixed training problems:
the plain one-problem-at-a-time GPU solver (svm_train, FIFO in arrival order)
against the continuous-batching server (svm_server_*), on the same trace and
the same eps / heuristic.  Inputs are uploaded before the clock starts;
latency is completion minus arrival, solves/s is problems over the makespan
(first arrival to last completion)."""
from __future__ import annotations

import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import datagen as g


def _make(j):
    return g.config5_problem(j)


def generate(num: int, workers: int = 16):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        cfgs = list(ex.map(_make, range(num), chunksize=4))
    return cfgs


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q))


def tune_classes(S, cfgs, probs, params, log=print) -> dict:
    """Team sizes of the batched solver measured by svm_autotune on the first problem of every
    class in the stream (row kind and n rounded up to a power of two), before the clock starts;
    the server then uses them for every problem of the class."""
    import math
    seen = {}
    for c, dp, p in zip(cfgs, probs, params):
        key = "%s_n2^%d" % (c.data.name.split("_", 1)[1], math.ceil(math.log2(c.data.n)))
        if key in seen:
            continue
        rc, info = S.svm_autotune(dp, p, S.SVM_TUNE_TEAM)
        assert rc == S.SVM_OK, S.strerror(rc)
        seen[key] = {"chosen": info["chosen"],
                     "us_per_iter": {str(x["shape"]): round(x["us_per_iter"], 2) for x in info["candidates"]}}
    log("serving: tuned team sizes of %d classes" % len(seen))
    return dict(sorted(seen.items()))


def run(num: int = 256, rate_hz: float = 200.0, log=print, slots: int = 0, budget_gb: float = 64.0,
        workers: int = 16, detail: list | None = None, plain: bool = True, tune: bool = True) -> dict:
    """Runs both paths on the same trace; with `detail` (a list) appends one record per problem:
    shape, team size, iterations and device / host times of both paths.  With `tune`, the
    batched path's team sizes come from svm_autotune per class (measured before the clock)."""
    import torch
    from . import svmhip as S
    t_gen = time.perf_counter()
    arrivals = g.config5_arrivals(num, rate_hz)
    cfgs = generate(num, workers)
    log("serving: generated %d problems in %.1f s" % (num, time.perf_counter() - t_gen))
    probs = [S.to_device(c.data) for c in cfgs]
    params = [S.params_for(c) for c in cfgs]
    torch.cuda.synchronize()
    S.svm_autotune_reset()
    tuned = tune_classes(S, cfgs, probs, params, log) if tune else None

    # ---- plain loop: one problem at a time, FIFO, each waits for its arrival; one workspace of
    # the largest size serves every solve, so no solve allocates inside the timed loop
    alphas_p = [torch.zeros(c.data.n, dtype=torch.float64, device="cuda") for c in cfgs]
    ws = torch.empty(max(S.svm_train_workspace_size(pr, pa) for pr, pa in zip(probs, params)),
                     dtype=torch.uint8, device="cuda")
    lat_p, duals_p, its_p, ms_p = [], [], 0, []
    t0 = time.perf_counter()
    for j, c in enumerate(cfgs if plain else []):
        now = time.perf_counter() - t0
        if now < arrivals[j]:
            time.sleep(arrivals[j] - now)
        rc, r = S.svm_train(probs[j], params[j], alphas_p[j], workspace=ws)
        assert rc in (S.SVM_OK, S.SVM_NOT_CONVERGED), S.strerror(rc)
        lat_p.append(time.perf_counter() - t0 - arrivals[j])
        duals_p.append(r.dual_obj)
        its_p += r.iterations
        ms_p.append((r.ms_total, r.iterations, r.grid_blocks))
        if (j + 1) % 32 == 0:
            log("serving: plain loop %d/%d done at %.1f s" % (j + 1, num, time.perf_counter() - t0))
    span_p = time.perf_counter() - t0
    torch.cuda.synchronize()
    if not plain:   # batched path only: no reference solves
        lat_p, duals_p, ms_p = [0.0] * num, [1.0] * num, [(0.0, 0, 0)] * num
        span_p = float("nan")

    # ---- server: submit at arrival, poll for completions
    alphas_s = [torch.zeros(c.data.n, dtype=torch.float64, device="cuda") for c in cfgs]
    slots = slots or 2 * torch.cuda.get_device_properties(0).multi_processor_count
    done_at = [None] * num
    res_s = [None] * num
    with S.Server(int(budget_gb * (1 << 30)), slots) as srv:
        tickets = {}
        nxt = 0
        t0 = time.perf_counter()
        last_log, last_t = 0, 0.0
        while nxt < num or tickets:
            now = time.perf_counter() - t0
            while nxt < num and arrivals[nxt] <= now:
                tickets[srv.submit(probs[nxt], params[nxt], alphas_s[nxt])] = nxt
                nxt += 1
            for t in list(tickets):
                got = srv.poll(t)
                if got is not None:
                    j = tickets.pop(t)
                    done_at[j] = time.perf_counter() - t0
                    res_s[j] = got
            done = sum(x is not None for x in done_at)
            if done - last_log >= 32 or time.perf_counter() - t0 > last_t + 20.0:
                last_log, last_t = done, time.perf_counter() - t0
                log("serving: server %d/%d done at %.1f s" % (done, num, last_t))
            time.sleep(0.0002)
        span_s = max(done_at)
        stats = srv.stats()
    torch.cuda.synchronize()
    bad = [j for j in range(num) if res_s[j][0] != S.SVM_OK]
    assert not bad, "server results not OK: %s" % [(j, S.strerror(res_s[j][0])) for j in bad[:5]]
    lat_s = [done_at[j] - arrivals[j] for j in range(num)]
    rel = [abs(res_s[j][1].dual_obj - duals_p[j]) / max(1e-300, abs(duals_p[j])) for j in range(num)]
    its_s = sum(res_s[j][1].iterations for j in range(num))
    if detail is not None:
        for j, c in enumerate(cfgs):
            r = res_s[j][1]
            detail.append({"j": j, "n": c.data.n, "d": c.data.d, "layout": c.data.layout, "C": c.C,
                           "gamma": c.gamma, "arrival": float(arrivals[j]), "done": done_at[j],
                           "team": r.grid_blocks, "iters": r.iterations, "ms_device": r.ms_step,
                           "plain_ms": ms_p[j][0], "plain_iters": ms_p[j][1], "plain_grid": ms_p[j][2]})
    out = {
        "problems": num, "rate_hz": rate_hz,
        "plain": {"solves_per_s": num / span_p, "makespan_s": span_p, "p50_latency_s": _pct(lat_p, 50),
                  "p99_latency_s": _pct(lat_p, 99), "iterations": its_p},
        "batched": {"solves_per_s": num / span_s, "makespan_s": span_s, "p50_latency_s": _pct(lat_s, 50),
                    "p99_latency_s": _pct(lat_s, 99), "iterations": its_s, "slots": slots, "stats": stats},
        "speedup_solves_per_s": span_p / span_s,
        "dual_rel_diff_max": max(rel), "dual_rel_diff_median": float(np.median(rel)),
        "dual_rel_diff_over_1e-6": int(sum(1 for v in rel if v > 1e-6)) if plain else None,
        "plain_workspace": "one preallocated workspace of the largest size",
        "tuned_team_sizes": tuned,
    }
    log("serving: plain %.2f solves/s (p99 %.2f s), batched %.2f solves/s (p99 %.2f s), speedup %.2fx"
        % (out["plain"]["solves_per_s"], out["plain"]["p99_latency_s"], out["batched"]["solves_per_s"],
           out["batched"]["p99_latency_s"], out["speedup_solves_per_s"]))
    return out
