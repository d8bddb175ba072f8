"""Several problems over one sample set (svm_train_shared) against the same problems solved one
after another (svm_train), on the sparse-binary workload at full size (n = 50,000, d = 300,
bitset rows): k = 1, 2, 4, 8 problems, problem 0 the workload's own labels and the others
seeded relabelings (10 % of the labels flipped, a one-vs-rest-like family over the same
rows) with C and gamma from a small grid; no shrinking (the shared pass runs Alg. 2).

    python -m paper_1406_5161_amd.shared_bench [--ks 1,2,4,8] [--n 50000]

Prints one JSON line per k: device time of the shared launches and of the k separate loops,
problem-iterations per second of each, and the row bytes read per problem-iteration (each
row's bitset, 4 bytes per word, read once per shared iteration for all live problems).
Every shared problem's alpha is checked equal to its own run's.
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import datagen as g


def relabel(y, seed, frac=0.1):
    r = np.random.default_rng([1406, 5161, 98, seed])
    z = y.copy()
    idx = r.choice(len(z), int(frac * len(z)), replace=False)
    z[idx] = -z[idx]
    return z


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ks", default="1,2,4,8")
    ap.add_argument("--n", type=int, default=50_000)
    a = ap.parse_args()
    import torch
    from . import svmhip as S
    S.lib()
    cfg = g.config2(n=a.n)
    data = cfg.data
    dp = S.to_device(data)
    grid = [(1.0, 1.0), (0.5, 1.0), (2.0, 2.0), (1.0, 0.5)]
    wpr = ((data.d + 31) // 32 + 3) // 4 * 4
    for k in [int(x) for x in a.ks.split(",")]:
        labels = [data.y if p == 0 else relabel(data.y, p) for p in range(k)]
        ys = [torch.from_numpy(np.ascontiguousarray(y, np.int8)).cuda() for y in labels]
        params = [S.make_params(cfg.C * grid[p % 4][0], cfg.gamma * grid[p % 4][1], cfg.eps) for p in range(k)]
        alphas = [torch.zeros(data.n, dtype=torch.float64, device="cuda") for _ in range(k)]
        ws = torch.empty(S.svm_train_shared_workspace_size(dp, ys, params), dtype=torch.uint8, device="cuda")
        rc, res = S.svm_train_shared(dp, ys, params, alphas, workspace=ws)   # warm-up
        assert rc == S.SVM_OK, S.strerror(rc)
        rc, res = S.svm_train_shared(dp, ys, params, alphas, workspace=ws)
        assert rc == S.SVM_OK, S.strerror(rc)
        torch.cuda.synchronize()
        shared_ms = res[0].ms_step
        iters = sum(r.iterations for r in res)
        rows = res[0].rows_streamed
        solo_ms, solo_iters = 0.0, 0
        for p in range(k):
            one = g.SvmData("solo", data.n, data.d, "csr", labels[p], row_ptr=data.row_ptr, col=data.col,
                            val=data.val)
            dq = S.to_device(one)
            al = torch.zeros(data.n, dtype=torch.float64, device="cuda")
            wq = torch.empty(S.svm_train_workspace_size(dq, params[p]), dtype=torch.uint8, device="cuda")
            S.svm_train(dq, params[p], al, workspace=wq)
            rc, r = S.svm_train(dq, params[p], al, workspace=wq)
            assert rc == S.SVM_OK
            torch.cuda.synchronize()
            assert np.array_equal(al.cpu().numpy(), alphas[p].cpu().numpy()), "shared result differs from its own run"
            solo_ms += r.ms_step
            solo_iters += r.iterations
        print(json.dumps({
            "k": k, "n": data.n, "d": data.d, "problem_iterations": iters,
            "shared_loop_ms": shared_ms, "separate_loops_ms": solo_ms,
            "shared_iterations_per_s": iters / (shared_ms * 1e-3),
            "separate_iterations_per_s": solo_iters / (solo_ms * 1e-3),
            "speedup": solo_ms / shared_ms,
            "row_bytes_per_problem_iteration": 4.0 * wpr * rows / iters,
            "row_bytes_per_iteration_separate": 4.0 * wpr * data.n,
            "launches": res[0].n_launches, "grid": res[0].grid_blocks}), flush=True)


if __name__ == "__main__":
    main()
