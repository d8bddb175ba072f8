"""Sampled checks at the full problem sizes of the three workloads (sparse binary n = 50,000,
text-like n = 200,000 -- the benchmark's default --, dense mixture n = 500,000), in the launch
configuration bench.py times (automatic grid, lanes per row, residency and head width; FP32
kernel values, FP64 f).  The trained model itself is compared with the oracle's at the sizes
the oracle can train (test_gpu_contract.py); here the checks hold at any size.

The oracle cannot solve these sizes in test time, so the checks are the ones that hold at
any size, with the oracle computing sampled outputs one by one from the GPU's alpha:
- box and equality constraints of the returned alpha;
- f of 256 seeded sample rows against the oracle's sum over the support vectors (abs 1e-4);
- the final KKT condition on those oracle-computed f values against the returned thresholds;
- decision values of 256 held-out queries against the oracle's classifier (abs 1e-4);
- beta, the dual objective and the support-vector counts against their definitions applied
  to the returned alpha and f."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_5161_amd import datagen as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1406_5161_amd import svmhip
    svmhip.lib()
    return svmhip


@pytest.mark.parametrize("which", [2, 3, 4])
def test_full_size_solution_against_sampled_oracle(S, which):
    cfg = g.CONFIGS[which]()
    data = cfg.data
    print("workload", cfg.name, "n", data.n, "d", data.d, flush=True)
    out = S.train_config(cfg)
    assert out.rc == S.SVM_OK, S.strerror(out.rc)
    r = out.result
    print("iterations", r["iterations"], "n_sv", r["n_sv"], "grid", r["grid_blocks"], "ms", r["ms_total"], flush=True)
    a, f = out.alpha, out.f
    y = data.y.astype(np.float64)
    C, eps = cfg.C, cfg.eps
    # box and equality
    assert a.min() >= 0.0 and a.max() <= C
    assert abs(float(np.dot(a, y))) <= 1e-9 * C * data.n
    # counts, beta and dual from their definitions on the returned alpha and f
    free = (a > 0) & (a < C)
    assert r["n_sv"] == int((a > 0).sum()) and r["n_bsv"] == int((a >= C).sum())
    beta = f[free].mean() if free.any() else 0.5 * (r["b_up"] + r["b_low"])
    assert abs(r["beta"] - beta) <= 1e-9 * max(1.0, abs(beta))
    D = a.sum() - 0.5 * np.dot(a * y, f + y)
    assert abs(r["dual_obj"] - D) <= 1e-9 * abs(D)
    # sampled rows: f against the oracle, and the KKT condition on the oracle's values
    rng = np.random.default_rng([1406, 5161, 90, which])
    rows = np.sort(rng.choice(data.n, 256, replace=False))
    sub = data.subset(rows)
    f_ref = O.decision(data, a, 0.0, cfg.gamma, sub) - y[rows]
    err = np.abs(f[rows] - f_ref).max()
    print("max |f - f_oracle| over samples", err, flush=True)
    assert err <= 1e-4
    ar, yr = a[rows], y[rows]
    in_up = ((ar > 0) & (ar < C)) | ((yr > 0) & (ar == 0)) | ((yr < 0) & (ar >= C))
    in_low = ((ar > 0) & (ar < C)) | ((yr > 0) & (ar >= C)) | ((yr < 0) & (ar == 0))
    tol = 2 * eps + 1e-4
    assert np.all(f_ref[in_up] >= r["b_low"] - tol)
    assert np.all(f_ref[in_low] <= r["b_up"] + tol)
    # held-out queries from the same generator
    q = cfg.queries.subset(np.arange(256))
    dv = S.decision_data(data, a, r["beta"], cfg.gamma, q)
    dv_ref = O.decision(data, a, r["beta"], cfg.gamma, q)
    derr = np.abs(dv - dv_ref).max()
    print("max |decision - oracle| over queries", derr, flush=True)
    assert derr <= 1e-4
