"""Kernel-row cache of the SMO loop (rows streamed from HBM): slot s mod S holds the kernel
row K(s, .) the loop computed when s was last in the working pair, and an iteration whose two
rows are cached reads no row data.  The cached values are the loop's own, so alpha, f, the
pair sequence and every count equal the run without the cache bit for bit, with the cache
holding every row (S = n) or few (S < n: slot collisions, including both rows of a pair in
one slot), for dense rows, wide CSR rows (slot map) and narrower CSR rows (column table), in
FP32 and FP64."""
import numpy as np
import pytest

from paper_1406_5161_amd import datagen as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1406_5161_amd import svmhip
    svmhip.lib()
    return svmhip


def sub(cfg, n):
    cfg.data = cfg.data.subset(np.arange(n))
    return cfg


def with_values(cfg, seed=4):
    r = np.random.default_rng([1406, 5161, 97, seed])
    d = cfg.data
    val = np.exp(0.5 * r.standard_normal(len(d.val))).astype(np.float32)
    cfg.data = g.SvmData(d.name + "_vals", d.n, d.d, "csr", d.y, row_ptr=d.row_ptr, col=d.col, val=val)
    return cfg


def run(S, cfg, prec, cache_mb, grid):
    import torch
    cap = 400_000
    tr = [torch.zeros(cap, dtype=torch.int32, device="cuda") for _ in range(2)] + \
         [torch.zeros(cap, dtype=torch.float64, device="cuda") for _ in range(2)]
    S.svm_debug_set_trace(cap, *tr)
    try:
        out = S.train_config(cfg, kernel_precision=prec, cache_mb=cache_mb, grid_blocks=grid,
                             flags=S.SVM_FLAG_NO_LDS_PAYLOAD | S.SVM_FLAG_NO_BITSETS)
    finally:
        S.svm_debug_set_trace(0)
    m = min(out.result["iterations"], cap)
    return out, tr[0][:m].cpu().numpy(), tr[1][:m].cpu().numpy()


CASES = [
    ("dense_mixture", lambda: sub(g.config4(heuristic=g.EARLIEST), 6000)),
    ("text_like", lambda: sub(g.config3(n=20_000), 6000)),
    ("column_table_values", lambda: with_values(sub(g.config2(), 5000))),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_cache_changes_nothing_but_the_bytes_read(S, case, prec):
    name, make = case
    cfg = make()
    n = cfg.data.n
    base, iu0, il0 = run(S, cfg, prec, 0, 16)
    assert base.rc == S.SVM_OK and base.result["cache_rows"] == 0
    vb = 8 if prec else 4
    full_mb = -(-n * n * vb // (1 << 20))             # every row has its own slot
    small_mb = max(1, n * (n // 7) * vb // (1 << 20))  # about n / 7 slots: collisions
    for mb in (full_mb, small_mb):
        out, iu, il = run(S, cfg, prec, mb, 16)
        r = out.result
        print(name, "prec", prec, "cache_mb", mb, "slots", r["cache_rows"], "iterations", r["iterations"],
              "both rows cached", r["cache_both"], "rows read", r["rows_read"], "of", r["rows_streamed"], flush=True)
        assert out.rc == S.SVM_OK
        assert r["cache_rows"] > 0 and r["cache_values"] > 0
        if mb == full_mb:   # reuse comes about n iterations later: only a full cache keeps it
            assert r["cache_both"] > 0 and r["rows_read"] < r["rows_streamed"]
        assert r["iterations"] == base.result["iterations"] and r["n_recon"] == base.result["n_recon"]
        assert np.array_equal(iu, iu0) and np.array_equal(il, il0)
        assert np.array_equal(out.alpha, base.alpha) and np.array_equal(out.f, base.f)
        assert r["dual_obj"] == base.result["dual_obj"]


def test_cache_is_ignored_for_rows_in_lds(S):
    cfg = sub(g.config2(), 3000)
    out = S.train_config(cfg, cache_mb=64)
    assert out.rc == S.SVM_OK and out.result["cache_rows"] == 0 and out.result["cache_values"] == 0
