"""The whole kernel matrix in the row cache (SVM_FLAG_KERNEL_MATRIX): FP32 kernel values from
the head/tail kernel sums, stored instead of summed, before the loop; every iteration then
reads both kernel rows and K(up, low) from the cache.  The FP32 trajectory is not the one
without the flag, so the trained model is held to the oracle's model (the stored text-like
n = 20,000 model, eq:lagdual / eq:classi) with the FP32 bounds of the default path, and to the
KKT conditions (eq:kktterm) on the oracle's own FP64 recompute of f."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
from test_gpu_contract import FP32_BOUNDS, P, decision_gap, load_case, sv_mismatch  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1406_5161_amd import svmhip
    svmhip.lib()
    return svmhip


@pytest.fixture(scope="module")
def text_case():
    return load_case("cfg3_n20000")


def kkt_gap(cfg, a):
    f = O.f_full(cfg.data, a, cfg.gamma)
    y = cfg.data.y.astype(np.float64)
    free = (a > 0) & (a < cfg.C)
    up = free | ((y > 0) & (a == 0)) | ((y < 0) & (a >= cfg.C))
    low = free | ((y > 0) & (a >= cfg.C)) | ((y < 0) & (a == 0))
    return f, f[low].max() - f[up].min()


def test_kernel_matrix_solve_against_the_oracle_model(S, text_case):
    cfg, ref = text_case
    n = cfg.data.n
    out = S.train_config(cfg, flags=S.SVM_FLAG_KERNEL_MATRIX, cache_mb=(n * n * 4 >> 20) + 16)
    assert out.rc == S.SVM_OK, S.strerror(out.rc)
    r = out.result
    assert r["kernel_matrix"] == 1 and r["cache_rows"] == n
    assert r["cache_both"] == r["iterations"] and r["rows_read"] == 0
    rel = abs(r["dual_obj"] - ref["dual_fresh"]) / abs(ref["dual_fresh"])
    mism = sv_mismatch(out.alpha, ref["alpha"], cfg.C)
    dgap = decision_gap(S, cfg, ref, out.alpha, r["beta"], S.SVM_KERNEL_FP32)
    f, gap = kkt_gap(cfg, out.alpha)
    P("kernel matrix: %.1f ms to fill, iterations %d (oracle %d), dual rel %.2e, sv mismatches %d, decision max "
      "abs %.2e, fresh KKT gap %.3e, max |f - oracle f| %.2e"
      % (r["ms_kmatrix"], r["iterations"], ref["iterations"], rel, mism, dgap, gap, np.abs(out.f - f).max()))
    b = FP32_BOUNDS["cfg3_n20000"]
    assert rel <= 1e-6
    assert mism <= b["sv_mismatch"] * n
    assert dgap <= b["decision"]
    assert gap <= 2 * cfg.eps + 1e-6
    assert np.abs(out.f - f).max() <= 1e-4


def test_kernel_matrix_results_do_not_depend_on_the_grid(S, text_case):
    cfg, _ = text_case
    n = cfg.data.n
    mb = (n * n * 4 >> 20) + 16
    o1 = S.train_config(cfg, flags=S.SVM_FLAG_KERNEL_MATRIX, cache_mb=mb, grid_blocks=8)
    o2 = S.train_config(cfg, flags=S.SVM_FLAG_KERNEL_MATRIX, cache_mb=mb, grid_blocks=37)
    assert o1.rc == S.SVM_OK and o2.rc == S.SVM_OK
    assert o1.result["kernel_matrix"] == 1 and o2.result["kernel_matrix"] == 1
    assert o1.result["iterations"] == o2.result["iterations"]
    assert np.array_equal(o1.alpha, o2.alpha)


def test_kernel_matrix_flag_needs_room_for_every_row(S, text_case):
    """With a cache of fewer than n slots the flag does nothing: the result is the one without it."""
    cfg, _ = text_case
    n = cfg.data.n
    mb = (n * n * 4 >> 20) // 2
    o1 = S.train_config(cfg, flags=S.SVM_FLAG_KERNEL_MATRIX, cache_mb=mb)
    o2 = S.train_config(cfg, cache_mb=mb)
    assert o1.rc == S.SVM_OK and o2.rc == S.SVM_OK
    assert o1.result["kernel_matrix"] == 0 and 0 < o1.result["cache_rows"] < n
    assert o1.result["iterations"] == o2.result["iterations"]
    assert np.array_equal(o1.alpha, o2.alpha)
