"""The contract at sizes the oracle cannot solve inside a test: the HIP library (through its
C-ABI) against the oracle's trained models stored by tests/golden/make_oracle_artifacts.py
(which calls only oracle/).  The stored dataset SHA-256 is checked against the regenerated
input first, so a stored model is only ever compared with the input it was trained on.

Contract: dual objective relative 1e-6; support-vector set identical except samples within
1e-6 of a bound; decision values absolute 1e-4 on held-out queries; the pair sequence
identical where the kernel values are FP64.

FP64 kernel values follow the oracle's trajectory and meet the whole contract.  FP32 kernel
values (the default) leave the oracle's trajectory at the first near-tie that FP32 rounding
flips and stop at another eps-optimal point: the dual still meets 1e-6 (it is unique up to the
eps band, which is far narrower here), while alpha and the decision values differ by up to
the eps band.  Those gaps are measured, printed and held to the bounds below (recorded in the
design notes), not to the 1e-4 contract."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1406_5161_amd import datagen as g

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_oracle_artifacts as A  # noqa: E402

pytestmark = pytest.mark.gpu

# FP32 kernel values (default path) against the oracle's model, about twice the measured gaps
# (support-vector samples outside the 1e-6 band as a fraction of n; decision max abs error on
# the held-out queries).  Measured on one MI355X: sparse binary n = 50,000: pairs part at
# iteration 2,598, 0 support-vector mismatches, decision 2.6e-3; text-like n = 20,000: 7,731,
# 0, 2.6e-4; dense mixture n = 50,000: 4,534, 0, 8.1e-4; the dual within 1.5e-7 in all three.
FP32_BOUNDS = {
    "cfg2_full": {"sv_mismatch": 0.001, "decision": 5e-3},
    "cfg3_n20000": {"sv_mismatch": 0.001, "decision": 1e-3},
    "cfg4_n50000": {"sv_mismatch": 0.001, "decision": 2e-3},
}


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1406_5161_amd import svmhip
    svmhip.lib()
    return svmhip


def P(*a):
    print(*a, flush=True)


def load_case(case):
    ref = A.load(case)
    factory, nq = A.CASES[case]
    cfg = factory()
    assert cfg.data.sha256() == ref["sha256"], "the stored model was trained on another input"
    return cfg, ref


def gpu_train(S, cfg, prec, trace_cap, **kw):
    import torch
    tr = [torch.zeros(trace_cap, dtype=torch.int32, device="cuda"),
          torch.zeros(trace_cap, dtype=torch.int32, device="cuda"),
          torch.zeros(trace_cap, dtype=torch.float64, device="cuda"),
          torch.zeros(trace_cap, dtype=torch.float64, device="cuda")]
    S.svm_debug_set_trace(trace_cap, *tr)
    try:
        out = S.train_config(cfg, kernel_precision=prec, **kw)
    finally:
        S.svm_debug_set_trace(0)
    m = min(out.result["iterations"], trace_cap)
    return out, tr[0][:m].cpu().numpy(), tr[1][:m].cpu().numpy()


def sv_mismatch(a_gpu, a_ref, C, tol=1e-6):
    near = (np.minimum(a_gpu, a_ref) < tol) & (np.maximum(a_gpu, a_ref) > 0)
    near |= (np.maximum(a_gpu, a_ref) > C - tol) & (np.minimum(a_gpu, a_ref) < C)
    diff = ((a_gpu > 0) != (a_ref > 0)) | ((a_gpu >= C) != (a_ref >= C))
    return int(np.sum(diff & ~near))


def first_divergence(iu, il, ref):
    m = min(len(iu), len(ref["i_up"]))
    bad = np.nonzero((iu[:m] != ref["i_up"][:m]) | (il[:m] != ref["i_low"][:m]))[0]
    return int(bad[0]) if len(bad) else -1


def decision_gap(S, cfg, ref, alpha, beta, prec):
    q = cfg.queries.subset(ref["q_rows"].astype(np.int64))
    dv = S.decision_data(cfg.data, alpha, beta, cfg.gamma, q, kernel_precision=prec)
    return float(np.abs(dv - ref["q_dec"]).max())


@pytest.mark.parametrize("case", ["cfg2_full", "cfg3_n20000", "cfg4_n50000"])
def test_fp64_kernel_values_meet_the_whole_contract(S, case):
    cfg, ref = load_case(case)
    P("case", case, cfg.name, "n", cfg.data.n, "oracle iterations", int(ref["iterations"]))
    cap = int(ref["iterations"]) + 16
    out, iu, il = gpu_train(S, cfg, S.SVM_KERNEL_FP64, cap)
    assert out.rc == S.SVM_OK, S.strerror(out.rc)
    r = out.result
    div = first_divergence(iu, il, ref)
    rel = abs(r["dual_obj"] - ref["dual_fresh"]) / abs(ref["dual_fresh"])
    mism = sv_mismatch(out.alpha, ref["alpha"], cfg.C)
    dgap = decision_gap(S, cfg, ref, out.alpha, r["beta"], S.SVM_KERNEL_FP64)
    P("  fp64: iterations %d (oracle %d), first divergence %d, dual rel %.2e, sv mismatches %d, "
      "decision max abs %.2e, max |alpha - oracle| %.2e"
      % (r["iterations"], ref["iterations"], div, rel, mism, dgap, np.abs(out.alpha - ref["alpha"]).max()))
    assert div == -1 and r["iterations"] == int(ref["iterations"])
    assert r["n_recon"] == int(ref["n_recon"])
    assert rel <= 1e-6
    assert mism == 0
    assert dgap <= 1e-4
    np.testing.assert_allclose(out.alpha, ref["alpha"], atol=1e-9)


@pytest.mark.parametrize("case", ["cfg2_full", "cfg3_n20000", "cfg4_n50000"])
def test_fp32_kernel_values_gaps_to_the_oracle_model(S, case):
    cfg, ref = load_case(case)
    cap = 4 * int(ref["iterations"]) + 1000
    out, iu, il = gpu_train(S, cfg, S.SVM_KERNEL_FP32, cap)
    assert out.rc == S.SVM_OK, S.strerror(out.rc)
    r = out.result
    div = first_divergence(iu, il, ref)
    rel = abs(r["dual_obj"] - ref["dual_fresh"]) / abs(ref["dual_fresh"])
    mism = sv_mismatch(out.alpha, ref["alpha"], cfg.C)
    dgap = decision_gap(S, cfg, ref, out.alpha, r["beta"], S.SVM_KERNEL_FP32)
    P("FP32-GAPS %s: iterations %d (oracle %d), first divergence %d, dual rel %.2e, sv mismatches %d of %d "
      "(%.3f%%), decision max abs %.2e, max |alpha - oracle| %.2e, head_cols %d"
      % (case, r["iterations"], ref["iterations"], div, rel, mism, cfg.data.n, 100.0 * mism / cfg.data.n, dgap,
         np.abs(out.alpha - ref["alpha"]).max(), r["head_cols"]))
    b = FP32_BOUNDS[case]
    assert rel <= 1e-6
    assert mism <= b["sv_mismatch"] * cfg.data.n
    assert dgap <= b["decision"]


def test_fp32_text_like_rows_from_hbm_many_workgroups(S):
    """Text-like rows (CSR with values, d = 47,000) at n = 20,000: the SMO loop on 24
    workgroups with the rows streamed from HBM (LDS holds only per-row state), 16 lanes per
    row; the model meets the dual contract against the oracle's model and the KKT conditions
    on a fresh FP64 recompute of f by the oracle."""
    cfg, ref = load_case("cfg3_n20000")
    out = S.train_config(cfg, grid_blocks=24, lanes_per_row=16, flags=S.SVM_FLAG_NO_LDS_PAYLOAD)
    assert out.rc == S.SVM_OK, S.strerror(out.rc)
    mode, grid, lpr = S.svm_debug_step_info()
    assert (mode, grid, lpr) == (1, 24, 16)
    r = out.result
    rel = abs(r["dual_obj"] - ref["dual_fresh"]) / abs(ref["dual_fresh"])
    a = out.alpha
    y = cfg.data.y.astype(np.float64)
    assert a.min() >= 0.0 and a.max() <= cfg.C and abs(float(np.dot(a, y))) <= 1e-9 * cfg.C * cfg.data.n
    f = O.f_full(cfg.data, a, cfg.gamma)
    free = (a > 0) & (a < cfg.C)
    up = free | ((y > 0) & (a == 0)) | ((y < 0) & (a >= cfg.C))
    low = free | ((y > 0) & (a >= cfg.C)) | ((y < 0) & (a == 0))
    gap = f[low].max() - f[up].min()
    P("rows from HBM: iterations %d, dual rel %.2e, fresh KKT gap %.3e, max |f - oracle f| %.2e"
      % (r["iterations"], rel, gap, np.abs(out.f - f).max()))
    assert rel <= 1e-6
    assert gap <= 2 * cfg.eps + 1e-6
    assert np.abs(out.f - f).max() <= 1e-4   # f_i + y_i is a decision value: the decision tolerance
