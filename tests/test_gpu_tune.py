"""The shape autotuner: svm_autotune times candidate launch shapes on the device and later
automatic solves of the same class use the fastest; the shape never changes alpha or f."""
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
    yield svmhip
    svmhip.svm_autotune_reset()


def test_grid_tuning_keeps_results(S):
    S.svm_autotune_reset()
    cfg = g.config2()
    cfg.data = cfg.data.subset(np.arange(20_000))
    before = S.train_config(cfg)
    g0 = S.svm_debug_step_info()[1]
    rc, info = S.svm_autotune(S.to_device(cfg.data), S.params_for(cfg), S.SVM_TUNE_GRID)
    assert rc == S.SVM_OK
    print("rule grid", g0, "tuned", info, flush=True)
    assert len(info["candidates"]) >= 2 and all(c["us_per_iter"] > 0 for c in info["candidates"])
    assert info["chosen"] == min(info["candidates"], key=lambda c: c["us_per_iter"])["shape"]
    after = S.train_config(cfg)
    assert S.svm_debug_step_info()[1] == info["chosen"]
    assert np.array_equal(before.alpha, after.alpha) and np.array_equal(before.f, after.f)
    assert before.result["iterations"] == after.result["iterations"]


def test_team_tuning_keeps_results(S):
    import torch
    S.svm_autotune_reset()
    cfg = g.config1(n=6000, d=128)
    dp = S.to_device(cfg.data)
    p = S.params_for(cfg)

    def batch():
        a = torch.zeros(cfg.data.n, dtype=torch.float64, device="cuda")
        rc, res = S.svm_train_batch([dp], [p], [a])
        assert rc == S.SVM_OK
        return a.cpu().numpy(), res[0]

    a0, r0 = batch()
    rc, info = S.svm_autotune(dp, p, S.SVM_TUNE_TEAM)
    assert rc == S.SVM_OK
    print("rule team", r0.grid_blocks, "tuned", info, flush=True)
    a1, r1 = batch()
    assert r1.grid_blocks == info["chosen"]
    assert np.array_equal(a0, a1) and r0.iterations == r1.iterations
