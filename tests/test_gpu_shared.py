"""Several training problems over one sample set in lockstep (svm_train_shared): one-vs-rest
style relabelings and C / gamma grids.  Each problem's alpha and f equal those of its own
svm_train run bit for bit (same arithmetic, same trajectory, same closing recompute), in FP32
and FP64, for binary CSR rows (bitsets) and dense rows, alone and among up to 8 problems that
converge at different iterations; with FP64 kernel values each also follows the oracle's
trajectory to its iteration count and alpha."""
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


def relabel(y, seed, frac=0.1):
    """Another labeling of the same samples: a seeded fraction of the labels flipped."""
    r = np.random.default_rng([1406, 5161, 98, seed])
    z = y.copy()
    idx = r.choice(len(z), int(frac * len(z)), replace=False)
    z[idx] = -z[idx]
    return z


def problems(kind, k):
    if kind == "binary":
        cfg = g.config2()
        data = cfg.data.subset(np.arange(6000))
        base = dict(C=1.0, gamma=1.0 / 300)
    else:
        cfg = g.config1(n=6000)
        data = cfg.data
        base = dict(C=1.0, gamma=0.05)
    grid = [(1.0, 1.0), (0.5, 1.0), (2.0, 2.0), (1.0, 0.5)]
    out = []
    for p in range(k):
        y = data.y if p == 0 else relabel(data.y, p)
        cm, gm = grid[p % len(grid)]
        out.append((y, base["C"] * cm, base["gamma"] * gm))
    return data, out


def solo(S, data, y, C, gamma, prec):
    d = g.SvmData("solo", data.n, data.d, data.layout, y, x=data.x, row_ptr=data.row_ptr, col=data.col,
                  val=data.val)
    return S.train_data(d, C, gamma, 1e-3, kernel_precision=prec)


def shared(S, data, probs, prec):
    import torch
    dp = S.to_device(data)
    ys = [torch.from_numpy(np.ascontiguousarray(y, np.int8)).cuda() for y, _, _ in probs]
    params = [S.make_params(C, gam, 1e-3, kernel_precision=prec) for _, C, gam in probs]
    alphas = [torch.zeros(data.n, dtype=torch.float64, device="cuda") for _ in probs]
    fs = [torch.zeros(data.n, dtype=torch.float64, device="cuda") for _ in probs]
    rc, res = S.svm_train_shared(dp, ys, params, alphas, fs)
    torch.cuda.synchronize()
    return rc, res, [a.cpu().numpy() for a in alphas], [f.cpu().numpy() for f in fs]


@pytest.mark.parametrize("k", [1, 3, 8])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("kind", ["binary", "dense"])
def test_each_problem_equals_its_own_run(S, kind, prec, k):
    data, probs = problems(kind, k)
    rc, res, alphas, fs = shared(S, data, probs, prec)
    assert rc == S.SVM_OK, S.strerror(rc)
    for p, (y, C, gamma) in enumerate(probs):
        one = solo(S, data, y, C, gamma, prec)
        assert one.rc == S.SVM_OK
        r = res[p]
        print(kind, "prec", prec, "k", k, "problem", p, "iterations", r.iterations, "(alone %d)" % one.result["iterations"],
              "launches", r.n_launches, flush=True)
        assert r.iterations == one.result["iterations"]
        assert np.array_equal(alphas[p], one.alpha) and np.array_equal(fs[p], one.f)
        assert r.dual_obj == one.result["dual_obj"] and r.beta == one.result["beta"]


def test_fp64_problems_follow_the_oracle(S):
    data, probs = problems("binary", 3)
    rc, res, alphas, _ = shared(S, data, probs, 1)
    assert rc == S.SVM_OK
    for p, (y, C, gamma) in enumerate(probs):
        d = g.SvmData("o", data.n, data.d, "csr", y, row_ptr=data.row_ptr, col=data.col, val=data.val)
        ref = O.train(d, C, gamma, 1e-3)
        assert res[p].iterations == ref.iterations
        np.testing.assert_allclose(alphas[p], ref.alpha, atol=1e-9)


def test_shared_rejects_shrinking_and_mixed_precision(S):
    import torch
    data, probs = problems("dense", 2)
    dp = S.to_device(data)
    ys = [torch.from_numpy(np.ascontiguousarray(y, np.int8)).cuda() for y, _, _ in probs]
    a = [torch.zeros(data.n, dtype=torch.float64, device="cuda") for _ in probs]
    p_shrink = [S.make_params(1.0, 0.05, shrink_mode=2, shrink_kind=0, shrink_param=2.0)] * 2
    assert S.svm_train_shared(dp, ys, p_shrink, a)[0] == S.SVM_EUNSUPPORTED
    p_mixed = [S.make_params(1.0, 0.05, kernel_precision=0), S.make_params(1.0, 0.05, kernel_precision=1)]
    assert S.svm_train_shared(dp, ys, p_mixed, a)[0] == S.SVM_EUNSUPPORTED
