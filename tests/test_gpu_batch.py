"""GPU tests of the batched solver (svm_train_batch) and the serving loop (svm_server_*).

A team of workgroups solves each problem; selection merges are exact and every row's f update
is its own, so alpha and f must be bit-identical alone, in a mix and for any team size; with
FP64 kernel values each problem follows the FP64 oracle's trajectory."""
import time

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


def mixed_problems(k=6, seed=0):
    """Small problems of the serving mix: dense d=20, dense d=128, CSR d=300 at 12%."""
    out = []
    for j in range(k):
        r = np.random.default_rng([1406, 5161, 77, seed, j])
        n = int(r.integers(600, 2500))
        kind = j % 3
        if kind == 0:
            data = g.gen_blobs(n, 20, r)
        elif kind == 1:
            data = g.gen_blobs(n, 128, r)
        else:
            data = g.gen_sparse_binary(n, 300, 0.12, r)
        C = [0.1, 1.0, 10.0][j % 3]
        gamma = float(10 ** r.uniform(-2.5, -1.0))
        heur = g.LAZY if j % 2 == 0 else g.EARLIEST
        out.append(g.SvmConfig("mix%d" % j, data, C=C, gamma=gamma, eps=1e-3, shrink_mode=g.SHRINK_MULTI,
                               shrink_kind=heur[0], shrink_param=heur[1]))
    return out


def run_batch(S, cfgs, prec, team=0):
    import torch
    probs = [S.to_device(c.data) for c in cfgs]
    params = [S.params_for(c, kernel_precision=prec, grid_blocks=team) for c in cfgs]
    alphas = [torch.zeros(c.data.n, dtype=torch.float64, device="cuda") for c in cfgs]
    fs = [torch.zeros(c.data.n, dtype=torch.float64, device="cuda") for c in cfgs]
    rc, res = S.svm_train_batch(probs, params, alphas, fs)
    torch.cuda.synchronize()
    return rc, res, [a.cpu().numpy() for a in alphas], [f.cpu().numpy() for f in fs]


def test_batch_fp64_follows_oracle(S):
    cfgs = mixed_problems(6, seed=1)
    rc, res, alphas, fs = run_batch(S, cfgs, S.SVM_KERNEL_FP64)
    assert rc == S.SVM_OK, S.strerror(rc)
    for c, r, a, f in zip(cfgs, res, alphas, fs):
        ref = O.train_config(c)
        print(c.name, c.data.n, c.data.d, "iters", r.iterations, ref.iterations, flush=True)
        assert r.iterations == ref.iterations
        assert r.n_recon == ref.n_recon
        np.testing.assert_allclose(a, ref.alpha, atol=1e-9)
        np.testing.assert_allclose(f, ref.f, atol=1e-9)
        D = O.dual(c.data, a, c.gamma)
        assert abs(D - O.dual(c.data, ref.alpha, c.gamma)) <= 1e-6 * abs(D)
        assert abs(r.beta - ref.beta) <= 1e-4


def team_problems():
    """Problems large enough for automatic teams of 2-3 workgroups (one of each kind), with
    shrink passes on every one (earliest schedule).  Their oracle trajectories do not change when
    every kernel value moves by one ulp, so the device exp (not correctly rounded in every case,
    unlike the host's) cannot flip a near-tie in the selection; an arbitrary problem can diverge
    that way after a few hundred iterations and still meets the dual tolerance."""
    out = []
    for j, (seed, n, kind) in enumerate([(10, 6500, 0), (1, 6100, 1), (2, 3500, 2)]):
        r = np.random.default_rng([1406, 5161, 78, seed])
        data = (g.gen_blobs(n, 20, r) if kind == 0 else g.gen_blobs(n, 128, r) if kind == 1
                else g.gen_sparse_binary(n, 300, 0.12, r))
        out.append(g.SvmConfig("team%d" % j, data, C=[1.0, 10.0, 1.0][j], gamma=[0.05, 0.01, 1 / 300][j], eps=1e-3,
                               shrink_mode=g.SHRINK_MULTI, shrink_kind=g.EARLIEST[0], shrink_param=g.EARLIEST[1]))
    return out


def test_batch_teams_fp64_follow_oracle(S):
    cfgs = team_problems()
    rc, res, alphas, fs = run_batch(S, cfgs, S.SVM_KERNEL_FP64)
    assert rc == S.SVM_OK, S.strerror(rc)
    for c, r, a, f in zip(cfgs, res, alphas, fs):
        ref = O.train_config(c)
        print(c.name, c.data.n, "team", r.grid_blocks, "iters", r.iterations, ref.iterations, flush=True)
        assert r.grid_blocks >= 2
        assert r.iterations == ref.iterations and r.n_recon == ref.n_recon
        assert r.shrink_passes == ref.shrink_passes and r.shrunk_total == ref.shrunk_total
        assert ref.shrink_passes > 0
        np.testing.assert_allclose(a, ref.alpha, atol=1e-9)
        np.testing.assert_allclose(f, ref.f, atol=1e-9)
        assert abs(r.dual_obj - ref.dual_obj) <= 1e-6 * abs(ref.dual_obj)
        assert abs(r.beta - ref.beta) <= 1e-4


def test_batch_alpha_f_do_not_depend_on_team_size(S):
    cfgs = team_problems()
    base = run_batch(S, cfgs, S.SVM_KERNEL_FP32, team=1)
    assert base[0] == S.SVM_OK
    for team in (2, 5, 16, 40):
        rc, res, alphas, fs = run_batch(S, cfgs, S.SVM_KERNEL_FP32, team=team)
        assert rc == S.SVM_OK
        for j in range(len(cfgs)):
            assert res[j].grid_blocks == team
            assert res[j].iterations == base[1][j].iterations
            assert np.array_equal(alphas[j], base[2][j]) and np.array_equal(fs[j], base[3][j])
            assert abs(res[j].dual_obj - base[1][j].dual_obj) <= 1e-9 * abs(base[1][j].dual_obj)


def test_batch_result_is_identical_alone_and_in_the_mix(S):
    cfgs = mixed_problems(9, seed=2)
    rc, res, alphas, fs = run_batch(S, cfgs, S.SVM_KERNEL_FP32)
    assert rc == S.SVM_OK
    for j in (0, 4, 8):
        rc1, res1, a1, f1 = run_batch(S, [cfgs[j]], S.SVM_KERNEL_FP32)
        assert rc1 == S.SVM_OK
        assert np.array_equal(a1[0], alphas[j]) and np.array_equal(f1[0], fs[j])
        assert res1[0].iterations == res[j].iterations and res1[0].beta == res[j].beta


def test_batch_fp32_matches_single_problem_solver(S):
    """The batched loop and the plain one-problem loop run the same method: same dual to 1e-6."""
    cfgs = mixed_problems(3, seed=3)
    rc, res, alphas, fs = run_batch(S, cfgs, S.SVM_KERNEL_FP32)
    assert rc == S.SVM_OK
    for c, r, a in zip(cfgs, res, alphas):
        single = S.train_config(c)
        D1, D2 = O.dual(c.data, a, c.gamma), O.dual(c.data, single.alpha, c.gamma)
        assert abs(D1 - D2) <= 1e-6 * abs(D2)


def test_server_continuous_batching_admission_and_identity(S):
    import torch
    cfgs = mixed_problems(8, seed=4)
    # reference: each problem alone through the batched entry point
    alone = [run_batch(S, [c], S.SVM_KERNEL_FP32)[2][0] for c in cfgs]
    # a budget that holds about two problems' solver state forces deferral
    budget = 2 * max(c.data.n for c in cfgs) * (8 * 4 + 4 * 128 + 16)
    probs = [S.to_device(c.data) for c in cfgs]
    alphas = [torch.zeros(c.data.n, dtype=torch.float64, device="cuda") for c in cfgs]
    torch.cuda.synchronize()
    with S.Server(budget, max_slots=3) as srv:
        tickets = []
        for c, p, a in zip(cfgs, probs, alphas):
            tickets.append(srv.submit(p, S.params_for(c), a))
            time.sleep(0.002)
            st = srv.stats()
            assert st["in_flight"] <= 3
        assert srv.drain() == S.SVM_OK
        st = srv.stats()
        print("server stats", st, flush=True)
        assert st["completed"] == len(cfgs)
        assert st["deferred"] >= 1
        for t in tickets:
            rc, r = srv.poll(t)
            assert rc == S.SVM_OK and r.iterations > 0
    torch.cuda.synchronize()
    for a, ref in zip(alphas, alone):
        assert np.array_equal(a.cpu().numpy(), ref)


def test_server_rejects_bad_problem_and_keeps_serving(S):
    import torch
    good = mixed_problems(2, seed=5)
    bad = g.SvmData("oneclass", 500, 20, "dense", np.ones(500, np.int8), x=good[0].data.x[:500].copy())
    # device buffers before the server starts: its loop holds all but a few compute units
    pb = S.to_device(bad)
    ab = torch.zeros(500, dtype=torch.float64, device="cuda")
    pg = [S.to_device(c.data) for c in good]
    ag = [torch.zeros(c.data.n, dtype=torch.float64, device="cuda") for c in good]
    torch.cuda.synchronize()
    with S.Server(1 << 30, max_slots=4) as srv:
        tb = srv.submit(pb, S.make_params(1.0, 0.1), ab)
        tg = [srv.submit(p, S.params_for(c), a) for p, c, a in zip(pg, good, ag)]
        assert srv.drain() == S.SVM_OK
        assert srv.poll(tb)[0] == S.SVM_EONECLASS
        for t in tg:
            assert srv.poll(t)[0] == S.SVM_OK
