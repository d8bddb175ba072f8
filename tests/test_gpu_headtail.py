"""Kernel sums over wide CSR rows with the frequent columns as dense rows on the matrix cores
and the rest as a sparse tail (reconstruction and recompute of Alg. 6, the classifier of
eq:classi), against the FP64 oracle.  Tiles of 64, 32 and 16 target rows (by how many tail
nonzeros a tile holds), the fallback to the sparse slot-map sums beyond that, ragged tiles,
split support-vector lists, and training with every head width."""
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


def P(*a):
    print(*a, flush=True)


def uniform_csr(n, d, nnz_row, seed, name):
    """Rows of exactly nnz_row columns drawn uniformly (so nearly every nonzero is in the tail),
    lognormal values, unit rows, random labels."""
    r = np.random.default_rng([1406, 5161, 96, seed])
    cols = np.sort(np.stack([r.choice(d, nnz_row, replace=False) for _ in range(n)]), axis=1).astype(np.int32)
    val = np.exp(0.5 * r.standard_normal((n, nnz_row)))
    val /= np.sqrt((val * val).sum(axis=1, keepdims=True))
    y = np.where(r.random(n) < 0.5, 1, -1).astype(np.int8)
    rp = (np.arange(n + 1) * nnz_row).astype(np.int32)
    return g.SvmData(name, n, d, "csr", y, row_ptr=rp, col=cols.ravel(), val=val.ravel().astype(np.float32))


@pytest.mark.parametrize("nq", [64 * 5 + 13, 64, 1])
def test_text_like_decision_on_the_dense_head(S, nq):
    cfg = g.config3(n=20_000)
    data = cfg.data.subset(np.arange(2600))
    rng = np.random.default_rng(31)
    alpha = np.where(rng.random(data.n) < 0.5, rng.uniform(0, cfg.C, data.n), 0.0)
    q = cfg.queries.subset(np.arange(nq))
    dv = S.decision_data(data, alpha, -0.125, cfg.gamma, q)
    dref = O.decision(data, alpha, -0.125, cfg.gamma, q)
    err = float(np.abs(dv - dref).max())
    P("nq", nq, "max |decision - oracle|", err)
    assert err <= 1e-4


@pytest.mark.parametrize("nnz_row,label", [(100, "tiles_of_32"), (200, "tiles_of_16"), (300, "slot_fallback")])
def test_long_tails_shrink_the_tile_or_fall_back(S, nnz_row, label):
    """64 rows of 100 tail nonzeros exceed the LDS table (4,096), so tiles hold 32 rows; 200
    nonzeros need tiles of 16; 300 exceed even those, and the sums take the slot-map path."""
    train = uniform_csr(900, 20_000, nnz_row, nnz_row, "train")
    q = uniform_csr(150, 20_000, nnz_row, nnz_row + 1, "queries")
    rng = np.random.default_rng(nnz_row)
    alpha = rng.uniform(0, 2.0, train.n)
    dv = S.decision_data(train, alpha, 0.25, 0.7, q)
    dref = O.decision(train, alpha, 0.25, 0.7, q)
    err = float(np.abs(dv - dref).max())
    P(label, "max |decision - oracle|", err)
    assert err <= 1e-4


@pytest.fixture(scope="module")
def text_problem():
    cfg = g.config3(n=20_000)
    cfg.data = cfg.data.subset(np.arange(6000))
    ref = O.train_config(cfg)
    return cfg, ref, O.dual(cfg.data, ref.alpha, cfg.gamma)


@pytest.mark.parametrize("H", [32, 64, 128, -1])
def test_training_with_each_head_width(S, text_problem, H):
    """Earliest shrinking with multi reconstruction on text-like rows: reconstruction and the
    closing recompute run on the dense head (H columns) plus the tail, or (H = -1) on the
    slot-map sums only; every width meets the dual contract, its f equals the oracle's sum
    over the support vectors, and a second run is bit-identical (the tail dots are exact
    fixed-point sums, so their order does not matter)."""
    cfg, ref, D_ref = text_problem
    out = S.train_config(cfg, head_cols=H)
    assert out.rc == S.SVM_OK, S.strerror(out.rc)
    r = out.result
    assert r["n_recon"] >= 1
    if H > 0:
        assert r["ksum_mfma"] == 2 and r["head_cols"] == H
    else:
        assert r["ksum_mfma"] == 0 and r["head_cols"] == 0
    rel = abs(O.dual(cfg.data, out.alpha, cfg.gamma) - D_ref) / abs(D_ref)
    rows = np.random.default_rng(7).choice(cfg.data.n, 400, replace=False)
    f_ref = O.decision(cfg.data, out.alpha, 0.0, cfg.gamma, cfg.data.subset(rows)) - cfg.data.y[rows]
    ferr = float(np.abs(out.f[rows] - f_ref).max())
    P("H", H, "iterations", r["iterations"], "(oracle %d)" % ref.iterations, "dual rel %.2e" % rel,
      "max |f - oracle| %.2e" % ferr, "recon ms %.1f" % r["ms_recon"])
    assert rel <= 1e-6
    assert ferr <= 1e-5
    again = S.train_config(cfg, head_cols=H)
    assert np.array_equal(again.alpha, out.alpha) and np.array_equal(again.f, out.f)


def test_head_cols_argument_is_checked(S):
    cfg = g.config3(n=20_000)
    cfg.data = cfg.data.subset(np.arange(300))
    assert S.train_config(cfg, head_cols=48).rc == S.SVM_EINVAL
