"""Seeded synthetic training problems shaped like the paper's workloads.

The paper evaluates on census, web, mushroom, handwritten-digit and IJCNN data
(Section "Datasets", Table 2).  None of those files is available, so every
problem here is generated from a fixed seed with the shapes, densities and
value distributions of those families:

* dense overlapping Gaussian blobs (digit / feature data),
* sparse binary rows with Zipf-distributed column ids (census / web / mushrooms),
* long sparse tf-idf-like rows, L2-normalised (text categorisation),
* a dense 8-component Gaussian mixture with many bounded support vectors,
* a Poisson stream of mixed problems for the serving path.

This module holds data generation only: no kernel values, no SMO arithmetic.
Both the FP64 CPU oracle and the GPU path are fed from it.  Every generator
draws from ``numpy.random.default_rng([1406, 5161, cfg, sub])`` (PCG64), builds
values in float64 and rounds them to float32 exactly once, so the oracle (which
reads the float32 values in float64) and the GPU see identical inputs.

Readings of details the workload descriptions leave open (recorded here and in
the design notes): the teacher has 10% non-zero N(0,1) coordinates and is
thresholded at its median (balanced classes); sparse row lengths follow
Binomial(d, density) or Poisson(mean) clipped to [1, d]; columns are drawn by
weighted sampling without replacement from a truncated Zipf(1.1) law and then
relabelled by a seeded permutation; tf-idf-like values are exp(N(0, 0.5^2));
the 8 mixture means lie on one seeded unit direction, spaced 1.0 apart.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# shrink_mode values of the C-ABI (none / single reconstruction / multi)
SHRINK_NONE, SHRINK_SINGLE, SHRINK_MULTI = 0, 1, 2
# shrink_kind values: fixed iteration count ("random: k") or fraction of n ("numsamples")
KIND_FIXED, KIND_FRACTION = 0, 1

# The two ends of the heuristic spectrum of Table 3: "earliest" shrinks every
# 2 iterations (random: 2, aggressive), "lazy" first shrinks after n/2
# iterations (numsamples: 50%, conservative).
EARLIEST = (KIND_FIXED, 2.0)
LAZY = (KIND_FRACTION, 0.5)


def rng_for(cfg: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([1406, 5161, int(cfg), int(sub)])


@dataclass
class SvmData:
    """One labelled sample set.  Dense: ``x`` is float32 (n, d) row-major.
    CSR: ``row_ptr`` int32 (n+1), ``col`` int32 sorted unique per row, ``val`` float32."""
    name: str
    n: int
    d: int
    layout: str
    y: np.ndarray
    x: Optional[np.ndarray] = None
    row_ptr: Optional[np.ndarray] = None
    col: Optional[np.ndarray] = None
    val: Optional[np.ndarray] = None

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.layout == "csr" else self.n * self.d

    def arrays(self):
        if self.layout == "dense":
            return {"x": self.x, "y": self.y}
        return {"row_ptr": self.row_ptr, "col": self.col, "val": self.val, "y": self.y}

    def sha256(self) -> str:
        h = hashlib.sha256()
        for k, a in sorted(self.arrays().items()):
            h.update(k.encode())
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def subset(self, rows: np.ndarray, name: str | None = None) -> "SvmData":
        rows = np.asarray(rows, dtype=np.int64)
        if self.layout == "dense":
            return SvmData(name or self.name, len(rows), self.d, "dense", self.y[rows].copy(),
                           x=np.ascontiguousarray(self.x[rows]))
        lens = (self.row_ptr[rows + 1] - self.row_ptr[rows]).astype(np.int64)
        rp = np.zeros(len(rows) + 1, np.int64)
        np.cumsum(lens, out=rp[1:])
        idx = np.concatenate([np.arange(self.row_ptr[r], self.row_ptr[r + 1]) for r in rows]) \
            if len(rows) else np.zeros(0, np.int64)
        return SvmData(name or self.name, len(rows), self.d, "csr", self.y[rows].copy(),
                       row_ptr=rp.astype(np.int32), col=self.col[idx].copy(), val=self.val[idx].copy())

    def to_dense(self) -> np.ndarray:
        if self.layout == "dense":
            return self.x
        out = np.zeros((self.n, self.d), np.float32)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        out[rows, self.col] = self.val
        return out


@dataclass
class SvmConfig:
    """A training problem plus its hyper-parameters (C, gamma = 1/(2 sigma^2), eps)
    and shrinking heuristic."""
    name: str
    data: SvmData
    C: float
    gamma: float
    eps: float = 1e-3
    shrink_mode: int = SHRINK_NONE
    shrink_kind: int = KIND_FIXED
    shrink_param: float = 0.0
    max_iter: int = 50_000_000
    queries: Optional[SvmData] = None
    extra: dict = field(default_factory=dict)


# ---------------------------------------------------------------- primitives

def _balanced_labels(n: int, rng: np.random.Generator) -> np.ndarray:
    y = np.ones(n, np.int8)
    y[n // 2:] = -1
    rng.shuffle(y)
    return y


def _teacher_labels(score: np.ndarray, flip_frac: float, rng: np.random.Generator) -> np.ndarray:
    """sign(score - median), 0 mapped to +1, then a seeded fraction flipped."""
    med = np.median(score)
    y = np.where(score - med >= 0, 1, -1).astype(np.int8)
    nflip = int(round(flip_frac * len(y)))
    if nflip:
        idx = rng.choice(len(y), size=nflip, replace=False)
        y[idx] = -y[idx]
    return y


def _zipf_cdf(d: int, s: float = 1.1) -> np.ndarray:
    p = np.arange(1, d + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(p)
    return c / c[-1]


def _sample_rows_without_replacement(lengths: np.ndarray, d: int, rng: np.random.Generator,
                                     s: float = 1.1) -> List[np.ndarray]:
    """For every row, draw ``lengths[i]`` distinct Zipf ranks in 0..d-1.

    Draws with replacement and keeps first occurrences: conditioned on the
    ranks already kept, the next new rank has probability proportional to its
    weight among the remaining ones, which is weighted sampling without
    replacement."""
    cdf = _zipf_cdf(d, s)
    n = len(lengths)
    out: List[Optional[np.ndarray]] = [None] * n
    todo = np.arange(n)
    mult = 2.0 if d > 4 * lengths.max() else 4.0
    while len(todo):
        L = lengths[todo]
        M = int(np.ceil(mult * L.max())) + 8
        cand = np.searchsorted(cdf, rng.random((len(todo), M)), side="right").astype(np.int64)
        np.minimum(cand, d - 1, out=cand)
        order = np.argsort(cand, axis=1, kind="stable")
        srt = np.take_along_axis(cand, order, axis=1)
        first_sorted = np.ones_like(srt, dtype=bool)
        first_sorted[:, 1:] = srt[:, 1:] != srt[:, :-1]
        first = np.zeros_like(first_sorted)
        np.put_along_axis(first, order, first_sorted, axis=1)
        rank = np.cumsum(first, axis=1)
        keep = first & (rank <= L[:, None])
        got = keep.sum(axis=1)
        ok = got >= L
        flat = cand[ok][keep[ok]]
        pieces = np.split(flat, np.cumsum(L[ok])[:-1])
        for r, piece in zip(todo[ok], pieces):
            out[r] = piece
        todo = todo[~ok]
        mult *= 2.0
    return out  # type: ignore[return-value]


def _assemble_csr(rows: List[np.ndarray], vals: List[np.ndarray], perm: np.ndarray):
    """Relabel columns by ``perm`` and sort each row by column id."""
    n = len(rows)
    lens = np.array([len(r) for r in rows], np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    c = perm[np.concatenate(rows)] if n else np.zeros(0, np.int64)
    v = np.concatenate(vals) if n else np.zeros(0)
    rid = np.repeat(np.arange(n), lens)
    o = np.lexsort((c, rid))
    return row_ptr.astype(np.int32), c[o].astype(np.int32), v[o]


# ---------------------------------------------------------------- families

def gen_blobs(n: int, d: int, rng: np.random.Generator, sep: float = 0.5, name="blobs") -> SvmData:
    """Two isotropic unit-variance Gaussian blobs with means +sep and -sep in every coordinate."""
    y = _balanced_labels(n, rng)
    x = y[:, None].astype(np.float64) * sep + rng.standard_normal((n, d))
    return SvmData(name, n, d, "dense", y, x=x.astype(np.float32))


def gen_sparse_binary(n: int, d: int, density: float, rng: np.random.Generator,
                      flip: float = 0.10, name="sparse_binary") -> SvmData:
    """Binary CSR rows: length ~ Binomial(d, density) (>= 1), Zipf(1.1) columns, value 1.0;
    labels from a sparse linear teacher with a fraction of flips."""
    L = np.clip(rng.binomial(d, density, size=n), 1, d).astype(np.int64)
    rows = _sample_rows_without_replacement(L, d, rng)
    perm = rng.permutation(d)
    vals = [np.ones(len(r)) for r in rows]
    row_ptr, col, val = _assemble_csr(rows, vals, perm)
    w = np.zeros(d)
    nz = rng.choice(d, size=max(1, int(round(0.1 * d))), replace=False)
    w[nz] = rng.standard_normal(len(nz))
    score = np.add.reduceat(w[col] * val, row_ptr[:-1]) if n else np.zeros(0)
    y = _teacher_labels(score, flip, rng)
    return SvmData(name, n, d, "csr", y, row_ptr=row_ptr, col=col, val=val.astype(np.float32))


def gen_text_like(n: int, d: int, mean_nnz: float, rng: np.random.Generator,
                  flip: float = 0.05, name="text_like") -> SvmData:
    """tf-idf-like CSR rows: length ~ Poisson(mean) clipped to [1, d], Zipf(1.1) columns,
    values exp(N(0, 0.5^2)), each row scaled to unit L2 norm; sparse linear teacher."""
    L = np.clip(rng.poisson(mean_nnz, size=n), 1, d).astype(np.int64)
    rows = _sample_rows_without_replacement(L, d, rng)
    perm = rng.permutation(d)
    lens = np.array([len(r) for r in rows], np.int64)
    v = np.exp(0.5 * rng.standard_normal(int(lens.sum())))
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    norm = np.sqrt(np.add.reduceat(v * v, starts))
    v = v / np.repeat(norm, lens)
    vals = np.split(v, np.cumsum(lens)[:-1])
    row_ptr, col, val = _assemble_csr(rows, vals, perm)
    w = np.zeros(d)
    nz = rng.choice(d, size=max(1, int(round(0.1 * d))), replace=False)
    w[nz] = rng.standard_normal(len(nz))
    score = np.add.reduceat(w[col] * val, row_ptr[:-1]) if n else np.zeros(0)
    y = _teacher_labels(score, flip, rng)
    return SvmData(name, n, d, "csr", y, row_ptr=row_ptr, col=col, val=val.astype(np.float32))


def gen_mixture(n: int, d: int, rng: np.random.Generator, k: int = 8, spacing: float = 1.0,
                name="mixture") -> SvmData:
    """k unit-variance Gaussian components with means j*spacing*u (u a seeded unit vector),
    j = 0..k-1; even j -> +1, odd j -> -1; equal weights (exactly n/k each when divisible)."""
    u = rng.standard_normal(d)
    u /= np.linalg.norm(u)
    comp = np.arange(n) % k
    rng.shuffle(comp)
    y = np.where(comp % 2 == 0, 1, -1).astype(np.int8)
    x = (comp[:, None] * spacing) * u[None, :] + rng.standard_normal((n, d))
    return SvmData(name, n, d, "dense", y, x=x.astype(np.float32))


# ---------------------------------------------------------------- named configurations

def config1(n: int = 2000, d: int = 20) -> SvmConfig:
    """Plain SMO, no shrinking: two blobs (means +-0.5, unit variance), gamma 0.05, C 1."""
    data = gen_blobs(n, d, rng_for(1, 0), name="cfg1")
    q = gen_blobs(10_000, d, rng_for(1, 1), name="cfg1_heldout")
    return SvmConfig("cfg1_blobs_n%d_d%d" % (n, d), data, C=1.0, gamma=0.05, eps=1e-3,
                     shrink_mode=SHRINK_NONE, queries=q)


def config2(n: int = 50_000, d: int = 300, heuristic=LAZY, mode=SHRINK_MULTI) -> SvmConfig:
    """Sparse binary (12% density, Zipf columns), gamma 1/d, C 1, lazy shrinking, multi."""
    data = gen_sparse_binary(n, d, 0.12, rng_for(2, 0), flip=0.10, name="cfg2")
    q = gen_sparse_binary(10_000, d, 0.12, rng_for(2, 1), flip=0.10, name="cfg2_heldout")
    return SvmConfig("cfg2_sparse_binary_n%d_d%d" % (n, d), data, C=1.0, gamma=1.0 / d, eps=1e-3,
                     shrink_mode=mode, shrink_kind=heuristic[0], shrink_param=heuristic[1], queries=q)


def config3(n: int = 200_000, d: int = 47_000, heuristic=EARLIEST, mode=SHRINK_MULTI) -> SvmConfig:
    """Text-like sparse (~75 nnz/row, lognormal values, unit rows), gamma 1, C 4."""
    data = gen_text_like(n, d, 75.0, rng_for(3, 0), flip=0.05, name="cfg3")
    q = gen_text_like(10_000, d, 75.0, rng_for(3, 1), flip=0.05, name="cfg3_heldout")
    return SvmConfig("cfg3_text_n%d_d%d" % (n, d), data, C=4.0, gamma=1.0, eps=1e-3,
                     shrink_mode=mode, shrink_kind=heuristic[0], shrink_param=heuristic[1], queries=q)


def config4(n: int = 500_000, d: int = 28, heuristic=LAZY, mode=SHRINK_MULTI) -> SvmConfig:
    """Dense 8-component mixture (4 per class, spacing 1.0), gamma 0.1, C 10."""
    data = gen_mixture(n, d, rng_for(4, 0), name="cfg4")
    q = gen_mixture(10_000, d, rng_for(4, 1), name="cfg4_heldout")
    return SvmConfig("cfg4_mixture_n%d_d%d" % (n, d), data, C=10.0, gamma=0.1, eps=1e-3,
                     shrink_mode=mode, shrink_kind=heuristic[0], shrink_param=heuristic[1], queries=q)


@dataclass
class ServeRequest:
    rid: int
    arrival_s: float
    config: SvmConfig


def config5_arrivals(num: int = 256, rate_hz: float = 200.0) -> np.ndarray:
    """Poisson arrival times (s) of the serving stream: exponential gaps, first arrival at 0."""
    r = rng_for(5, 0)
    gaps = r.exponential(1.0 / rate_hz, size=num)
    return np.cumsum(gaps) - gaps[0]


def config5_problem(j: int, n_lo: int = 1000, n_hi: int = 50_000) -> SvmConfig:
    """Problem j of the serving stream: n ~ U{n_lo..n_hi}, d in {20 dense, 128 dense, 300 sparse 12%},
    C in {0.1, 1, 10}, gamma = 10^U(-3, 0); lazy shrinking, multi."""
    pr = rng_for(5, 1 + j)
    n = int(pr.integers(n_lo, n_hi + 1))
    kind = int(pr.integers(0, 3))
    C = float([0.1, 1.0, 10.0][int(pr.integers(0, 3))])
    gamma = float(10.0 ** pr.uniform(-3.0, 0.0))
    if kind == 0:
        data = gen_blobs(n, 20, pr, name="req%d_dense20" % j)
    elif kind == 1:
        data = gen_blobs(n, 128, pr, name="req%d_dense128" % j)
    else:
        data = gen_sparse_binary(n, 300, 0.12, pr, flip=0.10, name="req%d_csr300" % j)
    return SvmConfig(data.name, data, C=C, gamma=gamma, eps=1e-3, shrink_mode=SHRINK_MULTI,
                     shrink_kind=LAZY[0], shrink_param=LAZY[1])


def config5(num: int = 256, rate_hz: float = 200.0, n_lo: int = 1000, n_hi: int = 50_000) -> List[ServeRequest]:
    """Poisson stream of mixed training problems (see config5_problem)."""
    arr = config5_arrivals(num, rate_hz)
    return [ServeRequest(j, float(arr[j]), config5_problem(j, n_lo, n_hi)) for j in range(num)]


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4}
