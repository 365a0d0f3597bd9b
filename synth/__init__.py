"""Seeded synthetic inputs for EBIC evaluation: matrices with planted trend
biclusters, populations of column series, and serving-job mixes.

This module only draws random data with the shapes and structure of the
benchmark collections the paper evaluates on (Sec. 2.1: UniBic-style
1000x100 narrow sets and small square sets, RecBic-style N(0,1) background,
noise 0.1-0.3, up to 2k columns, 20,000 x 250 gene-sized sets). It holds none
of the method's arithmetic (no trend test, no scoring) and is shared by the
oracle-side tests and the GPU path alike.

Generator recipe (NumPy PCG64 via ``default_rng(seed)``):
  1. draw the background matrix;
  2. for each planted bicluster draw its row count and column count uniformly
     in the stated ranges, its rows without replacement from rows not yet
     planted (row sets are disjoint), its columns without replacement (the
     drawn order is the trend order; columns may be shared between
     biclusters);
  3. for each planted row draw k background values, sort them ascending
     (descending for a reversed bicluster), write them in series order and add
     N(0, sigma) noise;
  4. cast to float32.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence

import numpy as np

# Seed bases: data 1000+i, population 2000+i, GA 3000+i, serving arrivals 4000,
# serving job j 5000+j.
DATA_SEED = 1000
POP_SEED = 2000
GA_SEED = 3000
ARRIVAL_SEED = 4000
JOB_SEED = 5000


@dataclasses.dataclass
class Planted:
    rows: np.ndarray      # sorted int64 row indices
    cols: np.ndarray      # int64 column series (trend order)
    reversed: bool


@dataclasses.dataclass
class MatrixCase:
    X: np.ndarray                 # float32 R x C, row-major
    truth: List[Planted]
    name: str

    @property
    def R(self) -> int:
        return int(self.X.shape[0])

    @property
    def C(self) -> int:
        return int(self.X.shape[1])

    def sha256(self) -> str:
        return hashlib.sha256(np.ascontiguousarray(self.X).tobytes()).hexdigest()


def _background(rng: np.random.Generator, kind: str, shape) -> np.ndarray:
    if kind == "uniform":
        return rng.random(shape)
    if kind == "normal":
        return rng.standard_normal(shape)
    if kind == "lognormal":
        return rng.lognormal(0.0, 1.0, shape)
    raise ValueError(kind)


PATTERNS = ("trend", "shift", "scale", "shift-scale", "constant-row")


def _pattern_rows(rng: np.random.Generator, pattern: str, nb: int, kb: int) -> np.ndarray:
    """nb x kb values whose every row increases along the columns (in the
    planted order) for the shift, scale and shift-scale patterns: column
    effects b_j drawn and sorted ascending, row effects a_i (positive for
    scale) and c_i drawn per row: shift a_i + b_j, scale a_i * b_j,
    shift-scale a_i * b_j + c_i. constant-row repeats one value per row (every
    step a tie)."""
    b = np.sort(rng.uniform(0.5, 2.0, kb))
    if pattern == "shift":
        return rng.normal(0.0, 1.0, (nb, 1)) + b
    if pattern == "scale":
        return rng.uniform(0.5, 2.0, (nb, 1)) * b
    if pattern == "shift-scale":
        return rng.uniform(0.5, 2.0, (nb, 1)) * b + rng.normal(0.0, 1.0, (nb, 1))
    if pattern == "constant-row":
        return np.repeat(rng.normal(0.0, 1.0, (nb, 1)), kb, axis=1)
    raise ValueError(f"unknown pattern {pattern!r}; one of {PATTERNS}")


def planted_matrix(R: int, C: int, *, background: str, n_planted: int,
                   rows_range: Sequence[int], cols_range: Sequence[int],
                   sigma: float, reverse_odd: bool = False, strict: bool = False,
                   seed: int, name: str = "", pattern: str = "trend") -> MatrixCase:
    """Background matrix with ``n_planted`` disjoint-row trend biclusters.

    ``pattern`` "trend": each planted row is its own sorted background draw;
    otherwise the bicluster's rows follow one of the paper's benchmark types
    (shift, scale, shift-scale, constant-row; see _pattern_rows).
    ``strict`` redraws a planted row until its values are pairwise distinct
    after the float32 cast (a strictly monotone planted trend with no ties).
    """
    rng = np.random.default_rng(seed)
    X = _background(rng, background, (R, C))
    available = np.ones(R, dtype=bool)
    truth: List[Planted] = []
    for b in range(n_planted):
        nb = int(rng.integers(rows_range[0], rows_range[1] + 1))
        kb = int(rng.integers(cols_range[0], cols_range[1] + 1))
        kb = min(kb, C)
        cand = np.flatnonzero(available)
        nb = min(nb, cand.size)
        rows = np.sort(rng.choice(cand, size=nb, replace=False))
        available[rows] = False
        cols = rng.choice(C, size=kb, replace=False)
        rev = bool(reverse_odd and (b % 2 == 1))
        if pattern != "trend":
            v = _pattern_rows(rng, pattern, nb, kb)
            if rev:
                v = v[:, ::-1]
            if sigma > 0:
                v = v + rng.normal(0.0, sigma, v.shape)
            X[np.ix_(rows, cols)] = v
            truth.append(Planted(rows=rows, cols=cols.astype(np.int64), reversed=rev))
            continue
        for r in rows:
            while True:
                v = np.sort(_background(rng, background, kb))
                if rev:
                    v = v[::-1]
                if sigma > 0:
                    v = v + rng.normal(0.0, sigma, kb)
                if not strict or np.unique(v.astype(np.float32)).size == kb:
                    break
            X[r, cols] = v
        truth.append(Planted(rows=rows, cols=cols.astype(np.int64), reversed=rev))
    return MatrixCase(X=np.ascontiguousarray(X.astype(np.float32)), truth=truth, name=name)


# ---------------------------------------------------------------------------
# The five workloads (tiny CPU case, plain-launch case, batched case, large
# expression-shaped case, serving mix).
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    R: int
    C: int
    background: str
    n_planted: int
    rows_range: tuple
    cols_range: tuple
    sigma: float
    reverse_odd: bool
    strict: bool
    population: int
    k_min: int
    k_max: int
    generations: int
    archive_size: int
    n_out: int
    negative_trends: int
    index: int


WORKLOADS = [
    Workload("tiny-100x20", 100, 20, "uniform", 1, (10, 10), (5, 5), 0.0, False, True,
             200, 2, 8, 50, 20, 1, 0, 0),
    Workload("plain-1000x100", 1000, 100, "normal", 5, (20, 100), (5, 15), 0.05, False, False,
             600, 3, 20, 200, 20, 5, 1, 1),
    Workload("batched-10000x500", 10000, 500, "lognormal", 10, (50, 500), (5, 40), 0.1, False,
             False, 4096, 3, 64, 100, 20, 10, 1, 2),
    Workload("large-40000x1000", 40000, 1000, "lognormal", 20, (100, 2000), (5, 60), 0.1, True,
             False, 8192, 3, 64, 20, 20, 20, 1, 3),
]


def workload(i: int) -> Workload:
    return WORKLOADS[i]


def workload_matrix(i: int, seed: Optional[int] = None) -> MatrixCase:
    w = WORKLOADS[i]
    return planted_matrix(w.R, w.C, background=w.background, n_planted=w.n_planted,
                          rows_range=w.rows_range, cols_range=w.cols_range, sigma=w.sigma,
                          reverse_odd=w.reverse_odd, strict=w.strict,
                          seed=DATA_SEED + i if seed is None else seed, name=w.name)


def random_series(rng: np.random.Generator, C: int, k: int) -> np.ndarray:
    return rng.choice(C, size=k, replace=False).astype(np.int64)


def population(C: int, P: int, k_min: int, k_max: int, *, seed: int,
               truth: Sequence[Planted] = (), planted_frac: float = 0.0) -> List[np.ndarray]:
    """``P`` column series of lengths uniform in [k_min, k_max].

    A ``planted_frac`` share is built from planted series: either a prefix of
    one, or the whole series (cut to k_max - 1) with one random unused column
    inserted at a random position. The rest are uniformly random distinct
    columns.
    """
    rng = np.random.default_rng(seed)
    k_max = min(k_max, C)
    out: List[np.ndarray] = []
    for _ in range(P):
        if truth and rng.random() < planted_frac:
            t = truth[int(rng.integers(len(truth)))]
            s = t.cols
            if rng.random() < 0.5:
                lo = max(k_min, 2)
                hi = max(lo, min(k_max, s.size))
                L = int(rng.integers(lo, hi + 1))
                seq = s[:L]
                if seq.size < L:
                    extra = np.setdiff1d(np.arange(C), seq)
                    seq = np.concatenate([seq, rng.choice(extra, L - seq.size, replace=False)])
            else:
                seq = s[:max(k_min - 1, min(s.size, k_max - 1))]
                unused = np.setdiff1d(np.arange(C), seq)
                c = int(rng.choice(unused))
                pos = int(rng.integers(seq.size + 1))
                seq = np.insert(seq, pos, c)
            out.append(seq.astype(np.int64))
        else:
            k = int(rng.integers(k_min, k_max + 1))
            out.append(random_series(rng, C, k))
    return out


def workload_population(i: int, case: Optional[MatrixCase] = None, P: Optional[int] = None,
                        seed: Optional[int] = None) -> List[np.ndarray]:
    w = WORKLOADS[i]
    truth = case.truth if case is not None else ()
    return population(w.C, w.population if P is None else P, w.k_min, w.k_max,
                      seed=POP_SEED + i if seed is None else seed, truth=truth,
                      planted_frac=0.1)


def to_csr(pop: Sequence[np.ndarray]):
    """Concatenate series into (offsets int32[P+1], cols uint16[sum k])."""
    lens = np.array([len(s) for s in pop], dtype=np.int64)
    offsets = np.zeros(len(pop) + 1, dtype=np.int32)
    np.cumsum(lens, out=offsets[1:])
    cols = np.concatenate([np.asarray(s, dtype=np.uint16) for s in pop]) if len(pop) else \
        np.zeros(0, dtype=np.uint16)
    return offsets, cols.astype(np.uint16)


# ---------------------------------------------------------------------------
# Serving mix: jobs on matrices of different shapes with Poisson arrivals.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class JobSpec:
    job: int
    R: int
    C: int
    n_planted: int
    population: int
    seed: int


def serving_jobs(n_jobs: int = 64, *, rows=(500, 50000), cols=(20, 2000),
                 pops=(256, 512, 1024, 2048, 4096), seed: int = ARRIVAL_SEED) -> List[JobSpec]:
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n_jobs):
        R = int(round(math.exp(rng.uniform(math.log(rows[0]), math.log(rows[1])))))
        C = int(round(math.exp(rng.uniform(math.log(cols[0]), math.log(cols[1])))))
        npl = int(rng.integers(1, 21))
        P = int(pops[int(rng.integers(len(pops)))])
        jobs.append(JobSpec(job=j, R=R, C=C, n_planted=npl, population=P, seed=JOB_SEED + j))
    return jobs


def job_matrix(spec: JobSpec) -> MatrixCase:
    R, C = spec.R, spec.C
    return planted_matrix(R, C, background="lognormal", n_planted=spec.n_planted,
                          rows_range=(max(10, R // 200), max(20, R // 20)),
                          cols_range=(3, max(3, min(60, C // 2))), sigma=0.1,
                          reverse_odd=True, seed=spec.seed, name=f"job{spec.job}")


def poisson_arrivals(n: int, mean_gap_s: float, seed: int = ARRIVAL_SEED + 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(mean_gap_s, n))


def random_matrix(R: int, C: int, seed: int, kind: str = "normal") -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_background(rng, kind, (R, C)).astype(np.float32))


def tie_matrix(R: int, C: int, levels: int, seed: int) -> np.ndarray:
    """Integer-valued float32 matrix with many ties (values 0..levels-1),
    plus signed zeros mixed in, for tie-rule edge tests."""
    rng = np.random.default_rng(seed)
    X = rng.integers(0, levels, size=(R, C)).astype(np.float32)
    z = rng.random((R, C)) < 0.1
    X[z] = np.where(rng.random(int(z.sum())) < 0.5, np.float32(0.0), np.float32(-0.0))
    return X
