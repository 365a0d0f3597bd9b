"""EBIC oracle -- TEST INFRASTRUCTURE ONLY.

A plain CPU implementation (``ebic_oracle.c``) of EBIC's fitness evaluation
and generational loop, written from the paper (Sec. 2.3 and 2.4 of
arXiv 2105.01196) and the readings listed at the top of that file. Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may load
it. It shares no code with the GPU library; the only module both sides use is
``synth`` (seeded random inputs, no method arithmetic).

Parity status: ``evaluate`` is pinned by brute force, Eulerian closed forms,
invariants and fitness identities; the size-score and overlap-penalty formulas
are a reading (the paper prints none). ``run`` is pinned by RNG known-answer
values, determinism and planted recovery; its trajectory is parity unpinned
against the paper.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ebic_oracle.c")
_LIB = os.path.join(_HERE, "libebic_oracle.so")
K_LIMIT = 512


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "approx_permille", "negative_trends", "overlap_permille", "min_rows", "k_score_min",
        "k_min", "k_max", "archive_size", "n_out", "population", "generations",
        "max_tabu_hits", "tournament", "max_attempts", "tie_rule")] + \
        [("op_permille", ctypes.c_int32 * 5)]


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.POINTER(ctypes.c_int32)),
                ("k", ctypes.POINTER(ctypes.c_int32)),
                ("cols", ctypes.POINTER(ctypes.c_uint16)),
                ("n", ctypes.POINTER(ctypes.c_int32)),
                ("score", ctypes.POINTER(ctypes.c_double)),
                ("rows", ctypes.POINTER(ctypes.c_uint8)),
                ("stats", ctypes.POINTER(ctypes.c_int64)),
                ("trace", ctypes.POINTER(ctypes.c_double))]


DEFAULTS = dict(approx_permille=850, negative_trends=0, overlap_permille=750, min_rows=5,
                k_score_min=2, k_min=2, k_max=8, archive_size=20, n_out=1, population=200,
                generations=50, max_tabu_hits=100000, tournament=4, max_attempts=1000,
                tie_rule=0)


def make_params(**kw) -> Params:
    """Parameters with the defaults above; op_permille (insertion, deletion,
    substitution, swap, crossover weights, per mille) defaults to 200 each."""
    d = dict(DEFAULTS)
    if "negative_trends" in kw and "k_score_min" not in kw:
        d["k_score_min"] = 3 if kw["negative_trends"] else 2
    d.update(kw)
    ops = d.pop("op_permille", (200,) * 5)
    p = Params(**d)
    p.op_permille[:] = list(ops)
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        L.oracle_evaluate.restype = ctypes.c_int
        L.oracle_evaluate.argtypes = [
            P(ctypes.c_float), ctypes.c_int, ctypes.c_int, ctypes.c_int,
            P(ctypes.c_int32), P(ctypes.c_uint16), ctypes.c_int, P(ctypes.c_uint8),
            P(ctypes.c_int32), P(ctypes.c_uint16), P(Params), ctypes.c_int,
            P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_uint8), P(ctypes.c_int32),
            P(ctypes.c_double)]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run.argtypes = [P(ctypes.c_float), ctypes.c_int, ctypes.c_int, P(Params),
                                 ctypes.c_uint64, ctypes.c_int, P(_Result)]
        L.oracle_splitmix64_next.restype = ctypes.c_uint64
        L.oracle_splitmix64_next.argtypes = [P(ctypes.c_uint64)]
        L.oracle_uniform.restype = ctypes.c_uint64
        L.oracle_uniform.argtypes = [P(ctypes.c_uint64), ctypes.c_uint64]
        L.oracle_crowding_keys.restype = ctypes.c_int
        L.oracle_crowding_keys.argtypes = [P(ctypes.c_int32), P(ctypes.c_uint16), ctypes.c_int,
                                           ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double)]
        L.oracle_mutants.restype = ctypes.c_int
        L.oracle_mutants.argtypes = [P(ctypes.c_int32), P(ctypes.c_uint16), ctypes.c_int,
                                     P(ctypes.c_double), ctypes.c_int, P(Params),
                                     ctypes.c_uint64, ctypes.c_int, P(ctypes.c_int32),
                                     P(ctypes.c_uint16)]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _csr(seqs: Sequence[Sequence[int]]):
    lens = [len(s) for s in seqs]
    off = np.zeros(len(seqs) + 1, dtype=np.int32)
    off[1:] = np.cumsum(lens)
    cols = (np.concatenate([np.asarray(s, dtype=np.uint16) for s in seqs])
            if seqs else np.zeros(0, np.uint16)).astype(np.uint16)
    if cols.size == 0:
        cols = np.zeros(1, np.uint16)
    return off, np.ascontiguousarray(cols)


@dataclasses.dataclass
class Archive:
    """Archived biclusters for the overlap penalty: row flags (K x R) and the
    column series of each member."""
    rows: np.ndarray                  # uint8 K x R
    series: List[Sequence[int]]

    @property
    def K(self) -> int:
        return len(self.series)

    @staticmethod
    def empty(R: int) -> "Archive":
        return Archive(np.zeros((0, R), np.uint8), [])


@dataclasses.dataclass
class Evaluation:
    fitness: np.ndarray   # float64 P
    count: np.ndarray     # int32 P
    support: np.ndarray   # uint8 P x R (1 = row supports the series)
    overlap: np.ndarray   # int32 P x K (rows shared with each archive member)
    score: np.ndarray     # float64 P (size score before the overlap penalty)


def evaluate(X: np.ndarray, seqs: Sequence[Sequence[int]], archive: Optional[Archive] = None,
             params: Optional[Params] = None, nthreads: int = 1) -> Evaluation:
    X = np.ascontiguousarray(X, dtype=np.float32)
    R, C = X.shape
    archive = archive or Archive.empty(R)
    params = params or make_params()
    P, K = len(seqs), archive.K
    off, cols = _csr(seqs)
    aoff, acols = _csr(archive.series)
    arows = np.ascontiguousarray(archive.rows, dtype=np.uint8).reshape(K, R)
    if arows.size == 0:
        arows = np.zeros((1, R), np.uint8)
    fit = np.zeros(max(P, 1), np.float64)
    cnt = np.zeros(max(P, 1), np.int32)
    sup = np.zeros((max(P, 1), R), np.uint8)
    ov = np.zeros((max(P, 1), max(K, 1)), np.int32)
    sc = np.zeros(max(P, 1), np.float64)
    rc = lib().oracle_evaluate(_ptr(X, ctypes.c_float), R, C, P, _ptr(off, ctypes.c_int32),
                               _ptr(cols, ctypes.c_uint16), K, _ptr(arows, ctypes.c_uint8),
                               _ptr(aoff, ctypes.c_int32), _ptr(acols, ctypes.c_uint16),
                               ctypes.byref(params), nthreads, _ptr(fit, ctypes.c_double),
                               _ptr(cnt, ctypes.c_int32), _ptr(sup, ctypes.c_uint8),
                               _ptr(ov, ctypes.c_int32) if K else None,
                               _ptr(sc, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_evaluate: invalid argument")
    return Evaluation(fit[:P], cnt[:P], sup[:P], ov[:P, :K], sc[:P])


@dataclasses.dataclass
class Bicluster:
    rows: np.ndarray      # sorted int64 row indices
    cols: np.ndarray      # int64 column series
    n: int
    score: float


@dataclasses.dataclass
class RunResult:
    biclusters: List[Bicluster]
    generations: int
    evaluations: int
    tabu_hits: int
    stop_reason: int
    trace: np.ndarray     # G x 4: population size, archive size, best score, tabu hits


def run(X: np.ndarray, params: Params, seed: int, nthreads: int = 1) -> RunResult:
    X = np.ascontiguousarray(X, dtype=np.float32)
    R, C = X.shape
    nb = max(params.n_out, 1)
    G = max(params.generations, 1)
    count = np.zeros(1, np.int32)
    k = np.zeros(nb, np.int32)
    cols = np.zeros((nb, K_LIMIT), np.uint16)
    n = np.zeros(nb, np.int32)
    score = np.zeros(nb, np.float64)
    rows = np.zeros((nb, R), np.uint8)
    stats = np.zeros(4, np.int64)
    trace = np.zeros((G, 4), np.float64)
    res = _Result(_ptr(count, ctypes.c_int32), _ptr(k, ctypes.c_int32),
                  _ptr(cols, ctypes.c_uint16), _ptr(n, ctypes.c_int32),
                  _ptr(score, ctypes.c_double), _ptr(rows, ctypes.c_uint8),
                  _ptr(stats, ctypes.c_int64), _ptr(trace, ctypes.c_double))
    rc = lib().oracle_run(_ptr(X, ctypes.c_float), R, C, ctypes.byref(params),
                          ctypes.c_uint64(seed), nthreads, ctypes.byref(res))
    if rc != 0:
        raise ValueError("oracle_run: invalid argument")
    bcs = [Bicluster(np.flatnonzero(rows[j]).astype(np.int64),
                     cols[j, :k[j]].astype(np.int64), int(n[j]), float(score[j]))
           for j in range(int(count[0]))]
    g = int(stats[0])
    return RunResult(bcs, g, int(stats[1]), int(stats[2]), int(stats[3]), trace[:g].copy())


def mutants(seqs: Sequence[Sequence[int]], C: int, params: Params, seed: int, n: int,
            key: Optional[Sequence[float]] = None) -> List[np.ndarray]:
    """n mutation attempts (tournament, operator, child) from the population
    seqs with tournament keys `key` (default all equal). An attempt in which
    no weighted operator applies gives an empty child."""
    off, cols = _csr(seqs)
    P = len(seqs)
    k = np.ascontiguousarray(key if key is not None else np.zeros(P), dtype=np.float64)
    lens = np.zeros(max(n, 1), np.int32)
    out = np.zeros((max(n, 1), K_LIMIT), np.uint16)
    rc = lib().oracle_mutants(_ptr(off, ctypes.c_int32), _ptr(cols, ctypes.c_uint16), P,
                              _ptr(k, ctypes.c_double), C, ctypes.byref(params),
                              ctypes.c_uint64(seed), n, _ptr(lens, ctypes.c_int32),
                              _ptr(out, ctypes.c_uint16))
    if rc != 0:
        raise ValueError("oracle_mutants: invalid argument")
    return [out[i, :min(lens[i], K_LIMIT)].astype(np.int64) for i in range(n)]


def crowding_keys(seqs: Sequence[Sequence[int]], C: int, fitness) -> np.ndarray:
    """Tournament keys of a population: each fitness halved once per column
    of the individual that more individuals hold than ceil(sum k / C)."""
    off, cols = _csr(seqs)
    fit = np.ascontiguousarray(fitness, dtype=np.float64)
    keys = np.zeros(max(len(seqs), 1), np.float64)
    if lib().oracle_crowding_keys(_ptr(off, ctypes.c_int32), _ptr(cols, ctypes.c_uint16),
                                  len(seqs), C, _ptr(fit, ctypes.c_double),
                                  _ptr(keys, ctypes.c_double)) != 0:
        raise ValueError("oracle_crowding_keys: invalid argument")
    return keys[:len(seqs)]


def splitmix64_stream(seed: int, count: int) -> List[int]:
    st = ctypes.c_uint64(seed)
    return [int(lib().oracle_splitmix64_next(ctypes.byref(st))) for _ in range(count)]


def uniform_stream(seed: int, bounds: Sequence[int]) -> List[int]:
    st = ctypes.c_uint64(seed)
    return [int(lib().oracle_uniform(ctypes.byref(st), ctypes.c_uint64(b))) for b in bounds]


def ce_score(found, truth):
    """Clustering error (Sec. 2.2, Eq. 1) of detected biclusters against the
    truth, each a sequence of (rows, cols): the confusion matrix counts the
    matrix cells (row, col) two biclusters share, D_max is its largest total
    over one-to-one assignments of detected to true biclusters (a library
    assignment solver is the one step taken from elsewhere), U is the set of
    all cells of all biclusters of both sets. Returns (D_max/|U|,
    (|U| - D_max)/|U|): the text reads 1 as a perfect match, the printed
    Eq. (1) is the second value. Both empty: (1.0, 0.0)."""
    from scipy.optimize import linear_sum_assignment

    def cells(b):
        rows, cols = b
        return {(int(r), int(c)) for r in rows for c in cols}

    fc = [cells(b) for b in found]
    tc = [cells(b) for b in truth]
    union = set().union(*fc, *tc)
    if not union:
        return 1.0, 0.0
    d_max = 0
    if fc and tc:
        m = np.array([[len(a & b) for b in tc] for a in fc], dtype=np.int64)
        i, j = linear_sum_assignment(m, maximize=True)
        d_max = int(m[i, j].sum())
    u = len(union)
    return d_max / u, (u - d_max) / u
