"""Python binding of the EBIC HIP library (``libebic.so``, C ABI in
include/ebic.h). Argument marshalling only: every step of the evaluation runs
in the library's kernels. PyTorch supplies device memory and streams.

The library must be built (``python -m paper_2105_01196_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebic.so")

EBIC_OK = 0
EBIC_PENDING = 1
EBIC_ERR_INVALID_ARG = -1
EBIC_ERR_NONFINITE = -2
EBIC_ERR_OOM = -3
EBIC_ERR_DEVICE = -4
EBIC_ERR_CAPACITY = -5
EBIC_MAX_K = 512
EBIC_MAX_ARCHIVE = 64
EBIC_MAX_COLS = 16384
EBIC_NOALLOC_MAX_JOBS = 64


class EbicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ebic error {code}: {msg}")
        self.code = code


_i32, _vp = ctypes.c_int32, ctypes.c_void_p


class ebic_params(ctypes.Structure):
    _fields_ = [(n, _i32) for n in (
        "approx_permille", "negative_trends", "overlap_permille", "min_rows", "k_score_min",
        "k_min", "k_max", "archive_size", "n_out", "population", "generations",
        "max_tabu_hits", "tournament", "max_attempts", "tie_rule")] + \
        [("op_permille", _i32 * 5)]


class ebic_matrix(ctypes.Structure):
    _fields_ = [("d_ranks", _vp), ("rows", _i32), ("cols", _i32), ("rows_pad", _i32),
                ("d_pairs", _vp), ("d_pairs_strict", _vp)]


class ebic_population(ctypes.Structure):
    _fields_ = [("size", _i32), ("length", _i32), ("d_offsets", _vp), ("d_cols", _vp),
                ("d_order", _vp)]


class ebic_archive(ctypes.Structure):
    _fields_ = [("size", _i32), ("length", _i32), ("d_support", _vp), ("d_offsets", _vp),
                ("d_cols", _vp)]


class ebic_eval_out(ctypes.Structure):
    _fields_ = [("d_fitness", _vp), ("d_count", _vp), ("d_support", _vp), ("d_overlap", _vp)]


class ebic_job(ctypes.Structure):
    _fields_ = [("matrix", ebic_matrix), ("population", ebic_population),
                ("archive", ebic_archive), ("params", ebic_params), ("out", ebic_eval_out)]


class ebic_bicluster(ctypes.Structure):
    _fields_ = [("n_rows", _i32), ("rows", ctypes.POINTER(_i32)), ("n_cols", _i32),
                ("cols", ctypes.POINTER(ctypes.c_uint16)), ("score", ctypes.c_double),
                ("row_dir", ctypes.POINTER(ctypes.c_uint8))]


ALLOC_FN = ctypes.CFUNCTYPE(_vp, _vp, ctypes.c_size_t, _vp)
RELEASE_FN = ctypes.CFUNCTYPE(None, _vp, _vp, _vp)


class ebic_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("ctx", _vp)]


class ebic_result(ctypes.Structure):
    _fields_ = [("count", _i32), ("biclusters", ctypes.POINTER(ebic_bicluster)),
                ("generations", _i32), ("evaluations", ctypes.c_int64),
                ("tabu_hits", ctypes.c_int64), ("stop_reason", _i32),
                ("trace", ctypes.POINTER(ctypes.c_double))]


class ebic_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", _i32),
                ("device_loop_population", _i32), ("device_loop_runners", _i32)]


class ebic_server_metrics(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("active", ctypes.c_int64), ("evaluations", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("p50_latency_s", ctypes.c_double),
                ("p99_latency_s", ctypes.c_double), ("mean_latency_s", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("hbm_in_use", ctypes.c_size_t),
                ("hbm_budget", ctypes.c_size_t), ("stage_s", ctypes.c_double),
                ("device_s", ctypes.c_double), ("host_s", ctypes.c_double),
                ("setup_s", ctypes.c_double), ("release_s", ctypes.c_double),
                ("device_loop_jobs", ctypes.c_int64), ("device_loop_s", ctypes.c_double)]


EBIC_STOP_GENERATIONS = 1
EBIC_STOP_TABU = 2
EBIC_STOP_EXHAUSTED = 3
EBIC_TIE_INDEX = 0
EBIC_TIE_STRICT = 1
EBIC_TIE_LOOSE = 2
EBIC_BATCH_GRAPH = 1
EBIC_BATCH_GATHER = 2
EBIC_BATCH_TUNE = 4

# Every symbol include/ebic.h declares, with its ctypes signature.
_SIGNATURES = {
    "ebic_version": (ctypes.c_int, []),
    "ebic_last_error": (ctypes.c_char_p, []),
    "ebic_matrix_bytes": (ctypes.c_size_t, [_i32, _i32]),
    "ebic_matrix_prepare": (ctypes.c_int, [_vp, _i32, _i32, _vp, ctypes.POINTER(ebic_matrix),
                                           _vp]),
    "ebic_population_upload": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _vp, _vp]),
    "ebic_evaluate": (ctypes.c_int, [ctypes.POINTER(ebic_matrix),
                                     ctypes.POINTER(ebic_population),
                                     ctypes.POINTER(ebic_archive), ctypes.POINTER(ebic_params),
                                     ctypes.POINTER(ebic_eval_out), _vp]),
    "ebic_support_rows": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i32, _vp, _vp, _vp]),
    "ebic_pairs_bytes": (ctypes.c_size_t, [_i32, _i32]),
    "ebic_pairs_words": (_i32, [_i32]),
    "ebic_pairs_strict_prepare": (ctypes.c_int, [ctypes.POINTER(ebic_matrix), _vp, _vp]),
    "ebic_pairs_prepare": (ctypes.c_int, [ctypes.POINTER(ebic_matrix), _vp, _vp]),
    "ebic_batch_create": (ctypes.c_int, [ctypes.POINTER(ebic_job), _i32, _i32,
                                         ctypes.POINTER(_vp)]),
    "ebic_batch_run": (ctypes.c_int, [_vp, _vp]),
    "ebic_batch_destroy": (ctypes.c_int, [_vp]),
    "ebic_evaluate_batched": (ctypes.c_int, [ctypes.POINTER(ebic_job), _i32, _vp]),
    "ebic_evaluate_batched_noalloc": (ctypes.c_int, [ctypes.POINTER(ebic_job), _i32, _vp]),
    "ebic_run": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(ebic_params), ctypes.c_uint64,
                                ctypes.POINTER(ebic_allocator), _vp,
                                ctypes.POINTER(ctypes.POINTER(ebic_result))]),
    "ebic_run_device": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(ebic_params), ctypes.c_uint64,
                                ctypes.POINTER(ebic_allocator), _vp,
                                ctypes.POINTER(ctypes.POINTER(ebic_result))]),
    "ebic_session_create": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(ebic_params),
                                           ctypes.c_uint64, ctypes.POINTER(ebic_allocator), _vp,
                                           ctypes.POINTER(_vp)]),
    "ebic_session_step": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32)]),
    "ebic_session_checkpoint": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ebic_session_restore": (ctypes.c_int, [_vp, _i32, _i32, _vp, ctypes.c_size_t,
                                            ctypes.POINTER(ebic_allocator), _vp,
                                            ctypes.POINTER(_vp)]),
    "ebic_session_result": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.POINTER(ebic_result))]),
    "ebic_session_free": (None, [_vp]),
    "ebic_result_free": (None, [ctypes.POINTER(ebic_result)]),
    "ebic_ce_score": (ctypes.c_int, [ctypes.POINTER(ebic_bicluster), _i32,
                                     ctypes.POINTER(ebic_bicluster), _i32, _i32, _i32,
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    "ebic_server_create": (ctypes.c_int, [ctypes.POINTER(ebic_server_config),
                                          ctypes.POINTER(_vp)]),
    "ebic_server_submit": (ctypes.c_int, [_vp, _vp, _i32, _i32, ctypes.POINTER(ebic_params),
                                          ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64)]),
    "ebic_server_poll": (ctypes.c_int, [_vp, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.POINTER(ebic_result))]),
    "ebic_server_wait": (ctypes.c_int, [_vp, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.POINTER(ebic_result))]),
    "ebic_server_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ebic_server_metrics)]),
    "ebic_server_destroy": (ctypes.c_int, [_vp]),
    "ebic_batch_profile": (ctypes.c_int, [_vp, _i32]),
    "ebic_batch_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                         ctypes.POINTER(_i32)]),
    "ebic_batch_set_tuning": (ctypes.c_int, [_vp, _i32, _i32, _i32]),
    "ebic_batch_timings": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(_i32)]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_2105_01196_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise EbicError(rc, lib().ebic_last_error().decode())
    return rc


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _to_device_bytes(a: np.ndarray, device) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.nbytes == 0:
        return torch.empty(8, dtype=torch.uint8, device=device)
    return torch.from_numpy(a.view(np.uint8).reshape(-1)).to(device)


DEFAULT_PARAMS = dict(approx_permille=850, negative_trends=0, overlap_permille=750,
                      min_rows=5, k_score_min=2, k_min=2, k_max=8, archive_size=20, n_out=1,
                      population=200, generations=50, max_tabu_hits=100000, tournament=4,
                      max_attempts=1000, tie_rule=0)


def make_params(**kw) -> ebic_params:
    """Parameters with the defaults above; op_permille (insertion, deletion,
    substitution, swap, crossover weights, per mille) defaults to 200 each."""
    d = dict(DEFAULT_PARAMS)
    if "negative_trends" in kw and "k_score_min" not in kw:
        d["k_score_min"] = 3 if kw["negative_trends"] else 2
    d.update(kw)
    ops = d.pop("op_permille", (200,) * 5)
    p = ebic_params(**d)
    p.op_permille[:] = list(ops)
    return p


def ebic_version() -> int:
    return lib().ebic_version()


def ebic_matrix_bytes(rows: int, cols: int) -> int:
    return int(lib().ebic_matrix_bytes(rows, cols))


@dataclasses.dataclass
class Matrix:
    """A prepared matrix: the rank array in device memory and its view."""
    ranks: torch.Tensor
    view: ebic_matrix
    pairs: Optional[torch.Tensor] = None
    pairs_strict: Optional[torch.Tensor] = None

    @property
    def rows(self) -> int:
        return self.view.rows

    @property
    def cols(self) -> int:
        return self.view.cols

    @property
    def words(self) -> int:
        return self.view.rows_pad // 64


def ebic_matrix_prepare(x: torch.Tensor, stream=None) -> Matrix:
    """Ingest a float32 rows x cols matrix already on the GPU."""
    assert x.is_cuda and x.dtype == torch.float32 and x.dim() == 2
    x = x.contiguous()
    R, C = x.shape
    nbytes = ebic_matrix_bytes(R, C)
    ranks = torch.empty(max(nbytes, 2), dtype=torch.uint8, device=x.device)
    view = ebic_matrix()
    _check(lib().ebic_matrix_prepare(x.data_ptr(), R, C, ranks.data_ptr(), ctypes.byref(view),
                                      _stream(stream)))
    return Matrix(ranks, view)


@dataclasses.dataclass
class Population:
    offsets: torch.Tensor
    cols: torch.Tensor
    view: ebic_population
    order: Optional[torch.Tensor] = None

    @property
    def size(self) -> int:
        return self.view.size


def csr(seqs: Sequence[Sequence[int]]):
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    off = np.zeros(len(seqs) + 1, dtype=np.int32)
    off[1:] = np.cumsum(lens)
    cols = (np.concatenate([np.asarray(s, dtype=np.uint16) for s in seqs])
            if len(seqs) else np.zeros(0, np.uint16)).astype(np.uint16)
    return off, cols


def ebic_population_upload(seqs_or_csr, cols: int, device="cuda", stream=None) -> Population:
    """Validate a population (list of series, or (offsets, cols) CSR arrays)
    and copy it to the GPU."""
    if isinstance(seqs_or_csr, tuple):
        off, cc = seqs_or_csr
    else:
        off, cc = csr(seqs_or_csr)
    off = np.ascontiguousarray(off, dtype=np.int32)
    cc = np.ascontiguousarray(cc, dtype=np.uint16)
    P = off.size - 1
    d_off = torch.empty(max(off.nbytes, 8), dtype=torch.uint8, device=device)
    d_cols = torch.empty(max(cc.nbytes, 8), dtype=torch.uint8, device=device)
    _check(lib().ebic_population_upload(off.ctypes.data, cc.ctypes.data if cc.size else None, P,
                                        cols, d_off.data_ptr(), d_cols.data_ptr(),
                                        _stream(stream)))
    view = ebic_population(P, int(cc.size), d_off.data_ptr(), d_cols.data_ptr(), None)
    return Population(d_off, d_cols, view)


def population_raw(off: np.ndarray, cc: np.ndarray, device="cuda") -> Population:
    """Copy a CSR population to the GPU without host validation (the device
    kernels guard every access and mark malformed individuals invalid)."""
    d_off = _to_device_bytes(np.asarray(off, np.int32), device)
    d_cols = _to_device_bytes(np.asarray(cc, np.uint16), device)
    view = ebic_population(int(np.asarray(off).size - 1), int(np.asarray(cc).size),
                           d_off.data_ptr(), d_cols.data_ptr(), None)
    return Population(d_off, d_cols, view)


def set_order(pop: Population, order: Optional[np.ndarray], device="cuda") -> None:
    """Attach a processing order (a permutation of 0..P-1) for the batched
    evaluator, or clear it with None."""
    if order is None:
        pop.view.d_order = None
        pop.order = None
        return
    d = torch.from_numpy(np.ascontiguousarray(order, dtype=np.int32)).to(device)
    pop.order = d
    pop.view.d_order = d.data_ptr()


def longest_first(seqs) -> np.ndarray:
    """Order that puts the longest series first (stable)."""
    lens = np.array([len(s) for s in seqs])
    return np.argsort(-lens, kind="stable").astype(np.int32)


@dataclasses.dataclass
class Archive:
    support: torch.Tensor     # int64 K x W (bit pattern of uint64 words)
    offsets: torch.Tensor
    cols: torch.Tensor
    view: ebic_archive

    @property
    def size(self) -> int:
        return self.view.size


def make_archive(support_words: np.ndarray, series: Sequence[Sequence[int]],
                 device="cuda") -> Archive:
    """Archive from host support bitmaps (K x W uint64) and member series."""
    K = len(series)
    sw = np.ascontiguousarray(support_words, dtype=np.uint64).reshape(K, -1)
    d_sup = torch.from_numpy(sw.view(np.int64).copy()).to(device) if K else \
        torch.zeros(1, dtype=torch.int64, device=device)
    off, cc = csr(series)
    d_off = _to_device_bytes(off, device)
    d_cols = _to_device_bytes(cc, device)
    view = ebic_archive(K, int(cc.size), d_sup.data_ptr(), d_off.data_ptr(), d_cols.data_ptr())
    return Archive(d_sup, d_off, d_cols, view)


def archive_from_device(support: torch.Tensor, sel: Sequence[int], pop_series,
                        device="cuda") -> Archive:
    sw = support[list(sel)].contiguous() if len(sel) else torch.zeros(1, dtype=torch.int64,
                                                                       device=device)
    series = [pop_series[i] for i in sel]
    off, cc = csr(series)
    d_off = _to_device_bytes(off, device)
    d_cols = _to_device_bytes(cc, device)
    view = ebic_archive(len(sel), int(cc.size), sw.data_ptr(), d_off.data_ptr(), d_cols.data_ptr())
    return Archive(sw, d_off, d_cols, view)


@dataclasses.dataclass
class EvalOut:
    fitness: torch.Tensor             # float64 P
    count: torch.Tensor               # int32 P
    support: Optional[torch.Tensor]   # int64 P x W (uint64 bit patterns)
    overlap: Optional[torch.Tensor]   # int32 P x K
    view: ebic_eval_out


def alloc_eval_out(P: int, words: int, K: int, support=True, overlap=True,
                   device="cuda") -> EvalOut:
    fit = torch.empty(max(P, 1), dtype=torch.float64, device=device)
    cnt = torch.empty(max(P, 1), dtype=torch.int32, device=device)
    sup = torch.empty((max(P, 1), words), dtype=torch.int64, device=device) if support else None
    ov = torch.empty((max(P, 1), max(K, 1)), dtype=torch.int32, device=device) \
        if overlap and K > 0 else None
    view = ebic_eval_out(fit.data_ptr(), cnt.data_ptr(), _dev(sup), _dev(ov))
    return EvalOut(fit, cnt, sup, ov, view)


def ebic_evaluate(m: Matrix, pop: Population, archive: Optional[Archive] = None,
                  params: Optional[ebic_params] = None, out: Optional[EvalOut] = None,
                  support=True, overlap=True, stream=None) -> EvalOut:
    """Plain evaluation of one population (one launch). Asynchronous on the
    stream; results are ready after a synchronize."""
    params = params or make_params()
    K = archive.size if archive is not None else 0
    if out is None:
        out = alloc_eval_out(pop.size, m.words, K, support, overlap, device=m.ranks.device)
    arch_view = archive.view if archive is not None else ebic_archive(0, 0, None, None, None)
    _check(lib().ebic_evaluate(ctypes.byref(m.view), ctypes.byref(pop.view),
                               ctypes.byref(arch_view), ctypes.byref(params),
                               ctypes.byref(out.view), _stream(stream)))
    return out


def ebic_pairs_bytes(rows: int, cols: int) -> int:
    return int(lib().ebic_pairs_bytes(rows, cols))


def ebic_pairs_words(rows: int) -> int:
    return int(lib().ebic_pairs_words(rows))


def ebic_pairs_prepare(m: Matrix, stream=None) -> Matrix:
    """Build the pair-comparison table of a prepared matrix (device memory
    from torch) and attach it to the matrix view."""
    nbytes = ebic_pairs_bytes(m.rows, m.cols)
    table = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device=m.ranks.device)
    _check(lib().ebic_pairs_prepare(ctypes.byref(m.view), table.data_ptr(), _stream(stream)))
    m.pairs = table
    return m


def ebic_pairs_strict_prepare(m: Matrix, stream=None) -> Matrix:
    """Build the strict pair table (the strict and loose tie rules take the
    pair form with both tables) and attach it to the matrix view."""
    nbytes = ebic_pairs_bytes(m.rows, m.cols)
    table = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device=m.ranks.device)
    _check(lib().ebic_pairs_strict_prepare(ctypes.byref(m.view), table.data_ptr(),
                                           _stream(stream)))
    m.pairs_strict = table
    return m


@dataclasses.dataclass
class Job:
    """One job of a batch; keeps the tensors its view points at alive."""
    matrix: Matrix
    pop: Population
    archive: Optional[Archive]
    params: ebic_params
    out: EvalOut

    def view(self) -> ebic_job:
        arch = self.archive.view if self.archive is not None else \
            ebic_archive(0, 0, None, None, None)
        return ebic_job(self.matrix.view, self.pop.view, arch, self.params, self.out.view)


def make_job(m: Matrix, pop: Population, archive: Optional[Archive] = None,
             params: Optional[ebic_params] = None, support=True, overlap=True) -> Job:
    params = params or make_params()
    K = archive.size if archive is not None else 0
    out = alloc_eval_out(pop.size, m.words, K, support, overlap, device=m.ranks.device)
    return Job(m, pop, archive, params, out)


class Batch:
    """A batch of jobs evaluated by one launch (ebic_batch_*)."""

    def __init__(self, jobs: Sequence[Job], graph: bool = False, gather: bool = False,
                 tune: bool = False):
        self.jobs = list(jobs)
        self._views = (ebic_job * len(self.jobs))(*[j.view() for j in self.jobs])
        flags = (EBIC_BATCH_GRAPH if graph else 0) | (EBIC_BATCH_GATHER if gather else 0) | \
            (EBIC_BATCH_TUNE if tune else 0)
        h = _vp()
        _check(lib().ebic_batch_create(self._views, len(self.jobs), flags, ctypes.byref(h)))
        self.handle = h

    def run(self, stream=None) -> None:
        _check(lib().ebic_batch_run(self.handle, _stream(stream)))

    def tuning(self):
        """(chunk groups per item, loads in flight, words per lane) in use;
        chunk groups 0 = the untuned default, chosen per job."""
        a, b, c = _i32(), _i32(), _i32()
        _check(lib().ebic_batch_tuning(self.handle, ctypes.byref(a), ctypes.byref(b),
                                       ctypes.byref(c)))
        return int(a.value), int(b.value), int(c.value)

    def set_tuning(self, chunks_per_item: int, loads_in_flight: int,
                   words_per_lane: int = 1) -> None:
        """Pin the item shape; later runs use it and do not tune."""
        _check(lib().ebic_batch_set_tuning(self.handle, chunks_per_item, loads_in_flight,
                                           words_per_lane))

    def profile(self, n: int) -> None:
        """Record kernel times for the next n runs."""
        _check(lib().ebic_batch_profile(self.handle, n))

    def timings(self, n: int) -> np.ndarray:
        """Kernel milliseconds of up to n recorded runs."""
        a = (ctypes.c_float * max(n, 1))()
        m = _i32(n)
        _check(lib().ebic_batch_timings(self.handle, a, ctypes.byref(m)))
        return np.array(a[:m.value])

    def close(self) -> None:
        if self.handle:
            lib().ebic_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ebic_evaluate_batched(jobs: Sequence[Job], stream=None) -> None:
    views = (ebic_job * len(jobs))(*[j.view() for j in jobs])
    _check(lib().ebic_evaluate_batched(views, len(jobs), _stream(stream)))


def ebic_evaluate_batched_noalloc(jobs: Sequence[Job], stream=None) -> None:
    """ebic_evaluate_batched without any allocation (job table in the
    library's fixed device array; at most EBIC_NOALLOC_MAX_JOBS jobs, each
    with its support output)."""
    views = (ebic_job * len(jobs))(*[j.view() for j in jobs])
    _check(lib().ebic_evaluate_batched_noalloc(views, len(jobs), _stream(stream)))


@dataclasses.dataclass
class Bicluster:
    rows: np.ndarray      # int64, ascending
    cols: np.ndarray      # int64, series order
    score: float
    row_dir: np.ndarray   # uint8 per row: 0 increasing trend, 1 reversed only

    @property
    def n(self) -> int:
        return int(self.rows.size)


@dataclasses.dataclass
class RunResult:
    biclusters: List[Bicluster]
    generations: int
    evaluations: int
    tabu_hits: int
    stop_reason: int
    trace: np.ndarray     # generations x 4


def _take_result(res) -> RunResult:
    """Copy a library-owned ebic_result into Python objects and free it."""
    try:
        r = res.contents
        bcs = []
        for j in range(r.count):
            b = r.biclusters[j]
            rows = np.ctypeslib.as_array(b.rows, (b.n_rows,)).astype(np.int64) if b.n_rows \
                else np.zeros(0, np.int64)
            cols = np.ctypeslib.as_array(b.cols, (b.n_cols,)).astype(np.int64)
            dirs = np.ctypeslib.as_array(b.row_dir, (b.n_rows,)).copy() if b.n_rows \
                else np.zeros(0, np.uint8)
            bcs.append(Bicluster(rows.copy(), cols.copy(), float(b.score), dirs))
        g = r.generations
        trace = np.ctypeslib.as_array(r.trace, (g * 4,)).reshape(g, 4).copy() if g else \
            np.zeros((0, 4))
        return RunResult(bcs, g, int(r.evaluations), int(r.tabu_hits), int(r.stop_reason), trace)
    finally:
        lib().ebic_result_free(res)


class TorchAllocator:
    """ebic_allocator backed by torch's caching allocator (device memory of
    a run then comes from, and returns to, torch's pool). Counts the calls."""

    def __init__(self, device=None):
        self.device = torch.cuda.current_device() if device is None else device
        self.allocs = 0
        self.releases = 0
        self.live = set()

        def _alloc(ctx, nbytes, stream):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                       stream if stream else None)
            except RuntimeError:
                return None
            self.allocs += 1
            self.live.add(int(p))
            return p

        def _release(ctx, ptr, stream):
            self.releases += 1
            self.live.discard(int(ptr))
            torch.cuda.caching_allocator_delete(ptr)

        self._a = ALLOC_FN(_alloc)
        self._r = RELEASE_FN(_release)
        self.view = ebic_allocator(self._a, self._r, None)


def _alloc_ref(alloc):
    return ctypes.byref(alloc.view) if alloc is not None else None


def ebic_run(x: np.ndarray, params: ebic_params, seed: int, stream=None,
             alloc: Optional[TorchAllocator] = None) -> RunResult:
    """The whole method on a host float32 matrix (synchronous)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    R, C = x.shape
    res = ctypes.POINTER(ebic_result)()
    _check(lib().ebic_run(x.ctypes.data, R, C, ctypes.byref(params), ctypes.c_uint64(seed),
                          _alloc_ref(alloc), _stream(stream), ctypes.byref(res)))
    return _take_result(res)


def ebic_run_device(x: np.ndarray, params: ebic_params, seed: int, stream=None,
                    alloc: Optional[TorchAllocator] = None) -> RunResult:
    """ebic_run with every generation after the first on the device; the
    same result for the same seed (synchronous)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    R, C = x.shape
    res = ctypes.POINTER(ebic_result)()
    _check(lib().ebic_run_device(x.ctypes.data, R, C, ctypes.byref(params),
                                 ctypes.c_uint64(seed), _alloc_ref(alloc), _stream(stream),
                                 ctypes.byref(res)))
    return _take_result(res)


def _bicluster_views(bics):
    """ctypes views of (rows, cols) pairs; the arrays are kept alive in keep."""
    keep, views = [], (ebic_bicluster * max(len(bics), 1))()
    for i, (rows, cols) in enumerate(bics):
        r = np.ascontiguousarray(rows, dtype=np.int32)
        c = np.ascontiguousarray(cols, dtype=np.uint16)
        keep += [r, c]
        views[i] = ebic_bicluster(int(r.size), r.ctypes.data_as(ctypes.POINTER(_i32)),
                                  int(c.size), c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                  0.0, None)
    return views, keep


def ebic_ce_score(found, truth, rows: int, cols: int):
    """(score D_max/|U|, Eq. 1 value (|U| - D_max)/|U|) of detected biclusters
    against the truth; each a sequence of (rows, cols) or Bicluster."""
    def pairs(bs):
        return [(b.rows, b.cols) if isinstance(b, Bicluster) else (b[0], b[1]) for b in bs]
    fv, k1 = _bicluster_views(pairs(found))
    tv, k2 = _bicluster_views(pairs(truth))
    score, ce = ctypes.c_double(), ctypes.c_double()
    _check(lib().ebic_ce_score(fv, len(found), tv, len(truth), rows, cols,
                               ctypes.byref(score), ctypes.byref(ce)))
    return score.value, ce.value


class Session:
    """A run of the method in steps, with checkpoints (ebic_session_*)."""

    def __init__(self, handle, alloc=None):
        self.handle = handle
        self.alloc = alloc  # kept alive while the session holds its memory

    @classmethod
    def create(cls, x: np.ndarray, params: ebic_params, seed: int, stream=None,
               alloc: Optional[TorchAllocator] = None) -> "Session":
        x = np.ascontiguousarray(x, dtype=np.float32)
        h = _vp()
        _check(lib().ebic_session_create(x.ctypes.data, x.shape[0], x.shape[1],
                                         ctypes.byref(params), ctypes.c_uint64(seed),
                                         _alloc_ref(alloc), _stream(stream), ctypes.byref(h)))
        return cls(h, alloc)

    @classmethod
    def restore(cls, x: np.ndarray, blob: bytes, stream=None,
                alloc: Optional[TorchAllocator] = None) -> "Session":
        x = np.ascontiguousarray(x, dtype=np.float32)
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        h = _vp()
        _check(lib().ebic_session_restore(x.ctypes.data, x.shape[0], x.shape[1], buf, len(blob),
                                          _alloc_ref(alloc), _stream(stream), ctypes.byref(h)))
        return cls(h, alloc)

    def step(self, steps: int) -> bool:
        """Up to `steps` evaluations; True once the run has finished."""
        done = _i32()
        _check(lib().ebic_session_step(self.handle, steps, ctypes.byref(done)))
        return bool(done.value)

    def checkpoint(self) -> bytes:
        n = ctypes.c_size_t(0)
        _check(lib().ebic_session_checkpoint(self.handle, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().ebic_session_checkpoint(self.handle, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def result(self) -> RunResult:
        res = ctypes.POINTER(ebic_result)()
        _check(lib().ebic_session_result(self.handle, ctypes.byref(res)))
        return _take_result(res)

    def close(self) -> None:
        if self.handle:
            lib().ebic_session_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Job server (ebic_server_*): continuous batching of runs on one GPU;
    jobs of at least device_loop_population individuals (0: none) run as
    device loops on device_loop_runners threads (0: 2)."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 0,
                 device_loop_population: int = 0, device_loop_runners: int = 0):
        cfg = ebic_server_config(hbm_budget, max_active, device_loop_population,
                                 device_loop_runners)
        h = _vp()
        _check(lib().ebic_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def submit(self, x: np.ndarray, params: ebic_params, seed: int) -> int:
        x = np.ascontiguousarray(x, dtype=np.float32)
        jid = ctypes.c_int64()
        _check(lib().ebic_server_submit(self.handle, x.ctypes.data, x.shape[0], x.shape[1],
                                        ctypes.byref(params), ctypes.c_uint64(seed),
                                        ctypes.byref(jid)))
        return int(jid.value)

    def poll(self, jid: int) -> Optional[RunResult]:
        res = ctypes.POINTER(ebic_result)()
        rc = _check(lib().ebic_server_poll(self.handle, jid, ctypes.byref(res)))
        return None if rc == EBIC_PENDING else _take_result(res)

    def wait(self, jid: int) -> RunResult:
        res = ctypes.POINTER(ebic_result)()
        _check(lib().ebic_server_wait(self.handle, jid, ctypes.byref(res)))
        return _take_result(res)

    def stats(self) -> dict:
        m = ebic_server_metrics()
        _check(lib().ebic_server_stats(self.handle, ctypes.byref(m)))
        return {n: getattr(m, n) for n, _ in ebic_server_metrics._fields_}

    def close(self) -> None:
        if self.handle:
            lib().ebic_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ebic_support_rows(support: torch.Tensor, sel: Sequence[int], counts: Sequence[int],
                      stream=None) -> List[np.ndarray]:
    """Row indices (ascending) of the selected individuals' supports."""
    P, W = support.shape
    dev = support.device
    sel_a = np.asarray(sel, dtype=np.int32)
    off = np.zeros(sel_a.size + 1, dtype=np.int32)
    off[1:] = np.cumsum(np.asarray(counts, dtype=np.int64))
    d_sel = torch.from_numpy(sel_a).to(dev) if sel_a.size else torch.zeros(1, dtype=torch.int32,
                                                                           device=dev)
    d_off = torch.from_numpy(off).to(dev)
    rows = torch.empty(max(int(off[-1]), 1), dtype=torch.int32, device=dev)
    _check(lib().ebic_support_rows(support.data_ptr(), P, W, d_sel.data_ptr(), int(sel_a.size),
                                   d_off.data_ptr(), rows.data_ptr(), _stream(stream)))
    torch.cuda.synchronize(dev)
    h = rows.cpu().numpy()
    return [h[off[i]:off[i + 1]].copy() for i in range(sel_a.size)]


def support_to_flags(words: torch.Tensor, rows: int) -> np.ndarray:
    """P x W support words (device or host) -> P x rows 0/1 flags on the host."""
    w = words.cpu().numpy().view(np.uint64) if isinstance(words, torch.Tensor) else words
    bits = np.unpackbits(w.view(np.uint8).reshape(w.shape[0], -1), axis=1, bitorder="little")
    return bits[:, :rows]


def flags_to_support(flags: np.ndarray, words: int) -> np.ndarray:
    """K x R 0/1 flags -> K x W uint64 words (bit r%64 of word r//64)."""
    K, R = flags.shape
    padded = np.zeros((K, words * 64), dtype=np.uint8)
    padded[:, :R] = flags
    return np.packbits(padded, axis=1, bitorder="little").view(np.uint64).reshape(K, words)
