"""ebic_run (host loop in the library, GPU evaluation) in lockstep with the
oracle's run: same seed -> same trajectory (population size, top-rank size,
best score and tabu hits after every generation), same stop, same
biclusters (rows, series, scores)."""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
NCPU = min(os.cpu_count() or 1, 16)


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2105_01196_amd import ebic
    return ebic


def _params(**kw):
    d = dict(approx_permille=850, negative_trends=0, overlap_permille=750, min_rows=5,
             k_min=2, k_max=8, archive_size=20, n_out=1, population=200, generations=50,
             max_tabu_hits=100000, tournament=4, max_attempts=1000)
    d.update(kw)
    d.setdefault("k_score_min", 3 if d["negative_trends"] else 2)
    return d


def _lockstep(E, X, kw, seed):
    got = E.ebic_run(X, E.make_params(**kw), seed)
    want = oracle.run(X, oracle.make_params(**kw), seed, nthreads=NCPU)
    assert got.generations == want.generations
    assert got.evaluations == want.evaluations
    assert got.tabu_hits == want.tabu_hits
    assert got.stop_reason == want.stop_reason
    np.testing.assert_array_equal(got.trace, want.trace)
    assert len(got.biclusters) == len(want.biclusters)
    for a, b in zip(got.biclusters, want.biclusters):
        np.testing.assert_array_equal(a.cols, b.cols)
        np.testing.assert_array_equal(a.rows, b.rows)
        assert a.score == b.score and a.n == b.n
    return got


def test_tiny_workload_lockstep(E):
    case = synth.workload_matrix(0)
    _lockstep(E, case.X, _params(n_out=5), synth.GA_SEED)


def test_strong_plant_recovered(E):
    case = synth.planted_matrix(100, 20, background="uniform", n_planted=1,
                                rows_range=(30, 30), cols_range=(5, 5), sigma=0.0, strict=True,
                                seed=1100)
    got = _lockstep(E, case.X, _params(), synth.GA_SEED)
    t = case.truth[0]
    top = got.biclusters[0]
    np.testing.assert_array_equal(top.cols, t.cols)
    assert set(t.rows.tolist()) <= set(top.rows.tolist())


def test_plain_workload_lockstep(E):
    w = synth.workload(1)
    case = synth.workload_matrix(1)
    kw = _params(negative_trends=1, k_min=w.k_min, k_max=w.k_max, population=w.population,
                 generations=w.generations, n_out=w.n_out)
    _lockstep(E, case.X, kw, synth.GA_SEED + 1)


def test_batched_workload_lockstep_few_generations(E):
    w = synth.workload(2)
    case = synth.workload_matrix(2)
    kw = _params(negative_trends=1, k_min=w.k_min, k_max=w.k_max, population=w.population,
                 generations=4, n_out=w.n_out)
    _lockstep(E, case.X, kw, synth.GA_SEED + 2)


def test_stops(E):
    X = synth.random_matrix(8, 4, seed=2)
    got = _lockstep(E, X, _params(k_min=2, k_max=4, population=10, generations=1000,
                                  max_tabu_hits=30), 1)
    assert got.stop_reason in (E.EBIC_STOP_TABU, E.EBIC_STOP_EXHAUSTED)
    # few distinct series: slots run out of attempts
    got = _lockstep(E, synth.random_matrix(6, 3, seed=3),
                    _params(k_min=2, k_max=3, population=40, generations=5, max_attempts=3), 7)
    assert got.stop_reason == E.EBIC_STOP_EXHAUSTED


def test_deterministic(E):
    case = synth.workload_matrix(0)
    a = E.ebic_run(case.X, E.make_params(**_params(generations=20, n_out=3)), 11)
    b = E.ebic_run(case.X, E.make_params(**_params(generations=20, n_out=3)), 11)
    np.testing.assert_array_equal(a.trace, b.trace)
    for x, y in zip(a.biclusters, b.biclusters):
        np.testing.assert_array_equal(x.rows, y.rows)
        np.testing.assert_array_equal(x.cols, y.cols)
