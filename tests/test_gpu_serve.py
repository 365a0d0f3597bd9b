"""Job server: each job's result is identical alone (ebic_run) and in the
mix; jobs queue under a small HBM budget and complete; an oversized job
fails alone; stats report latency percentiles."""
import os
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2105_01196_amd import ebic
    return ebic


def _kw(R, C, P, G, neg=1, **kw):
    d = dict(approx_permille=850, negative_trends=neg, overlap_permille=750, min_rows=5,
             k_min=3, k_max=min(20, C), archive_size=20, n_out=5, population=P,
             generations=G, max_tabu_hits=100000, tournament=4, max_attempts=1000,
             k_score_min=3 if neg else 2)
    d.update(kw)
    return d


def _mix():
    """Jobs on matrices of different shapes (planted, log-normal)."""
    shapes = [(500, 40, 128, 6), (1000, 100, 256, 5), (3000, 60, 192, 4), (200, 25, 96, 8),
              (2000, 300, 256, 3), (777, 33, 64, 7)]
    jobs = []
    for j, (R, C, P, G) in enumerate(shapes):
        case = synth.job_matrix(synth.JobSpec(job=j, R=R, C=C, n_planted=3, population=P,
                                              seed=synth.JOB_SEED + j))
        jobs.append((case.X, _kw(R, C, P, G), 700 + j))
    return jobs


def _same(a, b):
    assert a.generations == b.generations and a.tabu_hits == b.tabu_hits
    assert a.stop_reason == b.stop_reason and a.evaluations == b.evaluations
    np.testing.assert_array_equal(a.trace, b.trace)
    assert len(a.biclusters) == len(b.biclusters)
    for x, y in zip(a.biclusters, b.biclusters):
        np.testing.assert_array_equal(x.rows, y.rows)
        np.testing.assert_array_equal(x.cols, y.cols)
        assert x.score == y.score


def test_alone_equals_mix(E):
    jobs = _mix()
    alone = [E.ebic_run(X, E.make_params(**kw), seed) for X, kw, seed in jobs]
    srv = E.Server()
    ids = [srv.submit(X, E.make_params(**kw), seed) for X, kw, seed in jobs[:3]]
    time.sleep(0.05)  # the rest arrive while the first ones run
    ids += [srv.submit(X, E.make_params(**kw), seed) for X, kw, seed in jobs[3:]]
    mixed = [srv.wait(i) for i in ids]
    for a, b in zip(alone, mixed):
        _same(a, b)
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["p50_latency_s"] > 0 and st["p99_latency_s"] >= st["p50_latency_s"]
    assert st["ticks"] < sum(kw["generations"] + 1 for _, kw, _ in jobs)  # shared launches
    srv.close()
    # one of them against the oracle's loop
    X, kw, seed = jobs[0]
    want = oracle.run(X, oracle.make_params(**kw), seed)
    assert mixed[0].generations == want.generations
    np.testing.assert_array_equal(mixed[0].trace, want.trace)
    for x, y in zip(mixed[0].biclusters, want.biclusters):
        np.testing.assert_array_equal(x.rows, y.rows)
        np.testing.assert_array_equal(x.cols, y.cols)


def test_device_loop_jobs_in_the_mix(E):
    """With a low population threshold the server runs the larger jobs as
    device loops on its runner threads and the rest in ticks; a job beyond
    the device loop's limits (tournament of 20) stays in the ticks. Every
    result equals ebic_run alone."""
    jobs = _mix()
    X, kw, seed = jobs[1]
    jobs.append((X, dict(kw, tournament=20), 777))
    alone = [E.ebic_run(x, E.make_params(**k), sd) for x, k, sd in jobs]
    srv = E.Server(device_loop_population=150, device_loop_runners=2)
    ids = [srv.submit(x, E.make_params(**k), sd) for x, k, sd in jobs]
    for a, i in zip(alone, ids):
        _same(a, srv.wait(i))
    st = srv.stats()
    # populations 256, 192 and 256 within the limits; 256 with a tournament of 20 is not
    assert st["device_loop_jobs"] == 3 and st["completed"] == len(jobs) and st["failed"] == 0
    assert st["ticks"] > 0 and st["device_loop_s"] > 0
    srv.close()


def test_many_clashing_candidates_in_the_mix(E):
    """Top-rank list updates that walk past the candidates whose supports
    a tick gathers (no overlap allowed, 12 columns) give the same result as
    the job alone."""
    X = synth.random_matrix(20000, 12, seed=11)
    kw = _kw(20000, 12, 600, 3, k_min=3, k_max=6, overlap_permille=0, n_out=20)
    jobs = [(X, kw, 13)] + _mix()[:2]
    alone = [E.ebic_run(x, E.make_params(**k), sd) for x, k, sd in jobs]
    srv = E.Server()
    ids = [srv.submit(x, E.make_params(**k), sd) for x, k, sd in jobs]
    for a, i in zip(alone, ids):
        _same(a, srv.wait(i))
    srv.close()


def test_many_small_jobs_churn(E):
    """Forty small jobs of mixed shapes, at most eight resident: ticks take
    whichever jobs have finished their host steps, staging slots are reused
    many times over, and every job still equals its run alone."""
    rng = np.random.default_rng(91)
    jobs = []
    for j in range(40):
        R, C = int(rng.integers(60, 900)), int(rng.integers(8, 60))
        X = synth.random_matrix(R, C, seed=900 + j)
        kw = _kw(R, C, int(rng.choice([32, 64, 128, 256])), int(rng.integers(2, 7)),
                 neg=int(j % 2), k_max=min(12, C), tie_rule=int(j % 3))
        jobs.append((X, kw, 950 + j))
    alone = [E.ebic_run(X, E.make_params(**kw), seed) for X, kw, seed in jobs]
    srv = E.Server(max_active=8)
    ids = [srv.submit(X, E.make_params(**kw), seed) for X, kw, seed in jobs]
    for a, i in zip(alone, ids):
        _same(a, srv.wait(i))
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    srv.close()


def test_small_budget_queues(E):
    jobs = _mix()[:4]
    alone = [E.ebic_run(X, E.make_params(**kw), seed) for X, kw, seed in jobs]
    srv = E.Server(hbm_budget=6 << 20)  # room for about one job at a time
    ids = [srv.submit(X, E.make_params(**kw), seed) for X, kw, seed in jobs]
    st = srv.stats()
    assert st["queued"] + st["active"] + st["completed"] == len(jobs)
    for a, i in zip(alone, ids):
        _same(a, srv.wait(i))
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["active"] == 0
    # a result is published before its job's memory is freed (on the
    # server's releaser thread); the budget comes back right after
    deadline = time.monotonic() + 10
    while srv.stats()["hbm_in_use"] and time.monotonic() < deadline:
        time.sleep(0.01)
    assert srv.stats()["hbm_in_use"] == 0
    srv.close()


def test_oversized_job_fails_alone(E):
    jobs = _mix()[:2]
    srv = E.Server(hbm_budget=8 << 20, max_active=2)
    big = synth.random_matrix(20000, 200, seed=1)
    bid = srv.submit(big, E.make_params(**_kw(20000, 200, 4096, 3)), 1)
    ids = [srv.submit(X, E.make_params(**kw), seed) for X, kw, seed in jobs]
    with pytest.raises(E.EbicError) as ei:
        srv.wait(bid)
    assert ei.value.code == E.EBIC_ERR_CAPACITY
    for (X, kw, seed), i in zip(jobs, ids):
        _same(E.ebic_run(X, E.make_params(**kw), seed), srv.wait(i))
    srv.close()


def test_submit_validates(E):
    srv = E.Server()
    X = synth.random_matrix(50, 10, seed=1)
    with pytest.raises(E.EbicError) as ei:
        srv.submit(X, E.make_params(**_kw(50, 10, 32, 2, k_min=1)), 1)
    assert ei.value.code == E.EBIC_ERR_INVALID_ARG
    srv.close()


def test_close_with_queued_jobs(E):
    srv = E.Server(hbm_budget=6 << 20, max_active=1)
    for X, kw, seed in _mix()[:4]:
        srv.submit(X, E.make_params(**kw), seed)
    srv.close()  # active job finishes, queued ones are dropped; no hang, no fault


def test_nonfinite_job_fails_alone(E):
    """One matrix with a NaN among six valid jobs, all submitted at once so
    their ingests run on the preparer threads together: only that job fails,
    with EBIC_ERR_NONFINITE, and every other job equals its run alone."""
    jobs = _mix()
    bad = jobs[2][0].copy()
    bad[17, 3] = np.nan
    alone = [E.ebic_run(X, E.make_params(**kw), seed) for X, kw, seed in jobs]
    srv = E.Server()
    ids = [srv.submit(X, E.make_params(**kw), seed) for X, kw, seed in jobs[:3]]
    bid = srv.submit(bad, E.make_params(**jobs[2][1]), 5)
    ids += [srv.submit(X, E.make_params(**kw), seed) for X, kw, seed in jobs[3:]]
    with pytest.raises(E.EbicError) as ei:
        srv.wait(bid)
    assert ei.value.code == E.EBIC_ERR_NONFINITE
    for a, i in zip(alone, ids):
        _same(a, srv.wait(i))
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 1
    srv.close()


# Eight jobs of the 64-job serving mix (500-50,000 rows x 20-2,000 columns,
# populations 256-4,096, 30 generations), one at each eighth of the mix
# ordered by matrix size, from the smallest to the largest.
SERVING_GENS = 30


def _serving_sample():
    specs = synth.serving_jobs(64)
    by_size = sorted(specs, key=lambda s: (s.R * s.C, s.job))
    return [by_size[i] for i in (0, 9, 18, 27, 36, 45, 54, 63)]


def _serving_kw(s):
    return dict(approx_permille=850, negative_trends=1, overlap_permille=750, min_rows=5,
                k_score_min=3, k_min=3, k_max=min(64, s.C), archive_size=20, n_out=20,
                population=s.population, generations=SERVING_GENS, max_tabu_hits=10 ** 9,
                tournament=4, max_attempts=1000)


@pytest.fixture(scope="module")
def serving_sample_results(E):
    """The eight jobs through the server together."""
    specs = _serving_sample()
    mats = [synth.job_matrix(s).X for s in specs]
    srv = E.Server()
    ids = [srv.submit(X, E.make_params(**_serving_kw(s)), s.seed) for s, X in zip(specs, mats)]
    res = [srv.wait(i) for i in ids]
    srv.close()
    return specs, mats, res


@pytest.mark.slow
@pytest.mark.parametrize("which", range(8))
def test_serving_mix_job_equals_oracle(E, serving_sample_results, which):
    specs, mats, res = serving_sample_results
    s, X, got = specs[which], mats[which], res[which]
    want = oracle.run(X, oracle.make_params(**_serving_kw(s)), s.seed,
                      nthreads=min(os.cpu_count() or 1, 16))
    assert (got.generations, got.evaluations, got.tabu_hits, got.stop_reason) == \
        (want.generations, want.evaluations, want.tabu_hits, want.stop_reason)
    np.testing.assert_array_equal(got.trace, want.trace)
    assert len(got.biclusters) == len(want.biclusters)
    for x, y in zip(got.biclusters, want.biclusters):
        np.testing.assert_array_equal(x.rows, y.rows)
        np.testing.assert_array_equal(x.cols, y.cols)
        assert x.score == y.score
