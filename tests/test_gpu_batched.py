"""GPU parity of the pair table and the batched evaluator (both forms)
against the CPU oracle, bit for bit; multi-job batches, graph replays,
processing orders and malformed input."""
import itertools
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


def _kw(**kw):
    d = dict(approx_permille=850, negative_trends=1, overlap_permille=750, min_rows=5)
    d.update(kw)
    d.setdefault("k_score_min", 3 if d["negative_trends"] else 2)
    return d


def _matrix(E, X, pairs=True, strict=False):
    m = E.ebic_matrix_prepare(torch.from_numpy(np.ascontiguousarray(X)).cuda())
    if pairs:
        E.ebic_pairs_prepare(m)
    if strict:
        E.ebic_pairs_strict_prepare(m)
    return m


def _check_job(E, job, X, seqs, kw, arch=None, sample=None):
    P, R = len(seqs), X.shape[0]
    idx = np.arange(P) if sample is None else np.asarray(sample)
    ev = oracle.evaluate(X, [seqs[i] for i in idx], archive=arch,
                         params=oracle.make_params(**kw), nthreads=NCPU)
    cnt = job.out.count.cpu().numpy()[:P]
    fit = job.out.fitness.cpu().numpy()[:P]
    words = job.out.support.cpu().numpy().view(np.uint64)[:P]
    np.testing.assert_array_equal(cnt[idx], ev.count)
    np.testing.assert_array_equal(fit[idx].view(np.int64), ev.fitness.view(np.int64))
    np.testing.assert_array_equal(E.support_to_flags(words[idx], R), ev.support)
    allbits = np.unpackbits(words.view(np.uint8).reshape(P, -1), axis=1, bitorder="little")
    np.testing.assert_array_equal(allbits.sum(axis=1), cnt)
    assert not allbits[:, R:].any()
    if arch is not None and arch.K:
        np.testing.assert_array_equal(job.out.overlap.cpu().numpy()[:P, :arch.K][idx], ev.overlap)


def _run(E, X, seqs, kw, arch_flags=None, arch_series=None, gather=False, graph=False,
         order=False, sample=None, strict=False):
    m = _matrix(E, X, pairs=not gather, strict=strict and not gather)
    pop = E.ebic_population_upload(seqs, X.shape[1])
    if order:
        E.set_order(pop, E.longest_first(seqs))
    arch = None
    if arch_series:
        arch = E.make_archive(E.flags_to_support(arch_flags, m.words), arch_series)
    job = E.make_job(m, pop, arch, E.make_params(**kw))
    b = E.Batch([job], graph=graph, gather=gather)
    b.run()
    torch.cuda.synchronize()
    _check_job(E, job, X, seqs, kw, oracle.Archive(arch_flags, arch_series) if arch_series
               else None, sample)
    b.close()
    return job


def test_pair_table_bits(E):
    """Table bit (pair, row) = the oracle's support of the 2-column series
    (lo, hi) without reversed trends: the rows where lo precedes hi."""
    for X in (synth.workload_matrix(0).X, synth.tie_matrix(130, 9, levels=3, seed=5)):
        R, C = X.shape
        m = _matrix(E, X)
        torch.cuda.synchronize()
        pairs = list(itertools.combinations(range(C), 2))
        ev = oracle.evaluate(X, [list(p) for p in pairs],
                             params=oracle.make_params(approx_permille=1000, negative_trends=0,
                                                       min_rows=1, k_score_min=2))
        S = E.ebic_pairs_words(R)
        assert S % 16 == 0 and m.words <= S < m.words + 16
        table = m.pairs.cpu().numpy().view(np.uint64).reshape(len(pairs), S)[:, :m.words]
        table = np.ascontiguousarray(table)
        np.testing.assert_array_equal(E.support_to_flags(table, R), ev.support)
        bits = np.unpackbits(table.view(np.uint8).reshape(len(pairs), -1), axis=1,
                             bitorder="little")
        assert not bits[:, R:].any()
        assert E.ebic_pairs_bytes(R, C) == len(pairs) * S * 8
        # the strict table: the rows where lo's value is strictly smaller
        E.ebic_pairs_strict_prepare(m)
        torch.cuda.synchronize()
        ev = oracle.evaluate(X, [list(p) for p in pairs],
                             params=oracle.make_params(approx_permille=1000, negative_trends=0,
                                                       min_rows=1, k_score_min=2,
                                                       tie_rule=E.EBIC_TIE_STRICT))
        table = m.pairs_strict.cpu().numpy().view(np.uint64).reshape(len(pairs), S)[:, :m.words]
        table = np.ascontiguousarray(table)
        np.testing.assert_array_equal(E.support_to_flags(table, R), ev.support)
        bits = np.unpackbits(table.view(np.uint8).reshape(len(pairs), -1), axis=1,
                             bitorder="little")
        assert not bits[:, R:].any()


@pytest.mark.parametrize("gather", [False, True])
@pytest.mark.parametrize("kind", ["random", "ties"])
@pytest.mark.parametrize("approx,neg", [(1000, 0), (850, 1), (700, 0), (0, 1)])
def test_brute_force_tiny(E, gather, kind, approx, neg):
    X = synth.random_matrix(8, 6, seed=11) if kind == "random" else \
        synth.tie_matrix(8, 6, levels=3, seed=12)
    seqs = [list(s) for k in range(2, 7) for s in itertools.permutations(range(6), k)]
    _run(E, X, seqs, _kw(approx_permille=approx, negative_trends=neg, min_rows=1,
                         k_score_min=2), gather=gather)


@pytest.mark.parametrize("gather", [False, True])
def test_tiny_and_plain_workloads(E, gather):
    for i, neg in ((0, 0), (1, 1)):
        case = synth.workload_matrix(i)
        _run(E, case.X, synth.workload_population(i, case), _kw(negative_trends=neg),
             gather=gather)


@pytest.mark.parametrize("gather", [False, True])
def test_batched_workload_with_archive(E, gather):
    case = synth.workload_matrix(2)
    seqs = synth.workload_population(2, case)
    kw = _kw()
    ev = oracle.evaluate(case.X, seqs, params=oracle.make_params(**kw), nthreads=NCPU)
    top = [int(i) for i in np.argsort(-ev.score, kind="stable")[:20]]
    _run(E, case.X, seqs, kw, arch_flags=ev.support[top], arch_series=[seqs[i] for i in top],
         gather=gather, order=True)


def test_widest_matrix_with_long_archive(E):
    """EBIC_MAX_COLS columns (gather form; a pair table would not fit) and
    an archive whose members hold 10,240 columns in all, past what the
    kernel keeps in LDS."""
    R, C = 70, 16384
    X = synth.tie_matrix(R, C, levels=C // 4, seed=C)
    rng = np.random.default_rng(7)
    seqs = [list(rng.permutation(C)[:int(rng.integers(2, 40))]) for _ in range(60)] + \
        [list(rng.permutation(C)[:512]) for _ in range(2)]
    arch_series = [list(rng.permutation(C)[:512]) for _ in range(20)]
    kw = _kw(approx_permille=600, negative_trends=1, min_rows=1)
    arch_flags = oracle.evaluate(X, arch_series, params=oracle.make_params(**kw),
                                 nthreads=NCPU).support
    _run(E, X, seqs, kw, arch_flags=arch_flags, arch_series=arch_series, gather=True)


def test_large_workload_sampled(E):
    case = synth.workload_matrix(3)
    seqs = synth.workload_population(3, case)
    sample = np.sort(np.random.default_rng(8).choice(len(seqs), 384, replace=False))
    _run(E, case.X, seqs, _kw(), order=True, sample=sample)


@pytest.mark.slow
def test_large_workload_gather_equals_table_with_archives(E):
    """large-40000x1000 in full: 8,192 individuals as 8 populations of
    1,024, each against a 20-member archive (its own top 20 by score), in
    one launch of the pair form and one of the gather form. Count, support,
    overlap and fitness bits agree for every individual, and a sample of 256
    individuals matches the oracle with its archive."""
    case = synth.workload_matrix(3)
    X, R, C = case.X, case.R, case.C
    seqs = synth.workload_population(3, case)
    kw = _kw()
    m = _matrix(E, X)
    jobs_t, jobs_g, archs = [], [], []
    rng = np.random.default_rng(12)
    for j in range(8):
        part = seqs[j * 1024:(j + 1) * 1024]
        pop = E.ebic_population_upload(part, C)
        E.set_order(pop, E.longest_first(part))
        first = E.ebic_evaluate(m, pop, None, E.make_params(**kw))
        torch.cuda.synchronize()
        fit = first.fitness.cpu().numpy()[:len(part)]
        top = [int(i) for i in np.argsort(-fit, kind="stable")[:20]]
        arch = E.archive_from_device(first.support, top, part)
        flags = E.support_to_flags(first.support[top], R)
        archs.append((part, oracle.Archive(flags, [part[i] for i in top])))
        jobs_t.append(E.make_job(m, pop, arch, E.make_params(**kw)))
        jobs_g.append(E.make_job(m, pop, arch, E.make_params(**kw)))
    bt, bg = E.Batch(jobs_t), E.Batch(jobs_g, gather=True)
    bt.run()
    bg.run()
    torch.cuda.synchronize()
    for jt, jg in zip(jobs_t, jobs_g):
        assert torch.equal(jt.out.count, jg.out.count)
        assert torch.equal(jt.out.fitness, jg.out.fitness)
        assert torch.equal(jt.out.support, jg.out.support)
        assert torch.equal(jt.out.overlap, jg.out.overlap)
    pen = 0
    for j in (0, 5):
        part, arch = archs[j]
        sample = np.sort(rng.choice(len(part), 128, replace=False))
        _check_job(E, jobs_t[j], X, part, kw, arch=arch, sample=sample)
        cnt = jobs_t[j].out.count.cpu().numpy()[:len(part)]
        pen += int((jobs_t[j].out.fitness.cpu().numpy()[:len(part)] <
                    np.ldexp(cnt.astype(np.float64), [len(s) for s in part])).sum())
    assert pen > 0  # the archives penalise some individuals
    bt.close()
    bg.close()


@pytest.mark.parametrize("approx", [1000, 900, 700, 500, 300, 0])
def test_tolerance_regimes(E, approx):
    """Thermometer counters (t+1 <= 16) and exact bit-sliced counters (larger
    t), up to the longest series."""
    X = synth.random_matrix(777, 600, seed=6)
    rng = np.random.default_rng(approx)
    seqs = [list(rng.permutation(600)[:int(k)]) for k in rng.integers(2, 65, 120)]
    seqs += [list(rng.permutation(600)[:512]), list(np.argsort(X[3])[:300])]
    for neg in (0, 1):
        _run(E, X, seqs, _kw(approx_permille=approx, negative_trends=neg, min_rows=1))


def _descent_rows(C):
    """Row d (d < C) has exactly d descents along columns 0..C-1:
    d, d-1, ..., 0, d+1, ..., C-1; then the same rows negated, whose
    prefixes hold every count of ascents."""
    rows = [np.r_[np.arange(d, -1, -1), np.arange(d + 1, C)] for d in range(C)]
    X = np.array(rows, np.float32)
    return np.vstack([X, -X])


def _approx_for(k, t):
    """An approx (per mille) whose tolerance for length k is exactly t, or None."""
    for a in range(1000, -1, -1):
        if ((k - 1) * (1000 - a)) // 1000 == t:
            return a
    return None


@pytest.mark.parametrize("shape", [(1, 2, 1), (1, 4, 1), (2, 2, 1), (4, 4, 1), (1, 2, 2),
                                   (1, 4, 2), (2, 2, 2), (1, 8, 1), (2, 8, 1)])
def test_step_counts_at_counter_boundaries(E, shape):
    """Every count of steps against a trend, from 0 to k-1, meets tolerances
    at each counter width boundary (t = 2^P - 1 and 2^P) and beyond the
    widest pair-path counter, for every item shape."""
    C = 512
    X = _descent_rows(C)
    m = _matrix(E, X)
    rng = np.random.default_rng(11)
    for t in (0, 1, 2, 3, 4, 7, 8, 15, 16, 31, 32, 63, 64, 127, 128, 255, 256, 511):
        for k in sorted({min(C, t + 1), min(C, t + 2), min(C, 2 * t + 3), min(C, 4 * t + 5)}):
            a = _approx_for(k, t)
            if a is None or k < 2:
                continue
            cols = np.arange(k)
            seqs = [list(cols), list(cols[::-1]), list(rng.permutation(k)),
                    list(np.r_[cols[1:], cols[:1]])]
            pop = E.ebic_population_upload(seqs, C)
            for neg in (0, 1):
                kw = _kw(approx_permille=a, negative_trends=neg, min_rows=1)
                job = E.make_job(m, pop, None, E.make_params(**kw))
                b = E.Batch([job])
                b.set_tuning(*shape)
                assert b.tuning() == shape
                b.run()
                torch.cuda.synchronize()
                _check_job(E, job, X, seqs, kw)
                b.close()


def test_set_tuning_rejects_other_shapes(E):
    X = synth.random_matrix(100, 20, seed=3)
    m = _matrix(E, X)
    pop = E.ebic_population_upload([[0, 1, 2]], 20)
    b = E.Batch([E.make_job(m, pop, None, E.make_params(**_kw()))])
    for bad in ((3, 2, 1), (1, 3, 1), (0, 2, 1), (8, 4, 1), (1, 2, 3), (1, 2, 0), (1, 8, 2),
                (1, 16, 1)):
        with pytest.raises(Exception):
            b.set_tuning(*bad)
    b.set_tuning(2, 4, 2)
    assert b.tuning() == (2, 4, 2)
    b.close()


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_tie_rules(E, rule):
    """Tie-heavy rows and constant-row biclusters under each tie rule, in
    three forms: the pair table alone (the strict and loose rules then take
    the gather form), both pair tables (every rule in the pair form), and
    the gather form."""
    X = synth.tie_matrix(777, 64, levels=3, seed=31)
    case = synth.planted_matrix(500, 40, background="normal", n_planted=3,
                                rows_range=(40, 60), cols_range=(4, 12), sigma=0.0,
                                seed=32, pattern="constant-row")
    rng = np.random.default_rng(33 + rule)
    for M in (X, case.X):
        C = M.shape[1]
        seqs = [list(rng.permutation(C)[:int(k)]) for k in rng.integers(2, min(C, 64) + 1, 150)]
        seqs += [list(t.cols) for t in getattr(case, "truth", [])] if M is case.X else []
        for neg in (0, 1):
            for approx in (1000, 850, 500):
                kw = _kw(approx_permille=approx, negative_trends=neg, min_rows=1,
                         tie_rule=rule)
                _run(E, M, seqs, kw)
                _run(E, M, seqs, kw, strict=True)
                _run(E, M, seqs, kw, gather=True)


def test_mixed_tie_rules_in_one_batch(E):
    """Jobs under all three tie rules in one launch over a matrix with both
    pair tables: each job equals the oracle under its own rule."""
    X = synth.tie_matrix(700, 48, levels=4, seed=41)
    m = _matrix(E, X, strict=True)
    rng = np.random.default_rng(42)
    jobs, cases = [], []
    for rule in (E.EBIC_TIE_INDEX, E.EBIC_TIE_STRICT, E.EBIC_TIE_LOOSE, E.EBIC_TIE_STRICT):
        seqs = [list(rng.permutation(48)[:int(k)]) for k in rng.integers(2, 33, 120)]
        kw = _kw(approx_permille=800, negative_trends=int(rule != E.EBIC_TIE_LOOSE), min_rows=1,
                 tie_rule=rule)
        pop = E.ebic_population_upload(seqs, 48)
        jobs.append(E.make_job(m, pop, None, E.make_params(**kw)))
        cases.append((seqs, kw))
    b = E.Batch(jobs)
    b.run()
    torch.cuda.synchronize()
    for job, (seqs, kw) in zip(jobs, cases):
        _check_job(E, job, X, seqs, kw)
    b.close()


def test_pattern_biclusters(E):
    """The paper's benchmark types planted (shift, scale, shift-scale): their
    series keep every planted row, in both forms."""
    for pattern in ("shift", "scale", "shift-scale"):
        case = synth.planted_matrix(2000, 60, background="lognormal", n_planted=4,
                                    rows_range=(50, 200), cols_range=(5, 20), sigma=0.0,
                                    reverse_odd=True, seed=34, pattern=pattern)
        seqs = [list(t.cols) for t in case.truth]
        kw = _kw(approx_permille=1000, negative_trends=1, min_rows=1)
        job = _run(E, case.X, seqs, kw)
        flags = E.support_to_flags(job.out.support.cpu().numpy().view(np.uint64)[:len(seqs)],
                                   case.R)
        for i, t in enumerate(case.truth):
            assert flags[i][t.rows].all(), pattern


def test_multi_job_batch(E):
    """Jobs on different matrices and parameters in one launch, each equal to
    its own oracle evaluation; one job in gather form (no table)."""
    specs = [(0, _kw(negative_trends=0), True), (1, _kw(), True), (2, _kw(), False),
             (1, _kw(approx_permille=600, negative_trends=0), True)]
    jobs, data = [], []
    for i, kw, pairs in specs:
        case = synth.workload_matrix(i)
        seqs = synth.workload_population(i, case, P=300)
        m = _matrix(E, case.X, pairs=pairs)
        pop = E.ebic_population_upload(seqs, case.C)
        jobs.append(E.make_job(m, pop, None, E.make_params(**kw)))
        data.append((case.X, seqs, kw))
    b = E.Batch(jobs)
    b.run()
    torch.cuda.synchronize()
    for job, (X, seqs, kw) in zip(jobs, data):
        _check_job(E, job, X, seqs, kw)
    b.close()


@pytest.mark.parametrize("shape", [(1, 2, 1), (2, 4, 1), (4, 2, 1), (1, 2, 2), (2, 4, 2),
                                   (2, 8, 1)])
def test_uneven_jobs_interleaved(E, shape):
    """Jobs of uneven item counts (including an empty population) share one
    launch through the round-robin item schedule and its phases; each job
    equals its own oracle evaluation, archives and processing orders
    included."""
    specs = [(2, 37, True), (0, 0, False), (2, 513, True), (1, 5, False), (3, 200, True),
             (1, 300, True)]
    jobs, data = [], []
    for n, (wi, P, with_arch) in enumerate(specs):
        case = synth.workload_matrix(wi)
        seqs = synth.workload_population(wi, case, P=max(P, 1), seed=synth.POP_SEED + 50 + n)[:P]
        kw = _kw(approx_permille=(850, 700, 900, 1000, 850, 600)[n], negative_trends=n % 2)
        m = _matrix(E, case.X)
        pop = E.ebic_population_upload(seqs, case.C)
        if P:
            E.set_order(pop, E.longest_first(seqs))
        arch = oarch = None
        if with_arch and P:
            ev = oracle.evaluate(case.X, seqs, params=oracle.make_params(**kw), nthreads=NCPU)
            top = [int(i) for i in np.argsort(-ev.score, kind="stable")[:min(8, P)]]
            series = [seqs[i] for i in top]
            arch = E.make_archive(E.flags_to_support(ev.support[top], m.words), series)
            oarch = oracle.Archive(ev.support[top], series)
        jobs.append(E.make_job(m, pop, arch, E.make_params(**kw)))
        data.append((case.X, seqs, kw, oarch))
    b = E.Batch(jobs)
    b.set_tuning(*shape)
    b.run()
    torch.cuda.synchronize()
    for job, (X, seqs, kw, oarch) in zip(jobs, data):
        if seqs:
            _check_job(E, job, X, seqs, kw, oarch)
    b.close()


@pytest.mark.parametrize("shape", [(1, 2, 1), (2, 4, 1), (1, 2, 2)])
def test_mixed_row_counts_widen_items(E, shape):
    """Jobs of 40,000, 20,000, 10,000 and 1,000 rows in one launch: the
    larger jobs' items are widened to at most four per individual (ten and
    five 4,096-row chunks here) so the small job's workgroups carry no idle
    waves; every job equals the oracle, archives included (the 40,000-row
    job on a sample)."""
    specs = [(40000, 48, 300, True), (20000, 40, 200, False), (10000, 30, 150, True),
             (1000, 25, 120, True)]
    jobs, data = [], []
    for n, (R, C, P, with_arch) in enumerate(specs):
        X = synth.planted_matrix(R, C, background="lognormal", n_planted=3,
                                 rows_range=(R // 50, R // 10), cols_range=(4, 10), sigma=0.1,
                                 seed=70 + n).X
        rng = np.random.default_rng(80 + n)
        seqs = [list(map(int, rng.permutation(C)[:int(rng.integers(2, 17))])) for _ in range(P)]
        kw = _kw(approx_permille=(850, 700, 900, 800)[n], negative_trends=(1, 0, 1, 1)[n])
        m = _matrix(E, X)
        pop = E.ebic_population_upload(seqs, C)
        E.set_order(pop, E.longest_first(seqs))
        arch = oarch = None
        if with_arch:
            ev = oracle.evaluate(X, seqs[:60], params=oracle.make_params(**kw), nthreads=NCPU)
            top = [int(i) for i in np.argsort(-ev.score, kind="stable")[:8]]
            series = [seqs[i] for i in top]
            arch = E.make_archive(E.flags_to_support(ev.support[top], m.words), series)
            oarch = oracle.Archive(ev.support[top], series)
        jobs.append(E.make_job(m, pop, arch, E.make_params(**kw)))
        data.append((X, seqs, kw, oarch))
    b = E.Batch(jobs)
    b.set_tuning(*shape)
    b.run()
    torch.cuda.synchronize()
    for n, (job, (X, seqs, kw, oarch)) in enumerate(zip(jobs, data)):
        sample = np.arange(0, len(seqs), 5) if n == 0 else None
        _check_job(E, job, X, seqs, kw, oarch, sample=sample)
    b.close()


@pytest.mark.parametrize("R,shape", [(1000, (1, 2, 1)), (6000, (1, 2, 1)), (6000, (2, 4, 1)),
                                     (12000, (1, 4, 1)), (1000, (1, 2, 2))])
def test_several_individuals_per_workgroup(E, R, shape):
    """Rows of one or two 4,096-row chunks put four or two individuals in a
    workgroup (consecutive slots, each with its own waves and LDS, barriers
    shared), three chunks one; populations of 1-13 individuals leave the last
    workgroup partly idle, and two jobs share each launch, so a workgroup
    can hold individuals of both. Every job equals the oracle, archives and
    processing orders included."""
    case = synth.planted_matrix(R, 30, background="lognormal", n_planted=2,
                                rows_range=(20, 200), cols_range=(4, 12), sigma=0.1,
                                seed=77 + R)
    m = _matrix(E, case.X, pairs=True)
    for n, (P1, P2) in enumerate([(1, 2), (3, 5), (6, 1), (13, 7)]):
        jobs, data = [], []
        for j, P in enumerate((P1, P2)):
            seqs = synth.population(case.C, P, 2, 20, seed=synth.POP_SEED + 900 + 10 * n + j,
                                    truth=case.truth, planted_frac=0.3)
            kw = _kw(approx_permille=(850, 700)[j], negative_trends=j)
            pop = E.ebic_population_upload(seqs, case.C)
            E.set_order(pop, E.longest_first(seqs))
            arch = oarch = None
            if j == 0:
                ev = oracle.evaluate(case.X, seqs, params=oracle.make_params(**kw), nthreads=NCPU)
                top = [int(i) for i in np.argsort(-ev.score, kind="stable")[:min(4, P)]]
                series = [seqs[i] for i in top]
                arch = E.make_archive(E.flags_to_support(ev.support[top], m.words), series)
                oarch = oracle.Archive(ev.support[top], series)
            jobs.append(E.make_job(m, pop, arch, E.make_params(**kw)))
            data.append((seqs, kw, oarch))
        b = E.Batch(jobs, graph=n % 2 == 1)  # every other batch replays a graph
        b.set_tuning(*shape)
        for _ in range(2):
            b.run()
            torch.cuda.synchronize()
            for job, (seqs, kw, oarch) in zip(jobs, data):
                _check_job(E, job, case.X, seqs, kw, oarch)
        b.close()


def test_graph_replays_track_new_contents(E):
    """A graph-backed batch replayed over populations rewritten in place
    (same lengths, new columns): every replay equals the oracle."""
    case = synth.workload_matrix(1)
    kw = _kw()
    m = _matrix(E, case.X)
    rng = np.random.default_rng(3)
    lens = rng.integers(3, 21, 400)
    pops = [[list(rng.permutation(case.C)[:int(k)]) for k in lens] for _ in range(3)]
    pop = E.ebic_population_upload(pops[0], case.C)
    job = E.make_job(m, pop, None, E.make_params(**kw))
    b = E.Batch([job], graph=True)
    for rep in range(3):
        new = E.ebic_population_upload(pops[rep], case.C)
        pop.offsets.copy_(new.offsets)
        pop.cols.copy_(new.cols)
        torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        _check_job(E, job, case.X, pops[rep], kw)
        junk = torch.ones(1 << 20, device="cuda").sum()  # eager work between replays
        assert float(junk) == float(1 << 20)
    b.close()


def test_batched_equals_plain(E):
    case = synth.workload_matrix(2)
    seqs = synth.workload_population(2, case, P=1024)
    kw = E.make_params(**_kw())
    m = _matrix(E, case.X)
    pop = E.ebic_population_upload(seqs, case.C)
    plain = E.ebic_evaluate(m, pop, None, kw)
    job = E.make_job(m, pop, None, kw)
    E.ebic_evaluate_batched([job])
    torch.cuda.synchronize()
    for a, b in ((plain.count, job.out.count), (plain.fitness, job.out.fitness),
                 (plain.support, job.out.support)):
        assert torch.equal(a, b)


def test_malformed_individuals_marked(E):
    X = synth.random_matrix(3000, 10, seed=3)
    m = _matrix(E, X)
    good = [3, 1, 4]
    series = [good, [5], [2, 2, 7], [1, 10], [2, 7, 2], list(range(10)), good]
    off, cc = E.csr(series)
    pop = E.population_raw(off, cc)
    job = E.make_job(m, pop, None, E.make_params(**_kw(min_rows=1)))
    E.ebic_evaluate_batched([job])
    torch.cuda.synchronize()
    cnt = job.out.count.cpu().numpy()
    assert list(cnt[[1, 2, 3, 4]]) == [-1] * 4
    assert list(job.out.fitness.cpu().numpy()[[1, 2, 3, 4]]) == [-1.0] * 4
    assert not job.out.support.cpu().numpy()[[1, 2, 3, 4]].any()
    ev = oracle.evaluate(X, [good, list(range(10)), good],
                         params=oracle.make_params(**_kw(min_rows=1)))
    np.testing.assert_array_equal(cnt[[0, 5, 6]], ev.count)


def test_autotuned_batch_identical(E, tmp_path, monkeypatch):
    """A tuned batch (every item shape timed on the first run) gives the
    plain path's results bit for bit, records its choice in the JSON cache,
    and a graph-backed tuned batch replays the same results."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("EBIC_TUNE_CACHE", str(cache))
    case = synth.workload_matrix(2)
    seqs = synth.workload_population(2, case, P=777)
    kw = E.make_params(**_kw())
    m = _matrix(E, case.X)
    pop = E.ebic_population_upload(seqs, case.C)
    plain = E.ebic_evaluate(m, pop, None, kw)
    for graph in (False, True):
        job = E.make_job(m, pop, None, kw)
        b = E.Batch([job], tune=True, graph=graph)
        for _ in range(2):
            b.run()
            torch.cuda.synchronize()
            for x, y in ((plain.count, job.out.count), (plain.fitness, job.out.fitness),
                         (plain.support, job.out.support)):
                assert torch.equal(x, y)
        cpi, kb, wpl = b.tuning()
        assert cpi in (1, 2, 4) and kb in (2, 4, 8) and wpl in (1, 2)
        assert kb < 8 or wpl == 1
        b.close()
    text = cache.read_text()
    assert "_i777_j1" in text and "[" in text
