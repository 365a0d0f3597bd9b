"""GPU parity of the plain evaluator, ingest and support compaction against
the CPU oracle: counts, supports and overlaps bit-exact, FP64 fitness
bit-identical (relative tolerance 0). Every expected value comes from the
oracle on the same seeded inputs; archives are built from oracle supports."""
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
    d = dict(approx_permille=850, negative_trends=1, overlap_permille=750, min_rows=5)
    d.update(kw)
    if "k_score_min" not in d:
        d["k_score_min"] = 3 if d["negative_trends"] else 2
    return d


def _gpu_eval(E, X, seqs, kw, arch_flags=None, arch_series=None):
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    m = E.ebic_matrix_prepare(x)
    pop = E.ebic_population_upload(seqs, X.shape[1])
    arch = None
    if arch_series:
        arch = E.make_archive(E.flags_to_support(arch_flags, m.words), arch_series)
    out = E.ebic_evaluate(m, pop, arch, E.make_params(**kw))
    torch.cuda.synchronize()
    return out, m


def _check(E, X, seqs, kw, arch_flags=None, arch_series=None, sample=None):
    """Evaluate on the GPU; compare with the oracle on all (or sampled)
    individuals."""
    out, m = _gpu_eval(E, X, seqs, kw, arch_flags, arch_series)
    P, R = len(seqs), X.shape[0]
    idx = np.arange(P) if sample is None else np.asarray(sample)
    arch = oracle.Archive(arch_flags, arch_series) if arch_series else None
    ev = oracle.evaluate(X, [seqs[i] for i in idx], archive=arch,
                         params=oracle.make_params(**kw), nthreads=NCPU)
    cnt = out.count.cpu().numpy()[:P]
    fit = out.fitness.cpu().numpy()[:P]
    words = out.support.cpu().numpy().view(np.uint64)[:P]
    np.testing.assert_array_equal(cnt[idx], ev.count)
    np.testing.assert_array_equal(fit[idx].view(np.int64), ev.fitness.view(np.int64))
    flags = E.support_to_flags(words[idx], R)
    np.testing.assert_array_equal(flags, ev.support)
    # properties on every individual: count = |support|, padding bits clear
    allbits = np.unpackbits(words.view(np.uint8).reshape(P, -1), axis=1, bitorder="little")
    np.testing.assert_array_equal(allbits.sum(axis=1), cnt)
    assert not allbits[:, R:].any()
    if arch_series:
        ov = out.overlap.cpu().numpy()[:P, :len(arch_series)]
        np.testing.assert_array_equal(ov[idx], ev.overlap)
    return out, ev


def _all_series(C, kmax):
    import itertools
    out = []
    for k in range(2, kmax + 1):
        out += [list(s) for s in itertools.permutations(range(C), k)]
    return out


@pytest.mark.parametrize("kind", ["random", "ties"])
@pytest.mark.parametrize("approx,neg", [(1000, 0), (1000, 1), (850, 1), (700, 0), (0, 1)])
def test_brute_force_tiny(E, kind, approx, neg):
    X = synth.random_matrix(8, 6, seed=11) if kind == "random" else \
        synth.tie_matrix(8, 6, levels=3, seed=12)
    _check(E, X, _all_series(6, 6), _params(approx_permille=approx, negative_trends=neg,
                                              min_rows=1, k_score_min=2))


@pytest.mark.parametrize("rule", [1, 2])
@pytest.mark.parametrize("approx,neg", [(1000, 0), (1000, 1), (700, 0), (0, 1)])
def test_brute_force_tie_rules(E, rule, approx, neg):
    """Strict (a tie against both trends) and loose (against neither)."""
    X = synth.tie_matrix(8, 6, levels=3, seed=12)
    _check(E, X, _all_series(6, 6), _params(approx_permille=approx, negative_trends=neg,
                                              min_rows=1, k_score_min=2, tie_rule=rule))


def test_tiny_workload(E):
    case = synth.workload_matrix(0)
    seqs = synth.workload_population(0, case)
    _check(E, case.X, seqs, _params(negative_trends=0))


def test_plain_workload_1000x100(E):
    case = synth.workload_matrix(1)
    seqs = synth.workload_population(1, case)
    _check(E, case.X, seqs, _params())


def test_plain_workload_with_archive(E):
    """Overlap penalty against an archive of the 20 best (oracle-scored)
    individuals, members given as oracle supports."""
    case = synth.workload_matrix(1)
    seqs = synth.workload_population(1, case)
    kw = _params()
    ev = oracle.evaluate(case.X, seqs, params=oracle.make_params(**kw), nthreads=NCPU)
    top = [int(i) for i in np.argsort(-ev.score, kind="stable")[:20]]
    out, ev2 = _check(E, case.X, seqs, kw, arch_flags=ev.support[top],
                      arch_series=[seqs[i] for i in top])
    # members are penalised by their own archived copy
    assert np.all(ev2.fitness[top] <= ev.score[top] / 2)


def test_batched_workload_10000x500(E):
    case = synth.workload_matrix(2)
    seqs = synth.workload_population(2, case)
    _check(E, case.X, seqs, _params())


def test_large_workload_sampled(E):
    """40,000 x 1,000 with 8,192 individuals: GPU on all, oracle on a sample."""
    case = synth.workload_matrix(3)
    seqs = synth.workload_population(3, case)
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(len(seqs), 384, replace=False))
    _check(E, case.X, seqs, _params(), sample=sample)


@pytest.mark.parametrize("R,C", [(1, 2), (65, 3), (100, 2), (127, 9), (1000, 17)])
def test_ragged_shapes(E, R, C):
    X = synth.random_matrix(R, C, seed=R + C)
    rng = np.random.default_rng(R)
    seqs = [list(rng.permutation(C)[:int(rng.integers(2, C + 1))]) for _ in range(50)]
    for approx, neg in ((1000, 0), (800, 1)):
        _check(E, X, seqs, _params(approx_permille=approx, negative_trends=neg, min_rows=1,
                                   k_score_min=2))


@pytest.mark.parametrize("R,C", [(70, 16384), (129, 1025)])
def test_widest_rows(E, R, C):
    """Up to the widest matrix (EBIC_MAX_COLS columns): the ranks are the
    min-ranks (cells of the row strictly smaller, ties and signed zeros
    sharing one), and evaluation agrees with the oracle."""
    X = synth.tie_matrix(R, C, levels=C // 4, seed=C)
    x = torch.from_numpy(X).cuda()
    m = E.ebic_matrix_prepare(x)
    torch.cuda.synchronize()
    ranks = m.ranks.cpu().numpy().view(np.uint16).reshape(C, -1)[:, :R].T
    srt = np.sort(X, axis=1)
    want = np.stack([np.searchsorted(srt[r], X[r], side="left") for r in range(R)])
    np.testing.assert_array_equal(ranks, want)
    assert not m.ranks.cpu().numpy().view(np.uint16).reshape(C, -1)[:, R:].any()
    rng = np.random.default_rng(C)
    seqs = [list(rng.permutation(C)[:int(rng.integers(2, 40))]) for _ in range(60)] + \
        [list(rng.permutation(C)[:512]) for _ in range(2)]
    _check(E, X, seqs, _params(approx_permille=800, negative_trends=1, min_rows=1))


def test_longest_series(E):
    """k = 512 (the maximum), several tolerances."""
    X = synth.random_matrix(300, 600, seed=4)
    rng = np.random.default_rng(4)
    seqs = [list(rng.permutation(600)[:512]) for _ in range(4)] + \
        [list(np.argsort(X[0])[:512])]  # row 0 increasing along this one
    for approx in (1000, 700, 520, 0):
        _check(E, X, seqs, _params(approx_permille=approx, negative_trends=1, min_rows=1))


def test_ties_and_signed_zero(E):
    X = synth.tie_matrix(200, 12, levels=2, seed=9)
    X[:5] = 0.0
    X[5:10] = -0.0
    rng = np.random.default_rng(1)
    seqs = [list(rng.permutation(12)[:int(rng.integers(2, 13))]) for _ in range(200)]
    seqs += [list(range(12)), list(range(11, -1, -1))]
    for neg in (0, 1):
        _check(E, X, seqs, _params(approx_permille=900, negative_trends=neg, min_rows=1,
                                   k_score_min=2))


def test_invalid_individuals_marked(E):
    X = synth.random_matrix(70, 10, seed=3)
    x = torch.from_numpy(X).cuda()
    m = E.ebic_matrix_prepare(x)
    good = [3, 1, 4]
    series = [good, [5], [2, 2, 7], [1, 10], list(range(10)), good]
    off, cc = E.csr(series)
    pop = E.population_raw(off, cc)
    out = E.ebic_evaluate(m, pop, None, E.make_params(**_params(min_rows=1)))
    # an offset past the end of the column array is invalid too
    off2 = np.array([0, 3, 40], np.int32)
    pop2 = E.population_raw(off2, cc[:3])
    out2 = E.ebic_evaluate(m, pop2, None, E.make_params(**_params(min_rows=1)))
    torch.cuda.synchronize()
    cnt = out.count.cpu().numpy()
    fit = out.fitness.cpu().numpy()
    assert list(cnt[[1, 2, 3]]) == [-1, -1, -1]
    assert list(fit[[1, 2, 3]]) == [-1.0, -1.0, -1.0]
    assert not out.support.cpu().numpy()[[1, 2, 3]].any()
    ev = oracle.evaluate(X, [good, list(range(10)), good],
                         params=oracle.make_params(**_params(min_rows=1)))
    np.testing.assert_array_equal(cnt[[0, 4, 5]], ev.count)
    assert out2.count.cpu().numpy()[1] == -1 and out2.count.cpu().numpy()[0] == ev.count[0]


def test_empty_population(E):
    X = synth.random_matrix(64, 4, seed=2)
    m = E.ebic_matrix_prepare(torch.from_numpy(X).cuda())
    pop = E.population_raw(np.zeros(1, np.int32), np.zeros(0, np.uint16))
    E.ebic_evaluate(m, pop, None, E.make_params())
    torch.cuda.synchronize()


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_rejected(E, bad):
    X = synth.random_matrix(100, 5, seed=1)
    X[37, 2] = bad
    with pytest.raises(E.EbicError) as ei:
        E.ebic_matrix_prepare(torch.from_numpy(X).cuda())
    assert ei.value.code == E.EBIC_ERR_NONFINITE


def test_support_rows_compaction(E):
    case = synth.workload_matrix(1)
    seqs = synth.workload_population(1, case)[:100]
    kw = _params()
    out, m = _gpu_eval(E, case.X, seqs, kw)
    ev = oracle.evaluate(case.X, seqs, params=oracle.make_params(**kw), nthreads=NCPU)
    sel = [int(i) for i in np.argsort(-ev.count, kind="stable")[:12]] + [0, 99]
    rows = E.ebic_support_rows(out.support, sel, [int(ev.count[i]) for i in sel])
    for i, r in zip(sel, rows):
        np.testing.assert_array_equal(r, np.flatnonzero(ev.support[i]))


def test_repeated_launches_identical(E):
    case = synth.workload_matrix(2)
    seqs = synth.workload_population(2, case, P=512)
    kw = _params()
    x = torch.from_numpy(case.X).cuda()
    m = E.ebic_matrix_prepare(x)
    pop = E.ebic_population_upload(seqs, case.C)
    first = None
    for _ in range(10):
        out = E.ebic_evaluate(m, pop, None, E.make_params(**kw))
        torch.cuda.synchronize()
        cur = (out.count.cpu().numpy().tobytes(), out.fitness.cpu().numpy().tobytes(),
               out.support.cpu().numpy().tobytes())
        if first is None:
            first = cur
        assert cur == first
