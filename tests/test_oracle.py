"""Pins for the CPU oracle: each check rests on something other than the
oracle itself -- brute force with an independent formulation, textbook
Eulerian numbers, published RNG outputs, exact invariants and planted
recovery."""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth


def _eulerian_table(golden_dir):
    rows = {}
    with open(os.path.join(golden_dir, "eulerian_numbers.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, vals = line.split(":")
            rows[int(n)] = [int(v) for v in vals.split()]
    return rows


def _brute_support(X, series, approx, neg):
    """Independent formulation: order the series' cells of each row by
    (value, column index) with Python's sort, read off the induced
    permutation, and count its descents and ascents."""
    k = len(series)
    t = ((k - 1) * (1000 - approx)) // 1000
    out = []
    for row in X:
        order = sorted(range(k), key=lambda j: (float(row[series[j]]), series[j]))
        rank = [0] * k
        for pos, j in enumerate(order):
            rank[j] = pos
        desc = sum(rank[j] > rank[j + 1] for j in range(k - 1))
        asc = (k - 1) - desc
        out.append(int(desc <= t or (neg and asc <= t)))
    return np.array(out, dtype=np.uint8)


def _all_series(C, kmax):
    for k in range(2, kmax + 1):
        yield from itertools.permutations(range(C), k)


@pytest.mark.parametrize("kind", ["random", "ties"])
@pytest.mark.parametrize("approx,neg", [(1000, 0), (1000, 1), (850, 1), (700, 0), (500, 1),
                                        (0, 0)])
def test_brute_force_all_series(kind, approx, neg):
    C, R = 6, 8
    if kind == "random":
        X = synth.random_matrix(R, C, seed=11)
    else:
        X = synth.tie_matrix(R, C, levels=3, seed=12)
    seqs = [list(s) for s in _all_series(C, C)]
    p = oracle.make_params(approx_permille=approx, negative_trends=neg, min_rows=1,
                           k_score_min=2)
    ev = oracle.evaluate(X, seqs, params=p)
    for i, s in enumerate(seqs):
        want = _brute_support(X, s, approx, neg)
        np.testing.assert_array_equal(ev.support[i], want, err_msg=str(s))
        assert ev.count[i] == want.sum()


def test_eulerian_closed_form(golden_dir):
    A = _eulerian_table(golden_dir)
    for k in range(2, 8):
        perms = np.array(list(itertools.permutations(range(k))), dtype=np.float32)
        for approx in (1000, 900, 850, 700, 500, 300, 0):
            t = ((k - 1) * (1000 - approx)) // 1000
            for neg in (0, 1):
                p = oracle.make_params(approx_permille=approx, negative_trends=neg,
                                       min_rows=1, k_score_min=2)
                ev = oracle.evaluate(perms, [list(range(k))], params=p)
                # rows = all permutations; a row's descents along the series
                # are the descents of the permutation's inverse, which has the
                # same descent distribution
                want = sum(A[k][d] for d in range(k)
                           if d <= t or (neg and (k - 1 - d) <= t))
                assert ev.count[0] == want, (k, approx, neg)


def test_eulerian_printed_examples():
    """k=5: t=0 -> 1 (2 with reversed trends); t=1 -> 27 (54); k=6, t=1 -> 58 (116)."""
    for k, approx, want in ((5, 1000, (1, 2)), (5, 700, (27, 54)), (6, 800, (58, 116))):
        perms = np.array(list(itertools.permutations(range(k))), dtype=np.float32)
        got = []
        for neg in (0, 1):
            p = oracle.make_params(approx_permille=approx, negative_trends=neg, min_rows=1,
                                   k_score_min=2)
            got.append(int(oracle.evaluate(perms, [list(range(k))], params=p).count[0]))
        assert tuple(got) == want


def test_two_column_special_cases():
    X = synth.random_matrix(50, 7, seed=3)
    X[5, 2] = X[5, 4]  # a tie: the smaller column index comes first
    p0 = oracle.make_params(negative_trends=0, min_rows=1, k_score_min=2)
    p1 = oracle.make_params(negative_trends=1, min_rows=1, k_score_min=2)
    seqs = [[2, 4], [4, 2], [0, 6]]
    e0 = oracle.evaluate(X, seqs, params=p0)
    e1 = oracle.evaluate(X, seqs, params=p1)
    for i, (a, b) in enumerate(seqs):
        want = (X[:, a] < X[:, b]) | ((X[:, a] == X[:, b]) & (a < b))
        np.testing.assert_array_equal(e0.support[i].astype(bool), want)
        assert e1.count[i] == X.shape[0]


def test_invariants():
    rng = np.random.default_rng(5)
    X = synth.random_matrix(40, 9, seed=6)
    seqs = [list(rng.permutation(9)[:int(rng.integers(2, 10))]) for _ in range(60)]
    base = dict(min_rows=1, k_score_min=2)
    for neg in (0, 1):
        p = oracle.make_params(approx_permille=800, negative_trends=neg, **base)
        ev = oracle.evaluate(X, seqs, params=p)
        # row permutation permutes supports
        perm = rng.permutation(X.shape[0])
        evp = oracle.evaluate(X[perm], seqs, params=p)
        np.testing.assert_array_equal(evp.support, ev.support[:, perm])
        # within-row ranks (index tie-break) leave every support unchanged
        ranks = np.argsort(np.argsort(X, axis=1, kind="stable"), axis=1).astype(np.float32)
        np.testing.assert_array_equal(oracle.evaluate(ranks, seqs, params=p).support,
                                      ev.support)
        # column relabelling (tie-free matrix)
        cp = rng.permutation(X.shape[1])
        inv = np.argsort(cp)
        Xc = X[:, cp]
        seqs_c = [[int(inv[c]) for c in s] for s in seqs]
        np.testing.assert_array_equal(oracle.evaluate(Xc, seqs_c, params=p).support,
                                      ev.support)
        # count is the size of the support
        np.testing.assert_array_equal(ev.count, ev.support.sum(axis=1))
    # reversed trends: support = support(I) | support(reverse I) without them
    p0 = oracle.make_params(approx_permille=800, negative_trends=0, **base)
    p1 = oracle.make_params(approx_permille=800, negative_trends=1, **base)
    e_fwd = oracle.evaluate(X, seqs, params=p0)
    e_rev = oracle.evaluate(X, [s[::-1] for s in seqs], params=p0)
    e_neg = oracle.evaluate(X, seqs, params=p1)
    np.testing.assert_array_equal(e_neg.support, e_fwd.support | e_rev.support)
    np.testing.assert_array_equal(oracle.evaluate(X, [s[::-1] for s in seqs], params=p1).support,
                                  e_neg.support)
    # the count never falls as the tolerance grows
    prev = None
    for approx in (1000, 900, 800, 600, 400, 0):
        c = oracle.evaluate(X, seqs, params=oracle.make_params(approx_permille=approx,
                                                               negative_trends=1, **base)).count
        if prev is not None:
            assert np.all(c >= prev)
        prev = c


def _sequences(levels, k):
    """Every sequence over 0..levels-1 of length k, one per row."""
    return np.array(list(itertools.product(range(levels), repeat=k)), dtype=np.float32)


def test_tie_rules_closed_forms():
    """Rows = all 3^k sequences over {0, 1, 2}, exact trends (t = 0): the
    fitting rows are the strictly increasing sequences, C(3, k) of them, or
    the non-decreasing ones, C(k+2, k) by stars and bars, as each tie rule
    says; along the reversed series the column-index rule turns strict."""
    from math import comb
    for k in range(2, 6):
        X = _sequences(3, k)
        ident, rev = list(range(k)), list(range(k))[::-1]
        inc, nondec = comb(3, k), comb(k + 2, k)
        cases = [(1, ident, 0, inc), (2, ident, 0, nondec), (0, ident, 0, nondec),
                 (1, rev, 0, inc), (2, rev, 0, nondec), (0, rev, 0, inc),
                 # with reversed trends: both directions, the 3 constant rows
                 # counted once under the loose rule
                 (1, ident, 1, 2 * inc), (2, ident, 1, 2 * nondec - 3),
                 (0, ident, 1, nondec + inc)]
        for rule, series, neg, want in cases:
            p = oracle.make_params(approx_permille=1000, negative_trends=neg, min_rows=1,
                                   k_score_min=2, tie_rule=rule)
            assert oracle.evaluate(X, [series], params=p).count[0] == want, (k, rule, series, neg)


def test_tie_rules_agree_without_ties():
    rng = np.random.default_rng(21)
    X = synth.random_matrix(60, 10, seed=22)
    seqs = [list(rng.permutation(10)[:int(rng.integers(2, 11))]) for _ in range(80)]
    for neg in (0, 1):
        for approx in (1000, 800, 500):
            sup = [oracle.evaluate(X, seqs, params=oracle.make_params(
                approx_permille=approx, negative_trends=neg, min_rows=1, k_score_min=2,
                tie_rule=rule)).support for rule in (0, 1, 2)]
            np.testing.assert_array_equal(sup[0], sup[1])
            np.testing.assert_array_equal(sup[0], sup[2])


def test_tie_rules_nest():
    """A tie counts against both trends (strict), one (column index) or none
    (loose), so the supports nest: strict within index within loose."""
    rng = np.random.default_rng(23)
    X = synth.tie_matrix(80, 10, levels=3, seed=24)
    seqs = [list(rng.permutation(10)[:int(rng.integers(2, 11))]) for _ in range(80)]
    for neg in (0, 1):
        for approx in (1000, 800, 500):
            s0, s1, s2 = [oracle.evaluate(X, seqs, params=oracle.make_params(
                approx_permille=approx, negative_trends=neg, min_rows=1, k_score_min=2,
                tie_rule=rule)).support for rule in (0, 1, 2)]
            assert not (s1 & ~s0).any() and not (s0 & ~s2).any()
            assert (s1 != s2).any()


def test_fitness_identities():
    case = synth.workload_matrix(0)
    X = case.X
    planted = [int(c) for c in case.truth[0].cols]
    p = oracle.make_params(negative_trends=0)
    ev = oracle.evaluate(X, [planted, planted[:3], [0, 1]], params=p)
    # empty archive: no penalty
    np.testing.assert_array_equal(ev.fitness, ev.score)
    for i in range(3):
        if ev.score[i] > 0:
            k = [5, 3, 2][i]
            # the size score is an exact integer multiple of 2^k
            assert ev.score[i] == float(ev.count[i]) * 2.0 ** k
    # an archived copy of the individual covers all its cells: penalised
    arch = oracle.Archive(ev.support[:1].copy(), [planted])
    ev2 = oracle.evaluate(X, [planted], archive=arch, params=p)
    assert ev2.overlap[0, 0] == ev.count[0]
    assert ev2.fitness[0] == ev.score[0] / 2
    # full overlap is allowed at theta = 1000 per mille
    ev3 = oracle.evaluate(X, [planted], archive=arch,
                          params=oracle.make_params(negative_trends=0, overlap_permille=1000))
    assert ev3.fitness[0] == ev.score[0]
    # a member sharing no rows never penalises
    arch0 = oracle.Archive(np.zeros_like(ev.support[:1]), [planted])
    assert oracle.evaluate(X, [planted], archive=arch0, params=p).fitness[0] == ev.score[0]
    # each overlapping member halves again
    arch2 = oracle.Archive(np.repeat(ev.support[:1], 3, axis=0), [planted, planted, planted])
    assert oracle.evaluate(X, [planted], archive=arch2, params=p).fitness[0] == ev.score[0] / 8


def test_invalid_series_rejected():
    X = synth.random_matrix(10, 5, seed=1)
    for bad in ([1], [0, 0], [0, 5], list(range(5)) + [0]):
        with pytest.raises(ValueError):
            oracle.evaluate(X, [bad])


def test_splitmix64_known_answers(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64_seed0.txt")) as f:
        want = [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
    assert oracle.splitmix64_stream(0, len(want)) == want


def test_uniform_draw_distribution():
    bounds = [7] * 70000
    xs = np.array(oracle.uniform_stream(123, bounds))
    assert xs.min() == 0 and xs.max() == 6
    counts = np.bincount(xs, minlength=7)
    chi2 = ((counts - 10000.0) ** 2 / 10000.0).sum()
    assert chi2 < 30  # 6 dof, p ~ 4e-5
    # a power-of-two bound rejects nothing: the low bits of the raw stream
    raw = oracle.splitmix64_stream(9, 100)
    assert oracle.uniform_stream(9, [256] * 100) == [r & 255 for r in raw]
    assert oracle.uniform_stream(9, [1] * 5) == [0] * 5


def test_generator_determinism():
    a = synth.workload_matrix(0)
    b = synth.workload_matrix(0)
    assert a.sha256() == b.sha256()
    assert a.X.shape == (100, 20) and a.X.dtype == np.float32
    t = a.truth[0]
    assert t.rows.size == 10 and t.cols.size == 5
    vals = a.X[np.ix_(t.rows, t.cols)]
    assert np.all(np.diff(vals, axis=1) > 0)


def _c0_params(**kw):
    w = synth.workload(0)
    d = dict(approx_permille=850, negative_trends=w.negative_trends, overlap_permille=750,
             min_rows=5, k_min=w.k_min, k_max=w.k_max, archive_size=w.archive_size,
             n_out=w.n_out, population=w.population, generations=w.generations,
             max_tabu_hits=100000, tournament=4, max_attempts=1000)
    d.update(kw)
    return oracle.make_params(**d)


def test_run_planted_recovery():
    """Planted recovery: a 100 x 20 uniform matrix with one strictly increasing
    30-row x 5-column plant, run with the tiny workload's loop settings. The
    top bicluster must be the planted series with every planted row, for most
    (data seed, run seed) pairs. (The tiny workload's own 10-row plant is not
    a recovery case: under the n * 2^k size score its 2-4 column sub-series
    rank below the best random pairs, so the search stalls on those.)"""
    ok = 0
    for ds in range(5):
        case = synth.planted_matrix(100, 20, background="uniform", n_planted=1,
                                    rows_range=(30, 30), cols_range=(5, 5), sigma=0.0,
                                    strict=True, seed=1100 + ds)
        t = case.truth[0]
        follows = np.all(np.diff(case.X[:, t.cols], axis=1) > 0, axis=1)
        for seed in range(synth.GA_SEED, synth.GA_SEED + 4):
            res = oracle.run(case.X, _c0_params(), seed=seed)
            assert res.evaluations == int(res.trace[:, 0].sum())
            top = res.biclusters[0]
            if np.array_equal(top.cols, t.cols):
                # rows of the found bicluster: exactly those increasing
                # along the series (checked here with numpy, not the oracle)
                np.testing.assert_array_equal(top.rows, np.flatnonzero(follows))
                assert set(t.rows.tolist()) <= set(top.rows.tolist())
                ok += 1
    assert ok >= 14, ok


def test_run_deterministic():
    case = synth.workload_matrix(0)
    a = oracle.run(case.X, _c0_params(generations=20, n_out=5), seed=77)
    b = oracle.run(case.X, _c0_params(generations=20, n_out=5), seed=77)
    assert a.generations == b.generations and a.tabu_hits == b.tabu_hits
    np.testing.assert_array_equal(a.trace, b.trace)
    for x, y in zip(a.biclusters, b.biclusters):
        np.testing.assert_array_equal(x.rows, y.rows)
        np.testing.assert_array_equal(x.cols, y.cols)


def test_run_finds_best_on_tiny_matrix():
    """8 x 5 matrix: enumerate every series; the loop must reach the best
    size score within 50 generations (a soft check of the search)."""
    X = synth.random_matrix(8, 5, seed=21)
    seqs = [list(s) for s in _all_series(5, 5)]
    p = _c0_params(k_min=2, k_max=5, population=40, generations=50, min_rows=2, n_out=1)
    best = oracle.evaluate(X, seqs, params=p).score.max()
    res = oracle.run(X, p, seed=5)
    assert res.biclusters[0].score == best


def test_run_stops_on_tabu_hits():
    X = synth.random_matrix(8, 4, seed=2)
    p = _c0_params(k_min=2, k_max=4, population=10, generations=1000, max_tabu_hits=30)
    res = oracle.run(X, p, seed=1)
    assert res.stop_reason in (2, 3)
    assert res.generations < 1000
    if res.stop_reason == 2:
        assert res.tabu_hits == 30


def _random_bics(rng, n, R, C):
    return [(rng.choice(R, int(rng.integers(1, 9)), replace=False),
             rng.choice(C, int(rng.integers(1, 6)), replace=False)) for _ in range(n)]


def test_ce_score_special_cases():
    a = [([0, 1, 2], [0, 1]), ([5, 6], [2, 3, 4])]
    assert oracle.ce_score(a, a) == (1.0, 0.0)
    assert oracle.ce_score(a, [([8, 9], [5])]) == (0.0, 1.0)
    assert oracle.ce_score([], []) == (1.0, 0.0)
    assert oracle.ce_score(a, []) == (0.0, 1.0)
    # worked by hand: one shared cell (1, 1); 4 + 4 - 1 = 7 cells in all
    assert oracle.ce_score([([0, 1], [0, 1])], [([1, 2], [1, 2])]) == (1 / 7, 6 / 7)
    # order and repeats of rows / columns do not matter
    assert oracle.ce_score([([2, 0, 1, 1], [1, 0])], [([0, 1, 2], [0, 1])]) == (1.0, 0.0)


def test_ce_score_brute_force_assignment():
    """D_max against every injective assignment of the smaller set, on small
    random sets (including unequal sizes)."""
    rng = np.random.default_rng(41)
    for trial in range(60):
        nf, nt = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        f, t = _random_bics(rng, nf, 12, 8), _random_bics(rng, nt, 12, 8)
        cells = lambda b: {(int(r), int(c)) for r in b[0] for c in b[1]}
        m = [[len(cells(x) & cells(y)) for y in t] for x in f]
        best = 0
        if nf <= nt:
            for perm in itertools.permutations(range(nt), nf):
                best = max(best, sum(m[i][perm[i]] for i in range(nf)))
        else:
            for perm in itertools.permutations(range(nf), nt):
                best = max(best, sum(m[perm[j]][j] for j in range(nt)))
        u = len(set().union(*[cells(x) for x in f + t]))
        got = oracle.ce_score(f, t)
        if u:
            assert got == (best / u, (u - best) / u), trial


# --- boundaries of the size score, the overlap test and the bounded draw ---

def _increasing_rows(R, C, n):
    """R x C matrix whose first n rows increase along columns 0..C-1 and the
    rest decrease: along (0..k-1), exactly n rows keep the exact trend."""
    up = np.tile(np.arange(C, dtype=np.float32), (n, 1))
    down = np.tile(np.arange(C, 0, -1, dtype=np.float32), (R - n, 1))
    return np.vstack([up, down])


def test_size_score_thresholds():
    """s = n 2^k once n reaches min_rows and k reaches k_score_min; one
    below either threshold scores 0 (both comparisons inclusive)."""
    X = _increasing_rows(30, 6, 12)
    k = 4
    series = [list(range(k))]
    base = dict(approx_permille=1000, negative_trends=0, overlap_permille=750)
    for min_rows, want in ((11, 12 * 2 ** k), (12, 12 * 2 ** k), (13, 0)):
        ev = oracle.evaluate(X, series, params=oracle.make_params(
            min_rows=min_rows, k_score_min=2, **base))
        assert ev.count[0] == 12
        assert ev.score[0] == want and ev.fitness[0] == want, min_rows
    for ksm, want in ((k - 1, 12 * 2 ** k), (k, 12 * 2 ** k), (k + 1, 0)):
        ev = oracle.evaluate(X, series, params=oracle.make_params(
            min_rows=1, k_score_min=ksm, **base))
        assert ev.score[0] == want, ksm


def test_overlap_threshold_uses_shared_columns():
    """A member overlaps when 1000 h g > theta n k: h shared rows, g shared
    columns. Candidate (0, 1, 2, 3) on 10 fitting rows, theta 500 per mille:
    theta n k = 20,000. A member holding every row (h = 10) halves the score
    only when it shares 3 of the 4 columns (30,000); at 2 shared columns the
    product sits exactly on the bound (20,000, not above), and a member with
    every row but no shared column never penalises."""
    X = _increasing_rows(20, 8, 10)
    cand = [0, 1, 2, 3]
    p = oracle.make_params(approx_permille=1000, negative_trends=0, overlap_permille=500,
                           min_rows=1, k_score_min=2)
    ev = oracle.evaluate(X, [cand], params=p)
    n, s = int(ev.count[0]), float(ev.score[0])
    assert n == 10 and s == 10 * 2 ** 4
    rows = ev.support[:1].copy()
    cases = [([4, 5, 6, 7], s),        # g = 0
             ([0, 5, 6, 7], s),        # g = 1
             ([0, 1, 6, 7], s),        # g = 2: exactly on the bound
             ([7, 2, 1, 0], s / 2),    # g = 3 (order does not matter)
             ([3, 2, 1, 0, 4], s / 2)]  # g = 4
    for member, want in cases:
        got = oracle.evaluate(X, [cand], archive=oracle.Archive(rows, [member]), params=p)
        assert got.overlap[0, 0] == 10
        assert got.fitness[0] == want, member
    # the row side of the product: 9 shared rows and all 4 columns give
    # 36,000 > 20,000; 5 shared rows and 4 columns sit on the bound
    for h, want in ((9, s / 2), (5, s), (4, s)):
        part = np.zeros_like(rows)
        part[0, :h] = 1
        got = oracle.evaluate(X, [cand], archive=oracle.Archive(part, [cand]), params=p)
        assert got.overlap[0, 0] == h and got.fitness[0] == want, h


M64 = (1 << 64) - 1


def _splitmix64_ref(seed):
    """SplitMix64 in Python integers (the published generator: golden-ratio
    increment, variant-13 finaliser), as an independent implementation."""
    s = seed
    while True:
        s = (s + 0x9E3779B97F4A7C15) & M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        yield z ^ (z >> 31)


def _uniform_ref(gen, n):
    """x mod n of the first draw x at or above 2^64 mod n."""
    low = (1 << 64) % n
    while True:
        x = next(gen)
        if x >= low:
            return x % n


@pytest.mark.parametrize("n", [(1 << 63) + 1, 3 << 62, 10 ** 18 + 7])
def test_uniform_draw_rejection_large_bounds(n):
    """Bounds where rejection happens often (about 1/2, 1/4 and 1/41 of the
    draws): the oracle's stream equals a big-integer implementation, and for
    3 * 2^62 (where dropping the rejection would put half the draws below
    2^62) about a third of the draws fall below 2^62."""
    for seed in (1, 2, 3):
        ref = _splitmix64_ref(seed)
        want = [_uniform_ref(ref, n) for _ in range(1000)]
        assert oracle.uniform_stream(seed, [n] * 1000) == want
    if n == 3 << 62:
        xs = oracle.uniform_stream(77, [n] * 3000)
        frac = sum(x < (1 << 62) for x in xs) / len(xs)
        assert abs(frac - 1 / 3) < 0.05, frac


def test_reversed_series_share_a_tabu_entry():
    """Three columns, series of exactly three: six series, three up to
    reversal. With reversed trends on, a series and its reverse are one
    tabu entry, so once the first population holds one of each pair every
    mutant (a swap, or a full-length crossover child) is a tabu hit and the
    run stops after one generation; with them off three fresh series remain
    and the run goes on."""
    X = synth.random_matrix(12, 3, seed=4)
    base = dict(k_min=3, k_max=3, population=3, generations=20, max_tabu_hits=40,
                min_rows=1, n_out=3)
    for seed in (1, 2, 3, 4):
        on = oracle.run(X, _c0_params(negative_trends=1, k_score_min=3, **base), seed=seed)
        assert (on.generations, on.stop_reason, on.tabu_hits) == (1, 2, 40), seed
        off = oracle.run(X, _c0_params(negative_trends=0, k_score_min=2, **base), seed=seed)
        assert off.generations >= 2, seed


# --- the five operators (Sec. 2.3) and their weights ---

def _member_pop(rng, C, per, lens):
    """`per` random series of each length in `lens`."""
    return [list(map(int, rng.permutation(C)[:k])) for k in lens for _ in range(per)]


def _insertion_of(c, m):
    """Position where c inserts one new column into m, or None."""
    if len(c) != len(m) + 1:
        return None
    for pos in range(len(c)):
        if c[:pos] + c[pos + 1:] == m and c[pos] not in m:
            return pos
    return None


def _deletion_of(c, m):
    if len(c) != len(m) - 1:
        return None
    for pos in range(len(m)):
        if m[:pos] + m[pos + 1:] == c:
            return pos
    return None


def _substitution_of(c, m):
    if len(c) != len(m):
        return None
    diff = [i for i in range(len(m)) if c[i] != m[i]]
    return diff[0] if len(diff) == 1 and c[diff[0]] not in m else None


def _swap_of(c, m):
    if len(c) != len(m):
        return None
    diff = [i for i in range(len(m)) if c[i] != m[i]]
    if len(diff) == 2 and c[diff[0]] == m[diff[1]] and c[diff[1]] == m[diff[0]]:
        return tuple(diff)
    return None


def _crossover_cuts(c, I, J):
    """(a, b) with c = I[:a] followed by the columns of J[b:] not in I[:a]."""
    cuts = []
    for a in range(1, len(I)):
        for b in range(1, len(J)):
            head = I[:a]
            if head + [x for x in J[b:] if x not in head] == c:
                cuts.append((a, b))
    return cuts


OPS = ("insertion", "deletion", "substitution", "swap", "crossover")


@pytest.mark.parametrize("op", range(5))
def test_each_operator_alone(op):
    """With all the weight on one operator every child is that operator's
    result from some member of the population, and the drawn positions
    cover their whole ranges: insertion at 0..k (k = at the end), deletion,
    substitution and swap positions 0..k-1, crossover cuts 1..k-1."""
    rng = np.random.default_rng(31 + op)
    C = 30
    pop = _member_pop(rng, C, 3, [3, 4, 5, 6])
    w = [0] * 5
    w[op] = 1000
    p = oracle.make_params(k_min=2, k_max=8, tournament=1, op_permille=w)
    kids = [list(map(int, c)) for c in oracle.mutants(pop, C, p, seed=5 + op, n=3000)]
    seen = set()
    for c in kids:
        found = False
        for m in pop:
            if op == 0:
                pos = _insertion_of(c, m)
                ok = pos is not None
                if ok:
                    seen.add((len(m), pos))
            elif op == 1:
                pos = _deletion_of(c, m)
                ok = pos is not None
                if ok:
                    seen.add((len(m), pos))
            elif op == 2:
                pos = _substitution_of(c, m)
                ok = pos is not None
                if ok:
                    seen.add((len(m), pos))
            elif op == 3:
                ij = _swap_of(c, m)
                ok = ij is not None
                if ok:
                    seen.update((len(m), q) for q in ij)
            else:
                cuts = [ab for J in pop for ab in _crossover_cuts(c, m, J)]
                ok = bool(cuts)
                if ok:
                    seen.update((len(m), a) for a, _ in cuts)
            if ok:
                found = True
                break
        assert found, (OPS[op], c)
    for k in (3, 4, 5, 6):
        if op == 0:
            want = set(range(k + 1))
        elif op == 4:
            want = set(range(1, k))
        else:
            want = set(range(k))
        assert {pos for kk, pos in seen if kk == k} >= want, (OPS[op], k)


def test_operator_weights_distribution():
    """Members with disjoint columns, so a child's operator is read off its
    shape: one longer (insertion), one shorter (deletion), the same columns
    in another order (swap), one column replaced (substitution). Weights
    100/200/300/400/0 per mille give those shares of 20,000 children
    (chi-square, 3 degrees of freedom)."""
    C = 60
    pop = [list(range(4 * i, 4 * i + 4)) for i in range(15)]
    sets = [set(m) for m in pop]
    p = oracle.make_params(k_min=2, k_max=8, op_permille=[100, 200, 300, 400, 0])
    kids = oracle.mutants(pop, C, p, seed=9, n=20000)
    counts = np.zeros(4)
    for c in kids:
        c = list(map(int, c))
        if len(c) == 5:
            counts[0] += 1
        elif len(c) == 3:
            counts[1] += 1
        elif set(c) in sets:
            counts[3] += 1
        else:
            counts[2] += 1
    want = np.array([0.1, 0.2, 0.3, 0.4]) * len(kids)
    chi2 = (((counts - want) ** 2) / want).sum()
    assert chi2 < 16.3, counts  # p = 0.001


def test_operator_applicability():
    """At k = k_max insertion does not apply: with weights on insertion and
    deletion only, every child is a deletion; with all the weight on
    insertion no operator applies and every attempt gives no child."""
    C = 30
    pop = [list(range(3 * i, 3 * i + 6)) for i in range(4)]  # k = 6 = k_max
    p = oracle.make_params(k_min=2, k_max=6, op_permille=[500, 500, 0, 0, 0])
    for c in oracle.mutants(pop, C, p, seed=3, n=500):
        assert len(c) == 5
    p = oracle.make_params(k_min=2, k_max=6, op_permille=[1000, 0, 0, 0, 0])
    assert all(len(c) == 0 for c in oracle.mutants(pop, C, p, seed=3, n=50))
    # k = C: neither insertion nor substitution applies
    full = [[0, 1, 2], [2, 0, 1]]
    p = oracle.make_params(k_min=3, k_max=3, op_permille=[300, 0, 300, 400, 0])
    for c in oracle.mutants(full, 3, p, seed=4, n=300):
        assert sorted(c) == [0, 1, 2] and len(c) == 3


def test_operator_weights_validated_and_default():
    X = synth.random_matrix(20, 6, seed=1)
    for bad in ([200, 200, 200, 200, 199], [-1, 201, 200, 200, 400], [1001, 0, 0, 0, -1]):
        with pytest.raises(ValueError):
            oracle.run(X, _c0_params(k_max=4, generations=2, op_permille=bad), seed=1)
    a = oracle.run(X, _c0_params(k_max=4, generations=5, op_permille=[0] * 5), seed=2)
    b = oracle.run(X, _c0_params(k_max=4, generations=5), seed=2)
    np.testing.assert_array_equal(a.trace, b.trace)
    assert a.tabu_hits == b.tabu_hits


def test_crowding_keys_worked_examples():
    """Worked by hand. Four series over 4 columns, 8 entries: the mean share
    is ceil(8/4) = 2 and only column 0 (held 3 times) is overused, so the
    three series holding it are halved. Over 5 columns the share is
    ceil(8/5) = 2 as well, column 0 still the only one above it."""
    seqs = [[0, 1], [0, 2], [3, 0], [1, 2]]
    fit = np.array([16.0, 8.0, 0.0, 4.0])
    np.testing.assert_array_equal(oracle.crowding_keys(seqs, 4, fit), [8.0, 4.0, 0.0, 4.0])
    np.testing.assert_array_equal(oracle.crowding_keys(seqs, 5, fit), [8.0, 4.0, 0.0, 4.0])
    # 3 columns: share ceil(8/3) = 3; column 0 held 3 times is not above it
    seqs3 = [[0, 1], [0, 2], [2, 0], [1, 2]]
    np.testing.assert_array_equal(oracle.crowding_keys(seqs3, 3, fit), fit)
    # share ceil(9/4) = 3: column 0 (held 4 times) is overused, column 1
    # (held 3 times, exactly the share) is not
    seqs4 = [[0, 1, 2], [0, 1], [0, 1], [0, 3]]
    np.testing.assert_array_equal(oracle.crowding_keys(seqs4, 4, [64.0, 8.0, 8.0, 8.0]),
                                  [32.0, 4.0, 4.0, 4.0])
    # share ceil(10/4) = 3: columns 0 and 1 (held 4 times each) are both
    # overused, so every series is quartered
    seqs5 = [[0, 1, 2], [0, 1], [0, 1], [0, 1, 3]]
    np.testing.assert_array_equal(oracle.crowding_keys(seqs5, 4, [64.0, 8.0, 8.0, 8.0]),
                                  [16.0, 2.0, 2.0, 2.0])


def test_crowding_keys_invariants():
    """Relabelling columns leaves the keys unchanged; a population using
    every column equally is never penalised; e never exceeds k."""
    rng = np.random.default_rng(3)
    C = 30
    seqs = [list(map(int, rng.permutation(C)[:int(rng.integers(2, 9))])) for _ in range(50)]
    fit = np.ldexp(1.0, rng.integers(0, 30, 50)).astype(np.float64)
    keys = oracle.crowding_keys(seqs, C, fit)
    perm = rng.permutation(C)
    np.testing.assert_array_equal(oracle.crowding_keys([[int(perm[c]) for c in s] for s in seqs],
                                                       C, fit), keys)
    e = np.log2(fit / np.where(keys > 0, keys, 1.0))
    assert np.all(e >= 0) and np.all(e <= np.array([len(s) for s in seqs]))
    even = [[(i + j) % C for j in range(5)] for i in range(C)]  # each column 5 times
    np.testing.assert_array_equal(oracle.crowding_keys(even, C, np.ones(C)), np.ones(C))
