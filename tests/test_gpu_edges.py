"""GPU edge cases against the CPU oracle: denormal and signed-zero values on
every evaluation path, a matrix tall enough that an individual's rows take
more than 16 items and its support no longer fits the reduction's LDS copy,
ingests on several threads and streams at once, column byte offsets past
2^31, and pair tables on either side of 2^32 bytes."""
import os
import threading

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
    d = dict(approx_permille=850, negative_trends=1, overlap_permille=750, min_rows=1)
    d.update(kw)
    d.setdefault("k_score_min", 3 if d["negative_trends"] else 2)
    return d


def _outputs(E, out, P):
    return (out.count.cpu().numpy()[:P].copy(), out.fitness.cpu().numpy()[:P].view(np.int64).copy(),
            out.support.cpu().numpy().view(np.uint64)[:P].copy())


def _compare(E, got, ev, R, idx=None):
    cnt, fit, words = got
    idx = np.arange(cnt.size) if idx is None else np.asarray(idx)
    np.testing.assert_array_equal(cnt[idx], ev.count)
    np.testing.assert_array_equal(fit[idx], ev.fitness.view(np.int64))
    np.testing.assert_array_equal(E.support_to_flags(words[idx], R), ev.support)


def _paths(E, X, seqs, kw, arch_flags=None, arch_series=None, pairs=True):
    """(name, outputs) of the plain evaluator, the batched gather form and
    (when pairs) the batched pair form, with both pair tables for the
    strict and loose tie rules."""
    m = E.ebic_matrix_prepare(torch.from_numpy(np.ascontiguousarray(X)).cuda())
    pop = E.ebic_population_upload(seqs, X.shape[1])
    arch = None
    if arch_series:
        arch = E.make_archive(E.flags_to_support(arch_flags, m.words), arch_series)
    p = E.make_params(**kw)
    res = []
    out = E.ebic_evaluate(m, pop, arch, p)
    torch.cuda.synchronize()
    res.append(("plain", _outputs(E, out, len(seqs)), out))
    job = E.make_job(m, pop, arch, p)
    b = E.Batch([job], gather=True)
    b.run()
    torch.cuda.synchronize()
    res.append(("gather", _outputs(E, job.out, len(seqs)), job.out))
    b.close()
    if pairs:
        E.ebic_pairs_prepare(m)
        if kw.get("tie_rule", 0) != 0:
            E.ebic_pairs_strict_prepare(m)
        job = E.make_job(m, pop, arch, p)
        b = E.Batch([job])
        b.run()
        torch.cuda.synchronize()
        res.append(("pairs", _outputs(E, job.out, len(seqs)), job.out))
        b.close()
    return res


def _denormal_matrix(R, C, seed):
    """Values from a small set of edge floats: +-FLT_TRUE_MIN, a few other
    subnormals (repeated, so subnormal ties), +-0, +-FLT_MIN, the next float
    above FLT_MIN and +-1."""
    tiny = np.float32(np.finfo(np.float32).smallest_subnormal)
    fmin = np.finfo(np.float32).tiny
    vals = np.array([-1.0, -fmin, -3 * tiny, -tiny, -0.0, 0.0, tiny, 2 * tiny, 1000 * tiny,
                     fmin / 2, fmin, np.nextafter(fmin, np.float32(1)), 1.0], dtype=np.float32)
    assert all(np.isfinite(vals))
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(vals[rng.integers(0, vals.size, size=(R, C))])


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_denormal_and_signed_zero_values(E, rule):
    """Subnormal values compare exactly (a tie only when the bits are
    equal, or for -0 and +0), on the plain, gather and pair paths."""
    X = _denormal_matrix(300, 10, seed=17 + rule)
    rng = np.random.default_rng(rule)
    seqs = [list(map(int, rng.permutation(10)[:int(rng.integers(2, 11))])) for _ in range(300)]
    seqs += [list(range(10)), list(range(9, -1, -1))]
    for neg in (0, 1):
        kw = _kw(approx_permille=800, negative_trends=neg, tie_rule=rule)
        ev = oracle.evaluate(X, seqs, params=oracle.make_params(**kw))
        assert (ev.count > 0).any() and (ev.count < X.shape[0]).any()
        for name, got, _ in _paths(E, X, seqs, kw):
            _compare(E, got, ev, X.shape[0])


def test_denormal_ranks(E):
    """Ingest ranks: for every cell, the number of cells of its row with a
    smaller value, compared with numpy's float compares on the host."""
    X = _denormal_matrix(129, 13, seed=3)
    m = E.ebic_matrix_prepare(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    rp = (X.shape[0] + 63) // 64 * 64
    ranks = m.ranks.cpu().numpy().view(np.uint16)[:X.shape[1] * rp].reshape(X.shape[1], rp)
    want = (X[:, None, :] < X[:, :, None]).sum(axis=2)  # [r, c] = #{c' : X[r,c'] < X[r,c]}
    np.testing.assert_array_equal(ranks[:, :X.shape[0]].T, want)


def test_tall_matrix_items_and_supports_outside_lds(E):
    """140,000 rows: an individual's 2,188 row words take more than 16
    items of 4,096 rows (items widened), and its support is longer than the
    reduction's LDS copy (read back from global memory). Plain, gather and
    pair paths against the oracle, with a 20-member archive."""
    case = synth.planted_matrix(140000, 40, background="lognormal", n_planted=4,
                                rows_range=(500, 3000), cols_range=(4, 12), sigma=0.1,
                                reverse_odd=True, seed=140)
    X = case.X
    rng = np.random.default_rng(140)
    seqs = [list(map(int, rng.permutation(40)[:int(rng.integers(3, 41))])) for _ in range(200)]
    seqs += [list(map(int, t.cols)) for t in case.truth]
    kw = _kw(min_rows=5)
    ev0 = oracle.evaluate(X, seqs, params=oracle.make_params(**kw), nthreads=NCPU)
    top = [int(i) for i in np.argsort(-ev0.score, kind="stable")[:20]]
    arch_series = [seqs[i] for i in top]
    arch_flags = ev0.support[top]
    ev = oracle.evaluate(X, seqs, archive=oracle.Archive(arch_flags, arch_series),
                         params=oracle.make_params(**kw), nthreads=NCPU)
    assert (ev.fitness < ev.score).any()  # some individuals are penalised
    for name, got, out in _paths(E, X, seqs, kw, arch_flags, arch_series):
        _compare(E, got, ev, X.shape[0])
        np.testing.assert_array_equal(out.overlap.cpu().numpy()[:len(seqs), :20], ev.overlap)


@pytest.mark.parametrize("cols", [1290, 1300])
def test_pair_table_near_and_past_4_gib(E, cols):
    """40,000 rows make 5,120-byte pair rows: 1,290 columns give a 4.26 GB
    table, below 2^32 bytes, whose steps address pair rows by byte offset
    through one buffer resource (the last rows end close to 2^32); 1,300
    columns give 4.33 GB, past it, where steps address rows by pair index.
    Series reaching the table's last pairs, under every item shape, against
    the oracle."""
    R = 40000
    case = synth.planted_matrix(R, cols, background="normal", n_planted=2,
                                rows_range=(400, 800), cols_range=(4, 8), sigma=0.05, seed=cols)
    X = case.X
    rng = np.random.default_rng(cols)
    hi = np.arange(cols - 60, cols)
    seqs = [[cols - 2, cols - 1], [cols - 1, cols - 2], [cols - 3, cols - 1, cols - 2]]
    seqs += [list(map(int, rng.permutation(hi)[:int(rng.integers(2, 13))])) for _ in range(60)]
    seqs += [list(map(int, rng.permutation(cols)[:int(rng.integers(2, 13))])) for _ in range(60)]
    seqs += [list(map(int, t.cols)) for t in case.truth]
    kw = _kw(approx_permille=700, min_rows=1)
    ev = oracle.evaluate(X, seqs, params=oracle.make_params(**kw), nthreads=NCPU)
    assert ev.count.max() > 100
    m = E.ebic_matrix_prepare(torch.from_numpy(np.ascontiguousarray(X)).cuda())
    E.ebic_pairs_prepare(m)
    torch.cuda.synchronize()
    assert (E.ebic_pairs_bytes(R, cols) < 1 << 32) == (cols == 1290)
    pop = E.ebic_population_upload(seqs, cols)
    for shape in ((1, 2, 1), (2, 4, 1), (1, 8, 1), (1, 2, 2), (2, 4, 2)):
        print(f"pair table {cols} columns, shape {shape}", flush=True)
        job = E.make_job(m, pop, None, E.make_params(**kw))
        b = E.Batch([job])
        b.set_tuning(*shape)
        b.run()
        torch.cuda.synchronize()
        _compare(E, _outputs(E, job.out, len(seqs)), ev, R)
        b.close()


def test_concurrent_ingest_on_three_streams(E):
    """Three threads, each on a stream of its own, ingest at the same time:
    two clean matrices and one with a NaN, 12 times each. Every clean
    ingest gives the same ranks as one made alone; every NaN ingest fails
    with EBIC_ERR_NONFINITE and no clean one does."""
    mats = [synth.random_matrix(3000, 200, seed=s) for s in (1, 2, 3)]
    mats[1][1234, 77] = np.nan
    ref = {}
    for i in (0, 2):
        m = E.ebic_matrix_prepare(torch.from_numpy(mats[i]).cuda())
        torch.cuda.synchronize()
        ref[i] = m.ranks.cpu().numpy().copy()
    dev = [torch.from_numpy(x).cuda() for x in mats]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    results = [[] for _ in range(3)]

    def work(i):
        torch.cuda.set_device(0)
        for _ in range(12):
            try:
                m = E.ebic_matrix_prepare(dev[i], stream=streams[i])
                streams[i].synchronize()
                results[i].append(("ok", m.ranks.cpu().numpy()))
            except E.EbicError as e:
                results[i].append(("err", e.code))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(3)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for i in (0, 2):
        assert len(results[i]) == 12
        for kind, val in results[i]:
            assert kind == "ok", val
            np.testing.assert_array_equal(val, ref[i])
    assert results[1] == [("err", E.EBIC_ERR_NONFINITE)] * 12


@pytest.mark.slow
def test_column_offsets_past_2_gib(E):
    """2,097,152 rows x 520 columns: a column's byte offset in the rank
    matrix, c * rows_pad * 2, passes 2^31 from column 512 on. With many ties
    the column-index rule orders tied columns by those offsets, so they must
    compare as unsigned. Series across column 512, plain and gather paths,
    checked on 20,000 sampled rows."""
    R, C = 1 << 21, 520
    rng = np.random.default_rng(21)
    X = rng.integers(0, 3, size=(R, C), dtype=np.int8).astype(np.float32)
    cols = [int(c) for c in rng.permutation(np.arange(490, 520))]
    seqs = [cols[:k] for k in (2, 3, 5, 8)] + [cols[5:5 + k] for k in (2, 4, 6)] + \
        [[511, 512], [512, 511], [100, 515, 3, 519], list(range(505, 520))]
    rows = np.sort(rng.choice(R, 20000, replace=False))
    for neg in (0, 1):
        kw = _kw(approx_permille=700, negative_trends=neg)
        ev = oracle.evaluate(np.ascontiguousarray(X[rows]), seqs,
                             params=oracle.make_params(**kw), nthreads=NCPU)
        for name, (cnt, fit, words), _ in _paths(E, X, seqs, kw, pairs=False):
            flags = E.support_to_flags(words, R)[:, rows]
            np.testing.assert_array_equal(flags, ev.support, err_msg=name)
            np.testing.assert_array_equal(E.support_to_flags(words, R).sum(axis=1), cnt)
