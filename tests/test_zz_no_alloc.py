"""The allocation-free batched evaluation (ebic_evaluate_batched_noalloc,
through the C ABI) against ebic_evaluate_batched, bit for bit: two calls in
a row on the same GPU, the second with a smaller input, then the limits."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2105_01196_amd import ebic
    return ebic


_MATS = {}


def _matrix(E, wi, strict):
    key = (wi, strict)
    if key not in _MATS:
        case = synth.workload_matrix(wi)
        m = E.ebic_matrix_prepare(torch.from_numpy(case.X).cuda())
        E.ebic_pairs_prepare(m)
        if strict:
            E.ebic_pairs_strict_prepare(m)
        _MATS[key] = (case, m)
    return _MATS[key]


def _jobs(E, specs, seed):
    """One job per (workload, population size, archive size, tie rule); the
    archive is the population's own top members from a first plain
    evaluation."""
    jobs = []
    for n, (wi, P, K, tie) in enumerate(specs):
        case, m = _matrix(E, wi, tie != E.EBIC_TIE_INDEX)
        seqs = synth.workload_population(wi, case, P=P, seed=seed + n)
        params = E.make_params(approx_permille=(850, 700, 1000, 600)[n % 4],
                               negative_trends=(n + 1) % 2, overlap_permille=750, min_rows=5,
                               k_score_min=3 if (n + 1) % 2 else 2, tie_rule=tie)
        pop = E.ebic_population_upload(seqs, case.C)
        arch = None
        if K:
            first = E.ebic_evaluate(m, pop, None, params)
            torch.cuda.synchronize()
            fit = first.fitness.cpu().numpy()[:P]
            top = [int(i) for i in np.argsort(-fit, kind="stable")[:K]]
            arch = E.archive_from_device(first.support, top, seqs)
        E.set_order(pop, E.longest_first(seqs))
        jobs.append(E.make_job(m, pop, arch, params))
    return jobs


def _fresh(E, jobs):
    """The same inputs with outputs of their own."""
    return [E.make_job(j.matrix, j.pop, j.archive, j.params) for j in jobs]


def _same(a, b):
    assert torch.equal(a.out.count, b.out.count)
    assert torch.equal(a.out.fitness.view(torch.int64), b.out.fitness.view(torch.int64))
    assert torch.equal(a.out.support, b.out.support)
    if a.out.overlap is not None:
        assert torch.equal(a.out.overlap, b.out.overlap)


def test_noalloc_equals_batched_twice(E):
    stream = torch.cuda.current_stream()
    calls = [
        # batched-10000x500 with archives, plain-1000x100 under the strict
        # tie rule (both pair tables), tiny-100x20, large-40000x1000
        [(2, 1024, 20, E.EBIC_TIE_INDEX), (1, 600, 20, E.EBIC_TIE_STRICT),
         (0, 200, 0, E.EBIC_TIE_INDEX), (3, 300, 8, E.EBIC_TIE_INDEX)],
        # smaller: fewer jobs, smaller populations, column-index rule only
        [(1, 100, 5, E.EBIC_TIE_INDEX), (0, 37, 0, E.EBIC_TIE_INDEX)],
    ]
    for call, specs in enumerate(calls):
        print(f"no-alloc call {call}: {specs}", flush=True)
        ref = _jobs(E, specs, synth.POP_SEED + 300 + 10 * call)
        mine = _fresh(E, ref)
        E.ebic_evaluate_batched(ref, stream=stream)
        E.ebic_evaluate_batched_noalloc(mine, stream=stream)
        torch.cuda.synchronize()
        for a, b in zip(ref, mine):
            _same(a, b)
        assert int(ref[0].out.count.max()) > 0


def test_noalloc_limits(E):
    case, m = _matrix(E, 0, False)
    seqs = synth.workload_population(0, case, P=10)
    pop = E.ebic_population_upload(seqs, case.C)
    params = E.make_params(approx_permille=850, negative_trends=0, min_rows=5, k_score_min=2)
    many = [E.make_job(m, pop, None, params) for _ in range(E.EBIC_NOALLOC_MAX_JOBS + 1)]
    with pytest.raises(E.EbicError) as ei:
        E.ebic_evaluate_batched_noalloc(many)
    assert ei.value.code == E.EBIC_ERR_INVALID_ARG and "at most" in str(ei.value)
    no_sup = E.make_job(m, pop, None, params, support=False)
    with pytest.raises(E.EbicError) as ei:
        E.ebic_evaluate_batched_noalloc([no_sup])
    assert ei.value.code == E.EBIC_ERR_INVALID_ARG and "support" in str(ei.value)
    # the largest allowed call still runs and matches
    ok = many[:E.EBIC_NOALLOC_MAX_JOBS]
    ref = _fresh(E, ok)
    E.ebic_evaluate_batched(ref)
    E.ebic_evaluate_batched_noalloc(ok)
    torch.cuda.synchronize()
    for a, b in zip(ref, ok):
        _same(a, b)
