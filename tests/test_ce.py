"""The library's clustering error (ebic_ce_score, host code: confusion
matrix from row/column set sizes, its own Munkres solver, union of cells
row by row) against the oracle's (explicit cell sets, a library assignment
solver), exactly."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def E():
    from paper_2105_01196_amd import ebic
    return ebic


def _random_bics(rng, n, R, C, max_rows, max_cols):
    return [(rng.choice(R, int(rng.integers(1, max_rows + 1)), replace=False),
             rng.choice(C, int(rng.integers(1, max_cols + 1)), replace=False))
            for _ in range(n)]


def test_matches_oracle_on_random_sets(E):
    import oracle
    rng = np.random.default_rng(51)
    for trial in range(40):
        R, C = int(rng.integers(5, 400)), int(rng.integers(3, 60))
        nf, nt = int(rng.integers(0, 25)), int(rng.integers(0, 25))
        f = _random_bics(rng, nf, R, C, min(R, 60), min(C, 12))
        t = _random_bics(rng, nt, R, C, min(R, 60), min(C, 12))
        assert E.ebic_ce_score(f, t, R, C) == oracle.ce_score(f, t), trial


def test_overlapping_and_nested_biclusters(E):
    import oracle
    big = (np.arange(0, 50), np.arange(0, 10))
    inner = (np.arange(10, 20), np.arange(2, 5))
    shifted = (np.arange(25, 75), np.arange(5, 15))
    for f, t in [([big, inner], [big]), ([inner], [big, shifted]), ([big, shifted], [shifted, big])]:
        assert E.ebic_ce_score(f, t, 100, 20) == oracle.ce_score(f, t)


def test_rejects_indices_outside_the_matrix(E):
    with pytest.raises(Exception):
        E.ebic_ce_score([([0, 10], [0])], [], 10, 5)
    with pytest.raises(Exception):
        E.ebic_ce_score([([0], [5])], [], 10, 5)
