"""Pins of the oracle's random projection matrix (Sec. II-B, Alg. 1).

The generator is pinned to two sources outside the oracle: the published
Philox4x64-10 known-answer vector, and numpy's own Philox bit generator.  The
sparse Gaussian draw is pinned statistically against its definition.
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            vals = [int(x, 16) for x in line.replace("->", " ").split()]
            rows.append((vals[:4], vals[4:6], vals[6:10]))
    return rows


def test_philox_known_answer_vector():
    rows = _kat_rows()
    assert rows
    for ctr, key, want in rows:
        got = oracle.philox4x64_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
        assert [int(x) for x in got] == want


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox (4x64, 10 rounds) emits the block of counter c+1 first.
    rng = np.random.default_rng(5)
    for _ in range(50):
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        if ctr[0] == 0:
            continue
        bg = np.random.Philox(key=key, counter=np.array([ctr[0] - np.uint64(1), ctr[1], ctr[2], ctr[3]],
                                                        dtype=np.uint64))
        want = bg.random_raw(4)
        got = oracle.philox4x64_10(ctr, key)
        assert np.array_equal(got, want)


def test_density_is_binomial():
    # every entry is nonzero with probability a (Sec. II-B)
    d, T, depth = 128, 40, 10
    a = float(np.float32(1 / np.sqrt(d)))
    R = oracle.random_matrix(d, T, depth, a, seed=11)
    nnz = int((R != 0).sum())
    N = R.size
    mean, sd = N * a, np.sqrt(N * a * (1 - a))
    assert abs(nnz - mean) < 5 * sd
    # per-row counts follow Binomial(d, a): chi-square over count bins
    per_row = (R != 0).sum(axis=1)
    assert abs(per_row.mean() - d * a) < 5 * np.sqrt(d * a * (1 - a) / per_row.size)
    assert abs(per_row.var() - d * a * (1 - a)) < 0.35 * d * a * (1 - a)


def test_nonzeros_are_standard_normal():
    d, T, depth = 784, 50, 8
    a = float(np.float32(1 / np.sqrt(d)))
    R = oracle.random_matrix(d, T, depth, a, seed=12)
    z = R[R != 0].astype(np.float64)
    assert z.size > 5000
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)


def test_dense_case_a_equal_one():
    # a = 1 is the dense RP-tree variant: every entry is drawn
    R = oracle.random_matrix(64, 3, 4, 1.0, seed=3)
    assert np.count_nonzero(R) == R.size


def test_rows_independent_of_tree_count():
    # tree t's vectors depend on (seed, t, level, i) only, so the first trees of
    # a bigger index are the trees of a smaller one
    small = oracle.random_matrix(96, 3, 5, 0.1, seed=99)
    big = oracle.random_matrix(96, 7, 5, 0.1, seed=99)
    assert np.array_equal(small, big[: 3 * 5])
    other = oracle.random_matrix(96, 3, 5, 0.1, seed=100)
    assert not np.array_equal(small, other)


def test_levels_not_correlated():
    d = 1024
    R = oracle.random_matrix(d, 2, 6, 1.0, seed=21).astype(np.float64)
    C = np.corrcoef(R)
    off = C[~np.eye(C.shape[0], dtype=bool)]
    assert np.max(np.abs(off)) < 5 / np.sqrt(d)


@pytest.mark.parametrize("seed", [0, 1, 2**64 - 1])
def test_seed_full_width(seed):
    R = oracle.random_matrix(32, 2, 3, 0.5, seed=seed)
    assert np.all(np.isfinite(R))


# ---------------------------------------------------------------------------
# exact-count mode (the footnote of Sec. II-D): exactly ceil(a d) nonzeros per
# vector, the features with the smallest selection uniforms
# ---------------------------------------------------------------------------
def _uniforms_numpy(d, T, depth, seed):
    """Word 0 of every entry's block from numpy's Philox (pinned equal to the
    published generator above), as the 53-bit uniform, shape (T*depth, d)."""
    U = np.zeros((T * depth, d))
    for t in range(T):
        for lv in range(depth):
            for i in range(d):
                # numpy emits the block of counter c + 1 first: start one below
                # (i, lv, t, 0), read as a 256-bit number with word 0 lowest
                c = (i + (lv << 64) + (t << 128)) - 1
                words = [(c >> (64 * j)) & (2**64 - 1) for j in range(4)]
                bg = np.random.Philox(key=np.array([seed, 0], np.uint64), counter=np.array(words, np.uint64))
                U[t * depth + lv, i] = float(bg.random_raw(1)[0] >> np.uint64(11)) / 2.0**53
    return U


@pytest.mark.parametrize("d,a", [(128, 1 / np.sqrt(128)), (100, 0.05), (64, 0.5), (7, 0.3), (33, 1 / 33)])
def test_exact_mode_count(d, a):
    a = float(np.float32(a))
    R = oracle.random_matrix(d, 6, 5, a, seed=21, exact_nnz=True)
    m = min(d, max(1, int(np.ceil(np.float64(a) * d))))
    assert oracle.exact_nnz_count(d, a) == m
    assert np.all((R != 0).sum(axis=1) == m)


def test_exact_mode_selects_smallest_uniforms():
    d, T, depth, seed = 24, 3, 2, 77
    a = 0.2
    m = int(np.ceil(a * d))
    U = _uniforms_numpy(d, T, depth, seed)
    R = oracle.random_matrix(d, T, depth, a, seed, exact_nnz=True)
    for r in range(T * depth):
        want = set(np.lexsort((np.arange(d), U[r]))[:m].tolist())
        assert set(np.nonzero(R[r])[0].tolist()) == want


def test_exact_mode_nested_with_bernoulli():
    # the exact set is the m smallest uniforms, so for every threshold b the
    # Bernoulli set {u < b} either contains it or is contained in it
    d, T, depth, seed = 96, 4, 4, 5
    a = float(np.float32(1 / np.sqrt(d)))
    E = oracle.random_matrix(d, T, depth, a, seed, exact_nnz=True) != 0
    for b in (0.02, 0.05, 0.08, a, 0.12, 0.2, 0.5):
        B = oracle.random_matrix(d, T, depth, b, seed) != 0
        for r in range(T * depth):
            e, s = set(np.nonzero(E[r])[0]), set(np.nonzero(B[r])[0])
            assert e <= s or s <= e, (b, r)


def test_exact_mode_values_and_dense_case():
    d, T, depth, seed = 40, 3, 3, 9
    full = oracle.random_matrix(d, T, depth, 1.0, seed)
    assert np.array_equal(oracle.random_matrix(d, T, depth, 1.0, seed, exact_nnz=True), full)
    E = oracle.random_matrix(d, T, depth, 0.25, seed, exact_nnz=True)
    nz = E != 0
    assert np.array_equal(E[nz], full[nz])


def test_exact_mode_positions_uniform():
    # each feature is chosen with probability m / d, independently of its index
    d, T, depth = 50, 200, 10
    a = 0.1
    E = oracle.random_matrix(d, T, depth, a, seed=3, exact_nnz=True) != 0
    counts = E.sum(axis=0)
    assert stats.chisquare(counts).pvalue > 1e-3
