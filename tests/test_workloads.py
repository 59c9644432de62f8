"""The seeded input generators: determinism, shape, structure, stochastic rows."""
import numpy as np
import pytest

from paper_2507_22538_amd import workloads as W


def _row_sums(d):
    rid = np.repeat(np.arange(d.S * d.A), np.diff(d.row_ptr))
    return np.bincount(rid, weights=d.val, minlength=d.S * d.A)


def test_hash_python_matches_c():
    lib = W._load()
    for args in [(0, 0, 0, 0), (1, 2, 3, 4), (2**63, 17, 2**40 + 3, 99)]:
        assert W.key(*args) == lib.ipigen_key(*args)


def test_random_sparse_structure_and_determinism():
    a = W.random_sparse(500, 3, 8, 0.9, seed=4)
    b = W.random_sparse(500, 3, 8, 0.9, seed=4)
    c = W.random_sparse(500, 3, 8, 0.9, seed=5)
    for x, y in [(a.row_ptr, b.row_ptr), (a.col, b.col), (a.val, b.val), (a.g, b.g)]:
        assert np.array_equal(x, y)
    assert not np.array_equal(a.col, c.col)
    assert a.nnz == 500 * 3 * 8
    for r in range(a.S * a.A):
        cs = a.col[a.row_ptr[r]:a.row_ptr[r + 1]]
        assert np.all(np.diff(cs) > 0)  # distinct and sorted
    assert np.all(a.val > 0)
    np.testing.assert_allclose(_row_sums(a), 1.0, atol=1e-14)
    assert np.all((a.g >= 0) & (a.g < 1))


def test_random_sparse_variable_rows_and_full_rows():
    d = W.random_sparse(40, 2, 1, 0.9, seed=1, k_hi=40)
    lens = np.diff(d.row_ptr)
    assert lens.min() >= 1 and lens.max() <= 40 and len(set(lens)) > 5
    np.testing.assert_allclose(_row_sums(d), 1.0, atol=1e-13)
    full = W.random_sparse(16, 2, 16, 0.9, seed=2)  # k = S: every column present
    for r in range(32):
        assert np.array_equal(full.col[full.row_ptr[r]:full.row_ptr[r + 1]], np.arange(16))


def test_birth_death_band():
    d = W.birth_death(100, 4, seed=0)
    assert d.nnz == 100 * 4 * 24
    np.testing.assert_allclose(_row_sums(d), 1.0, atol=1e-14)
    for s in (0, 5, 50, 99):
        cs = d.col[d.row_ptr[s * 4]:d.row_ptr[s * 4 + 1]]
        assert len(cs) == 24 and np.all(np.diff(cs) == 1)
        assert cs[0] == min(max(s - 12, 0), 100 - 24)
    # binomial weights: p_a falls with a, so the mean offset falls with a
    s = 50
    means = []
    for a in range(4):
        b, e = d.row_ptr[s * 4 + a], d.row_ptr[s * 4 + a + 1]
        means.append(np.dot(d.val[b:e], d.col[b:e] - s))
    assert all(x > y for x, y in zip(means, means[1:]))


def test_pendulum_structure():
    d = W.pendulum(16, 11)
    assert d.S == 256 and d.nnz == 256 * 11 * 4
    assert np.all(np.diff(d.row_ptr) == 4)
    np.testing.assert_allclose(_row_sums(d), 1.0, atol=1e-14)
    assert np.all(d.val >= 0)
    for r in range(0, d.S * d.A, 37):
        cs = d.col[d.row_ptr[r]:d.row_ptr[r + 1]]
        assert np.all(np.diff(cs) > 0)
    # cost at theta = pi, v ~ 0, zero torque is the minimum over the grid
    assert d.g.min() >= 0


def test_maze_structure():
    d = W.maze(9, 11, wall_frac=0.25, seed=3)
    assert d.S == 99 and d.A == 5 and d.nnz == 99 * 5
    assert np.all(d.val == 1.0)
    assert np.all(d.g[(d.S - 1) * 5:] == -100.0)


def test_named_config_params():
    p = [W.c4_params(i) for i in range(512)]
    assert all(2000 <= x["S"] <= 200000 for x in p)
    assert all(4 <= x["A"] <= 16 and 4 <= x["k"] <= 32 for x in p)
    assert {x["gamma"] for x in p} == {0.9, 0.99, 0.999}
    q = [W.c5_params(i) for i in range(200)]
    assert all(1000 <= x["S"] <= 5e6 and 4 <= x["A"] <= 32 and 8 <= x["k"] <= 32 for x in q)
    assert all(0.95 <= x["gamma"] <= 0.9999 for x in q)
