"""Pins for the oracle's Hines solve (Sec. II: parent-before-child numbering,
extended Thomas algorithm) against dense LU and the textbook banded solve."""
import numpy as np
import pytest
import scipy.linalg

import oracle


def random_tree_system(rng, n):
    parent = np.full(n, -1, np.int64)
    for i in range(1, n):
        parent[i] = rng.integers(0, i)
    sig = rng.uniform(0.5, 50.0, n)
    sig[0] = 0.0
    cdt = rng.uniform(0.1, 20.0, n)
    d = cdt.copy()
    for i in range(1, n):
        d[i] += sig[i]
        d[parent[i]] += sig[i]
    u = -sig
    A = np.diag(d)
    for i in range(1, n):
        A[i, parent[i]] = A[parent[i], i] = u[i]
    return parent, d, u, A


@pytest.mark.parametrize("n", [1, 2, 3, 7, 19, 40])
def test_hines_matches_dense_lu(n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        parent, d, u, A = random_tree_system(rng, n)
        b = rng.normal(size=n) * 50
        x = oracle.hines_solve(parent, d, u, b)
        ref = np.linalg.solve(A, b)
        assert np.max(np.abs(x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_unbranched_matches_banded_thomas():
    rng = np.random.default_rng(7)
    n = 300
    parent = np.arange(-1, n - 1, dtype=np.int64)
    sig = rng.uniform(1, 10, n)
    sig[0] = 0
    d = rng.uniform(0.1, 1, n)
    for i in range(1, n):
        d[i] += sig[i]
        d[i - 1] += sig[i]
    b = rng.normal(size=n)
    ab = np.zeros((3, n))
    ab[0, 1:] = -sig[1:]
    ab[1] = d
    ab[2, :-1] = -sig[1:]
    ref = scipy.linalg.solve_banded((1, 1), ab, b)
    x = oracle.hines_solve(parent, d, -sig, b)
    assert np.max(np.abs(x - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_solve_is_symmetric_dot_product():
    """<A^-1 x, y> = <x, A^-1 y>: the adjoint reuses the same solve."""
    rng = np.random.default_rng(3)
    parent, d, u, A = random_tree_system(rng, 60)
    x, y = rng.normal(size=60), rng.normal(size=60)
    lhs = oracle.hines_solve(parent, d, u, x) @ y
    rhs = x @ oracle.hines_solve(parent, d, u, y)
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)
