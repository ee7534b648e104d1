"""The oracle's parallel loops (OpenMP over rows or planes of one colour, the
residual and the interpolation) give bitwise the results of one thread: the
points of one colour do not couple, so the order in which threads update them
cannot matter."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1803_02481_amd import inputs


@pytest.fixture
def threads():
    prev = O.set_threads(1)
    yield
    O.set_threads(prev)


def test_2d_solve_and_mixed_solve_bitwise_for_any_thread_count(threads):
    n = 257
    planes = O.fv5(inputs.cells_log10_blocks(n, n, 16, seed=1))
    b = inputs.load_uniform(n, n, seed=2)
    res = {}
    for t in (1, 3, max(2, os.cpu_count() or 2)):
        O.set_threads(t)
        h = O.Hierarchy(planes)
        u, hist = h.solve(b, tol=1e-10)
        um, hm, cyc, steps = h.solve_mixed(b, tol=1e-10)
        res[t] = (u, hist, um, hm, cyc, steps)
    ref = res[1]
    for t, got in res.items():
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), t
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3]), t
        assert got[4:] == ref[4:], t


def test_3d_solve_bitwise_for_any_thread_count(threads):
    m = 33
    planes = O.fv7(inputs.cells3_log10_blocks(m, m, m, block=4, seed=51))
    b = inputs.load3_uniform(m, m, m, seed=53)
    res = {}
    for t in (1, 4):
        O.set_threads(t)
        u, hist = O.Hierarchy3(planes).solve(b, tol=1e-10)
        res[t] = (u, hist)
    assert np.array_equal(res[1][0], res[4][0]) and np.array_equal(res[1][1], res[4][1])
