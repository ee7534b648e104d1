"""The test-side helpers agree with each other: the vectorised residual used on
large problems equals the residual of the explicitly assembled sparse matrix."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import helpers as H


@pytest.mark.parametrize("npt", [5, 9])
def test_vectorised_residual_equals_sparse_matrix_residual(npt):
    rng = np.random.default_rng(npt)
    n = 17
    planes = O.fv5(10 ** rng.uniform(-2, 2, (n - 1, n - 1)))
    if npt == 9:
        h = O.Hierarchy(O.fv5(10 ** rng.uniform(-2, 2, (2 * n - 2, 2 * n - 2))))
        st = h.stencil(h.L - 2)
        planes = np.zeros((5, n, n))
        planes[0] = st[:, :, 1, 1]
        planes[1, :, 1:] = -st[:, 1:, 1, 0]
        planes[2, 1:, :] = -st[1:, :, 0, 1]
        planes[3, 1:, 1:] = -st[1:, 1:, 0, 0]
        planes[4, 1:, :-1] = -st[1:, :-1, 0, 2]
    b = rng.standard_normal((n, n))
    u = rng.standard_normal((n, n))
    u[0] = u[-1] = 0
    u[:, 0] = u[:, -1] = 0
    A = H.matrix_from_planes(planes)
    want = H.to_interior(b) - A @ H.to_interior(u)
    got = H.residual_from_planes(planes, b, u)
    assert np.abs(H.to_interior(got) - want).max() <= 1e-14 * np.abs(want).max()
    assert np.all(got[0] == 0) and np.all(got[-1] == 0) and np.all(got[:, 0] == 0) and np.all(got[:, -1] == 0)
