"""The allocation-free entry point hipbmg_residual_norm_noalloc, through the C
interface, against the allocating hipbmg_residual_norm: the same kernels on a
fixed per-device array, so the same bits, on consecutive calls whose inputs
shrink (what a call leaves in the array must not leak into the next), and a
clear error beyond the array's size."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1803_02481_amd import hipbmg as HB
from tests import helpers as H

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _case(n, m, npt, seed):
    rng = np.random.default_rng(seed)
    planes = O.fv5(10.0 ** rng.uniform(-2, 2, size=(m - 1, n - 1)))
    if npt == 9:
        planes = np.concatenate([planes, 0.1 * np.abs(rng.standard_normal((2, m, n)))])
    b = rng.standard_normal((m, n))
    u = rng.standard_normal((m, n))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return planes, b, u, dev(planes), dev(b), dev(u)


def test_noalloc_equals_the_allocating_entry_point_on_consecutive_calls():
    # a large grid, then a smaller one (fewer partials than the first call
    # left in the array), then the large one again
    for (n, m, npt, seed) in [(4097, 1025, 5, 1), (129, 65, 9, 2), (33, 17, 5, 3), (4097, 1025, 5, 1)]:
        planes, b, u, gp, gb, gu = _case(n, m, npt, seed)
        want = HB.residual_norm(gp, gb, gu)
        got = HB.residual_norm(gp, gb, gu, noalloc=True)
        assert got == want, (n, m, got, want)
        # and both are the residual of the host's assembly of the same operator
        r = H.residual_from_planes(planes, b, u)
        assert got[0] == pytest.approx(float(np.linalg.norm(r)), rel=1e-12)
        assert got[1] == pytest.approx(float(np.linalg.norm(b[1:-1, 1:-1])), rel=1e-12)


def test_noalloc_rejects_grids_beyond_its_array():
    # checked from the sizes alone, before any device work: the pointers are
    # never read
    planes, b, u, gp, gb, gu = _case(33, 33, 5, 4)
    out = (ctypes.c_double * 2)()
    lib = HB.lib()
    st = lib.hipbmg_residual_norm_noalloc(32769, 32769, 5, ctypes.c_void_p(gp.data_ptr()),
                                          ctypes.c_void_p(gb.data_ptr()), ctypes.c_void_p(gu.data_ptr()), out,
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == HB.EINVAL
    assert b"allocation-free limit" in lib.hipbmg_last_error()
    # the entry point still works after the rejected call
    assert HB.residual_norm(gp, gb, gu, noalloc=True) == HB.residual_norm(gp, gb, gu)
