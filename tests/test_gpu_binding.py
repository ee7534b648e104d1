"""The binding's argument checks and the batched solver's tolerance handling.

The C interface takes bare device pointers and sizes, so the binding checks
every tensor's dtype, device and shape against what the library will read or
write through it and raises before any library call.  A batched handle replays
its V-cycle from a captured graph; the convergence test inside must apply the
tolerance of the current solve.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1803_02481_amd import hipbmg as HB
from paper_1803_02481_amd import inputs
from tests.test_gpu_parity import batch_case, c, g, oracle_relres, rand_cells

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_mismatched_shapes_raise_before_any_library_call():
    n = 33
    planes = O.fv5(rand_cells(n, n, 0))
    hier = HB.Hierarchy(g(planes))
    good = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    bad = torch.zeros((n, n - 2), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        hier.solve(bad)
    with pytest.raises(ValueError):
        hier.solve(good, bad)
    with pytest.raises(ValueError):
        hier.op_smooth(hier.L - 1, bad, good)
    with pytest.raises(ValueError):
        hier.op_interp_smooth(hier.L - 1, good, good, good, good)   # xc has the fine shape
    with pytest.raises(ValueError):
        hier.op_smooth(hier.L, good, good)                          # no such level
    with pytest.raises(TypeError):
        hier.solve(good.float())
    theta = torch.zeros((n - 1, n - 1), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        HB.grad_logD(theta[:-1], good, good)
    with pytest.raises(ValueError):
        HB.grad_logD(theta, good, bad)
    with pytest.raises(ValueError):
        HB.SolveFV.apply(theta, bad)
    with pytest.raises(ValueError):
        HB.SolveFVBatched.apply(theta[None], good[None, :, :-1])
    # the handle still works after the rejected calls
    u, info = hier.solve(g(inputs.load_uniform(n, n, seed=1)))
    assert info.relres <= 1e-10


def test_batched_arguments_are_checked():
    sizes = [(33, 33), (65, 33)]
    planes, bs = batch_case(sizes, seed0=90)
    p9 = np.zeros((5,) + planes[1].shape[1:])
    p9[:3] = planes[1]
    with pytest.raises(ValueError):
        HB.BatchHierarchy([g(planes[0]), g(p9)])      # 5- and 9-point problems in one batch
    bh = HB.BatchHierarchy([g(p) for p in planes])
    with pytest.raises(ValueError):
        bh.solve([g(bs[0])])                           # one right-hand side for two problems
    with pytest.raises(ValueError):
        bh.solve([g(bs[1]), g(bs[0])])                 # shapes swapped
    us, infos = bh.solve([g(b) for b in bs])
    for k in range(2):
        assert oracle_relres(planes[k], bs[k], c(us[k])) <= 1.2e-10


def test_3d_shapes_are_checked():
    m = 9
    planes3 = O.fv7(inputs.cells3_log10_blocks(m, m, m, block=4, seed=41))
    h3 = HB.Hierarchy3(g(planes3))
    with pytest.raises(ValueError):
        h3.solve(torch.zeros((m, m, m - 2), dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        h3.residual(h3.L - 1, torch.zeros((m, m, m), dtype=torch.float64, device=DEV),
                    torch.zeros((m, m), dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("precision", [HB.FP64, HB.MIXED])
@pytest.mark.parametrize("use_graph", [1, 0])
def test_batched_solves_apply_each_call_tolerance(precision, use_graph):
    # one handle, solved at a loose then a tight tolerance and back: every
    # problem ends at the tolerance of its own call.  A graph captured during
    # the first solve must not keep that solve's tolerance.
    sizes = [(65, 65), (129, 97), (33, 33)]
    planes, bs = batch_case(sizes, seed0=120)
    bh = HB.BatchHierarchy([g(p) for p in planes], precision=precision, use_graph=use_graph)
    cycles = {}
    for tol in (1e-6, 1e-10, 1e-6, 1e-10):
        us, infos = bh.solve([g(b) for b in bs], tol=tol)
        assert bh.status == HB.OK
        for k in range(len(sizes)):
            rr = oracle_relres(planes[k], bs[k], c(us[k]))
            assert rr <= 1.2 * tol, (tol, k, rr)
            assert infos[k].relres <= tol, (tol, k, infos[k].relres)
            # an FP64 solve contracts by ~0.1 per cycle, so a loose one stops
            # well above the tight tolerance (a refinement step of mixed
            # precision may jump past both)
            if tol == 1e-6 and precision == HB.FP64:
                assert rr > 1e-9, (k, rr)
        key = tuple(i.cycles for i in infos)
        assert cycles.setdefault(tol, key) == key, (tol, key, cycles[tol])
    assert all(a <= b for a, b in zip(cycles[1e-6], cycles[1e-10])), cycles
    if precision == HB.FP64:
        assert all(a < b for a, b in zip(cycles[1e-6], cycles[1e-10])), cycles


@pytest.mark.parametrize("npt,nx,ny", [(5, 65, 65), (5, 257, 193), (9, 129, 97), (5, 3, 3), (9, 1025, 35)])
def test_residual_norm_matches_host_residual(npt, nx, ny):
    from tests import helpers as H
    from tests.test_gpu_parity import make_planes
    planes = make_planes(nx, ny, npt, seed=nx + ny) if nx > 3 else O.fv5(rand_cells(nx, ny, 1))
    rng = np.random.default_rng(nx * ny)
    b = rng.standard_normal((ny, nx))
    u = rng.standard_normal((ny, nx))
    rn, bn = HB.residual_norm(g(planes), g(b), g(u))
    # the boundary ring of u is read as zero, of b ignored
    r = H.residual_from_planes(planes, b, u)
    want_r = float(np.linalg.norm(r))
    want_b = float(np.linalg.norm(b[1:-1, 1:-1]))
    assert rn == pytest.approx(want_r, rel=1e-13) and bn == pytest.approx(want_b, rel=1e-13), (rn, want_r, bn, want_b)
    # the same bits on a second call
    assert HB.residual_norm(g(planes), g(b), g(u)) == (rn, bn)
    with pytest.raises(ValueError):
        HB.residual_norm(g(planes), g(b[:-1]), g(u))
