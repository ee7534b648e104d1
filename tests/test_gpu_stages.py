"""GPU checks of the agglomeration stages (section 4 on one GPU): levels
between the grid-wide kernels and the collapsed workgroup run on several
workgroups of one launch, with a grid barrier where the single workgroup has
a workgroup barrier.

Every point's arithmetic in a stage is the arithmetic the collapsed
workgroup does for that level, so a solve with stages above collapse level
l* must give bitwise the iterate of the plain collapse of the same levels;
whole solves are also checked on the oracle's residual."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1803_02481_amd import hipbmg as HB
from paper_1803_02481_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def case(n, seed):
    planes = O.fv5(inputs.cells_lognormal(n, n, 1.0, seed=seed))
    b = inputs.load_uniform(n, n, seed=seed + 1)
    return planes, b


def run(planes, b, cycles, **prm):
    h = HB.Hierarchy(g(planes), max_cycles=cycles, **prm)
    u, info = h.solve(g(b), tol=1e-30, check=False)
    torch.cuda.synchronize()
    return u, info


@pytest.mark.parametrize("precision", [HB.FP64, HB.MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("wg", [2, 8, 256])
def test_stage_iterate_equals_plain_collapse(wg, precision):
    planes, b = case(257, 40)
    print("stage of %d workgroups on levels 5..3, l* = 2" % wg, flush=True)
    u0, i0 = run(planes, b, 4, collapse_level=5, cluster_wg=0, precision=precision)
    u1, i1 = run(planes, b, 4, collapse_level=2, cluster_wg=wg, cluster_top=5, precision=precision)
    assert i0.cluster_stages == 0 and i1.cluster_stages == 1
    assert list(i1.cluster_wg)[:1] == [wg] and list(i1.cluster_hi)[:1] == [5]
    assert torch.equal(u0, u1)
    assert i0.history() == i1.history()


def test_several_stages_equal_plain_collapse(monkeypatch):
    planes, b = case(513, 42)
    u0, i0 = run(planes, b, 3, collapse_level=6, cluster_wg=0)
    monkeypatch.setenv("HIPBMG_STAGES", "128:6,16:4,2:3")
    print("stages 128:6, 16:4, 2:3 above l* = 1", flush=True)
    u1, i1 = run(planes, b, 3, collapse_level=1)
    assert i1.cluster_stages == 3
    assert list(i1.cluster_wg)[:3] == [128, 16, 2] and list(i1.cluster_hi)[:3] == [6, 4, 3]
    assert torch.equal(u0, u1)


def test_stage_solve_reaches_tolerance():
    n = 1025
    planes = O.fv5(inputs.cells_log10_blocks(n, n, 16, -2.0, 2.0, seed=1))
    b = inputs.load_uniform(n, n, seed=2)
    print("1025^2 blocks, stage of 32 workgroups on levels 7..4, l* = 3", flush=True)
    h = HB.Hierarchy(g(planes), collapse_level=3, cluster_wg=32, cluster_top=7)
    u, info = h.solve(g(b), tol=1e-10)
    ref, iref = HB.Hierarchy(g(planes), collapse_level=7, cluster_wg=0).solve(g(b), tol=1e-10)
    assert info.cycles == iref.cycles
    assert torch.equal(u, ref)
    ora = O.Hierarchy(planes)
    r = ora.residual(ora.L - 1, b, u.cpu().numpy())
    rr = float(np.linalg.norm(r[1:-1, 1:-1]) / np.linalg.norm(b[1:-1, 1:-1]))
    print("oracle relres %.3e after %d cycles" % (rr, info.cycles))
    assert rr <= 1.2e-10


def test_stage_parameters_are_checked():
    planes, _ = case(129, 44)
    gp = g(planes)
    for prm in ({"collapse_level": 2, "cluster_wg": 3, "cluster_top": 4},     # not a power of two
                {"collapse_level": 2, "cluster_wg": 512, "cluster_top": 4},   # beyond 256
                {"cluster_wg": 8, "cluster_top": 4},                          # no collapse level
                {"collapse_level": 4, "cluster_wg": 8, "cluster_top": 4},     # top not above l*
                {"collapse_level": 2, "cluster_wg": 8, "cluster_top": 6},     # the finest level
                {"collapse_level": 2, "cluster_wg": -2}):
        with pytest.raises(HB.HipBMGError) as e:
            HB.Hierarchy(gp, **prm)
        assert e.value.status == HB.EINVAL, prm


def test_search_reports_a_consistent_path():
    HB.calibrate()
    planes, b = case(1025, 46)
    u, info = run(planes, b, 2)
    print("search: l* %d, %d stages %s %s, %.1f us, %d states expanded"
          % (info.collapse_level, info.cluster_stages, list(info.cluster_wg), list(info.cluster_hi),
             info.search_us, info.search_expanded))
    assert info.search_expanded > 0 and np.isfinite(info.search_us) and info.search_us > 0
    wg, hi = list(info.cluster_wg)[: info.cluster_stages], list(info.cluster_hi)[: info.cluster_stages]
    assert all(w >= 2 for w in wg) and wg == sorted(wg, reverse=True) and len(set(wg)) == len(wg)
    assert all(info.collapse_level < x <= info.levels - 2 for x in hi) and hi == sorted(hi, reverse=True)
    # the plain argmin over l* is one of the paths the search considered
    assert info.search_us <= min(list(info.model_us)[: info.levels]) * (1 + 1e-12)


def test_calibration_measures_stage_terms():
    cal = HB.calibrate()
    for k in range(8):
        wg = 2 << k
        a, bw = cal["alpha_stage_us_%dwg_fp64" % wg], cal["stage_GBps_%dwg_fp64" % wg]
        print("%3d workgroups: %.3f us per barrier phase, %.1f GB/s" % (wg, a, bw))
        assert a > 0.0 or bw > 0.0

