"""GPU checks of streaming-pass variants that must not change the iteration:
the up leg forming r/C from the rows it loads instead of reading a stored
plane, the last cycle of a capped solve run as the pipelined pass's first
stage alone, the pipelined pass forming a zero-excess operator's diagonal
instead of loading it, the tile kernels of the small coarse levels, and the
large coarse levels forming the diagonal of their deep vertices.  Each is
compared bitwise with the path it replaces."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1803_02481_amd import hipbmg as HB
from paper_1803_02481_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def c(t):
    return t.detach().cpu().numpy()


def run(planes, b, cycles, tol=1e-30, **prm):
    h = HB.Hierarchy(g(planes), max_cycles=cycles, **prm)
    u, info = h.solve(g(b), tol=tol, check=False)
    torch.cuda.synchronize()
    return u, info


@pytest.mark.parametrize("precision", [HB.FP64, HB.MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny", [(257, 257), (385, 193)])
def test_up_leg_r_over_c_formed_from_rows_is_bitwise_the_stored_one(nx, ny, precision, monkeypatch):
    # the up leg's r/C from the loaded pre-relaxed iterate (no q plane) on every
    # coarse level, against the stored q on every level: the same expressions
    # on the same values.  The computed diagonal is kept on every level (an r/C
    # level would otherwise store its deep vertices' diagonal as the sum of its
    # connections, a different operator at the rounding level)
    monkeypatch.setenv("HIPBMG_NO_ZC9", "1")
    planes = O.fv5(inputs.cells_log10_blocks(nx, ny, 16, seed=60))
    b = inputs.load_uniform(nx, ny, seed=61)
    res = {}
    for name, lim in (("stored", "1000000000000"), ("formed", "0")):
        monkeypatch.setenv("HIPBMG_RC_MIN", lim)
        for rb in ("1", "5"):
            monkeypatch.setenv("HIPBMG_RB", rb)
            res[(name, rb)] = run(planes, b, 4, collapse_level=1, precision=precision)
    for rb in ("1", "5"):
        assert torch.equal(res[("stored", rb)][0], res[("formed", rb)][0]), rb
        assert res[("stored", rb)][1].history() == res[("formed", rb)][1].history()
    assert torch.equal(res[("formed", "1")][0], res[("formed", "5")][0])



@pytest.mark.parametrize("n", [129, 257])
def test_last_cycle_pass_is_bitwise_the_rebuild(n, monkeypatch):
    planes = O.fv5(inputs.cells_log10_blocks(n, n, 16, seed=70))
    b = inputs.load_uniform(n, n, seed=71)
    out = {}
    for name, flag in (("rebuild", "1"), ("last_pass", "0")):
        monkeypatch.setenv("HIPBMG_NO_LAST_PASS", flag)
        # mixed: the inner FP32 solves stop at a cycle cap of 8 (all but
        # possibly the last, which may reach its looser tolerance first)
        out[(name, "mixed")] = run(planes, b, 500, tol=1e-10, precision=HB.MIXED, inner_max_cycles=8)
        # FP64 capped before the tolerance
        out[(name, "fp64")] = run(planes, b, 5, tol=1e-30)
    for prec in ("mixed", "fp64"):
        (u0, i0), (u1, i1) = out[("rebuild", prec)], out[("last_pass", prec)]
        print("%s: %d cycles, relres %.3e" % (prec, i1.cycles, i1.relres))
        assert i0.cycles == i1.cycles and i0.outer_steps == i1.outer_steps
        assert torch.equal(u0, u1), prec
        assert i0.history() == i1.history(), prec
        assert i0.relres == i1.relres


@pytest.mark.parametrize("precision", [HB.FP64, HB.MIXED])
@pytest.mark.parametrize("nx,ny,gpu_fv", [(257, 257, False), (225, 161, True), (129, 385, False), (65, 129, False)])
def test_zero_excess_pass_is_bitwise_the_loading_pass(nx, ny, gpu_fv, precision, monkeypatch):
    # a finite-volume operator's diagonal is the sum of its connections: the
    # pipelined pass forms it instead of loading it, with the same bits
    cells = inputs.cells_log10_blocks(nx, ny, 8, seed=nx + ny)
    planes = HB.fv5_from_cells(g(cells)) if gpu_fv else g(O.fv5(cells))
    b = g(inputs.load_uniform(nx, ny, seed=7))
    res = {}
    for noz in ("1", "0"):
        monkeypatch.setenv("HIPBMG_NO_ZEXC", noz)
        h = HB.Hierarchy(planes, precision=precision)
        h.profile(True)
        u, info = h.solve(b, tol=1e-10)
        per = h.profile_read(precision)["fused3"][2]
        res[noz] = (u, info.history(), info.cycles, per)
    assert torch.equal(res["0"][0], res["1"][0])
    assert res["0"][1:3] == res["1"][1:3]
    w = 8 if precision == HB.FP64 else 4
    assert res["1"][3] - res["0"][3] == w * nx * ny     # one plane fewer per launch


def test_operator_with_a_reaction_term_keeps_loading_the_diagonal(monkeypatch):
    # C = sum of connections + h^2 c (a reaction term): not a zero excess
    n = 129
    planes = O.fv5(inputs.cells_log10_blocks(n, n, 8, seed=3))
    planes[0, 1:-1, 1:-1] += 1e-3
    b = g(inputs.load_uniform(n, n, seed=4))
    monkeypatch.setenv("HIPBMG_NO_ZEXC", "0")
    h = HB.Hierarchy(g(planes))
    h.profile(True)
    u, info = h.solve(b, tol=1e-10)
    per = h.profile_read(0)["fused3"][2]
    assert per == 68 * n * n
    A = H.matrix_from_planes(planes)
    bi = H.to_interior(c(b))
    assert np.linalg.norm(bi - A @ H.to_interior(c(u))) <= 1.2e-10 * np.linalg.norm(bi)


@pytest.mark.parametrize("nx,ny,seed", [(257, 257, 1), (225, 161, 2), (129, 385, 3), (65, 129, 4), (513, 97, 5)])
def test_formed_weights_pass_is_bitwise_the_loading_pass(nx, ny, seed, monkeypatch):
    # the FP64 pipelined pass forms the finest level's interpolation weights
    # from the rows it loads with the setup's own expressions: the same bits
    # as reading the stored weights, with and without the formed diagonal,
    # through whole solves and through capped solves that end on the
    # pipelined pass's last-cycle and rebuild variants
    planes = g(O.fv5(inputs.cells_log10_blocks(nx, ny, 4, seed=seed)))
    b = g(inputs.load_uniform(nx, ny, seed=seed + 10))
    for noz in ("0", "1"):
        monkeypatch.setenv("HIPBMG_NO_ZEXC", noz)
        for cap in (None, 3):
            res = {}
            for nowf in ("1", "0"):
                monkeypatch.setenv("HIPBMG_WFORM", "0" if nowf == "1" else "1")
                prm = {} if cap is None else {"max_cycles": cap}
                h = HB.Hierarchy(planes, **prm)
                h.profile(True)
                u, info = h.solve(b, tol=1e-10 if cap is None else 1e-30, check=cap is None)
                per = h.profile_read(0)["fused3" if cap is None else "fused3_last"][2]
                res[nowf] = (u, info.history(), info.cycles, per)
            assert torch.equal(res["0"][0], res["1"][0]), (noz, cap)
            assert res["0"][1:3] == res["1"][1:3], (noz, cap)
            assert res["1"][3] - res["0"][3] == 16 * nx * ny     # the weight planes are not read


@pytest.mark.parametrize("precision", [HB.FP64, HB.MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("nw", ["4", "8"])
@pytest.mark.parametrize("nx,ny,cells", [(257, 257, "blocks"), (257, 225, "lognormal"), (193, 97, "blocks"),
                                         (449, 129, "checker")])
def test_tile_kernels_are_bitwise_the_streaming_kernels(nx, ny, cells, nw, precision, monkeypatch):
    # every coarse 9-point level on the tile kernels (whole tiles relaxed in
    # two row phases per sweep) against every level on the streaming kernels:
    # the same expressions on the same values, so the same bits; the collapse
    # level is fixed, as the model prices the two kinds differently
    if cells == "blocks":
        D = inputs.cells_log10_blocks(nx, ny, 16, seed=61)
    elif cells == "lognormal":
        D = inputs.cells_lognormal(nx, ny, 1.0, seed=62)
    else:
        D = inputs.cells_two_phase_blocks(nx, ny, 16, seed=63)
    planes = O.fv5(D)
    b = inputs.load_uniform(nx, ny, seed=64)
    for pipelined in ("0", "1"):
        monkeypatch.setenv("HIPBMG_NO_FUSE3", "0" if pipelined == "1" else "1")
        limits = ("HIPBMG_TILE_MAX", "HIPBMG_TILE_UP_MAX", "HIPBMG_TILE_UP_MAX64")
        for k in limits:
            monkeypatch.setenv(k, "0")
        u0, i0 = run(planes, b, 6, precision=precision, collapse_level=1)
        for k in limits:
            monkeypatch.setenv(k, str(1 << 40))
        monkeypatch.setenv("HIPBMG_TILE_NW", nw)
        u1, i1 = run(planes, b, 6, precision=precision, collapse_level=1)
        monkeypatch.delenv("HIPBMG_TILE_NW")
        for k in limits:
            monkeypatch.delenv(k)
        assert i1.cycles == i0.cycles
        assert list(i1.history()) == list(i0.history())
        assert torch.equal(u1, u0), float((u1 - u0).abs().max())
    # and a whole solve to the tolerance, with the default choice of levels,
    # meets it by the host's residual
    u, info = run(planes, b, 500, tol=1e-10, precision=precision)
    r = H.residual_from_planes(planes, b, c(u))
    assert np.linalg.norm(r) <= 1.2e-10 * np.linalg.norm(b[1:-1, 1:-1])


@pytest.mark.parametrize("precision", [HB.FP64, HB.MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny", [(257, 257), (385, 193)])
def test_coarse_deep_diagonal_formed_is_bitwise_the_loaded_one(nx, ny, precision, monkeypatch):
    # every coarse level on the r/C kernels (HIPBMG_RC_MIN lowered); their
    # deep vertices' diagonal is stored as the ordered sum of the connections
    # at setup, and the kernels form it instead of loading it: the same bits
    # as loading it from the same stored operator
    planes = O.fv5(inputs.cells_log10_blocks(nx, ny, 16, seed=71))
    b = inputs.load_uniform(nx, ny, seed=72)
    monkeypatch.setenv("HIPBMG_RC_MIN", "1000")
    for pipelined in ("0", "1"):
        monkeypatch.setenv("HIPBMG_NO_FUSE3", "0" if pipelined == "1" else "1")
        monkeypatch.setenv("HIPBMG_ZC9_LOAD", "1")
        u0, i0 = run(planes, b, 6, precision=precision, collapse_level=1)
        monkeypatch.delenv("HIPBMG_ZC9_LOAD")
        u1, i1 = run(planes, b, 6, precision=precision, collapse_level=1)
        assert list(i1.history()) == list(i0.history())
        assert torch.equal(u1, u0), float((u1 - u0).abs().max())
    # the stored diagonal: the ordered sum of the eight connections at the
    # deep vertices of every such level, within rounding of the oracle's
    # Galerkin diagonal everywhere
    h = HB.Hierarchy(g(planes), collapse_level=1)
    ora = O.Hierarchy(planes)
    for l in range(1, h.L - 1):
        C, W, S, SW, SE = (c(t) for t in h.stencil(l))
        ny_, nx_ = C.shape
        if nx_ * ny_ < 1000:
            continue
        rs = (W[2:-2, 2:-2] + W[2:-2, 3:-1] + S[2:-2, 2:-2] + S[3:-1, 2:-2] + SW[2:-2, 2:-2] + SW[3:-1, 3:-1]
              + SE[2:-2, 2:-2] + SE[3:-1, 1:-3])
        assert np.array_equal(C[2:-2, 2:-2], rs), l
        Co = ora.stencil(l)[:, :, 1, 1]
        assert np.all(np.abs(C[1:-1, 1:-1] - Co[1:-1, 1:-1]) <= 1e-12 * np.abs(Co[1:-1, 1:-1])), l
    # a whole solve meets the tolerance by the host's residual
    monkeypatch.delenv("HIPBMG_NO_FUSE3")
    u, info = run(planes, b, 500, tol=1e-10, precision=precision)
    r = H.residual_from_planes(planes, b, c(u))
    assert np.linalg.norm(r) <= 1.2e-10 * np.linalg.norm(b[1:-1, 1:-1])
