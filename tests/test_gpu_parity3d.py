"""GPU parity of the 3D path (include/hipbmg3d.h) against the 3D FP64 oracle,
through the C interface: finite volumes, every level's interpolation weights
and Galerkin operator, each solve-phase operation, whole solves cycle by
cycle, edge cases, and at the full 257^3 size sampled values that a local
oracle window reproduces plus the true residual of the answer.

Tolerances: the GPU sums the same terms in other orders (27-point stencils,
Galerkin triple sums), so single operations agree to a few ulps of their
magnitudes (1e-13 relative); relative residual histories agree to 5e-14 of
their largest entry over a solve (measured <= 5.7e-15: errors grow with the
condition of the coarse operators but stay far below the 1e-10 stopping
test's resolution).
"""
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


def c(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def problem(shape, seed, kind="blocks"):
    nz, ny, nx = shape
    if kind == "blocks":
        D = inputs.cells3_log10_blocks(nx, ny, nz, block=4, seed=seed)
    elif kind == "lognormal":
        D = inputs.cells3_lognormal(nx, ny, nz, sigma=1.0, seed=seed)
    else:
        D = np.ones((nz - 1, ny - 1, nx - 1))
    b = inputs.load3_uniform(nx, ny, nz, seed=seed + 1)
    return D, b


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("shape", [(9, 9, 9), (17, 9, 33)])
def test_fv7_matches_the_oracle_bitwise(shape):
    D, _ = problem(shape, 40)
    assert np.array_equal(c(HB.fv7_from_cells(g(D))), O.fv7(D))


@pytest.mark.parametrize("shape,npt", [((17, 17, 17), 7), ((9, 17, 33), 7), ((17, 17, 17), 27)])
def test_hierarchy_matches_the_oracle(shape, npt):
    D, _ = problem(shape, 41)
    planes = O.fv7(D)
    if npt == 27:
        # a 27-point finest operator: the oracle's first Galerkin level of a finer problem
        fine = O.Hierarchy3(O.fv7(inputs.cells3_log10_blocks(*(2 * s - 1 for s in shape[::-1]), block=4,
                                                              seed=42)))
        st = fine.stencil(fine.L - 2).reshape(shape + (27,))
        planes = np.concatenate([st[None, ..., 13]] + [-st[None, ..., o] for o in range(13)])
    ora = O.Hierarchy3(planes)
    gpu = HB.Hierarchy3(g(planes))
    assert gpu.L == ora.L
    for l in range(ora.L):
        assert gpu.size(l) == ora.size(l)
        want = np.moveaxis(ora.stencil(l).reshape(ora.size(l) + (27,)), -1, 0)
        got = c(gpu.stencil(l))
        assert rel_err(got, want) <= 1e-13, l
        if l:
            want = np.moveaxis(ora.interp(l).reshape(ora.size(l) + (8,)), -1, 0)
            got = c(gpu.interp(l))
            assert np.abs(got - want).max() <= 1e-13, l


@pytest.mark.parametrize("shape", [(17, 17, 17), (9, 17, 33)])
def test_single_operations_match_the_oracle(shape):
    D, b = problem(shape, 43, "lognormal")
    planes = O.fv7(D)
    ora = O.Hierarchy3(planes)
    gpu = HB.Hierarchy3(g(planes))
    rng = np.random.default_rng(44)
    for l in range(ora.L - 1, -1, -1):
        sz = ora.size(l)
        bl = np.zeros(sz)
        bl[1:-1, 1:-1, 1:-1] = rng.standard_normal(tuple(s - 2 for s in sz))
        x0 = np.zeros(sz)
        x0[1:-1, 1:-1, 1:-1] = rng.standard_normal(tuple(s - 2 for s in sz))
        for sweeps in (1, 2):
            assert rel_err(c(gpu.smooth(l, g(bl), g(x0), sweeps)), ora.smooth(l, bl, x0, sweeps)) <= 1e-13, l
        r = ora.residual(l, bl, x0)
        assert rel_err(c(gpu.residual(l, g(bl), g(x0))), r) <= 1e-13, l
        if l:
            assert rel_err(c(gpu.restrict(l, g(r))), ora.restrict(l, r)) <= 1e-13, l
            csz = ora.size(l - 1)
            xc = np.zeros(csz)
            xc[1:-1, 1:-1, 1:-1] = rng.standard_normal(tuple(s - 2 for s in csz))
            for rc in (0, 1):
                want = ora.interp_correct(l, x0, r, xc, rc)
                assert rel_err(c(gpu.interp_correct(l, g(x0), g(r), g(xc), rc)), want) <= 1e-13, (l, rc)
    sz = ora.size(0)
    b0 = np.zeros(sz)
    b0[1:-1, 1:-1, 1:-1] = rng.standard_normal(tuple(s - 2 for s in sz))
    assert rel_err(c(gpu.coarse_solve(g(b0))), ora.coarse_solve(b0)) <= 1e-13


@pytest.mark.parametrize("shape,kind,prm", [
    ((17, 17, 17), "blocks", {}),
    ((33, 33, 33), "lognormal", {}),
    ((9, 17, 33), "blocks", {}),
    ((17, 17, 17), "const", {"residual_correction": 0}),
    ((33, 17, 17), "blocks", {"coarsest_n": 5}),
    ((17, 17, 17), "lognormal", {"nu1": 1, "nu2": 2}),
])
def test_solve_history_matches_the_oracle(shape, kind, prm):
    D, b = problem(shape, 45, kind)
    planes = O.fv7(D)
    ora = O.Hierarchy3(planes, coarsest_n=prm.get("coarsest_n", 3), nu1=prm.get("nu1", 2),
                       nu2=prm.get("nu2", 1), rescorr=prm.get("residual_correction", 1))
    u_ref, hist = ora.solve(b, tol=1e-10)
    gpu = HB.Hierarchy3(g(planes), **prm)
    u, info = gpu.solve(g(b), tol=1e-10)
    h = np.array(info.history())
    print("%s %s: %d cycles (oracle %d), relres %.3e" % (shape, kind, info.cycles, len(hist), info.relres))
    assert info.cycles == len(hist)
    print("history: max difference %.3e of the largest, %.3e relative" % (np.abs(h - hist).max() / hist.max(),
                                                                         (np.abs(h - hist) / hist).max()))
    # measured <= 2.3e-15 of the largest and <= 2.8e-7 relative per cycle
    assert np.abs(h - hist).max() <= 5e-14 * hist.max()
    assert np.all(np.abs(h - hist) <= 1e-6 * hist)
    assert info.relres <= 1e-10
    # the answer's residual under the oracle's operator
    r = ora.residual(ora.L - 1, b, c(u))
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)


def test_solve_from_a_27_point_finest_operator_matches_the_oracle():
    # a 27-point finest operator (the oracle's first Galerkin level of a finer
    # block medium) on a non-cubic grid: the whole solve cycle by cycle
    fine = O.Hierarchy3(O.fv7(inputs.cells3_log10_blocks(33, 17, 33, block=4, seed=56)))
    st = fine.stencil(fine.L - 2)
    shape = st.shape[:3]
    flat = st.reshape(shape + (27,))
    planes = np.concatenate([flat[None, ..., 13]] + [-flat[None, ..., o] for o in range(13)])
    b = inputs.load3_uniform(shape[2], shape[1], shape[0], seed=57)
    ora = O.Hierarchy3(planes)
    _, hist = ora.solve(b, tol=1e-10)
    gpu = HB.Hierarchy3(g(planes))
    u, info = gpu.solve(g(b), tol=1e-10)
    h = np.array(info.history())
    print("27-point history: max difference %.3e of the largest" % (np.abs(h - hist).max() / hist.max()))
    assert info.cycles == len(hist) and np.abs(h - hist).max() <= 5e-14 * hist.max()   # measured 1.6e-15
    r = ora.residual(ora.L - 1, b, c(u))
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)


def test_edge_cases():
    # a 3^3 grid: one unknown, one level, the Cholesky solve alone
    D, b = problem((3, 3, 3), 46, "lognormal")
    planes = O.fv7(D)
    gpu = HB.Hierarchy3(g(planes))
    assert gpu.L == 1
    u, info = gpu.solve(g(b), tol=1e-12)
    assert info.cycles == 1 and abs(c(u)[1, 1, 1] - b[1, 1, 1] / planes[0, 1, 1, 1]) <= 1e-15 * abs(c(u)[1, 1, 1])
    # zero right-hand side: u = 0 without cycles
    D, b = problem((9, 9, 9), 47)
    gpu = HB.Hierarchy3(g(O.fv7(D)))
    u, info = gpu.solve(torch.zeros((9, 9, 9), dtype=torch.float64, device=DEV), u0=g(np.ones((9, 9, 9))))
    assert info.cycles == 0 and float(c(u).max()) == 0.0
    # an initial guess (boundary entries ignored) and a cycle cap: ENOCONV with the capped iterate
    D, b = problem((17, 17, 17), 48, "lognormal")
    planes = O.fv7(D)
    u0 = np.random.default_rng(49).standard_normal((17, 17, 17))
    ora = O.Hierarchy3(planes)
    u_ref, hist = ora.solve(b, u0=u0, tol=1e-30, max_cycles=3)
    gpu = HB.Hierarchy3(g(planes), max_cycles=3)
    u, info = gpu.solve(g(b), u0=g(u0), tol=1e-30, check=False)
    assert info.cycles == 3 and rel_err(c(u), u_ref) <= 1e-11
    with pytest.raises(HB.HipBMGError) as e:
        gpu.solve(g(b), u0=g(u0), tol=1e-30)
    assert e.value.status == HB.ENOCONV
    # an odd size whose half is even stops coarsening there: 7 -> 4
    D, b = problem((7, 13, 7), 50)
    planes = O.fv7(D)
    ora = O.Hierarchy3(planes)
    gpu = HB.Hierarchy3(g(planes))
    assert gpu.L == ora.L == 2 and gpu.size(0) == (4, 7, 4)
    u, info = gpu.solve(g(b))
    _, hist = ora.solve(b)
    assert info.cycles == len(hist)


def test_full_size_257_sampled_against_oracle_windows_and_true_residual():
    # 257^3 vertices (16.97 M), the size the benchmark runs
    n = 257
    D = inputs.cells3_log10_blocks(n, n, n, block=8, seed=51)
    Dg = g(D)
    planes = HB.fv7_from_cells(Dg)
    gpu = HB.Hierarchy3(planes)
    L = gpu.L
    assert L == 8
    # sampled: a window of 16^3 cells starting at an even vertex reproduces,
    # away from its own boundary, the weights and the first Galerkin operator
    rng = np.random.default_rng(52)
    P = gpu.interp(L - 1)
    A1 = gpu.stencil(L - 2)
    for _ in range(3):
        c0 = 2 * rng.integers(0, (n - 1 - 16) // 2, size=3)
        win = D[c0[0]:c0[0] + 16, c0[1]:c0[1] + 16, c0[2]:c0[2] + 16]
        ora = O.Hierarchy3(O.fv7(win))
        Pw = np.moveaxis(ora.interp(ora.L - 1).reshape(17, 17, 17, 8), -1, 0)
        Aw = np.moveaxis(ora.stencil(ora.L - 2).reshape(9, 9, 9, 27), -1, 0)
        got = c(P[:, c0[0] + 6:c0[0] + 11, c0[1] + 6:c0[1] + 11, c0[2] + 6:c0[2] + 11])
        assert np.abs(got - Pw[:, 6:11, 6:11, 6:11]).max() <= 1e-13
        cc = c0 // 2
        got = c(A1[:, cc[0] + 4, cc[1] + 4, cc[2] + 4])
        want = Aw[:, 4, 4, 4]
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    del P, A1
    # the answer's true residual, from the finite-volume planes with torch ops
    b = g(inputs.load3_uniform(n, n, n, seed=53))
    u, info = gpu.solve(b, tol=1e-10)
    print("257^3: %d cycles, relres %.3e" % (info.cycles, info.relres))
    C, W, S, B = planes
    Au = C * u
    Au[:, :, 1:] -= W[:, :, 1:] * u[:, :, :-1]
    Au[:, :, :-1] -= W[:, :, 1:] * u[:, :, 1:]
    Au[:, 1:, :] -= S[:, 1:, :] * u[:, :-1, :]
    Au[:, :-1, :] -= S[:, 1:, :] * u[:, 1:, :]
    Au[1:] -= B[1:] * u[:-1]
    Au[:-1] -= B[1:] * u[1:]
    r = (b - Au)[1:-1, 1:-1, 1:-1]
    rel = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b[1:-1, 1:-1, 1:-1]))
    assert info.relres <= 1e-10 and abs(rel - info.relres) <= 1e-3 * info.relres
    # contrast 1e4 between 8^3-cell blocks: tens of cycles (78 for the 2D analogue at 4097^2)
    assert info.cycles <= 80


def test_graph_replay_is_bitwise_the_eager_cycle():
    # the captured cycle replays on later solves (with eager work between
    # them) and gives bitwise the eager launches' iterates and histories
    D, b = problem((33, 17, 17), 54, "lognormal")
    planes = g(O.fv7(D))
    eager = HB.Hierarchy3(planes, use_graph=0)
    u_e, i_e = eager.solve(g(b))
    graph = HB.Hierarchy3(planes, use_graph=1)
    for rep in range(3):
        u_g, i_g = graph.solve(g(b))
        assert torch.equal(u_g, u_e), rep
        assert i_g.history() == i_e.history(), rep
        graph.smooth(graph.L - 1, g(b), g(np.zeros((33, 17, 17))), 1)
        torch.cuda.synchronize()


@pytest.mark.parametrize("shape,kind", [((33, 33, 33), "lognormal"), ((17, 33, 65), "blocks")])
def test_collapse_level_leaves_the_iteration_bitwise_unchanged(shape, kind):
    # levels 0..l* in one workgroup do the grid-wide kernels' arithmetic in
    # the same order: iterate and history are identical for every l*
    D, b = problem(shape, 55, kind)
    planes = g(O.fv7(D))
    ref = None
    L = HB.Hierarchy3(planes).L
    for ls in range(L):
        h = HB.Hierarchy3(planes, collapse_level=ls)
        u, info = h.solve(g(b))
        assert info.collapse_level == ls
        if ref is None:
            ref = (u, info.history())
        else:
            assert torch.equal(u, ref[0]), ls
            assert info.history() == ref[1], ls
    with pytest.raises(HB.HipBMGError) as e:
        HB.Hierarchy3(planes, collapse_level=L)
    assert e.value.status == HB.EINVAL
    # the model's choice is one of them and reports its predictions
    u, info = HB.Hierarchy3(planes).solve(g(b))
    assert 0 <= info.collapse_level < L and torch.equal(u, ref[0])
    assert all(info.model_us[l] > 0 for l in range(L))


@pytest.mark.parametrize("case", range(12))
def test_random_shapes_and_parameters_match_the_oracle(case):
    # seeded random odd sizes (3..41 per side, coarsening stopping wherever a
    # side turns even), media, V(nu1,nu2), r/C, coarsest size and collapse level
    rng = np.random.default_rng(600 + case)
    nx, ny, nz = (int(2 * rng.integers(1, 21) + 1) for _ in range(3))
    kind = ["blocks", "lognormal", "const"][case % 3]
    D, b = problem((nz, ny, nx), 610 + case, kind)
    prm = {"nu1": int(rng.integers(1, 4)), "nu2": int(rng.integers(1, 3)),
           "residual_correction": int(rng.integers(0, 2)), "coarsest_n": int(rng.choice([3, 5]))}
    planes = O.fv7(D)
    ora = O.Hierarchy3(planes, coarsest_n=prm["coarsest_n"], nu1=prm["nu1"], nu2=prm["nu2"],
                       rescorr=prm["residual_correction"])
    nunk = np.prod([s - 2 for s in ora.size(0)])
    if nunk > 4096:
        pytest.skip("coarsest level beyond the direct solver's limit")
    _, hist = ora.solve(b, tol=1e-10, max_cycles=200)
    gpu_L = HB.Hierarchy3(g(planes), **prm).L
    prm["collapse_level"] = int(rng.integers(0, min(gpu_L, 8)))
    gpu = HB.Hierarchy3(g(planes), max_cycles=200, **prm)
    u, info = gpu.solve(g(b), tol=1e-10, check=False)
    h = np.array(info.history())
    print((nz, ny, nx), kind, prm, info.cycles, len(hist))
    assert info.cycles == len(hist)
    # relative residuals near the rounding level (a direct solve on one
    # level) differ by rounding alone: an absolute floor of 1e-14
    print("random case history: max difference %.3e of the largest" % (np.abs(h - hist).max() / hist.max()))
    assert np.abs(h - hist).max() <= 5e-14 * hist.max() + 1e-14     # measured <= 5.7e-15


def _solve_bytes(planes, b):
    h = HB.Hierarchy3(planes)
    h.profile(True)
    u, info = h.solve(b)
    pr = h.profile_read()
    return u, info, pr["relax_colour"][2], pr["residual"][2]


@pytest.mark.parametrize("shape,kind,gpu_fv", [((33, 33, 33), "blocks", False), ((17, 33, 65), "lognormal", True)])
def test_formed_diagonal_is_bitwise_the_loaded_one(shape, kind, gpu_fv, monkeypatch):
    # finite volumes store C as W_p + W_e + S_p + S_n + B_p + B_t; the setup
    # checks that bitwise and the finest relaxation and residual kernels then
    # form the diagonal instead of loading it: the same iteration bit for bit,
    # with one plane fewer read
    D, b = problem(shape, 56, kind)
    planes = HB.fv7_from_cells(g(D)) if gpu_fv else g(O.fv7(D))
    n = shape[0] * shape[1] * shape[2]
    monkeypatch.setenv("HIPBMG_NO_ZEXC", "1")
    u0, i0, rb0, sb0 = _solve_bytes(planes, g(b))
    monkeypatch.delenv("HIPBMG_NO_ZEXC")
    u1, i1, rb1, sb1 = _solve_bytes(planes, g(b))
    assert i0.cycles == i1.cycles and i0.history() == i1.history()
    assert torch.equal(u0, u1)
    assert rb0 == 56 * n / 4 and rb1 == 48 * n / 4      # mean of the four colour-group launches
    assert sb0 - sb1 == 8 * n
    # an operator whose diagonal is not that sum (a reaction term) keeps
    # loading it and still reaches the tolerance by the oracle's residual
    p2 = planes.clone()
    p2[0, 1:-1, 1:-1, 1:-1] += 0.5
    ora = O.Hierarchy3(c(p2))
    u2, i2, rb2, _ = _solve_bytes(p2, g(b))
    assert rb2 == 56 * n / 4
    r = ora.residual(ora.L - 1, b, c(u2))
    bi = b[1:-1, 1:-1, 1:-1]
    assert np.linalg.norm(r) <= 1.2e-10 * np.linalg.norm(bi), np.linalg.norm(r) / np.linalg.norm(bi)
