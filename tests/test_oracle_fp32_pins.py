"""Pins of the oracle's FP32 edge-form mode (the inner solver of mixed
precision) against facts that do not come from its own code: exact arithmetic
on dyadic data, the floating-point forward-error bound of each operation, the
zero row sums of pure diffusion, the convergence of the refinement and a
sparse direct solve.

The representation follows the reading used for mixed precision: setup in
FP64, each level demoted once to connections c_pq (float) and an excess
E_p = A(p,p) - sum_q c_pq (double, then float), (A x)_p formed as
sum_q c_pq (x_p - x_q) + E_p x_p.  The method's steps are those of Algorithm 1
(section 2) with the r/C term (section 3).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1803_02481_amd import inputs
from tests import helpers as H

U32 = 2.0 ** -24


def _ring0(a):
    a[0, :] = a[-1, :] = a[:, 0] = a[:, -1] = 0
    return a


def _rand32(rng, shape, lo=-1.0, hi=1.0, integer=False):
    if integer:
        v = rng.integers(int(lo), int(hi) + 1, size=shape).astype(np.float32)
    else:
        v = rng.uniform(lo, hi, size=shape).astype(np.float32)
    return _ring0(v)


# --------------------------------------------------------------------------
# exact arithmetic: D = 1 gives dyadic operators and weights, so on integer
# data every float operation is exact and must equal the FP64 oracle bitwise
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [17, 33])
def test_fp32_equals_fp64_on_dyadic_data(n):
    h = O.Hierarchy(O.fv5(np.ones((n - 1, n - 1))))
    rng = np.random.default_rng(n)
    fine = h.L - 1
    ny, nx = h.size(fine)
    x = _rand32(rng, (ny, nx), -4, 4, integer=True)
    b = _rand32(rng, (ny, nx), -8, 8, integer=True)
    # the finest diagonal is 4 everywhere, so a four-colour sweep divides by a
    # power of two only: exact while the values keep few bits
    assert np.array_equal(h.smooth32(fine, b, x, 1), h.smooth(fine, b.astype(np.float64), x.astype(np.float64), 1))
    r32 = h.residual32(fine, b, x)
    r64 = h.residual(fine, b.astype(np.float64), x.astype(np.float64))
    assert np.array_equal(r32, r64)
    # restriction by the weights 1, 1/2, 1/4
    assert np.array_equal(h.restrict32(fine, r32), h.restrict(fine, r64))
    # interpolation and the r/C term with C = 4
    xc = _rand32(rng, h.size(fine - 1), -4, 4, integer=True)
    got = h.interp_correct32(fine, x, r32, xc, 1)
    want = h.interp_correct(fine, x.astype(np.float64), r64, xc.astype(np.float64), 1)
    assert np.array_equal(got, want)
    # every Galerkin level of D = 1 is dyadic (closed form), so its edge form
    # holds the FP64 entries exactly and its residual on integer data is exact
    for l in range(fine - 1, 0, -1):
        A32, P32 = h.level32(l)
        A64 = h.stencil(l)
        conn = -A64.copy()
        conn[:, :, 1, 1] = 0.0
        exc = A64[:, :, 1, 1] - conn.sum(axis=(2, 3))
        want = conn.copy()
        want[:, :, 1, 1] = exc
        assert np.array_equal(A32.astype(np.float64), want), l
        assert np.array_equal(P32.astype(np.float64), h.interp(l)), l
        cy, cx = h.size(l)
        xl = _rand32(rng, (cy, cx), -4, 4, integer=True)
        bl = _rand32(rng, (cy, cx), -8, 8, integer=True)
        assert np.array_equal(h.residual32(l, bl, xl), h.residual(l, bl.astype(np.float64), xl.astype(np.float64))), l


def test_fp32_dyadic_catches_a_dropped_excess():
    # next to the boundary the excess carries the Dirichlet connection; the
    # residual there differs from the one without it by c * x, far above any
    # rounding, so the dyadic check above covers the excess term
    n = 17
    h = O.Hierarchy(O.fv5(np.ones((n - 1, n - 1))))
    A32, _ = h.level32(h.L - 1)
    assert A32[1, 5, 1, 1] == 1.0 and A32[1, 1, 1, 1] == 2.0 and A32[5, 5, 1, 1] == 0.0


# --------------------------------------------------------------------------
# forward-error bounds on random high-contrast media: each float operation is
# the FP64 one on the same (widened) inputs, within a few units of float
# rounding of the sum of the magnitudes of its terms
# --------------------------------------------------------------------------
def _terms(A64, A32, x, b):
    """|b| + sum_q |c_pq| |x_p - x_q| + |E_p x_p| over the interior."""
    ny, nx = x.shape
    xd = x.astype(np.float64)
    T = np.abs(b).astype(np.float64)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            xq = np.zeros_like(xd)
            xq[1:-1, 1:-1] = xd[1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx]
            T += np.abs(A64[:, :, dy + 1, dx + 1]) * np.abs(xd - xq)
    T += np.abs(A32[:, :, 1, 1].astype(np.float64) * xd)
    return T


@pytest.mark.parametrize("npt", [5, 9])
def test_fp32_operations_within_forward_error_bound(npt):
    n = 65
    D = inputs.cells_log10_blocks(n, n, 4, seed=3)
    planes = O.fv5(D)
    if npt == 9:
        # a 9-point finest operator: the first Galerkin level of a finer grid
        big = O.Hierarchy(O.fv5(inputs.cells_log10_blocks(2 * n - 1, 2 * n - 1, 8, seed=3)))
        st = big.stencil(big.L - 2)
        planes = np.stack([st[:, :, 1, 1], -st[:, :, 1, 0], -st[:, :, 0, 1], -st[:, :, 0, 0], -st[:, :, 0, 2]])
    h = O.Hierarchy(planes)
    rng = np.random.default_rng(npt)
    for l in range(h.L - 1, 0, -1):
        ny, nx = h.size(l)
        A32, P32 = h.level32(l)
        A64 = h.stencil(l)
        x = _rand32(rng, (ny, nx))
        b = _rand32(rng, (ny, nx))
        # residual: <= ~12 roundings of the terms (9 products and sums, the
        # connection and excess roundings, the final difference); measured
        # <= 3.4 units
        r32 = h.residual32(l, b, x)
        r64 = h.residual(l, b.astype(np.float64), x.astype(np.float64))
        T = _terms(A64, A32, x, b)
        assert np.all(np.abs(r32 - r64) <= 16 * U32 * T), l
        # restriction: four weights per fine vertex, each rounded once
        Pabs = np.abs(h.interp(l))
        bc64 = h.restrict(l, r32.astype(np.float64))
        bcT = np.zeros_like(bc64)
        for bb in (0, 1):
            for aa in (0, 1):
                contrib = Pabs[1:-1, 1:-1, bb, aa] * np.abs(r32[1:-1, 1:-1])
                jj, ii = np.mgrid[1:ny - 1, 1:nx - 1]
                np.add.at(bcT, ((jj >> 1) + bb, (ii >> 1) + aa), contrib)
        assert np.all(np.abs(h.restrict32(l, r32) - bc64) <= 16 * U32 * bcT), l
        # interpolation and r/C
        xc = _rand32(rng, h.size(l - 1))
        got = h.interp_correct32(l, x, r32, xc, 1)
        want = h.interp_correct(l, x.astype(np.float64), r32.astype(np.float64), xc.astype(np.float64), 1)
        C = A64[:, :, 1, 1]
        Cs = np.where(C > 0, C, 1.0)
        xcT = np.zeros_like(want)
        xcd = np.abs(xc.astype(np.float64))
        jj, ii = np.mgrid[0:ny, 0:nx]
        for bb in (0, 1):
            for aa in (0, 1):
                J = np.minimum((jj >> 1) + bb, xc.shape[0] - 1)
                I = np.minimum((ii >> 1) + aa, xc.shape[1] - 1)
                xcT += Pabs[:, :, bb, aa] * xcd[J, I]
        bound = 16 * U32 * (np.abs(x) + xcT + np.abs(r32) / Cs)
        assert np.all(np.abs(got - want) <= bound), l


# --------------------------------------------------------------------------
# the property the edge form exists for: rows of pure diffusion away from the
# boundary keep a zero row sum to FP64 rounding after demotion
# --------------------------------------------------------------------------
def test_fp32_edge_form_keeps_zero_row_sums():
    n = 129
    h = O.Hierarchy(O.fv5(inputs.cells_log10_blocks(n, n, 8, seed=9)))
    for l in range(h.L - 1, 0, -1):
        ny, nx = h.size(l)
        if ny < 9:
            continue
        one = _ring0(np.ones((ny, nx), np.float32))
        rs = -h.residual32(l, np.zeros_like(one), one)        # A32 applied to the constant 1
        C = h.stencil(l)[:, :, 1, 1]
        core = (slice(3, -3), slice(3, -3))
        # what is left is the FP64 Galerkin row sum itself, whose rounding
        # accumulates over the products (measured <= 4.9e-13 C at the 9^2
        # level of this 129^2 medium); rounding every matrix entry to float
        # instead would leave row sums of about 1e-7 C
        assert np.abs(rs[core] / C[core]).max() <= 1e-11, l


# --------------------------------------------------------------------------
# the inner V-cycle and the refinement
# --------------------------------------------------------------------------
def test_fp32_vcycle_contracts_like_fp64():
    n = 129
    planes = O.fv5(np.exp(np.random.default_rng(4).standard_normal((n - 1, n - 1))))
    h = O.Hierarchy(planes)
    b = inputs.load_uniform(n, n, seed=5)
    rn = np.linalg.norm(b[1:-1, 1:-1])
    e, hist = h.inner32(b.astype(np.float32), 6, rn)
    # lognormal sigma = 1: the FP64 V-cycle contracts by <= 0.15 per cycle;
    # the FP32 one does the same until float rounding is reached
    rates = hist[1:] / hist[:-1]
    assert hist[0] <= 0.15 and np.all(rates[hist[1:] > 1e-5] <= 0.15), hist
    # one FP32 cycle is the FP64 cycle to float accuracy
    e1, _ = h.inner32(b.astype(np.float32), 1, rn)
    u1 = h.vcycle(b, np.zeros_like(b))
    assert np.abs(e1 - u1).max() <= 1e-5 * np.abs(u1).max()


@pytest.mark.parametrize("kind", ["blocks", "checkerboard"])
def test_mixed_solve_reaches_the_fp64_answer(kind):
    n = 257
    if kind == "blocks":
        D = inputs.cells_log10_blocks(n, n, 16, seed=1)
    else:
        D = inputs.cells_two_phase_blocks(n, n, 16, seed=3)
    planes = O.fv5(D)
    b = inputs.load_uniform(n, n, seed=2)
    h = O.Hierarchy(planes)
    u, hist, cycles, steps = h.solve_mixed(b, tol=1e-10)
    # the relative residual by an independently assembled sparse matrix
    A = H.matrix_from_planes(planes)
    bi = H.to_interior(b)
    rel = np.linalg.norm(bi - A @ H.to_interior(u)) / np.linalg.norm(bi)
    assert rel <= 1e-10 and hist[-1] <= 1e-10 and steps == len(hist) - 1
    # each refinement step cuts the FP64 residual by at least 1e-2 or reaches
    # the tolerance (inner solves stop at 1e-4 relative, or at tol / (2 rel)
    # when that is looser; the FP32 operator is a close model of the FP64 one
    # because of the edge form)
    assert np.all(hist[1:] <= np.maximum(1e-2 * hist[:-1], 1e-10)), hist
    # the answer is the direct solution to the conditioning of the residual
    ud = spla.spsolve(A.tocsc(), bi)
    assert np.abs(H.to_interior(u) - ud).max() <= 1e-6 * np.abs(ud).max()
