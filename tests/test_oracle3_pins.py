"""Pins of the 3D FP64 CPU oracle against facts fixed by mathematics and by
the method's definition, independent of the oracle's own code: closed forms
(trilinear weights and a Kronecker-product Galerkin operator for D=1,
one-dimensional flux weights for coefficients varying along x only), library
routines on explicitly assembled matrices, invariants and brute force.

Paper sections cited: section 2 (operator-induced interpolation, Galerkin
coarse operator, Algorithm 1 V-cycle), section 3 (the 3D interpolation cost,
interpolation with the r/C term, Cholesky coarse solve), section 5 (vertex-
centred finite volumes for -div(D grad u) with zero Dirichlet data).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1803_02481_amd import inputs


def offsets():
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yield dx, dy, dz


def interior_index(shape):
    nz, ny, nx = shape
    idx = -np.ones(shape, dtype=np.int64)
    idx[1:-1, 1:-1, 1:-1] = np.arange((nz - 2) * (ny - 2) * (nx - 2)).reshape(nz - 2, ny - 2, nx - 2)
    return idx


def matrix3(st):
    """Sparse matrix over interior unknowns from [nz][ny][nx][3][3][3] entries."""
    nz, ny, nx = st.shape[:3]
    idx = interior_index((nz, ny, nx))
    rows, cols, vals = [], [], []
    for dx, dy, dz in offsets():
        a = st[1:-1, 1:-1, 1:-1, dz + 1, dy + 1, dx + 1]
        q = idx[1 + dz:nz - 1 + dz, 1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx]
        m = (q >= 0) & (a != 0)
        rows.append(idx[1:-1, 1:-1, 1:-1][m])
        cols.append(q[m])
        vals.append(a[m])
    n = (nz - 2) * (ny - 2) * (nx - 2)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def interp3(P, cshape):
    """Sparse P (fine interior x coarse interior) from [..][2][2][2] rows."""
    nz, ny, nx = P.shape[:3]
    fi = interior_index((nz, ny, nx))
    ci = interior_index(cshape)
    rows, cols, vals = [], [], []
    K, J, I = np.meshgrid(np.arange(1, nz - 1), np.arange(1, ny - 1), np.arange(1, nx - 1), indexing="ij")
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                w = P[1:-1, 1:-1, 1:-1, c, b, a]
                kc, jc, ic = (K >> 1) + c, (J >> 1) + b, (I >> 1) + a
                ok = (kc < cshape[0]) & (jc < cshape[1]) & (ic < cshape[2]) & (w != 0)
                col = ci[np.minimum(kc, cshape[0] - 1), np.minimum(jc, cshape[1] - 1), np.minimum(ic, cshape[2] - 1)]
                assert np.all(col[ok] >= 0), "weight on a coarse boundary vertex"
                rows.append(fi[1:-1, 1:-1, 1:-1][ok])
                cols.append(col[ok])
                vals.append(w[ok])
    nf = (nz - 2) * (ny - 2) * (nx - 2)
    nc = (cshape[0] - 2) * (cshape[1] - 2) * (cshape[2] - 2)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nf, nc))


def lap1(n):
    """1D Dirichlet Laplacian tridiag(-1, 2, -1) over the n-2 interior vertices."""
    m = n - 2
    return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]).toarray()


def lin1(n):
    """1D linear interpolation, interior fine vertices x interior coarse vertices."""
    nc = (n + 1) // 2
    P = np.zeros((n - 2, nc - 2))
    for I in range(1, nc - 1):
        P[2 * I - 1, I - 1] = 1.0
        P[2 * I - 2, I - 1] = 0.5
        P[2 * I, I - 1] = 0.5
    return P


def rhs(shape, seed):
    nz, ny, nx = shape
    return inputs.load3_uniform(nx, ny, nz, seed=seed)


# --------------------------------------------------------------------------
# Section 5: vertex-centred finite volumes in 3D
# --------------------------------------------------------------------------
def test_fv7_constant_D_is_the_seven_point_laplacian():
    C, W, S, B = O.fv7(np.ones((6, 6, 6)))
    assert np.all(C[1:-1, 1:-1, 1:-1] == 6.0)
    assert np.all(W[1:-1, 1:-1, 1:] == 1.0)
    assert np.all(S[1:-1, 1:, 1:-1] == 1.0)
    assert np.all(B[1:, 1:-1, 1:-1] == 1.0)


def test_fv7_one_cell_gives_a_quarter_to_each_of_its_twelve_edges():
    # the dual face of each of the twelve edges of a cell cuts a quarter of it
    D = np.zeros((4, 4, 4))
    D[1, 2, 1] = 8.0  # cell x in [1,2], y in [2,3], z in [1,2] ([ck][cj][ci])
    C, W, S, B = O.fv7(D)
    for j in (2, 3):
        for k in (1, 2):
            assert W[k, j, 2] == 2.0      # x-edge (1,j,k)-(2,j,k), stored at its east end
    for i in (1, 2):
        for k in (1, 2):
            assert S[k, 3, i] == 2.0      # y-edge (i,2,k)-(i,3,k), stored at its north end
    for i in (1, 2):
        for j in (2, 3):
            assert B[2, j, i] == 2.0      # z-edge (i,j,1)-(i,j,2), stored at its upper end
    assert np.count_nonzero(W) == 4 and np.count_nonzero(S) == 4 and np.count_nonzero(B) == 4
    # the diagonal is the sum of the six connections of the vertex
    assert C[2, 2, 1] == W[2, 2, 1] + W[2, 2, 2] + S[2, 2, 1] + S[2, 3, 1] + B[2, 2, 1] + B[3, 2, 1] == 6.0


# --------------------------------------------------------------------------
# Section 2: operator-induced interpolation, D = 1 -> trilinear
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [9, 17])
def test_interp_constant_D_is_trilinear_on_every_level(n):
    h = O.Hierarchy3(O.fv7(np.ones((n - 1,) * 3)))
    for l in range(1, h.L):
        P = h.interp(l)
        nz, ny, nx = h.size(l)
        cz, cy, cx = h.size(l - 1)
        for k in range(1, nz - 1):
            for j in range(1, ny - 1):
                for i in range(1, nx - 1):
                    for c in (0, 1):
                        for b in (0, 1):
                            for a in (0, 1):
                                # the tensor product of 1D linear weights
                                w = 1.0
                                for t, e in ((i, a), (j, b), (k, c)):
                                    w *= (0.5 if t & 1 else (1.0 if e == 0 else 0.0))
                                I, J, K = (i >> 1) + a, (j >> 1) + b, (k >> 1) + c
                                if not (1 <= I <= cx - 2 and 1 <= J <= cy - 2 and 1 <= K <= cz - 2):
                                    w = 0.0
                                assert P[k, j, i, c, b, a] == w, (l, i, j, k, a, b, c)


@pytest.mark.parametrize("n", [9, 17])
def test_galerkin_constant_D_is_the_kronecker_product_form(n):
    # A = L x I x I + I x L x I + I x I x L with trilinear P = P1 x P1 x P1, so
    # P^T A P = Lc x Mc x Mc + ... with Lc = P1^T L P1, Mc = P1^T M P1 (exact
    # in dyadic arithmetic), level after level
    h = O.Hierarchy3(O.fv7(np.ones((n - 1,) * 3)))
    L1, M1 = lap1(n), np.eye(n - 2)
    nf = n
    for l in range(h.L - 2, -1, -1):
        P1 = lin1(nf)
        L1, M1 = P1.T @ L1 @ P1, P1.T @ M1 @ P1
        nf = (nf + 1) // 2
        want = np.kron(np.kron(M1, M1), L1) + np.kron(np.kron(M1, L1), M1) + np.kron(np.kron(L1, M1), M1)
        got = matrix3(h.stencil(l)).toarray()
        assert np.array_equal(got, want), l


# --------------------------------------------------------------------------
# Section 2: coefficients varying along x only -> 1D flux weights
# --------------------------------------------------------------------------
def test_interp_x_layered_media_uses_one_dimensional_flux_weights():
    # D = D(x): the collapsed relations reduce to the 1D flux balance along x,
    # a_W / (a_W + a_E), times the linear 1/2 along every odd y or z index
    n = 17
    nc = (n + 1) // 2
    rng = np.random.default_rng(5)
    dx = 10.0 ** rng.uniform(-3, 3, size=n - 1)
    D = np.broadcast_to(dx[None, None, :], (n - 1, n - 1, n - 1)).copy()
    h = O.Hierarchy3(O.fv7(D))
    P = h.interp(h.L - 1)
    checked = 0
    for k in range(1, n - 1):
        for j in range(1, n - 1):
            for i in range(1, n - 1, 2):
                wx = (dx[i - 1] / (dx[i - 1] + dx[i]), dx[i] / (dx[i - 1] + dx[i]))
                for c in range(1 + (k & 1)):
                    for b in range(1 + (j & 1)):
                        for a in (0, 1):
                            w = wx[a] * (0.5 if j & 1 else 1.0) * (0.5 if k & 1 else 1.0)
                            I, J, K = (i >> 1) + a, (j >> 1) + b, (k >> 1) + c
                            if not (1 <= I <= nc - 2 and 1 <= J <= nc - 2 and 1 <= K <= nc - 2):
                                w = 0.0
                            # the collapse cancels the y and z connections (a factor 3 of
                            # the diagonal): a few ulps
                            assert abs(P[k, j, i, c, b, a] - w) <= 2e-15, (i, j, k, a, b, c)
                            checked += 1
    assert checked > 1000


# --------------------------------------------------------------------------
# Section 2: Galerkin product against scipy on assembled matrices
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(9, 9, 9), (9, 17, 5), (17, 9, 9)])
def test_galerkin_matches_sparse_triple_product(shape):
    nz, ny, nx = shape
    D = inputs.cells3_log10_blocks(nx, ny, nz, block=2, lo=-2, hi=2, seed=21)
    h = O.Hierarchy3(O.fv7(D))
    for l in range(h.L - 1, 0, -1):
        A = matrix3(h.stencil(l))
        P = interp3(h.interp(l), h.size(l - 1))
        want = (P.T @ A @ P).toarray()
        got = matrix3(h.stencil(l - 1)).toarray()
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-14 * scale, l


def test_coarse_operators_are_symmetric_with_zero_interior_row_sums():
    n = 17
    D = inputs.cells3_lognormal(n, n, n, sigma=1.5, seed=22)
    h = O.Hierarchy3(O.fv7(D))
    for l in range(h.L - 1):
        st = h.stencil(l)
        A = matrix3(st).toarray()
        C = np.abs(np.diag(A)).max()
        assert np.abs(A - A.T).max() <= 1e-14 * C, l
        nz, ny, nx = h.size(l)
        if min(nz, ny, nx) >= 7:
            rs = st.sum(axis=(3, 4, 5))
            assert np.abs(rs[3:-3, 3:-3, 3:-3]).max() <= 1e-13 * C, l


def test_import_of_27_point_planes_reproduces_the_hierarchy_below():
    # a coarse operator written as 14 planes (C, then -A(p, p+d) for the lower
    # half d = 0..12 of the linear offsets) builds the same levels again
    n = 17
    D = inputs.cells3_log10_blocks(n, n, n, block=4, seed=23)
    h = O.Hierarchy3(O.fv7(D))
    st = h.stencil(h.L - 2)
    nz, ny, nx = st.shape[:3]
    flat = st.reshape(nz, ny, nx, 27)
    planes = np.zeros((14, nz, ny, nx))
    planes[0] = flat[..., 13]
    for o in range(13):
        planes[1 + o] = -flat[..., o]
    h2 = O.Hierarchy3(planes)
    assert h2.L == h.L - 1
    # the lower half is taken as given; the upper half is its mirror, which the
    # triple sum reproduces up to the rounding of a separate summation
    top = h2.stencil(h2.L - 1).reshape(nz, ny, nx, 27)
    assert np.array_equal(top[..., :14], flat[..., :14])
    for l in range(h2.L):
        a, b = h2.stencil(l), h.stencil(l)
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max(), l
        if l:
            assert np.abs(h2.interp(l) - h.interp(l)).max() <= 1e-13, l


# --------------------------------------------------------------------------
# Restriction is the transpose of interpolation (section 2)
# --------------------------------------------------------------------------
def test_restriction_is_the_adjoint_of_interpolation():
    n = 17
    D = inputs.cells3_lognormal(n, n, n, seed=24)
    h = O.Hierarchy3(O.fv7(D))
    rng = np.random.default_rng(25)
    l = h.L - 1
    r = np.zeros((n, n, n))
    r[1:-1, 1:-1, 1:-1] = rng.standard_normal((n - 2,) * 3)
    cs = h.size(l - 1)
    v = np.zeros(cs)
    v[1:-1, 1:-1, 1:-1] = rng.standard_normal(tuple(s - 2 for s in cs))
    Pv = h.interp_correct(l, np.zeros((n, n, n)), np.zeros((n, n, n)), v, rescorr=0)
    lhs = float(np.sum(h.restrict(l, r) * v))
    rhs_ = float(np.sum(r * Pv))
    assert abs(lhs - rhs_) <= 1e-12 * abs(lhs)


# --------------------------------------------------------------------------
# Algorithm 1: the V-cycle reaches the direct solution
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,coarsest", [((9, 9, 9), 3), ((17, 9, 9), 3), ((17, 17, 17), 5)])
def test_vcycle_reaches_the_direct_solution(shape, coarsest):
    nz, ny, nx = shape
    D = inputs.cells3_log10_blocks(nx, ny, nz, block=4, seed=26)
    planes = O.fv7(D)
    h = O.Hierarchy3(planes, coarsest_n=coarsest)
    b = rhs(shape, 27)
    u, hist = h.solve(b, tol=1e-10)
    assert hist[-1] <= 1e-10 and len(hist) < 40
    A = matrix3(O.Hierarchy3(planes, coarsest_n=max(shape)).stencil(0))
    ud = spla.spsolve(A.tocsc(), b[1:-1, 1:-1, 1:-1].ravel())
    r = b[1:-1, 1:-1, 1:-1].ravel() - A @ u[1:-1, 1:-1, 1:-1].ravel()
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)
    assert np.abs(u[1:-1, 1:-1, 1:-1].ravel() - ud).max() <= 1e-6 * np.abs(ud).max()


def test_single_level_is_the_cholesky_solve():
    # a grid no coarser than coarsest_n is solved directly in one cycle
    planes = O.fv7(inputs.cells3_lognormal(5, 5, 5, seed=28))
    h = O.Hierarchy3(planes, coarsest_n=5)
    assert h.L == 1
    b = rhs((5, 5, 5), 29)
    u, hist = h.solve(b, tol=1e-12)
    assert len(hist) == 1 and hist[0] <= 1e-14


def test_convergence_rates_are_grid_independent():
    rates = []
    for n in (17, 33):
        h = O.Hierarchy3(O.fv7(np.ones((n - 1,) * 3)))
        u, hist = h.solve(rhs((n, n, n), 30), tol=1e-10)
        rates.append((hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1)))
    assert max(rates) <= 0.08 and abs(rates[0] - rates[1]) <= 0.03
    n = 17
    h = O.Hierarchy3(O.fv7(inputs.cells3_lognormal(n, n, n, sigma=1.0, seed=31)))
    u, hist = h.solve(rhs((n, n, n), 32), tol=1e-10)
    assert (hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1)) <= 0.2


def test_manufactured_solution_converges_at_second_order():
    # u = sin(pi x) sin(pi y) sin(pi z), D = 1: -lap u = 3 pi^2 u, b = h^2 f
    errs = []
    for n in (9, 17, 33):
        h_ = 1.0 / (n - 1)
        x = np.linspace(0, 1, n)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        ue = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
        b = h_ * h_ * 3 * np.pi ** 2 * ue
        b[0], b[-1], b[:, 0], b[:, -1], b[:, :, 0], b[:, :, -1] = 0, 0, 0, 0, 0, 0
        u, hist = O.Hierarchy3(O.fv7(np.ones((n - 1,) * 3))).solve(b, tol=1e-12)
        errs.append(np.abs(u - ue).max())
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.8 <= e0 / e1 <= 4.2, errs


def test_rescorr_term_changes_only_the_path_not_the_answer():
    n = 17
    planes = O.fv7(inputs.cells3_lognormal(n, n, n, seed=33))
    b = rhs((n, n, n), 34)
    u1, h1 = O.Hierarchy3(planes, rescorr=1).solve(b, tol=1e-11)
    u0, h0 = O.Hierarchy3(planes, rescorr=0).solve(b, tol=1e-11)
    assert h1[-1] <= 1e-11 and h0[-1] <= 1e-11
    assert not np.array_equal(h1[:2], h0[:2])
    assert np.abs(u1 - u0).max() <= 1e-8 * np.abs(u1).max()
