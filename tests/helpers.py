"""Test-side assembly of explicit sparse matrices, used to check the oracle
with library routines (scipy.sparse products, triangular and dense solves)."""
import numpy as np
import scipy.sparse as sp


def interior_index(ny, nx):
    idx = -np.ones((ny, nx), dtype=np.int64)
    idx[1:-1, 1:-1] = np.arange((ny - 2) * (nx - 2)).reshape(ny - 2, nx - 2)
    return idx


def matrix_from_planes(planes):
    """Sparse matrix over interior unknowns from {C, W, S[, SW, SE]} planes."""
    ny, nx = planes.shape[1:]
    C, W, S = planes[0], planes[1], planes[2]
    SW = planes[3] if planes.shape[0] == 5 else np.zeros_like(C)
    SE = planes[4] if planes.shape[0] == 5 else np.zeros_like(C)
    idx = interior_index(ny, nx)
    rows, cols, vals = [], [], []
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            p = idx[j, i]
            ent = {(0, 0): C[j, i], (-1, 0): -W[j, i], (1, 0): -W[j, i + 1],
                   (0, -1): -S[j, i], (0, 1): -S[j + 1, i],
                   (-1, -1): -SW[j, i], (1, 1): -SW[j + 1, i + 1],
                   (1, -1): -SE[j, i], (-1, 1): -SE[j + 1, i - 1]}
            for (dx, dy), v in ent.items():
                q = idx[j + dy, i + dx]
                if q >= 0 and v != 0.0:
                    rows.append(p); cols.append(q); vals.append(v)
    n = (ny - 2) * (nx - 2)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def matrix_from_stencil(st):
    """Sparse matrix from the oracle's [ny][nx][3][3] matrix-entry stencil."""
    ny, nx = st.shape[:2]
    idx = interior_index(ny, nx)
    rows, cols, vals = [], [], []
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    v = st[j, i, dy + 1, dx + 1]
                    q = idx[j + dy, i + dx]
                    if v != 0.0:
                        assert q >= 0, "entry towards a boundary vertex"
                        rows.append(idx[j, i]); cols.append(q); vals.append(v)
    n = (ny - 2) * (nx - 2)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def interp_matrix(P, cshape):
    """Sparse P (fine interior x coarse interior) from rows [ny][nx][2][2]."""
    ny, nx = P.shape[:2]
    cny, cnx = cshape
    fidx = interior_index(ny, nx)
    cidx = interior_index(cny, cnx)
    rows, cols, vals = [], [], []
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            for b in (0, 1):
                for a in (0, 1):
                    w = P[j, i, b, a]
                    if w != 0.0:
                        q = cidx[(j >> 1) + b, (i >> 1) + a]
                        assert q >= 0, "weight on a boundary coarse vertex"
                        rows.append(fidx[j, i]); cols.append(q); vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=((ny - 2) * (nx - 2), (cny - 2) * (cnx - 2)))


def to_interior(v):
    return v[1:-1, 1:-1].ravel()


def from_interior(x, ny, nx):
    out = np.zeros((ny, nx))
    out[1:-1, 1:-1] = x.reshape(ny - 2, nx - 2)
    return out


def residual_from_planes(planes, b, u):
    """b - A u over interior vertices (zero on the boundary ring), vectorised,
    with A the operator of the planes {C, W, S[, SW, SE]} (matrix entries
    C, -W(p), -W(p+e), -S(p), -S(p+n), ...) and u = 0 on the boundary."""
    u = np.array(u, dtype=np.float64)
    u[0, :] = u[-1, :] = 0.0
    u[:, 0] = u[:, -1] = 0.0
    C, W, S = planes[0], planes[1], planes[2]
    I = (slice(1, -1), slice(1, -1))
    Au = (C[I] * u[I] - W[I] * u[1:-1, :-2] - W[1:-1, 2:] * u[1:-1, 2:]
          - S[I] * u[:-2, 1:-1] - S[2:, 1:-1] * u[2:, 1:-1])
    if planes.shape[0] == 5:
        SW, SE = planes[3], planes[4]
        Au -= SW[I] * u[:-2, :-2] + SW[2:, 2:] * u[2:, 2:] + SE[I] * u[:-2, 2:] + SE[2:, :-2] * u[2:, :-2]
    r = np.zeros_like(u)
    r[I] = b[I] - Au
    return r
