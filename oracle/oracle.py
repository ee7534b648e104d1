"""ctypes wrapper around the FP64 CPU oracles (``bmg_oracle.c`` in 2D,
``bmg_oracle3d.c`` in 3D).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the GPU library never does.  It shares no
code with the GPU path.

Arrays are numpy float64, row-major ``[ny][nx]`` over the vertex grid including
the boundary ring, matching the plane format of the library's C interface.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "bmg_oracle.c"), os.path.join(_HERE, "bmg_oracle3d.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force=False):
    """Compile the oracle with gcc (plain IEEE double, no FMA contraction,
    OpenMP for the loops whose points are independent)."""
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]
                              + _SRCS + ["-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        L.oracle_setup.restype = ctypes.c_void_p
        L.oracle_setup.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)]
        L.oracle_free.argtypes = [ctypes.c_void_p]
        L.oracle_num_levels.argtypes = [ctypes.c_void_p]
        L.oracle_num_levels.restype = ctypes.c_int
        L.oracle_level_size.argtypes = [ctypes.c_void_p, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.oracle_get_stencil.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.oracle_get_interp.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.oracle_solve.argtypes = [ctypes.c_void_p, _D, _D, ctypes.c_double, ctypes.c_int, _D]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_smooth.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D, ctypes.c_int]
        L.oracle_residual.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D, _D]
        L.oracle_restrict.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D]
        L.oracle_interp_correct.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D, _D, ctypes.c_int]
        L.oracle_coarse_solve.argtypes = [ctypes.c_void_p, _D, _D]
        L.oracle_vcycle.argtypes = [ctypes.c_void_p, _D, _D]
        L.oracle_fv5.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        L.oracle_grad_logD.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
        L.oracle_fv5_aniso.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, ctypes.c_double,
                                       _D, _D, _D]
        F = ctypes.POINTER(ctypes.c_float)
        L.oracle32_demote.argtypes = [ctypes.c_void_p]
        L.oracle32_get_level.argtypes = [ctypes.c_void_p, ctypes.c_int, F, F]
        L.oracle32_smooth.argtypes = [ctypes.c_void_p, ctypes.c_int, F, F, ctypes.c_int]
        L.oracle32_residual.argtypes = [ctypes.c_void_p, ctypes.c_int, F, F, F]
        L.oracle32_restrict.argtypes = [ctypes.c_void_p, ctypes.c_int, F, F]
        L.oracle32_interp_correct.argtypes = [ctypes.c_void_p, ctypes.c_int, F, F, F, ctypes.c_int]
        L.oracle32_vcycle.argtypes = [ctypes.c_void_p, F, F]
        L.oracle32_inner.argtypes = [ctypes.c_void_p, F, F, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        L.oracle32_inner.restype = ctypes.c_int
        L.oracle_solve_mixed.argtypes = [ctypes.c_void_p, _D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int)]
        L.oracle_solve_mixed.restype = ctypes.c_int
        I = ctypes.c_int
        IP = ctypes.POINTER(ctypes.c_int)
        L.oracle3_fv7.argtypes = [I, I, I, _D, _D, _D, _D, _D]
        L.oracle3_setup.restype = ctypes.c_void_p
        L.oracle3_setup.argtypes = [I, I, I, I, _D, I, I, I, I, IP]
        L.oracle3_free.argtypes = [ctypes.c_void_p]
        L.oracle3_num_levels.argtypes = [ctypes.c_void_p]
        L.oracle3_num_levels.restype = I
        L.oracle3_level_size.argtypes = [ctypes.c_void_p, I, IP, IP, IP]
        L.oracle3_get_stencil.argtypes = [ctypes.c_void_p, I, _D]
        L.oracle3_get_interp.argtypes = [ctypes.c_void_p, I, _D]
        L.oracle3_solve.argtypes = [ctypes.c_void_p, _D, _D, ctypes.c_double, I, _D]
        L.oracle3_solve.restype = I
        L.oracle3_smooth.argtypes = [ctypes.c_void_p, I, _D, _D, I]
        L.oracle3_residual.argtypes = [ctypes.c_void_p, I, _D, _D, _D]
        L.oracle3_restrict.argtypes = [ctypes.c_void_p, I, _D, _D]
        L.oracle3_interp_correct.argtypes = [ctypes.c_void_p, I, _D, _D, _D, I]
        L.oracle3_coarse_solve.argtypes = [ctypes.c_void_p, _D, _D]
        L.oracle3_vcycle.argtypes = [ctypes.c_void_p, _D, _D]
    return _lib


def set_threads(n):
    """Threads of the oracle's parallel loops (results do not depend on it);
    returns the previous count."""
    return lib().oracle_set_threads(int(n))


def _p(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f(a):
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def fv5(cellD):
    """5-point finite-volume planes (C, W, S) from per-cell diffusivity [(ny-1),(nx-1)]."""
    cellD = np.ascontiguousarray(cellD, dtype=np.float64)
    ny, nx = cellD.shape[0] + 1, cellD.shape[1] + 1
    out = np.zeros((3, ny, nx))
    lib().oracle_fv5(nx, ny, _p(cellD), _p(out[0]), _p(out[1]), _p(out[2]))
    return out


def fv5_aniso(Dx, Dy, hx, hy):
    """5-point finite-volume planes (C, W, S) for D = diag(Dx, Dy) per cell
    [(ny-1),(nx-1)] on a grid of spacings hx, hy (section 5)."""
    Dx = np.ascontiguousarray(Dx, dtype=np.float64)
    Dy = np.ascontiguousarray(Dy, dtype=np.float64)
    ny, nx = Dx.shape[0] + 1, Dx.shape[1] + 1
    out = np.zeros((3, ny, nx))
    lib().oracle_fv5_aniso(nx, ny, _p(Dx), _p(Dy), float(hx), float(hy), _p(out[0]), _p(out[1]), _p(out[2]))
    return out


def grad_logD(cellD, u, lam):
    cellD = np.ascontiguousarray(cellD, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    ny, nx = u.shape
    g = np.zeros((ny - 1, nx - 1))
    lib().oracle_grad_logD(nx, ny, _p(cellD), _p(u), _p(lam), _p(g))
    return g


class Hierarchy:
    """Oracle multigrid hierarchy built from the finest stencil planes.

    planes: [3 or 5][ny][nx] = {C, W, S[, SW, SE]} with positive connections.
    Level 0 is the coarsest, level L-1 the finest.
    """

    def __init__(self, planes, coarsest_n=3, nu1=2, nu2=1, rescorr=1):
        planes = np.ascontiguousarray(planes, dtype=np.float64)
        npt = {3: 5, 5: 9}[planes.shape[0]]
        self.ny, self.nx = planes.shape[1:]
        st = ctypes.c_int(0)
        self._h = lib().oracle_setup(self.nx, self.ny, npt, _p(planes), coarsest_n, nu1, nu2,
                                     rescorr, ctypes.byref(st))
        self.status = st.value
        if not self._h:
            raise ValueError("oracle_setup rejected the arguments (status %d)" % st.value)
        self.L = lib().oracle_num_levels(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().oracle_free(self._h)
            self._h = None

    def size(self, l):
        a, b = ctypes.c_int(), ctypes.c_int()
        lib().oracle_level_size(self._h, l, ctypes.byref(a), ctypes.byref(b))
        return b.value, a.value  # (ny, nx)

    def stencil(self, l):
        """[ny][nx][3][3] matrix entries A(p, p + (dx, dy)) at [.., dy+1, dx+1]."""
        ny, nx = self.size(l)
        out = np.zeros((ny, nx, 9))
        lib().oracle_get_stencil(self._h, l, _p(out))
        return out.reshape(ny, nx, 3, 3)

    def interp(self, l):
        """[ny][nx][2][2] interpolation rows of level l onto corners of level l-1,
        weight on coarse vertex ((i>>1)+a, (j>>1)+b) at [.., b, a]."""
        ny, nx = self.size(l)
        out = np.zeros((ny, nx, 4))
        lib().oracle_get_interp(self._h, l, _p(out))
        return out.reshape(ny, nx, 2, 2)

    def solve(self, b, u0=None, tol=1e-10, max_cycles=500):
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.zeros_like(b) if u0 is None else np.array(u0, dtype=np.float64, order="C")
        hist = np.zeros(max_cycles)
        n = lib().oracle_solve(self._h, _p(b), _p(u), tol, max_cycles, _p(hist))
        return u, hist[:n]

    def vcycle(self, b, u):
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.array(u, dtype=np.float64, order="C")
        lib().oracle_vcycle(self._h, _p(b), _p(u))
        return u

    def smooth(self, l, b, x, sweeps=1):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x, dtype=np.float64, order="C")
        lib().oracle_smooth(self._h, l, _p(b), _p(x), sweeps)
        return x

    def residual(self, l, b, x):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        r = np.zeros_like(b)
        lib().oracle_residual(self._h, l, _p(b), _p(x), _p(r))
        return r

    def restrict(self, l, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        bc = np.zeros(self.size(l - 1))
        lib().oracle_restrict(self._h, l, _p(r), _p(bc))
        return bc

    def interp_correct(self, l, x, r, xc, rescorr=1):
        x = np.array(x, dtype=np.float64, order="C")
        r = np.ascontiguousarray(r, dtype=np.float64)
        xc = np.ascontiguousarray(xc, dtype=np.float64)
        lib().oracle_interp_correct(self._h, l, _p(x), _p(r), _p(xc), rescorr)
        return x

    def coarse_solve(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        lib().oracle_coarse_solve(self._h, _p(b), _p(x))
        return x

    # ---- FP32 edge form (inner solver of mixed precision) ----------------
    def demote(self):
        """Build the FP32 edge-form copy of every level (once per hierarchy)."""
        if not getattr(self, "_has32", False):
            lib().oracle32_demote(self._h)
            self._has32 = True

    def level32(self, l):
        """FP32 edge form of level l: ([ny][nx][3][3] with the connections
        -A(p, p+d) off the centre and the excess at the centre, [ny][nx][2][2]
        interpolation rows), both float32."""
        self.demote()
        ny, nx = self.size(l)
        A = np.zeros((ny, nx, 9), np.float32)
        P = np.zeros((ny, nx, 4), np.float32)
        lib().oracle32_get_level(self._h, l, _f(A), _f(P))
        return A.reshape(ny, nx, 3, 3), P.reshape(ny, nx, 2, 2)

    def smooth32(self, l, b, x, sweeps=1):
        self.demote()
        b = np.ascontiguousarray(b, dtype=np.float32)
        x = np.array(x, dtype=np.float32, order="C")
        lib().oracle32_smooth(self._h, l, _f(b), _f(x), sweeps)
        return x

    def residual32(self, l, b, x):
        self.demote()
        b = np.ascontiguousarray(b, dtype=np.float32)
        x = np.ascontiguousarray(x, dtype=np.float32)
        r = np.zeros_like(b)
        lib().oracle32_residual(self._h, l, _f(b), _f(x), _f(r))
        return r

    def restrict32(self, l, r):
        self.demote()
        r = np.ascontiguousarray(r, dtype=np.float32)
        bc = np.zeros(self.size(l - 1), np.float32)
        lib().oracle32_restrict(self._h, l, _f(r), _f(bc))
        return bc

    def interp_correct32(self, l, x, r, xc, rescorr=1):
        self.demote()
        x = np.array(x, dtype=np.float32, order="C")
        r = np.ascontiguousarray(r, dtype=np.float32)
        xc = np.ascontiguousarray(xc, dtype=np.float32)
        lib().oracle32_interp_correct(self._h, l, _f(x), _f(r), _f(xc), rescorr)
        return x

    def vcycle32(self, b, x):
        self.demote()
        b = np.ascontiguousarray(b, dtype=np.float32)
        x = np.array(x, dtype=np.float32, order="C")
        lib().oracle32_vcycle(self._h, _f(b), _f(x))
        return x

    def inner32(self, r, cycles, rnorm, inner_tol=0.0):
        """One refinement step's inner solve of A e = r from e = 0: returns
        (e, inner relative residual after each cycle)."""
        self.demote()
        r = np.ascontiguousarray(r, dtype=np.float32)
        e = np.zeros_like(r)
        hist = np.zeros(max(cycles, 1))
        k = lib().oracle32_inner(self._h, _f(r), _f(e), cycles, float(rnorm), float(inner_tol), _p(hist))
        return e, hist[:k]

    def solve_mixed(self, b, u0=None, tol=1e-10, max_cycles=500, inner_max=32, inner_tol=1e-4, adapt=True):
        """FP64 iterative refinement around FP32 inner solves: returns
        (u, outer relative residual before each step and at the end, FP32
        cycles run, inner solves).  Each inner solve stops at inner_tol or,
        with adapt, already at tol / (2 outer relres) when that is looser."""
        self.demote()
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.zeros_like(b) if u0 is None else np.array(u0, dtype=np.float64, order="C")
        hist = np.zeros(max_cycles + 2)
        steps = ctypes.c_int(0)
        cyc = lib().oracle_solve_mixed(self._h, _p(b), _p(u), tol, max_cycles, inner_max, inner_tol,
                                       1 if adapt else 0, _p(hist), ctypes.byref(steps))
        return u, hist[:steps.value + 1], cyc, steps.value


# --------------------------------------------------------------------------
# 3D
# --------------------------------------------------------------------------

def fv7(cellD):
    """7-point finite-volume planes (C, W, S, B) [4][nz][ny][nx] from per-cell
    diffusivity [(nz-1)][(ny-1)][(nx-1)]."""
    cellD = np.ascontiguousarray(cellD, dtype=np.float64)
    nz, ny, nx = cellD.shape[0] + 1, cellD.shape[1] + 1, cellD.shape[2] + 1
    out = np.zeros((4, nz, ny, nx))
    lib().oracle3_fv7(nx, ny, nz, _p(cellD), _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3]))
    return out


class Hierarchy3:
    """3D oracle hierarchy built from the finest stencil planes.

    planes: [4][nz][ny][nx] = {C, W, S, B} (7-point), or [14][nz][ny][nx] =
    {C, then -A(p, p+d) for the 13 lower-half offsets d in linear order
    (dz+1)*9+(dy+1)*3+(dx+1) = 0..12} (27-point).  Level 0 is the coarsest.
    """

    def __init__(self, planes, coarsest_n=3, nu1=2, nu2=1, rescorr=1):
        planes = np.ascontiguousarray(planes, dtype=np.float64)
        npt = {4: 7, 14: 27}[planes.shape[0]]
        self.nz, self.ny, self.nx = planes.shape[1:]
        st = ctypes.c_int(0)
        self._h = lib().oracle3_setup(self.nx, self.ny, self.nz, npt, _p(planes), coarsest_n, nu1, nu2,
                                      rescorr, ctypes.byref(st))
        self.status = st.value
        if not self._h:
            raise ValueError("oracle3_setup rejected the arguments (status %d)" % st.value)
        self.L = lib().oracle3_num_levels(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().oracle3_free(self._h)
            self._h = None

    def size(self, l):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lib().oracle3_level_size(self._h, l, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return c.value, b.value, a.value  # (nz, ny, nx)

    def stencil(self, l):
        """[nz][ny][nx][3][3][3] matrix entries A(p, p + d) at [.., dz+1, dy+1, dx+1]."""
        nz, ny, nx = self.size(l)
        out = np.zeros((nz, ny, nx, 27))
        lib().oracle3_get_stencil(self._h, l, _p(out))
        return out.reshape(nz, ny, nx, 3, 3, 3)

    def interp(self, l):
        """[nz][ny][nx][2][2][2] interpolation rows of level l, weight on coarse
        vertex ((i>>1)+a, (j>>1)+b, (k>>1)+c) at [.., c, b, a]."""
        nz, ny, nx = self.size(l)
        out = np.zeros((nz, ny, nx, 8))
        lib().oracle3_get_interp(self._h, l, _p(out))
        return out.reshape(nz, ny, nx, 2, 2, 2)

    def solve(self, b, u0=None, tol=1e-10, max_cycles=500):
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.zeros_like(b) if u0 is None else np.array(u0, dtype=np.float64, order="C")
        hist = np.zeros(max_cycles)
        n = lib().oracle3_solve(self._h, _p(b), _p(u), tol, max_cycles, _p(hist))
        return u, hist[:n]

    def vcycle(self, b, u):
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.array(u, dtype=np.float64, order="C")
        lib().oracle3_vcycle(self._h, _p(b), _p(u))
        return u

    def smooth(self, l, b, x, sweeps=1):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x, dtype=np.float64, order="C")
        lib().oracle3_smooth(self._h, l, _p(b), _p(x), sweeps)
        return x

    def residual(self, l, b, x):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        r = np.zeros_like(b)
        lib().oracle3_residual(self._h, l, _p(b), _p(x), _p(r))
        return r

    def restrict(self, l, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        bc = np.zeros(self.size(l - 1))
        lib().oracle3_restrict(self._h, l, _p(r), _p(bc))
        return bc

    def interp_correct(self, l, x, r, xc, rescorr=1):
        x = np.array(x, dtype=np.float64, order="C")
        r = np.ascontiguousarray(r, dtype=np.float64)
        xc = np.ascontiguousarray(xc, dtype=np.float64)
        lib().oracle3_interp_correct(self._h, l, _p(x), _p(r), _p(xc), rescorr)
        return x

    def coarse_solve(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        lib().oracle3_coarse_solve(self._h, _p(b), _p(x))
        return x
