"""Thin Python binding of the hipbmg C interface (include/hipbmg.h).

Argument marshalling only: every step of setup and solve runs in the HIP
library ``libhipbmg.so`` built in-tree for gfx950.  torch supplies device
memory (tensor data pointers, and through hipbmg_set_allocator the handles'
own memory from its caching allocator, registered when the library is
loaded) and the current stream.  Loading fails loudly if the library is
missing; there is no fallback.
"""
import atexit
import ctypes
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhipbmg.so")
_lib = None

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, ENOCONV, ENAN = range(7)
FP64, MIXED = 0, 1
MAX_LEVELS = 24
MAX_HIST = 1024


class Params(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("coarsest_n", ctypes.c_int),
                ("collapse_level", ctypes.c_int), ("residual_correction", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_max_cycles", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("use_graph", ctypes.c_int), ("cluster_wg", ctypes.c_int), ("cluster_top", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("outer_steps", ctypes.c_int), ("relres", ctypes.c_double),
                ("levels", ctypes.c_int), ("collapse_level", ctypes.c_int),
                ("model_us", ctypes.c_double * MAX_LEVELS), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("relres_hist", ctypes.c_double * MAX_HIST),
                ("rb_down", ctypes.c_int * MAX_LEVELS), ("rb_up", ctypes.c_int * MAX_LEVELS),
                ("rb_pipelined", ctypes.c_int), ("cluster_stages", ctypes.c_int),
                ("cluster_wg", ctypes.c_int * 4), ("cluster_hi", ctypes.c_int * 4),
                ("search_us", ctypes.c_double), ("search_expanded", ctypes.c_int),
                ("path_us", ctypes.c_double)]

    def history(self):
        n = self.outer_steps if self.outer_steps else self.cycles
        return list(self.relres_hist[: min(n, MAX_HIST)])


class HipBMGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("hipbmg status %d: %s" % (status, msg))
        self.status = status


_VP = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "hipbmg_default_params": (None, [ctypes.POINTER(Params)]),
    "hipbmg_setup": (_I, [_I, _I, _I, _VP, ctypes.POINTER(Params), _VP, ctypes.POINTER(_VP)]),
    "hipbmg_solve": (_I, [_VP, _VP, _VP, ctypes.c_double, _VP, ctypes.POINTER(Info)]),
    "hipbmg_destroy": (_I, [_VP]),
    "hipbmg_level_size": (_I, [_VP, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "hipbmg_get_stencil": (_I, [_VP, _I, _VP, _VP]),
    "hipbmg_get_interp": (_I, [_VP, _I, _VP, _VP]),
    "hipbmg_op_smooth": (_I, [_VP, _I, _VP, _VP, _I, _VP]),
    "hipbmg_op_smooth_restrict": (_I, [_VP, _I, _VP, _VP, _I, _VP, _VP, _VP]),
    "hipbmg_op_interp_smooth": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _I, ctypes.POINTER(ctypes.c_double), _VP]),
    "hipbmg_get_level32": (_I, [_VP, _I, _VP, _VP, _VP]),
    "hipbmg_op32_smooth": (_I, [_VP, _I, _VP, _VP, _I, _VP]),
    "hipbmg_op32_smooth_restrict": (_I, [_VP, _I, _VP, _VP, _I, _VP, _VP, _VP]),
    "hipbmg_op32_interp_smooth": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _I, ctypes.POINTER(ctypes.c_double), _VP]),
    "hipbmg_op32_inner": (_I, [_VP, _VP, _VP, _I, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(_I), _VP]),
    "hipbmg_fv5_from_cells": (_I, [_I, _I, _VP, _I, _VP, _VP]),
    "hipbmg_residual_norm": (_I, [_I, _I, _I, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "hipbmg_residual_norm_noalloc": (_I, [_I, _I, _I, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "hipbmg_fv5_aniso": (_I, [_I, _I, _VP, _VP, ctypes.c_double, ctypes.c_double, _VP, _VP]),
    "hipbmg_grad_logD": (_I, [_I, _I, _VP, _VP, _VP, _VP, _VP]),
    "hipbmg_fv5_from_cells_batched": (_I, [_I, _I, _I, _VP, _I, _VP, _VP]),
    "hipbmg_grad_logD_batched": (_I, [_I, _I, _I, _VP, _VP, _VP, _VP, _VP]),
    "hipbmg_profile": (_I, [_VP, _I]),
    "hipbmg_profile_read": (_I, [_VP, _I, _I, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]),
    "hipbmg_profile_levels": (_I, [_VP, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
    "hipbmg_model_levels": (_I, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]),
    "hipbmg_calibrate": (_I, [_VP, ctypes.POINTER(ctypes.c_double)]),
    "hipbmg_setup_batched": (_I, [_I, ctypes.POINTER(_I), ctypes.POINTER(_I), _I, ctypes.POINTER(_VP),
                                  ctypes.POINTER(Params), _VP, ctypes.POINTER(_VP)]),
    "hipbmg_solve_batched": (_I, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.c_double, _VP,
                                  ctypes.POINTER(Info)]),
    "hipbmg_destroy_batched": (_I, [_VP]),
    "hipbmg_batch_tile_shape": (_I, [_VP, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "hipbmg_set_allocator": (_I, [_VP, _VP, _VP]),
    "hipbmg_last_error": (ctypes.c_char_p, []),
    "hipbmg_paper_model": (_I, [_I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), _I, _I, _I, _I, _I,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]),
    "hipbmg_paper_enumerate": (_I, [_I, ctypes.POINTER(_I), ctypes.POINTER(_I), _I, ctypes.POINTER(_I),
                                    ctypes.POINTER(_I)]),
    "hipbmg_paper_search": (_I, [ctypes.c_void_p, ctypes.POINTER(_I), ctypes.POINTER(_I), _I,
                                 ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double)]),
    "hipbmg_paper_astar": (_I, [ctypes.c_void_p, ctypes.POINTER(_I), ctypes.POINTER(_I), _I,
                                ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(_I)]),
    "hipbmg_paper_path_cost": (_I, [ctypes.c_void_p, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                    ctypes.POINTER(_I), _I, ctypes.POINTER(ctypes.c_double)]),
    # 3D path (include/hipbmg3d.h)
    "hipbmg3d_fv7_from_cells": (_I, [_I, _I, _I, _VP, _VP, _VP]),
    "hipbmg3d_setup": (_I, [_I, _I, _I, _I, _VP, ctypes.POINTER(Params), _VP, ctypes.POINTER(_VP)]),
    "hipbmg3d_solve": (_I, [_VP, _VP, _VP, ctypes.c_double, _VP, ctypes.POINTER(Info)]),
    "hipbmg3d_destroy": (_I, [_VP]),
    "hipbmg3d_num_levels": (_I, [_VP, ctypes.POINTER(_I)]),
    "hipbmg3d_level_size": (_I, [_VP, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "hipbmg3d_get_stencil": (_I, [_VP, _I, _VP, _VP]),
    "hipbmg3d_get_interp": (_I, [_VP, _I, _VP, _VP]),
    "hipbmg3d_op_smooth": (_I, [_VP, _I, _VP, _VP, _I, _VP]),
    "hipbmg3d_op_residual": (_I, [_VP, _I, _VP, _VP, _VP, _VP]),
    "hipbmg3d_op_restrict": (_I, [_VP, _I, _VP, _VP, _VP]),
    "hipbmg3d_op_interp_correct": (_I, [_VP, _I, _VP, _VP, _VP, _I, _VP]),
    "hipbmg3d_op_coarse_solve": (_I, [_VP, _VP, _VP, _VP]),
    "hipbmg3d_profile": (_I, [_VP, _I]),
    "hipbmg3d_profile_read": (_I, [_VP, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(ctypes.c_double)]),
}

# hipbmg_alloc_fn / hipbmg_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator = None   # the registered callbacks, kept alive while registered
_open_handles = weakref.WeakSet()
_atexit_registered = False


def _close_open_handles():
    # handles whose memory came from a Python allocator call back into Python
    # when they are destroyed: do it at exit, before the interpreter tears down
    for h in list(_open_handles):
        try:
            h.close()
        except Exception:
            pass


def lib():
    """Load libhipbmg.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhipbmg.so is not built (run python -m paper_1803_02481_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        # handle memory from torch's caching allocator: hierarchies rebuilt
        # every step (the adjoint's setups) then reuse pooled blocks instead
        # of paying hipMalloc and a synchronising hipFree per block
        use_torch_allocator()
    return _lib


def set_allocator(alloc=None, free=None):
    """Register Python callables as the library's device allocator for handle
    memory: alloc(nbytes) -> device address (int, 256-byte aligned; 0 or an
    exception on failure), free(address).  No arguments restores hipMalloc.
    Blocks are returned to the allocator that made them when their handle is
    closed, so keep the callables valid until then."""
    global _allocator, _atexit_registered
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        _check(lib().hipbmg_set_allocator(None, None, None))
        return

    def _a(nbytes, ctx):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:
            return None

    def _f(ptr, ctx):
        try:
            free(int(ptr))
        except Exception:
            pass

    if not _atexit_registered:
        atexit.register(_close_open_handles)
        _atexit_registered = True
    cbs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(lib().hipbmg_set_allocator(ctypes.cast(cbs[0], ctypes.c_void_p), ctypes.cast(cbs[1], ctypes.c_void_p),
                                      None))
    # earlier callbacks may still own blocks of open handles: keep them all alive
    _allocator = (cbs, _allocator)


def use_torch_allocator():
    """Take handle memory from PyTorch's caching allocator, on the device that
    is current when the library allocates, so that it is pooled with the
    caller's tensors.  This is the binding's default; set_allocator() with no
    arguments returns to hipMalloc."""

    def alloc(nbytes):
        return torch.cuda.caching_allocator_alloc(nbytes, device=torch.cuda.current_device())

    set_allocator(alloc, torch.cuda.caching_allocator_delete)


def _check(status):
    if status != OK:
        raise HipBMGError(status, lib().hipbmg_last_error().decode())


def _ptr(t, dtype=torch.float64, shape=None, name="array"):
    """Device pointer of a contiguous CUDA tensor, checked against the dtype and
    shape the library will read or write through it (the C interface takes
    bare pointers and sizes, so a mismatch here would be an out-of-bounds
    access there)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s: expected a CUDA tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s: expected a contiguous %s tensor" % (name, dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s: expected shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_params(**kw):
    p = Params()
    lib().hipbmg_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Hierarchy:
    """Multigrid hierarchy on the GPU (hipbmg_setup / hipbmg_solve)."""

    def __init__(self, coeffs, **params):
        if coeffs.dim() != 3 or coeffs.shape[0] not in (3, 5):
            raise ValueError("coeffs must be [3 or 5][ny][nx]")
        self.npt = 5 if coeffs.shape[0] == 3 else 9
        self.ny, self.nx = int(coeffs.shape[1]), int(coeffs.shape[2])
        self.params = default_params(**params)
        self.device = coeffs.device
        h = ctypes.c_void_p()
        _check(lib().hipbmg_setup(self.nx, self.ny, self.npt, _ptr(coeffs, name="coeffs"), ctypes.byref(self.params),
                                  _stream(), ctypes.byref(h)))
        self._h = h
        _open_handles.add(self)
        self.L = self._levels()

    def _levels(self):
        L = 0
        while lib().hipbmg_level_size(self._h, L, None, None) == OK:
            L += 1
        return L

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().hipbmg_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self, l):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().hipbmg_level_size(self._h, l, ctypes.byref(a), ctypes.byref(b)))
        return b.value, a.value   # (ny, nx)

    def solve(self, b, u=None, tol=1e-10, check=True):
        """Returns (u, info).  u is updated in place if given."""
        if u is None:
            u = torch.zeros_like(b)
        shp = (self.ny, self.nx)
        info = Info()
        st = lib().hipbmg_solve(self._h, _ptr(b, shape=shp, name="b"), _ptr(u, shape=shp, name="u"), tol, _stream(),
                                ctypes.byref(info))
        if check and st != OK:
            _check(st)
        info.status = st
        return u, info

    def stencil(self, l):
        ny, nx = self.size(l)
        out = torch.zeros((5, ny, nx), dtype=torch.float64, device=self.device)
        _check(lib().hipbmg_get_stencil(self._h, l, _ptr(out), _stream()))
        return out

    def interp(self, l):
        cny, cnx = self.size(l - 1)
        out = torch.zeros((8, cny, cnx), dtype=torch.float64, device=self.device)
        _check(lib().hipbmg_get_interp(self._h, l, _ptr(out), _stream()))
        return out

    def profile(self, enable=True, levels=False):
        """Record finest-level kernel times (levels=True: every level's legs
        and the collapse launch too)."""
        _check(lib().hipbmg_profile(self._h, (2 if levels else 1) if enable else 0))

    def profile_levels(self, precision=0):
        """[(down_ms, up_ms, collapse_ms, launches down/up/collapse)] per level."""
        ms = (ctypes.c_double * (3 * MAX_LEVELS))()
        n = (ctypes.c_longlong * (3 * MAX_LEVELS))()
        _check(lib().hipbmg_profile_levels(self._h, precision, ms, n))
        return [(ms[3 * l], ms[3 * l + 1], ms[3 * l + 2], n[3 * l], n[3 * l + 1], n[3 * l + 2])
                for l in range(self.L)]

    def model_levels(self):
        """The model's terms (us per V-cycle): grid-wide kernels and collapsed
        form of every level, and the collapsed launch holding the coarsest."""
        grid = (ctypes.c_double * MAX_LEVELS)()
        wg = (ctypes.c_double * MAX_LEVELS)()
        base = (ctypes.c_double * 1)()
        _check(lib().hipbmg_model_levels(self._h, grid, wg, base))
        return {"grid_us": list(grid)[: self.L], "collapsed_us": list(wg)[: self.L], "base_us": base[0]}

    KERNELS = ("relax", "relax_zero", "relax_restrict", "relax_restrict_zero", "interp_relax",
               "interp_relax_norm", "relax_norm", "relax2_restrict", "relax2_restrict_zero", "fused3",
               "fused3_rebuild", "relax2_restrict_noq", "relax2_restrict_noq_zero", "interp_rc_relax",
               "fused3_last")

    def profile_read(self, precision=0):
        """{kernel name: (total_ms, launches, bytes_per_launch)} for launched kernels."""
        out = {}
        for k, name in enumerate(self.KERNELS):
            ms, n, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
            _check(lib().hipbmg_profile_read(self._h, precision, k, ctypes.byref(ms), ctypes.byref(n),
                                             ctypes.byref(by)))
            if n.value:
                out[name] = (ms.value, n.value, by.value)
        return out

    def _fields(self, l, dtype, **arrays):
        """Pointers of level-l fields (coarse=True entries: level l-1), shapes checked."""
        if not 0 <= l < self.L:
            raise ValueError("level %d out of range [0, %d)" % (l, self.L))
        out = []
        for name, (t, coarse) in arrays.items():
            if coarse and l < 1:
                raise ValueError("level 0 has no coarser level")
            out.append(_ptr(t, dtype, self.size(l - 1 if coarse else l), name))
        return out

    def op_smooth(self, l, b, x, sweeps=1):
        x = x.clone()
        pb, px = self._fields(l, torch.float64, b=(b, False), x=(x, False))
        _check(lib().hipbmg_op_smooth(self._h, l, pb, px, sweeps, _stream()))
        return x

    def op_smooth_restrict(self, l, b, x, sweeps=1):
        x = x.clone()
        q = torch.zeros_like(x)
        cny, cnx = self.size(l - 1)
        bc = torch.zeros((cny, cnx), dtype=torch.float64, device=x.device)
        pb, px, pq, pc = self._fields(l, torch.float64, b=(b, False), x=(x, False), q=(q, False), bc=(bc, True))
        _check(lib().hipbmg_op_smooth_restrict(self._h, l, pb, px, sweeps, pq, pc, _stream()))
        return x, q, bc

    def op_interp_smooth(self, l, b, x, q, xc, rescorr=1, want_norm=False):
        x = x.clone()
        ss = ctypes.c_double(0.0)
        pb, px, pq, pc = self._fields(l, torch.float64, b=(b, False), x=(x, False), q=(q, False), xc=(xc, True))
        _check(lib().hipbmg_op_interp_smooth(self._h, l, pb, px, pq, pc, rescorr,
                                             ctypes.byref(ss) if want_norm else None, _stream()))
        return (x, ss.value) if want_norm else x

    # ---- FP32 edge-form levels (mixed-precision handles) -----------------
    def level32(self, l):
        """(planes [5][ny][nx] = {E, W, S, SW, SE}, weights [8][cny][cnx] or None
        on level 0), float32."""
        if not 0 <= l < self.L:
            raise ValueError("level %d out of range [0, %d)" % (l, self.L))
        ny, nx = self.size(l)
        st = torch.zeros((5, ny, nx), dtype=torch.float32, device=self.device)
        wt = None
        if l >= 1:
            cny, cnx = self.size(l - 1)
            wt = torch.zeros((8, cny, cnx), dtype=torch.float32, device=self.device)
        _check(lib().hipbmg_get_level32(self._h, l, _ptr(st, torch.float32),
                                        _ptr(wt, torch.float32) if wt is not None else None, _stream()))
        return st, wt

    def op32_smooth(self, l, b, x, sweeps=1):
        x = x.clone()
        pb, px = self._fields(l, torch.float32, b=(b, False), x=(x, False))
        _check(lib().hipbmg_op32_smooth(self._h, l, pb, px, sweeps, _stream()))
        return x

    def op32_smooth_restrict(self, l, b, x, sweeps=1):
        x = x.clone()
        q = torch.zeros_like(x)
        cny, cnx = self.size(l - 1)
        bc = torch.zeros((cny, cnx), dtype=torch.float32, device=x.device)
        pb, px, pq, pc = self._fields(l, torch.float32, b=(b, False), x=(x, False), q=(q, False), bc=(bc, True))
        _check(lib().hipbmg_op32_smooth_restrict(self._h, l, pb, px, sweeps, pq, pc, _stream()))
        return x, q, bc

    def op32_interp_smooth(self, l, b, x, q, xc, rescorr=1, want_norm=False):
        x = x.clone()
        ss = ctypes.c_double(0.0)
        pb, px, pq, pc = self._fields(l, torch.float32, b=(b, False), x=(x, False), q=(q, False), xc=(xc, True))
        _check(lib().hipbmg_op32_interp_smooth(self._h, l, pb, px, pq, pc, rescorr,
                                               ctypes.byref(ss) if want_norm else None, _stream()))
        return (x, ss.value) if want_norm else x

    def op32_inner(self, r, cycles, rnorm, inner_tol=0.0):
        """The inner FP32 solve of one refinement step, A e = r from e = 0:
        (e, inner relative residual after each cycle)."""
        e = torch.zeros_like(r)
        pr, pe = self._fields(self.L - 1, torch.float32, r=(r, False), e=(e, False))
        hist = (ctypes.c_double * max(1, int(cycles)))()
        done = ctypes.c_int(0)
        _check(lib().hipbmg_op32_inner(self._h, pr, pe, int(cycles), float(rnorm), float(inner_tol), hist,
                                       ctypes.byref(done), _stream()))
        return e, list(hist)[: done.value]


class BatchHierarchy:
    """Many independent problems of different sizes solved together
    (hipbmg_setup_batched / hipbmg_solve_batched)."""

    def __init__(self, coeffs_list, **params):
        n = len(coeffs_list)
        if n == 0:
            raise ValueError("empty batch")
        for k, c in enumerate(coeffs_list):
            if c.dim() != 3 or c.shape[0] not in (3, 5):
                raise ValueError("coeffs_list[%d] must be [3 or 5][ny][nx]" % k)
            if c.shape[0] != coeffs_list[0].shape[0]:
                raise ValueError("every problem of a batch needs the same stencil (plane count)")
        npt = 5 if coeffs_list[0].shape[0] == 3 else 9
        self.shapes = [(int(c.shape[1]), int(c.shape[2])) for c in coeffs_list]
        nx = (_I * n)(*[s[1] for s in self.shapes])
        ny = (_I * n)(*[s[0] for s in self.shapes])
        ptrs = (_VP * n)(*[_ptr(c, name="coeffs_list[%d]" % k).value for k, c in enumerate(coeffs_list)])
        self.params = default_params(**params)
        h = ctypes.c_void_p()
        _check(lib().hipbmg_setup_batched(n, nx, ny, npt, ptrs, ctypes.byref(self.params), _stream(),
                                          ctypes.byref(h)))
        self._h = h
        _open_handles.add(self)
        self.n = n

    def tile_shape(self, problem, level):
        """(strips per workgroup, row-block cap, row-pair steps per tile of
        this level) chosen by the autotuner (hipbmg_batch_tile_shape)."""
        w, cap, rb = _I(), _I(), _I()
        _check(lib().hipbmg_batch_tile_shape(self._h, int(problem), int(level), ctypes.byref(w), ctypes.byref(cap),
                                             ctypes.byref(rb)))
        return w.value, cap.value, rb.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().hipbmg_destroy_batched(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b_list, u_list=None, tol=1e-10, check=True):
        if u_list is None:
            u_list = [torch.zeros_like(b) for b in b_list]
        n = self.n
        if len(b_list) != n or len(u_list) != n:
            raise ValueError("the batch has %d problems: got %d right-hand sides, %d iterates"
                             % (n, len(b_list), len(u_list)))
        bp = (_VP * n)(*[_ptr(b, shape=self.shapes[k], name="b_list[%d]" % k).value for k, b in enumerate(b_list)])
        up = (_VP * n)(*[_ptr(u, shape=self.shapes[k], name="u_list[%d]" % k).value for k, u in enumerate(u_list)])
        infos = (Info * n)()
        st = lib().hipbmg_solve_batched(self._h, bp, up, tol, _stream(), infos)
        if check and st != OK:
            _check(st)
        self.status = st
        return u_list, list(infos)


def calibrate():
    """Measure the performance-model parameters on the current device; later
    hierarchies choose their collapse level with them."""
    out = (ctypes.c_double * 64)()
    _check(lib().hipbmg_calibrate(_stream(), out))
    return {k: out[i] for i, k in enumerate(CALIBRATION_KEYS)}


CALIBRATION_KEYS = ("alpha_launch_us", "hbm_GBps", "cache_GBps",
                    "step_dn_us_fp64", "step_up_us_fp64", "step_dn_us_fp32", "step_up_us_fp32",
                    "t_base_us_fp64", "t_base_us_fp32",
                    "alpha_bar_us_fp64_lds", "alpha_bar_us_fp64_global",
                    "alpha_bar_us_fp32_lds", "alpha_bar_us_fp32_global",
                    "wg_GBps_fp64_lds", "wg_GBps_fp64_global", "wg_GBps_fp32_lds", "wg_GBps_fp32_global",
                    "bare_barrier_lds_us", "bare_barrier_l2_us", "bare_wg_l2_GBps", "plain_sweep_step_us",
                    "t0_dn_us_fp64", "t0_up_us_fp64", "t0_dn_us_fp32", "t0_up_us_fp32") + tuple(
    "%s_%dwg_%s" % (what, 2 << k, prec) for prec in ("fp64", "fp32") for what in ("alpha_stage_us", "stage_GBps")
    for k in range(8))


def residual_norm(coeffs, b, u, noalloc=False):
    """(||b - A u||_2, ||b||_2) over interior vertices for the operator of the
    stencil planes coeffs ([3 or 5][ny][nx]).  noalloc: the entry point that
    allocates no device memory (hipbmg_residual_norm_noalloc)."""
    if coeffs.dim() != 3 or coeffs.shape[0] not in (3, 5):
        raise ValueError("coeffs must be [3 or 5][ny][nx]")
    ny, nx = int(coeffs.shape[1]), int(coeffs.shape[2])
    out = (ctypes.c_double * 2)()
    fn = lib().hipbmg_residual_norm_noalloc if noalloc else lib().hipbmg_residual_norm
    _check(fn(nx, ny, 5 if coeffs.shape[0] == 3 else 9, _ptr(coeffs, name="coeffs"),
              _ptr(b, shape=(ny, nx), name="b"), _ptr(u, shape=(ny, nx), name="u"), out, _stream()))
    return out[0], out[1]


def fv5_from_cells(cell, is_log=False):
    """5-point finite-volume planes {C, W, S} ([3][ny][nx]) from per-cell D or ln D."""
    if cell.dim() != 2:
        raise ValueError("cell must be [ny-1][nx-1]")
    ny, nx = cell.shape[0] + 1, cell.shape[1] + 1
    out = torch.empty((3, ny, nx), dtype=torch.float64, device=cell.device)
    _check(lib().hipbmg_fv5_from_cells(nx, ny, _ptr(cell), 1 if is_log else 0, _ptr(out), _stream()))
    return out


def fv5_from_cells_batched(cells, is_log=False):
    """fv5_from_cells for a batch of one size in one launch: cells [B][ny-1][nx-1]
    -> planes [B][3][ny][nx]."""
    if cells.dim() != 3 or cells.shape[0] < 1:
        raise ValueError("cells must be [B][ny-1][nx-1]")
    nb, ny, nx = cells.shape[0], cells.shape[1] + 1, cells.shape[2] + 1
    out = torch.empty((nb, 3, ny, nx), dtype=torch.float64, device=cells.device)
    _check(lib().hipbmg_fv5_from_cells_batched(nb, nx, ny, _ptr(cells, name="cells"), 1 if is_log else 0,
                                               _ptr(out), _stream()))
    return out


def fv5_aniso(dx_cell, dy_cell, hx, hy):
    """5-point finite-volume planes {C, W, S} for D = diag(Dx, Dy) per cell on a
    grid of spacings hx, hy (the stretched grids of section 5)."""
    if dx_cell.dim() != 2:
        raise ValueError("dx_cell must be [ny-1][nx-1]")
    ny, nx = dx_cell.shape[0] + 1, dx_cell.shape[1] + 1
    if tuple(dy_cell.shape) != tuple(dx_cell.shape):
        raise ValueError("dx_cell and dy_cell must have the same shape")
    out = torch.empty((3, ny, nx), dtype=torch.float64, device=dx_cell.device)
    _check(lib().hipbmg_fv5_aniso(nx, ny, _ptr(dx_cell), _ptr(dy_cell), float(hx), float(hy), _ptr(out),
                                  _stream()))
    return out


def grad_logD(theta, u, lam):
    """dL/dtheta per cell ([ny-1][nx-1]) from the solution u and the adjoint lam ([ny][nx])."""
    if u.dim() != 2:
        raise ValueError("u must be [ny][nx]")
    ny, nx = u.shape
    g = torch.empty_like(theta)
    _check(lib().hipbmg_grad_logD(nx, ny, _ptr(theta, shape=(ny - 1, nx - 1), name="theta"),
                                  _ptr(u, name="u"), _ptr(lam, shape=(ny, nx), name="lam"),
                                  _ptr(g, shape=(ny - 1, nx - 1), name="grad"), _stream()))
    return g


def grad_logD_batched(theta, u, lam):
    """grad_logD for a batch of one size in one launch: theta [B][ny-1][nx-1],
    u and lam [B][ny][nx] -> [B][ny-1][nx-1]."""
    if u.dim() != 3 or u.shape[0] < 1:
        raise ValueError("u must be [B][ny][nx]")
    nb, ny, nx = u.shape
    g = torch.empty((nb, ny - 1, nx - 1), dtype=torch.float64, device=u.device)
    _check(lib().hipbmg_grad_logD_batched(nb, nx, ny, _ptr(theta, shape=(nb, ny - 1, nx - 1), name="theta"),
                                          _ptr(u, name="u"), _ptr(lam, shape=(nb, ny, nx), name="lam"),
                                          _ptr(g), _stream()))
    return g


class SolveFV(torch.autograd.Function):
    """u = A(theta)^{-1} b with A the 5-point finite-volume operator of
    -div(exp(theta) grad u) and zero Dirichlet data.  Backward: one adjoint
    solve with the same hierarchy (A is symmetric) and the per-cell gradient
    kernel."""

    @staticmethod
    def forward(ctx, theta, b, tol=1e-10, params=None):
        if theta.dim() != 2 or tuple(b.shape) != (theta.shape[0] + 1, theta.shape[1] + 1):
            raise ValueError("theta must be [ny-1][nx-1] and b [ny][nx]")
        coeffs = fv5_from_cells(theta.detach().contiguous(), is_log=True)
        hier = Hierarchy(coeffs, **(params or {}))
        u, info = hier.solve(b.detach().contiguous(), tol=tol)
        ctx.hier = hier
        ctx.tol = tol
        ctx.save_for_backward(theta, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        theta, u = ctx.saved_tensors
        lam, _ = ctx.hier.solve(grad_u.contiguous(), tol=ctx.tol)
        g_theta = grad_logD(theta.detach().contiguous(), u, lam)
        ctx.hier.close()
        return g_theta, lam, None, None


class SolveFVBatched(torch.autograd.Function):
    """u_k = A(theta_k)^{-1} b_k for a batch of problems of one size
    (theta: [B, ny-1, nx-1] per-cell ln D, b: [B, ny, nx]).  Forward: one
    hierarchy per problem, all problems solved together by the batched solver.
    Backward: the adjoint problems A(theta_k) lambda_k = dL/du_k, batched on the
    same hierarchies (A is symmetric), then the per-cell gradient kernel."""

    @staticmethod
    def forward(ctx, theta, b, tol=1e-10, params=None):
        if theta.dim() != 3 or tuple(b.shape) != (theta.shape[0], theta.shape[1] + 1, theta.shape[2] + 1):
            raise ValueError("theta must be [B][ny-1][nx-1] and b [B][ny][nx]")
        th = theta.detach().contiguous()
        bb = b.detach().contiguous()
        nb = th.shape[0]
        planes = fv5_from_cells_batched(th, is_log=True)
        coeffs = [planes[k] for k in range(nb)]
        hier = BatchHierarchy(coeffs, **(params or {}))
        del coeffs, planes
        u = torch.zeros_like(bb)
        hier.solve([bb[k] for k in range(nb)], [u[k] for k in range(nb)], tol=tol)
        ctx.hier = hier
        ctx.tol = tol
        ctx.save_for_backward(theta, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        theta, u = ctx.saved_tensors
        gu = grad_u.contiguous()
        nb = gu.shape[0]
        lam = torch.zeros_like(gu)
        ctx.hier.solve([gu[k] for k in range(nb)], [lam[k] for k in range(nb)], tol=ctx.tol)
        th = theta.detach().contiguous()
        g_theta = grad_logD_batched(th, u.contiguous(), lam)
        ctx.hier.close()
        return g_theta, lam, None, None


# --------------------------------------------------------------------------
# 3D (include/hipbmg3d.h)
# --------------------------------------------------------------------------
KERNELS3 = ("relax_colour", "residual", "restrict", "interp", "coarse_levels")


def fv7_from_cells(cells):
    """7-point finite-volume planes {C, W, S, B} [4][nz][ny][nx] from per-cell D
    [(nz-1)][(ny-1)][(nx-1)] (a CUDA float64 tensor)."""
    if cells.dim() != 3:
        raise ValueError("cells must be [nz-1][ny-1][nx-1]")
    nz, ny, nx = (int(d) + 1 for d in cells.shape)
    out = torch.empty((4, nz, ny, nx), dtype=torch.float64, device=cells.device)
    _check(lib().hipbmg3d_fv7_from_cells(nx, ny, nz, _ptr(cells), _ptr(out), _stream()))
    return out


class Hierarchy3:
    """3D multigrid hierarchy on the GPU (hipbmg3d_setup / hipbmg3d_solve).

    planes: [4][nz][ny][nx] {C, W, S, B} (7-point) or [14][nz][ny][nx] (27-point:
    C, then -A(p, p+d) for the lower-half offsets d, linear index 0..12)."""

    def __init__(self, planes, **params):
        if planes.dim() != 4 or planes.shape[0] not in (4, 14):
            raise ValueError("planes must be [4 or 14][nz][ny][nx]")
        self.npt = 7 if planes.shape[0] == 4 else 27
        self.nz, self.ny, self.nx = (int(d) for d in planes.shape[1:])
        self.params = default_params(**params)
        self.device = planes.device
        h = ctypes.c_void_p()
        _check(lib().hipbmg3d_setup(self.nx, self.ny, self.nz, self.npt, _ptr(planes), ctypes.byref(self.params),
                                    _stream(), ctypes.byref(h)))
        self._h = h
        _open_handles.add(self)
        n = ctypes.c_int()
        _check(lib().hipbmg3d_num_levels(self._h, ctypes.byref(n)))
        self.L = n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().hipbmg3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self, l):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().hipbmg3d_level_size(self._h, l, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return c.value, b.value, a.value   # (nz, ny, nx)

    def _field(self, l):
        return torch.zeros(self.size(l), dtype=torch.float64, device=self.device)

    def stencil(self, l):
        """[27][nz][ny][nx]: out[(dz+1)*9+(dy+1)*3+(dx+1)] = A(p, p+d)."""
        out = torch.empty((27,) + self.size(l), dtype=torch.float64, device=self.device)
        _check(lib().hipbmg3d_get_stencil(self._h, l, _ptr(out), _stream()))
        return out

    def interp(self, l):
        """[8][nz][ny][nx]: weight of fine vertex (i,j,k) on ((i>>1)+a, (j>>1)+b, (k>>1)+c) at [4c+2b+a]."""
        out = torch.empty((8,) + self.size(l), dtype=torch.float64, device=self.device)
        _check(lib().hipbmg3d_get_interp(self._h, l, _ptr(out), _stream()))
        return out

    def solve(self, b, u0=None, tol=1e-10, check=True):
        u = torch.zeros_like(b) if u0 is None else u0.clone()
        shp = (self.nz, self.ny, self.nx)
        info = Info()
        st = lib().hipbmg3d_solve(self._h, _ptr(b, shape=shp, name="b"), _ptr(u, shape=shp, name="u0"), float(tol),
                                  _stream(), ctypes.byref(info))
        if st != OK and (check or st not in (ENOCONV,)):
            _check(st)
        return u, info

    def _lv(self, l, t, name, coarse=False):
        if not 0 <= l < self.L or (coarse and l < 1):
            raise ValueError("level %d out of range" % l)
        return _ptr(t, shape=self.size(l - 1 if coarse else l), name=name)

    def smooth(self, l, b, x, sweeps=1):
        x = x.clone()
        _check(lib().hipbmg3d_op_smooth(self._h, l, self._lv(l, b, "b"), self._lv(l, x, "x"), sweeps, _stream()))
        return x

    def residual(self, l, b, x):
        r = self._field(l)
        _check(lib().hipbmg3d_op_residual(self._h, l, self._lv(l, b, "b"), self._lv(l, x, "x"), _ptr(r), _stream()))
        return r

    def restrict(self, l, r):
        bc = self._field(l - 1)
        _check(lib().hipbmg3d_op_restrict(self._h, l, self._lv(l, r, "r"), _ptr(bc), _stream()))
        return bc

    def interp_correct(self, l, x, r, xc, rescorr=1):
        x = x.clone()
        _check(lib().hipbmg3d_op_interp_correct(self._h, l, self._lv(l, x, "x"), self._lv(l, r, "r"),
                                                self._lv(l, xc, "xc", coarse=True), rescorr, _stream()))
        return x

    def coarse_solve(self, b):
        x = self._field(0)
        _check(lib().hipbmg3d_op_coarse_solve(self._h, self._lv(0, b, "b"), _ptr(x), _stream()))
        return x

    def profile(self, enable=True):
        _check(lib().hipbmg3d_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kernel class: (ms, launches, algorithmic bytes per launch)}
        accumulated since profile(True)."""
        out = {}
        for k, name in enumerate(KERNELS3):
            ms, n, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
            _check(lib().hipbmg3d_profile_read(self._h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
            out[name] = (ms.value, n.value, by.value)
        return out


# --------------------------------------------------------------------------
# the paper's distributed model (host only)
# --------------------------------------------------------------------------
PAPER_TERMS = ("smooth", "residual", "restrict", "interp", "agglomerate", "cgsolve")


def paper_model(N, P, ns, ncolors=4, nu1=2, nu2=1, redundant=0, alpha=0.65e-6, beta=5.65e-9, gamma=0.44e-9):
    """T_V-cycle of the paper's model (section 3).  N, P: per level (0 coarsest)
    global grid points and processor grid, each a list of D-tuples.  Returns
    (total seconds, [per-level dict of the six terms])."""
    L, D = len(N), len(N[0])
    Na = (ctypes.c_int * (L * D))(*[int(v) for row in N for v in row])
    Pa = (ctypes.c_int * (L * D))(*[int(v) for row in P for v in row])
    terms = (ctypes.c_double * (L * 6))()
    total = ctypes.c_double()
    _check(lib().hipbmg_paper_model(D, L, Na, Pa, ns, ncolors, nu1, nu2, redundant, alpha, beta, gamma, terms,
                                    ctypes.byref(total)))
    return total.value, [dict(zip(PAPER_TERMS, terms[6 * l: 6 * l + 6])) for l in range(L)]


def paper_enumerate(N, P, max_grids=64):
    """Coarse processor grids of section 4's enumeration, [(p_0, .., p_{D-1}), ...]."""
    D = len(N)
    Na = (ctypes.c_int * D)(*[int(v) for v in N])
    Pa = (ctypes.c_int * D)(*[int(v) for v in P])
    g = (ctypes.c_int * (max_grids * D))()
    cnt = ctypes.c_int()
    _check(lib().hipbmg_paper_enumerate(D, Na, Pa, max_grids, g, ctypes.byref(cnt)))
    return [tuple(g[k * D:(k + 1) * D]) for k in range(cnt.value)]


class PaperSetup(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int), ("limit", ctypes.c_int), ("coarsest", ctypes.c_int), ("ns", ctypes.c_int),
                ("ncolors", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("redundant", ctypes.c_int),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double)]


def _paper_setup(D, limit, coarsest, ns, ncolors, nu1, nu2, redundant, alpha, beta, gamma):
    return PaperSetup(D, limit, coarsest, ns, ncolors, nu1, nu2, redundant, alpha, beta, gamma)


def paper_search(N, P, limit=9, coarsest=3, ns=9, ncolors=4, nu1=2, nu2=1, redundant=0, alpha=0.65e-6,
                 beta=5.65e-9, gamma=0.44e-9):
    """Cheapest redistribution path of section 4's search over the paper's
    model: (model seconds per V-cycle, [processor grids after the first])."""
    D = len(N)
    st = _paper_setup(D, limit, coarsest, ns, ncolors, nu1, nu2, redundant, alpha, beta, gamma)
    Na = (ctypes.c_int * D)(*N)
    Pa = (ctypes.c_int * D)(*P)
    path = (ctypes.c_int * (64 * D))()
    ln = ctypes.c_int()
    t = ctypes.c_double()
    _check(lib().hipbmg_paper_search(ctypes.byref(st), Na, Pa, 64, path, ctypes.byref(ln), ctypes.byref(t)))
    return t.value, [tuple(path[k * D:(k + 1) * D]) for k in range(ln.value)]


def paper_astar(N, P, limit=9, coarsest=3, ns=9, ncolors=4, nu1=2, nu2=1, redundant=0, alpha=0.65e-6,
                beta=5.65e-9, gamma=0.44e-9):
    """The same search by A*: (model seconds per V-cycle, [processor grids
    after the first], states expanded)."""
    D = len(N)
    st = _paper_setup(D, limit, coarsest, ns, ncolors, nu1, nu2, redundant, alpha, beta, gamma)
    Na = (ctypes.c_int * D)(*N)
    Pa = (ctypes.c_int * D)(*P)
    path = (ctypes.c_int * (64 * D))()
    ln = ctypes.c_int()
    t = ctypes.c_double()
    ex = ctypes.c_int()
    _check(lib().hipbmg_paper_astar(ctypes.byref(st), Na, Pa, 64, path, ctypes.byref(ln), ctypes.byref(t),
                                    ctypes.byref(ex)))
    return t.value, [tuple(path[k * D:(k + 1) * D]) for k in range(ln.value)], ex.value


def paper_path_cost(N, P, seq, limit=9, coarsest=3, ns=9, ncolors=4, nu1=2, nu2=1, redundant=0, alpha=0.65e-6,
                    beta=5.65e-9, gamma=0.44e-9):
    """Model seconds per V-cycle along the given processor grids (after the first)."""
    D = len(N)
    st = _paper_setup(D, limit, coarsest, ns, ncolors, nu1, nu2, redundant, alpha, beta, gamma)
    Na = (ctypes.c_int * D)(*N)
    Pa = (ctypes.c_int * D)(*P)
    flat = [v for g in seq for v in g]
    path = (ctypes.c_int * max(1, len(flat)))(*flat)
    t = ctypes.c_double()
    _check(lib().hipbmg_paper_path_cost(ctypes.byref(st), Na, Pa, path, len(seq), ctypes.byref(t)))
    return t.value
