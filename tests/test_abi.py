"""CPU checks of the C boundary: the library is built, loads, and exports every
entry point declared in include/hipbmg.h and include/hipbmg3d.h (no device
calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", "hipbmg.h"), os.path.join(ROOT, "include", "hipbmg3d.h")]
LIB = os.path.join(ROOT, "paper_1803_02481_amd", "libhipbmg.so")


def declared_functions():
    names = set()
    for hdr in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(hdr).read(), flags=re.S)
        names |= set(re.findall(r"\b(hipbmg(?:3d)?_[A-Za-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("hipbmg_setup", "hipbmg_solve", "hipbmg_destroy", "hipbmg_fv5_from_cells",
                 "hipbmg_grad_logD", "hipbmg_last_error", "hipbmg_default_params",
                 "hipbmg3d_setup", "hipbmg3d_solve", "hipbmg3d_destroy", "hipbmg3d_fv7_from_cells"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhipbmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhipbmg.so not built")
def test_binding_signatures_cover_the_header():
    from paper_1803_02481_amd import hipbmg
    assert set(hipbmg._SIGS) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhipbmg.so not built")
def test_default_params_and_errors_without_device():
    from paper_1803_02481_amd import hipbmg
    p = hipbmg.default_params()
    assert (p.nu1, p.nu2, p.coarsest_n, p.collapse_level, p.max_cycles) == (2, 1, 3, -1, 500)
    lib = hipbmg.lib()
    h = ctypes.c_void_p()
    # argument validation happens before any device call
    assert lib.hipbmg_setup(64, 65, 5, ctypes.c_void_p(8), None, None, ctypes.byref(h)) == hipbmg.EINVAL
    assert b"odd" in lib.hipbmg_last_error()
    assert lib.hipbmg_setup(65, 65, 7, ctypes.c_void_p(8), None, None, ctypes.byref(h)) == hipbmg.EINVAL
    assert lib.hipbmg_setup(65, 65, 5, None, None, None, ctypes.byref(h)) == hipbmg.EINVAL
    assert lib.hipbmg_solve(None, None, None, 1e-10, None, None) == hipbmg.EINVAL
    assert lib.hipbmg_destroy(None) == hipbmg.OK
    # the 3D entry points validate before any device call as well
    p3 = ctypes.byref(p)
    assert lib.hipbmg3d_setup(33, 33, 32, 7, ctypes.c_void_p(8), p3, None, ctypes.byref(h)) == hipbmg.EINVAL
    assert b"odd" in lib.hipbmg_last_error()
    assert lib.hipbmg3d_setup(33, 33, 33, 9, ctypes.c_void_p(8), p3, None, ctypes.byref(h)) == hipbmg.EINVAL
    pm = hipbmg.default_params(precision=hipbmg.MIXED)
    assert lib.hipbmg3d_setup(33, 33, 33, 7, ctypes.c_void_p(8), ctypes.byref(pm), None,
                              ctypes.byref(h)) == hipbmg.EINVAL
    assert b"FP64" in lib.hipbmg_last_error()
    pc = hipbmg.default_params(coarsest_n=33)
    assert lib.hipbmg3d_setup(33, 33, 33, 7, ctypes.c_void_p(8), ctypes.byref(pc), None,
                              ctypes.byref(h)) == hipbmg.EINVAL
    assert b"unknowns" in lib.hipbmg_last_error()
    assert lib.hipbmg3d_solve(None, None, None, 1e-10, None, None) == hipbmg.EINVAL
    assert lib.hipbmg3d_destroy(None) == hipbmg.OK


def test_binding_structs_match_the_header_layout(tmp_path):
    """sizeof and every field offset of the parameter and info structs, as the
    C compiler lays them out, equal those of the ctypes mirrors."""
    from paper_1803_02481_amd import hipbmg
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include "hipbmg.h"', "int main(void) {"]
    for cname, py in (("hipbmg_params", hipbmg.Params), ("hipbmg_info", hipbmg.Info),
                      ("hipbmg_paper_setup", hipbmg.PaperSetup)):
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0; }"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                  text=True).stdout.splitlines())
    for cname, py in (("hipbmg_params", hipbmg.Params), ("hipbmg_info", hipbmg.Info),
                      ("hipbmg_paper_setup", hipbmg.PaperSetup)):
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)


def test_set_allocator_validates_its_arguments():
    import ctypes
    from paper_1803_02481_amd import hipbmg as HB
    L = HB.lib()
    fa = HB.ALLOC_FN(lambda n, ctx: 0)
    ff = HB.FREE_FN(lambda p, ctx: None)
    assert L.hipbmg_set_allocator(ctypes.cast(fa, ctypes.c_void_p), None, None) == HB.EINVAL
    assert L.hipbmg_set_allocator(None, ctypes.cast(ff, ctypes.c_void_p), None) == HB.EINVAL
    assert L.hipbmg_set_allocator(ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ff, ctypes.c_void_p), None) == HB.OK
    assert L.hipbmg_set_allocator(None, None, None) == HB.OK
    with pytest.raises(ValueError):
        HB.set_allocator(lambda n: 0)
    HB.use_torch_allocator()   # the binding's default
