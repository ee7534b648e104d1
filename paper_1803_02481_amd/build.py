"""Build libhipbmg.so in-tree: hand-written HIP for gfx950 plus the host runtime.

    python -m paper_1803_02481_amd.build
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhipbmg.so")
OBJ = os.path.join(ROOT, "_build")

HIP_SOURCES = ["bmg_stream.hip", "bmg_setup.hip", "bmg_collapse.hip", "bmg_misc.hip",
               "bmg_host.hip", "bmg_calib.hip", "bmg3d.hip", "bmg_resnorm.hip"]
CXX_SOURCES = ["bmg_model.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-I" + INC,
             # fuse a*b+c only within one source expression: every inlined or
             # peeled copy of a step then rounds alike, so results do not
             # depend on the tiling
             "-ffp-contract=on",
             # no packed-FP32 instructions (v_pk_*_f32) in device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    if src.endswith(".cpp"):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-I" + INC, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC] + HIP_FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in HIP_SOURCES + CXX_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
