"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracles (2D, its FP32 mode, 3D) and the host-only model code (the
single-GPU model, its redistribution search, the paper's distributed model,
enumeration and searches) are compiled with -fsanitize=address,undefined
together with drivers that call every entry point on small ragged problems,
the paper's own problems and random setups.  A sanitizer report aborts the
program (no recovery), and leak checking is on."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(cmd, exe):
    subprocess.run(cmd, check=True, cwd=ROOT)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=ENV)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracles_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    out = _run(["gcc", "-std=c99", "-ffp-contract=off", "-fopenmp"] + SAN +
               ["tests/sanitize_oracle.c", "oracle/bmg_oracle.c", "oracle/bmg_oracle3d.c", "-o", str(exe), "-lm"],
               exe)
    assert "checksum" in out


@pytest.mark.parametrize("driver", ["sanitize_model.cpp", "model_search_check.cpp"])
def test_model_code_under_sanitizers(tmp_path, driver):
    exe = tmp_path / "model_san"
    _run(["g++", "-std=c++17", "-I", "include", "-I", "paper_1803_02481_amd/csrc"] + SAN +
         ["tests/" + driver, "paper_1803_02481_amd/csrc/bmg_model.cpp", "-o", str(exe)], exe)
