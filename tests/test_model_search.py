"""CPU checks of the performance model's redistribution search (section 4):
the A* search over (level, workgroups) states against the enumeration of
every path, compiled on the host from the library's model source."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_astar_matches_exhaustive_search(tmp_path):
    exe = tmp_path / "model_search_check"
    src = [os.path.join(ROOT, "tests", "model_search_check.cpp"),
           os.path.join(ROOT, "paper_1803_02481_amd", "csrc", "bmg_model.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1803_02481_amd", "csrc")] + src + ["-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "fails 0" in r.stdout
