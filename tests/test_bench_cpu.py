"""Host logic of bench.py (CPU): the step-source hash that ties the committed
counter summaries to the sources they were taken from, and the refusal of a
multi-GPU run."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_only_drops_comments_and_keeps_code():
    src = "int a = 1;  // one\n/* a block\n   comment */\n\nint b = a / 2;  /* half */\n"
    assert bench._code_only(src) == "int a = 1;\nint b = a / 2;"


def test_hash_ignores_comments_but_not_code():
    src = open(os.path.join(ROOT, "paper_2311_12180_amd", "csrc", "kernels.hip")).read()
    commented = src.replace("namespace pdlp {", "// a note\nnamespace pdlp {  /* and another */", 1)
    assert commented != src
    assert bench._code_only(commented) == bench._code_only(src)
    changed = src.replace("constexpr int kDecideBlock = 1024;", "constexpr int kDecideBlock = 512;", 1)
    assert changed != src
    assert bench._code_only(changed) != bench._code_only(src)


def test_step_hash_is_deterministic():
    h = bench.step_kernels_hash()
    assert len(h) == 16 and h == bench.step_kernels_hash()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
