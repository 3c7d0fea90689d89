"""CPU test of the serving loop's batching and admission policy
(paper_2603_02048_amd/csrc/serve_policy.h, pure host C++), built with g++."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_batching_policy(tmp_path):
    exe = str(tmp_path / "serve_policy_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2603_02048_amd", "csrc"),
                           os.path.join(ROOT, "tests", "serve_policy_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().startswith("OK")
