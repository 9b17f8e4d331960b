"""The product server's scheduling core (arena bounded by the HBM budget, arrival-ordered
admission, batch limits), built for the host and checked against an independent model:
shadow ranges over a fake address space and an event-driven replay of the server loop
with Poisson arrivals (see tests/sched_host_check.cpp)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduling_core(tmp_path):
    exe = str(tmp_path / "sched_host_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-I",
                           os.path.join(ROOT, "paper_0901_1413_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sched_host_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.splitlines()
    assert lines[-1] == "ok all", out.stdout
    names = [l.split()[1] for l in lines if l.startswith("ok ")]
    assert names.count("arena_random") == 2 and names.count("server_replay") == 3
    assert "arena_reset" in names and "queue" in names
