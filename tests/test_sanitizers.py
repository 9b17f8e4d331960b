"""Host code under sanitizers (CPU only, no GPU needed).

- AddressSanitizer + UndefinedBehaviorSanitizer: the oracle (tests/oracle_host_check.c),
  the scheduling core and arena (sched_host_check.cpp), the server's worker core with a fake
  executor (server_host_check.cpp), the field formulas (field_host_check.cpp), the
  Strassen-Winograd schedule (sw_host_check.cpp), and the library's own host code - the
  tuning-cache parser, configuration choice and every argument check of the C ABI
  (abi_host_check.cpp, linked with the library's host sources built with host-only
  sanitizers and its kernel objects as built).
- ThreadSanitizer: the server's worker core with four submitting threads and a polling
  thread against the fake executor, including a failed launch and a batch that never
  completes (the watchdog); the persistent workgroups' drain loop (drain_host_check.cpp).
"""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0901_1413_amd", "csrc")
TESTS = os.path.join(ROOT, "tests")
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
# ROCm's clang: it links the library's objects (built by hipcc with its sanitizer
# instrumentation), and its ThreadSanitizer runtime intercepts pthread_cond_clockwait, which
# libstdc++ uses for waits on the steady clock (the host gcc's runtime does not, and then
# takes a mutex released inside such a wait for one still held)
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def run(exe, env=ENV, timeout=300):
    out = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert out.stdout.splitlines()[-1] == "ok all" or "FAIL" not in out.stdout, out.stdout[-2000:]
    return out.stdout


def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_host_check")
    subprocess.check_call(["gcc", "-std=c99", "-fopenmp", "-Wall", "-Werror", *ASAN,
                           os.path.join(TESTS, "oracle_host_check.c"), os.path.join(ROOT, "oracle", "gfq_oracle.c"),
                           "-o", exe])
    assert run(exe).splitlines()[-1] == "ok all"


@pytest.mark.parametrize("src", ["sched_host_check.cpp", "server_host_check.cpp", "field_host_check.cpp",
                                 "sw_host_check.cpp", "drain_host_check.cpp"])
def test_host_checks_asan_ubsan(tmp_path, src):
    exe = str(tmp_path / src.replace(".cpp", ""))
    subprocess.check_call(["g++", "-std=c++17", "-pthread", "-Wall", "-Werror", "-Wno-unknown-pragmas", *ASAN, "-I", CSRC,
                           os.path.join(TESTS, src), "-o", exe])
    out = run(exe)
    if src in ("sched_host_check.cpp", "server_host_check.cpp", "drain_host_check.cpp"):
        assert out.splitlines()[-1] == "ok all"


def test_server_core_tsan(tmp_path):
    exe = str(tmp_path / "server_host_check_tsan")
    subprocess.check_call([CLANGXX, "-std=c++17", "-pthread", "-Wall", "-Werror", "-fsanitize=thread", "-g", "-O1",
                           "-I", CSRC, os.path.join(TESTS, "server_host_check.cpp"), "-o", exe])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    out = run(exe, env=env)
    assert out.splitlines()[-1] == "ok all"
    assert "ok watchdog" in out and "ok launch_failure" in out and out.count("ok traffic") == 2


def test_drain_loop_tsan(tmp_path):
    """The persistent workgroups' drain loop (the device kernel's own code, gfq_drain.h) on
    host threads under ThreadSanitizer: the published index is ordered by the barriers."""
    exe = str(tmp_path / "drain_host_check_tsan")
    subprocess.check_call([CLANGXX, "-std=c++17", "-pthread", "-Wall", "-Werror", "-fsanitize=thread", "-g", "-O1",
                           "-I", CSRC, os.path.join(TESTS, "drain_host_check.cpp"), "-o", exe])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    out = run(exe, env=env)
    assert out.splitlines()[-1] == "ok all" and out.count("ok drain") == 5


HOST_SOURCES = ["gfq_api.cpp", "gfq_tune.cpp", "gfq_batch_host.cpp", "gfq_server.cpp"]


def test_library_host_code_asan_ubsan(tmp_path):
    """The library's host sources rebuilt with host-only sanitizers (the device code of every
    kernel object is as built), driven through the C ABI without a GPU."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_0901_1413_amd import build as libbuild
    objdir = os.path.join(ROOT, "paper_0901_1413_amd", "_build")
    kernel_objs = [o for o in sorted(glob.glob(os.path.join(objdir, "*.o")))
                   if os.path.basename(o).replace(".o", ".cpp") not in HOST_SOURCES]
    if len(kernel_objs) < len(libbuild.SOURCES) - len(HOST_SOURCES):
        libbuild.build()
        kernel_objs = [o for o in sorted(glob.glob(os.path.join(objdir, "*.o")))
                       if os.path.basename(o).replace(".o", ".cpp") not in HOST_SOURCES]
    hipcc = libbuild.HIPCC
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

    def cc(src, obj):
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-pthread",
                               *host_san, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", "-o", obj, src],
                              stderr=subprocess.DEVNULL)

    jobs = [(os.path.join(CSRC, s), str(tmp_path / s.replace(".cpp", ".o"))) for s in HOST_SOURCES]
    jobs.append((os.path.join(TESTS, "abi_host_check.cpp"), str(tmp_path / "abi_host_check.o")))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda j: cc(*j), jobs))
    exe = str(tmp_path / "abi_host_check")
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(hipcc)), "lib")
    subprocess.check_call([CLANGXX, "-fsanitize=address,undefined", "-pthread", "-o", exe, *[o for _, o in jobs],
                           *kernel_objs, "-L", rocm_lib, "-lamdhip64", "-Wl,-rpath," + rocm_lib])
    # the HIP runtime's own allocations at exit are not the library's: no leak check here
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", ABI_CHECK_TMP=str(tmp_path))
    out = run(exe, env=env)
    assert out.splitlines()[-1] == "ok all"
    assert "ok tune_cache" in out and "ok choose_config" in out and "ok validation" in out
    assert "ok plan_batch" in out
