"""Host code under sanitizers (CPU only): the serving scheduler's threads
under ThreadSanitizer, the FP64 reference and the library's host-side
arithmetic (the plain method's parameter draws and per-sample constants)
under AddressSanitizer and UndefinedBehaviorSanitizer.  Each driver is built
here, run on the workloads of the benchmark and the tests, and must exit
cleanly with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

from paper_2604_27193_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
CSRC = os.path.join(ROOT, "paper_2604_27193_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
CLANG = "/opt/rocm/llvm/bin/clang++"


def workloads():
    return [W.single(100), W.single(100, impact_exit=True), W.single(100, obstacle="none"),
            W.sweep(n=100)[37], W.sweep(n=100)[255], W.paper_preset(100),
            W.paper_preset(100, integrator="euler"), W.perception(100),
            dict(W.perception(100), p_dropout=0.9, frame_period=0.001),
            W.closed_loop(100), W.rare_event(100), W.uneven_batch(3)[2],
            dict(W.single(100), nofma=True)]


def run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, env=env)
    return r.returncode, r.stdout + r.stderr


def clean(rc, out):
    assert rc == 0, out[-3000:]
    for word in ("Sanitizer", "runtime error", "WARNING: ThreadSanitizer"):
        assert word not in out, out[-3000:]


def test_scheduler_threads_under_tsan(tmp_path):
    exe = str(tmp_path / "sched_tsan")
    rc, out = run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                   "-I", INCLUDE, "-I", CSRC, "-I", TESTS,
                   os.path.join(TESTS, "sanitize_sched.cpp"), "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    rc, out = run([exe], env=env)
    clean(rc, out)
    assert "bad 0" in out


def test_reference_under_asan_ubsan(tmp_path):
    from oracle import oracle
    path = tmp_path / "scenarios.bin"
    path.write_bytes(b"".join(bytes(oracle.scenario(d)) for d in workloads()))
    exe = str(tmp_path / "oracle_asan")
    rc, out = run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-builtin",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                   "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "aeb_oracle.c"),
                   os.path.join(TESTS, "sanitize_oracle.c"), "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = run([exe, str(path), "3000"])
    clean(rc, out)
    assert f"scenarios {len(workloads())}, failures 0" in out


@pytest.mark.skipif(not shutil.which(CLANG) and not os.path.exists(CLANG),
                    reason="ROCm clang++ not installed")
def test_host_sampler_under_asan_ubsan(tmp_path):
    from paper_2604_27193_amd import binding
    path = tmp_path / "scenarios.bin"
    path.write_bytes(b"".join(bytes(binding.scenario(d)) for d in workloads()))
    exe = str(tmp_path / "sampler_asan")
    rc, out = run([CLANG, "-x", "c++", "-std=c++17", "-O1", "-g", "-ffp-contract=off",
                   "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", INCLUDE, "-I", CSRC,
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
                   os.path.join(TESTS, "sanitize_sampler.cpp"), "-o", exe])
    assert rc == 0, out
    rc, out = run([exe, str(path), "20000"])
    clean(rc, out)
    assert f"scenarios {len(workloads())}, bad draws 0" in out
