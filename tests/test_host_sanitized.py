"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): tests/host_check/host_check.cpp drives the C ABI's size queries,
option checks and error paths against a build whose host code is
instrumented, and must finish without a failed check or a sanitizer report."""
import os
import shutil
import subprocess

import pytest

from paper_2501_16122_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(300)
def test_host_entry_points_under_sanitizers(tmp_path):
    if not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    for src in build.SANITIZE_REUSE:
        if not os.path.exists(os.path.join(build.BUILD, src.replace(".hip", ".o"))):
            pytest.skip("the regular build's objects are missing (run build() first)")
    lib = build.build_host_sanitized(str(tmp_path))
    exe = str(tmp_path / "host_check")
    # the driver is plain C++: built by the clang that hipcc drives, so that
    # both link the same sanitizer runtime
    clang = os.path.join(os.path.dirname(os.path.realpath(build.HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/lib/llvm/bin/clang++"
    cmd = [clang, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++20", "-fsanitize=address",
           "-fsanitize=undefined", "-shared-libsan", "-I", build.INCLUDE,
           os.path.join(HERE, "host_check", "host_check.cpp"), lib, f"-Wl,-rpath,{tmp_path}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    env = dict(os.environ)
    rt_dirs = [os.path.dirname(rt)] if rt and os.path.exists(rt) else []
    env["LD_LIBRARY_PATH"] = os.pathsep.join(rt_dirs + [env.get("LD_LIBRARY_PATH", "")])
    # leaks of the HIP runtime's own start-up are outside the checked code
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out
    assert "host checks ok" in run.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
