"""The host C++ (assembly, validation, planning, the C ABI's host paths)
under AddressSanitizer and UndefinedBehaviorSanitizer: the host-side tests
run again against a build of the library whose host sources are instrumented
(paper_2310_09410_amd.build.build_sanitized; nothing on the GPU is), and
every sanitizer report fails the test."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_paths_are_clean_under_asan_and_ubsan(tmp_path):
    from paper_2310_09410_amd import build
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    try:
        lib = build.build_sanitized()
    except RuntimeError as e:
        pytest.skip(str(e))
    gxx = shutil.which("g++")
    pre = [subprocess.run([gxx, f"-print-file-name={n}"], capture_output=True, text=True, check=True).stdout.strip()
           for n in ("libasan.so", "libstdc++.so")]
    logs = str(tmp_path / "san")
    env = dict(os.environ, LD_PRELOAD=" ".join(pre), LDOPF_LIBRARY=lib,
               ASAN_OPTIONS=f"detect_leaks=0:log_path={logs}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={logs}")
    probe = subprocess.run([sys.executable, "-c", "from paper_2310_09410_amd import _native; print(_native.LIB_PATH)"],
                           env=env, capture_output=True, text=True, cwd=ROOT)
    assert probe.stdout.strip() == lib, probe.stderr
    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_host.py")],
                         env=env, capture_output=True, text=True, cwd=ROOT, timeout=600)
    reports = glob.glob(logs + "*")
    text = "".join(open(f).read() for f in reports)
    assert run.returncode == 0 and not reports, (run.stdout[-2000:], text[:4000])
