"""The library's host policy under AddressSanitizer and
UndefinedBehaviorSanitizer.

The policy code (status strings, the uneven batch's work-queue builder, the
server's pool allocator, admission rule and latency percentile; one
HIP-free source file) is built alone with g++ and both sanitizers into a
CPU-only library, and the CPU tests of that policy run in a child process
that loads it (ADCT_POLICY_LIB) with the sanitizer runtimes preloaded.  Any
report aborts the child.  A second child loads a small library with a
planted heap overread, to show that a report does abort in this setup.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_07414_amd", "csrc")
POLICY_SRC = os.path.join(CSRC, "adct_policy.cpp")
SAN_FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-shared", "-fPIC"]
POLICY_TESTS = ["tests/test_serve_policy.py", "tests/test_abi.py::test_work_queue_small_exact",
                "tests/test_abi.py::test_work_queue_covers_every_tile_once", "tests/test_abi.py::test_work_queue_errors"]


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def san(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not available")
    d = tmp_path_factory.mktemp("sanitized")
    lib = str(d / "libadct_policy_san.so")
    subprocess.run(["g++", *SAN_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, POLICY_SRC, "-o", lib],
                   check=True)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONDONTWRITEBYTECODE="1")
    return {"lib": lib, "dir": d, "env": env}


def test_policy_tests_run_clean_under_sanitizers(san):
    env = dict(san["env"], ADCT_POLICY_LIB=san["lib"])
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *POLICY_TESTS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout and "failed" not in r.stdout
    # the instrumented library, not libadct.so, served the calls
    probe = ("from paper_1606_07414_amd import adct; assert adct.percentile([3.0, 1.0, 2.0], 50) == 2.0; "
             "assert adct._POLICY is not None and adct._LIB is None; print('instrumented')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "instrumented" in r.stdout, r.stderr[-2000:]


def test_a_planted_overread_aborts_the_child(san):
    src = san["dir"] / "overread.cpp"
    src.write_text(textwrap.dedent("""
        #include <vector>
        extern "C" int overread(int n) { std::vector<int> v(n, 1); return v.data()[n]; }
    """))
    lib = str(san["dir"] / "liboverread.so")
    subprocess.run(["g++", *SAN_FLAGS, str(src), "-o", lib], check=True)
    code = f"import ctypes; print(ctypes.CDLL({lib!r}).overread(4))"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=san["env"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
