"""The host-side C code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (oracle/build_sanitized.sh, gcc) runs its pin tests and the
  harness's host tests with gcc's libasan and libubsan preloaded.
* The library's host code (embedding, layout, tables, handle preparation,
  argument checks; paper_1603_03755_amd.build.build_host_sanitized, clang)
  runs the host-forced failure tests and the host-only queries with clang's
  ASan runtime preloaded.

Each runs in a subprocess (the sanitizer runtime must be loaded first); a
sanitizer report aborts it.  No GPU is touched."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, args, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + args,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return r.returncode, r.stdout[-3000:] + r.stderr[-3000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    subprocess.run(["sh", os.path.join(ROOT, "oracle", "build_sanitized.sh"), str(tmp_path)], check=True)
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    libubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    tests = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_")) + ["tests/test_harness_host.py"]
    rc, out = _run({"SQA_ORACLE_LIB": str(tmp_path / "liboracle_asan.so"), "LD_PRELOAD": f"{libasan}:{libubsan}"},
                   tests, timeout=900)
    assert rc == 0, out
    assert "passed" in out


def _clang_asan_runtime():
    base = "/opt/rocm/lib/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for ver in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


@pytest.mark.skipif(_clang_asan_runtime() is None, reason="clang's ASan runtime not found")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_1603_03755_amd import build as B
    if not os.path.exists(os.path.join(B.HERE, "_build", "sqa_kernels.hip.o")):
        pytest.skip("the library's device objects are not built")
    lib = B.build_host_sanitized(str(tmp_path))
    rc, out = _run({"SQA_LIBRARY": lib, "LD_PRELOAD": _clang_asan_runtime()},
                   ["tests/test_host_failures.py", "tests/test_abi.py::test_random_trees_match_oracle_on_host",
                    "tests/test_abi.py::test_host_only_queries"], timeout=600)
    assert rc == 0, out
    assert "passed" in out
