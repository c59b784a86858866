"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

Each is built with the sanitizers into a temporary directory, and the CPU
tests that exercise it run against that build in a child process with the
sanitizer runtime preloaded: every oracle pin (fixtures, closed forms,
brute force, invariants, batches on threads), and the library's argument
checks that return before any device call.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(cmd):
    try:
        path = subprocess.check_output(cmd, text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _child(env_extra, tests, timeout=900):
    """Run the given CPU tests in a child process; (exit status, output)."""
    env = dict(os.environ, **env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    # --capture=sys leaves file descriptor 2 alone, where a sanitizer report goes
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "--capture=sys",
                        "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def _clean(rc, out):
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[:4000]
    assert rc == 0, out[-4000:]
    assert " passed" in out


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime(["gcc", "-print-file-name=libasan.so"])
    if not asan:
        pytest.skip("gcc's ASan runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", lib, os.path.join(ROOT, "oracle", "oracle.c")])
    _clean(*_child({"LD_PRELOAD": asan, "INSP_ORACLE_LIB": lib},
                   ["tests/test_oracle.py", "tests/test_mlp_oracle.py"]))


def test_a_planted_overflow_is_reported(tmp_path):
    # negative control: the same build and child run, with the oracle's
    # row buffer (one row's successors) allocated for a single element
    asan = _runtime(["gcc", "-print-file-name=libasan.so"])
    if not asan:
        pytest.skip("gcc's ASan runtime is not installed")
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    old = "int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[n] > 0 ? rp[n] : 1));"
    assert src.count(old) == 1
    bad = tmp_path / "oracle_bad.c"
    bad.write_text(src.replace(old, "int32_t *row = (int32_t *)malloc(sizeof(int32_t));"))
    lib = str(tmp_path / "liboracle_bad.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", lib, str(bad)])
    rc, out = _child({"LD_PRELOAD": asan, "INSP_ORACLE_LIB": lib}, ["tests/test_oracle.py"])
    assert rc != 0 and "AddressSanitizer: heap-buffer-overflow" in out, out[-2000:]


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    import glob
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's ASan runtime is not installed")
    from paper_2404_03226_amd import build
    lib = build.build(sanitize=True, out=str(tmp_path / "libinspirit_san.so"))
    _clean(*_child({"LD_PRELOAD": rt[-1], "INSP_LIB": lib}, ["tests/test_abi.py"]))
