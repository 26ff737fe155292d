"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code.

* The oracle's C library is built with gcc's sanitizers (-O1, one thread)
  and every one of its entry points is driven on small graphs, including
  edgeless and two-vertex-component ones; the digests of all results must
  equal those of the ordinary build.
* The HIP library is built with the sanitizers on its host code (device code
  is not instrumented) and the CPU tests of the C ABI run against it:
  symbol export, argument validation of every entry point, workspace-size
  and budget-table calls.  A sanitizer report aborts the child process.
"""
import glob
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1601_05527_amd")
ASAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, extra_env):
    env = dict(os.environ)
    env.update(ASAN_ENV)
    env.update(extra_env)
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_oracle_under_asan_ubsan():
    import oracle
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    san = oracle.build(force=True, sanitize=True)
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(rt) and os.path.exists(rt), rt
    script = os.path.join(ROOT, "tests", "sanitized_calls.py")
    plain = _run([sys.executable, script], {"ORACLE_LIBRARY": ""})
    assert plain.returncode == 0, plain.stderr[-4000:]
    checked = _run([sys.executable, script], {"ORACLE_LIBRARY": san, "LD_PRELOAD": rt})
    assert checked.returncode == 0, checked.stderr[-4000:]
    a = json.loads(plain.stdout.strip().splitlines()[-1])
    b = json.loads(checked.stdout.strip().splitlines()[-1])
    assert b["library"] == san
    assert a["library"] != san
    assert a["digests"] == b["digests"]
    assert "runtime error" not in checked.stderr


def _stale(lib):
    if not os.path.exists(lib):
        return True
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + [os.path.join(ROOT, "include", "ad.h")]
    return max(os.path.getmtime(s) for s in srcs) > os.path.getmtime(lib)


def test_library_host_code_under_asan_ubsan():
    from paper_1601_05527_amd import build_lib
    if not os.path.exists(build_lib.HIPCC):
        pytest.skip("hipcc not found")
    lib = build_lib.SAN_LIB
    if _stale(lib):
        build_lib.build_sanitized()
    rt = build_lib.sanitizer_runtime()
    r = _run([sys.executable, "-m", "pytest", "-q", "-s", "-p", "no:cacheprovider",
              os.path.join("tests", "test_abi_cpu.py")],
             {"AD_LIBRARY": lib, "LD_PRELOAD": rt})
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "passed" in r.stdout and "failed" not in r.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out
