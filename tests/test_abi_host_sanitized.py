"""The host-side ABI checks (tests/test_abi_host.py) once more, against a
build of the library whose host C++ (argument validation, workspace sizing,
tile cache, entry points) carries AddressSanitizer and
UndefinedBehaviorSanitizer instrumentation: any out-of-bounds access, use
after free or undefined behaviour on those paths aborts the run.  CPU only."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_checks_pass_under_asan_and_ubsan():
    sys.path.insert(0, os.path.join(ROOT, "paper_2508_18071_amd"))
    import build
    try:
        lib = build.build_sanitized()
        rt = build.asan_runtime()
    except RuntimeError as e:
        pytest.skip(f"sanitized build unavailable: {e}")
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "library is not instrumented"
    env = dict(os.environ, EVS_LIB_PATH=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = ("import paper_2508_18071_amd as m, sys; assert m.LIB_PATH == sys.argv[1], m.LIB_PATH; "
            "m.lib(); print('loaded', m.LIB_PATH)")
    r = subprocess.run([sys.executable, "-c", code, lib], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "loaded" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
