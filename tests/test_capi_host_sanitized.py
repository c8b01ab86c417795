"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

build.py's host-sanitized build instruments the host side of liblbm (the
C-ABI argument validation, layout and launch rules, the equal-area
construction, the JSON tune cache) and a child pytest runs the host-only
C-ABI tests (test_capi_host.py) against it, with clang's shared ASan runtime
preloaded and every report fatal.  No GPU is touched: those tests stop
before any device work.
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hip_build_module():
    import importlib.util

    path = os.path.join(ROOT, "paper_1904_11792_amd", "build.py")
    spec = importlib.util.spec_from_file_location("_lbm_hip_build_san", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_host_code_is_clean_under_asan_and_ubsan():
    lib = _hip_build_module().build(sanitize_host=True)
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    assert rt, "clang's shared ASan runtime is missing"
    env = dict(os.environ, LBM_LIBRARY=lib, LD_PRELOAD=rt[-1],
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = ("import sys; sys.path.insert(0, %r); from paper_1904_11792_amd import lbm; "
             "print(lbm.LIB_PATH)" % ROOT)
    # the instrumented build needs the runtime: without the preload it does not load ...
    bare = dict(env)
    del bare["LD_PRELOAD"]
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, timeout=300, env=bare)
    assert r.returncode != 0 and "__asan" in r.stderr, r.stderr[-2000:]
    # ... and with it the binding loads that build
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == lib, r.stdout + r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_capi_host.py")],
                       capture_output=True, text=True, timeout=900, cwd=ROOT, env=env)
    report = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, report
    assert "passed" in r.stdout and "failed" not in r.stdout, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
