"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the library is rebuilt with the sanitizers on its host
compilation (the GPU code is unchanged) and tests/test_abi.py runs against it
in a child process with the clang ASan runtime preloaded. Every argument
check, size computation and error path of the boundary then runs
instrumented; a sanitizer report fails the child."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_under_host_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_1310_7114_amd import build as b

    lib = b.build_sanitized(verbose=False)
    env = dict(os.environ)
    env.update({"ITC_LIB_PATH": lib, "LD_PRELOAD": b.asan_runtime(),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
