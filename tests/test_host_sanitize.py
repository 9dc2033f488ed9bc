"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

``build.build_host_sanitized()`` compiles the library with both sanitizers on its host pass
(plan creation and validation, grid-length factoring, bin choice, workspace layout, batch
grouping, the tuning caches' parsing and writing, argument checks); the CPU tests of the C
ABI and of the host logic then run against that copy in a child process with the ASan
runtime preloaded, and any sanitizer report fails them.  Leak detection is off: the Python
interpreter itself holds memory at exit.  The first run builds (about a minute); later runs
reuse the build while the sources are unchanged.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from paper_1810_09891_amd import build as B  # noqa: E402

RUNNER = r"""
import sys
sys.path.insert(0, %(root)r)
from paper_1810_09891_amd import _lib
_lib.LIB_PATH = %(lib)r
import pytest
rc = pytest.main(["-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", %(abi)r, %(host)r])
loaded = [l.split()[-1] for l in open("/proc/self/maps") if "libnfft_mi355x" in l]
print("LOADED", sorted(set(loaded)))
sys.exit(rc)
"""


def test_host_code_clean_under_sanitizers():
    rt = B.host_asan_runtime()
    if rt is None or not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc or clang ASan runtime")
    lib = B.build_host_sanitized()
    code = RUNNER % {"root": ROOT, "lib": lib, "abi": os.path.join(HERE, "test_abi_cpu.py"),
                     "host": os.path.join(HERE, "test_host.py")}
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT,
                       timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-5000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-5000:]
    assert "LOADED ['%s']" % lib in out, out[-2000:]
