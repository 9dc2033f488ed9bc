"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (with leak
detection): ``sanitize_oracle.c`` drives every exported routine of ``oracle/nfft_oracle.c``
on small inputs (every window, d = 1..3, power-of-two and other grid lengths, nodes outside
[-1/2, 1/2), stencils wider than the grid), built with gcc and ``-fno-sanitize-recover``, so
that any out-of-bounds access, leak, overflow or other undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sanitize_oracle")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", os.path.join(ROOT, "oracle", "nfft_oracle.c"),
           os.path.join(HERE, "sanitize_oracle.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("no sanitizer runtime for gcc: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "Sanitizer" not in out, out[-4000:]
    assert out.strip().splitlines()[-1] == "done"
    assert out.count(" E2 ") == 24  # 4 windows x 6 plan shapes
