"""The CPU oracle built with gcc's address, leak and undefined-behaviour sanitizers and run
through every exported function on small frames, error paths included (tests/oracle_selfcheck.c).
CPU only; skipped where the sanitizer runtime is missing."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "orc_selfcheck")
        cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-ffp-contract=off", "-o", exe, os.path.join(HERE, "oracle_selfcheck.c"),
               os.path.join(ROOT, "oracle", "gsc_oracle.c"), "-lm"]
        build = subprocess.run(cmd, capture_output=True, text=True)
        if build.returncode != 0:
            if "asan" in build.stderr or "ubsan" in build.stderr:
                pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
            raise AssertionError(build.stderr)
        # (the sanitizer runtime need not come first among preloaded libraries)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert run.returncode == 0, run.stdout + run.stderr
        assert "oracle self-check ok" in run.stdout
