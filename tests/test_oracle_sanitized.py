"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): tests/c/oracle_sanitized.c runs the whole chain, with and
without per-pair coefficients, on a small torus; any out-of-bounds access,
leak or undefined behaviour aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_chain_is_clean_under_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]
    r = subprocess.run([cc, *flags, "-I", os.path.join(ROOT, "oracle"),
                        os.path.join(ROOT, "tests", "c", "oracle_sanitized.c"),
                        os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    if "does not come first" in run.stderr:
        pytest.skip("the sanitizer runtime cannot be first in this process environment")
    assert run.returncode == 0, run.stdout + run.stderr
    assert "oracle chain: ok" in run.stdout
