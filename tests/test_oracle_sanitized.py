"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer and
driven through every operator, function, base scheme and the shuffle (CPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", exe,
                           os.path.join(HERE, "oracle_sanitized_driver.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    # the process environment is passed on unchanged apart from the
    # sanitizer options (ASan need not come first among loaded libraries)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout[-2000:] + r.stderr[-4000:]
