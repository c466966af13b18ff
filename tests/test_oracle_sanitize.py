"""The oracle under host sanitizers: tests/oracle_sanitize.c calls every
oracle entry point (runs of each birth model, scheme, migration setting and
asynchronous ticks; sample, MRCA bounds, reconstruction; ragged,
degenerate, past-the-horizon and invalid inputs), built with gcc's
AddressSanitizer (leak detection on) and UndefinedBehaviorSanitizer with
every report fatal."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wextra",
           "-Werror", "-o", exe, os.path.join(HERE, "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "hsga_oracle.c"), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "cannot find" in build.stderr and "asan" in build.stderr:
        pytest.skip("gcc has no sanitizer runtime here")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stderr[-4000:]
    assert run.stdout.strip() == "ok"
