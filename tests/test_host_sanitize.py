"""The library's host-only code (the site rule's closed form and the Newick
writer) under host sanitizers: tests/host_sanitize.cpp built with hipcc,
AddressSanitizer and UndefinedBehaviorSanitizer on the host side (every
report fatal), and separately with ThreadSanitizer while eight threads
build and read the rule-table cache at once.  Device code is compiled
without sanitizers and never launched: no GPU is needed."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2404_10861_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")


def build(exe, host_flags, defines=()):
    cmd = [HIPCC, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-fno-gpu-sanitize",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    for f in host_flags:
        cmd += ["-Xarch_host", f]
    cmd += list(defines) + ["-o", exe, os.path.join(HERE, "host_sanitize.cpp"),
                            os.path.join(CSRC, "hsga_rule.cpp"), os.path.join(CSRC, "hsga_tree.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if res.returncode != 0 and "cannot find" in res.stderr and "san" in res.stderr:
        pytest.skip("no sanitizer runtime here")
    assert res.returncode == 0, res.stderr[-4000:]


def run(exe, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert res.stdout.strip() == "ok"


def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_asan")
    build(exe, ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                "-fno-omit-frame-pointer"])
    run(exe, {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})


def test_rule_cache_under_tsan(tmp_path):
    exe = str(tmp_path / "host_tsan")
    build(exe, ["-fsanitize=thread"], defines=["-DTHREADS"])
    run(exe, {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
