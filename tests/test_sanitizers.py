"""AddressSanitizer and UndefinedBehaviorSanitizer over host code, on the CPU:
the oracle (every entry point on seeded random inputs, exact-size buffers)
and the serving engine's host code (the race driver against the host
backend; the sanitizers are applied to host code only)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-o", str(exe),
                           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
                           os.path.join(ROOT, "oracle", "ace_oracle.c"), "-lpthread"])
    run = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1"})
    out = run.stdout + run.stderr
    assert run.returncode == 0 and "ok" in run.stdout, out[-4000:]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc absent")
def test_serving_engine_under_asan_ubsan(tmp_path):
    exe = tmp_path / "engine_sanitize"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"),
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-o", str(exe), os.path.join(ROOT, "tests", "stream_race_driver.cpp"),
           os.path.join(ROOT, "paper_2603_10242_amd", "csrc", "ace_api.hip"), "-lpthread"]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert build.returncode == 0, build.stderr[-2000:]
    # leak checking off: the HIP runtime keeps allocations until exit
    run = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    out = run.stdout + run.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert run.returncode == 0 and "bad 0" in out, out[-2000:]
