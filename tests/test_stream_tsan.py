"""ThreadSanitizer over the serving engine's host code: the race driver
(stream_race_driver.cpp) is built together with the library sources, the
sanitizer applied to host code only, and run on the CPU with the engine's
host backend.  No GPU is used."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc absent")
def test_serving_engine_has_no_data_races(tmp_path):
    exe = tmp_path / "race_driver"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"),
           "-Xarch_host", "-fsanitize=thread",
           "-o", str(exe), os.path.join(ROOT, "tests", "stream_race_driver.cpp"),
           os.path.join(ROOT, "paper_2603_10242_amd", "csrc", "ace_api.hip"), "-lpthread"]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if build.returncode != 0 and "fsanitize" in build.stderr and "unsupported" in build.stderr:
        pytest.skip("ThreadSanitizer unavailable")
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    out = run.stdout + run.stderr
    assert "WARNING: ThreadSanitizer" not in out, out[-4000:]
    assert run.returncode == 0, out[-2000:]
    assert "bad 0" in out
