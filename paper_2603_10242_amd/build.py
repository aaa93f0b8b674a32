"""Builds libace.so (hipcc, gfx950) and the workload's OpenSSL client helper, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build_libace(verbose: bool = False) -> str:
    out = os.path.join(HERE, "libace.so")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + HIP_FLAGS + ["-o", tmp, os.path.join(HERE, "csrc", "ace_api.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "not a recognized feature for this target"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, out)
    return out


def build_all(verbose: bool = False) -> list[str]:
    from . import workload
    return [build_libace(verbose), workload.build_client(force=True)]


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_2603_10242_amd import build as b  # noqa
    for p in b.build_all(verbose=True):
        print(p)
