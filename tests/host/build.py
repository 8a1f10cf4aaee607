"""Builds the GPU test instruments of tests/host (gfx950): libclockprobe.so
from clock_probe.hip and libtimelineprobe.so from timeline_probe.hip.  Called
by the repository's build() beside the library's own build; nothing here is
part of the library."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLOCK_PROBE = os.path.join(HERE, "libclockprobe.so")
TIMELINE_PROBE = os.path.join(HERE, "libtimelineprobe.so")


def _build_one(src: str, out: str, verbose: bool) -> str:
    tmp = out + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2112_15079_amd", "csrc"),
           "-o", tmp, os.path.join(HERE, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


def build(verbose: bool = False) -> str:
    _build_one("timeline_probe.hip", TIMELINE_PROBE, verbose)
    return _build_one("clock_probe.hip", CLOCK_PROBE, verbose)


if __name__ == "__main__":
    build(verbose=True)
