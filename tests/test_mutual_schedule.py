"""The each-pair-once pass's workgroup decode, checked on the CPU.

tests/host/mutual_schedule.hip includes the kernel source and runs its
host-and-device decode on the host for 2,500 sizes and two shapes: every
range pair (g, r), r >= g, runs once, whole or as both halves of a split
pair (sub-phases 0-1 and 2-3, each over all its targets and sources), and
every body receives each of its partial slots exactly once (both halves'
targets and reactions, the diagonal workgroup's zero-filled extra slots).
Nothing runs on a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


def test_mutual_decode_covers_every_pair_and_slot_once(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "mutual_schedule")
    build = subprocess.run(
        [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "paper_2112_15079_amd", "csrc"),
         "-I", os.path.join(ROOT, "include"), "-o", exe,
         os.path.join(ROOT, "tests", "host", "mutual_schedule.hip")],
        capture_output=True, text=True, timeout=600)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(run.stdout[-3000:])
    assert run.returncode == 0 and "ok (" in run.stdout, run.stdout[-2000:]
    # the headline size: 768 whole pairs, 93 split over three super-diagonals
    assert "n=10425 tile(4,4) R=41 pairs=861 F=768 D=3 kD=14 grid=954 slots=47" in run.stdout
