"""When the waves of the FP64 each-pair-once force pass (shape (4, 4),
N = 10,425) enter, start their sweep (sources and targets staged in LDS),
end it and exit, and on which CU and SIMD (test instrument
tests/host/libtimelineprobe.so, built by the repository's build(): the
library's own workgroup body with its marks recording s_memrealtime).  It
splits the pass's issue efficiency into the start (every workgroup loads at
once), the sweep, and the end of the partly filled last round, per CU.  The
records are checked for consistency; the figures are printed."""
import collections
import ctypes
import os

import numpy as np
import pytest

import solar_ics as S

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "tests", "host", "libtimelineprobe.so")


def q(x):
    x = np.asarray(x, dtype=np.float64)
    return (f"mean {x.mean():6.2f}  p10 {np.percentile(x, 10):6.2f}  p50 {np.median(x):6.2f}  "
            f"p90 {np.percentile(x, 90):6.2f}  max {x.max():6.2f}")


def test_force_pass_wave_timeline():
    torch = pytest.importorskip("torch")
    assert torch.cuda.is_available()
    assert os.path.exists(LIB), f"{LIB} is missing: run __graft_entry__.build()"
    lib = ctypes.CDLL(LIB)
    lib.timeline_probe_force.argtypes = [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
        ctypes.c_int64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    lib.timeline_probe_force.restype = ctypes.c_int
    s = S.config(1)
    pos = np.ascontiguousarray(s.pos, dtype=np.float64)
    gm = np.ascontiguousarray(s.G * s.mass, dtype=np.float64)
    out = np.zeros(4096 * 32, dtype=np.uint64)
    grid, us = ctypes.c_int(0), ctypes.c_double(0.0)
    rc = lib.timeline_probe_force(pos.ctypes.data, gm.ctypes.data, s.n, 1500, out.ctypes.data,
                                  out.size, ctypes.byref(grid), ctypes.byref(us))
    assert rc == 0
    rec = out[: 32 * grid.value].reshape(grid.value, 4, 8).astype(np.int64)
    t = rec[:, :, :4]
    assert (t > 0).all(), "every wave records its four marks"
    assert (np.diff(t, axis=2) >= 0).all(), "entry <= sweep start <= sweep end <= exit"
    base = t[:, :, 0].min()
    t = (t - base) / 100.0   # the 100 MHz counter, in us
    span = t[:, :, 3].max()
    assert span <= 1.5 * us.value + 5.0
    code = rec[:, 0, 6]
    half = code % 10 - 1
    whole = half < 0
    hw, xcc = rec[:, :, 4], rec[:, :, 5] & 0xF
    simd = (hw >> 4) & 3
    four = np.mean([len(set(x)) == 4 for x in simd.tolist()])
    cu = [(int(a), int(b)) for a, b in zip(xcc[:, 0], (hw[:, 0] >> 8) & 0xFF)]
    print(f"n={s.n}: {grid.value} workgroups ({whole.sum()} whole range pairs, "
          f"{(~whole).sum()} halves) on {len(set(cu))} CUs; recorded launch {us.value:.2f} us "
          f"(events), first entry to last exit {span:.2f} us; workgroups whose four waves "
          f"ran on four SIMDs: {100 * four:.0f} %")
    print(f"entry                      {q(t[:, :, 0].ravel())}")
    print(f"sweep start                {q(t[:, :, 1].ravel())}")
    print(f"staging (entry to start)   {q((t[:, :, 1] - t[:, :, 0]).ravel())}")
    print(f"sweep, whole pairs         {q((t[whole][:, :, 2] - t[whole][:, :, 1]).ravel())}")
    print(f"sweep, halves              {q((t[~whole][:, :, 2] - t[~whole][:, :, 1]).ravel())}")
    print(f"sweep end to exit          {q((t[:, :, 3] - t[:, :, 2]).ravel())}")
    print(f"exit                       {q(t[:, :, 3].ravel())}")
    by_cu = collections.defaultdict(list)
    for b, c in enumerate(cu):
        by_cu[c].append(b)
    classes = collections.defaultdict(list)
    for c, wgs in by_cu.items():
        nw = int(whole[wgs].sum())
        nh = len(wgs) - nw
        classes[(nw, nh)].append(t[wgs][:, :, 3].max())
    for (nw, nh), ends in sorted(classes.items(), reverse=True):
        print(f"CUs holding {nw} whole pair(s) and {nh} half(s): {len(ends):3d}, "
              f"last exit {q(ends)}")
    assert sum(len(v) for v in classes.values()) == len(set(cu))
