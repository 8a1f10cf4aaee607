"""The shader clock under the FP64 each-pair-once force pass (test
instrument tests/host/libclockprobe.so, built by the repository's build():
the library's own workgroup body with s_memtime / s_memrealtime read by each
workgroup).  The roofline's FP64 peak (78.6 TFLOP/s) assumes 2.4 GHz; this
measures the clock the chip holds while running the pass, from idle through
~1.2 s of back-to-back launches at N = 10,425, so that the kernel's fraction
of peak can be split into clock and issue efficiency."""
import ctypes
import os

import numpy as np
import pytest

import solar_ics as S

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "tests", "host", "libclockprobe.so")


def test_sustained_shader_clock_under_force_pass():
    torch = pytest.importorskip("torch")
    assert torch.cuda.is_available()
    assert os.path.exists(LIB), f"{LIB} is missing: run __graft_entry__.build()"
    lib = ctypes.CDLL(LIB)
    D = ctypes.POINTER(ctypes.c_double)
    lib.clock_probe_force.argtypes = [D, D, ctypes.c_int64, ctypes.c_int, ctypes.c_int, D, D, D, D]
    lib.clock_probe_force.restype = ctypes.c_int
    s = S.config(1)
    pos = np.ascontiguousarray(s.pos, dtype=np.float64)
    gm = np.ascontiguousarray(s.G * s.mass, dtype=np.float64)
    batches, per = 24, 50
    out = [np.zeros(batches) for _ in range(4)]
    ptr = lambda a: a.ctypes.data_as(D)
    rc = lib.clock_probe_force(ptr(pos), ptr(gm), s.n, batches, per, *[ptr(o) for o in out])
    assert rc == 0
    us, mean, lo, hi = out
    for b in range(batches):
        print(f"batch {b:2d} (launches {b * per + 1}-{(b + 1) * per}): {us[b]:.2f} us per launch; "
              f"sclk mean {mean[b]:.3f} GHz (workgroups {lo[b]:.3f} .. {hi[b]:.3f})", flush=True)
    tail = mean[batches // 2:]
    print(f"sustained (second half): sclk {tail.mean():.3f} GHz, {us[batches // 2:].mean():.2f} us "
          f"per launch; first batch {mean[0]:.3f} GHz, {us[0]:.2f} us", flush=True)
    assert np.all((mean > 0.5) & (mean < 3.0))
    assert np.all(lo <= mean + 1e-9) and np.all(mean <= hi + 1e-9)
