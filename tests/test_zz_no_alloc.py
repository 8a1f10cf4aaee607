"""nbody_verlet_run_static (no workspace, nothing allocated): its results
equal nbody_verlet_run's bit for bit, over two and more calls in a row on the
shared static scratch, the later ones on smaller systems; runs too large for
the scratch are refused with the inputs untouched.  Called through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import solar_ics as S

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2112_15079_amd")
from paper_2112_15079_amd import _capi as C  # noqa: E402

DEV = "cuda:0"


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def run_static(p, v, m, G, dt, steps, precision):
    prec = {"fp64": C.NBODY_FP64, "split": C.NBODY_SPLIT,
            "compensated": C.NBODY_SPLIT_COMPENSATED}[precision]
    small = 0.0 if prec == C.NBODY_FP64 else nb.SMALL_MASS_MSUN
    return C.load().nbody_verlet_run_static(p.data_ptr(), v.data_ptr(), m.data_ptr(),
                                            int(m.shape[0]), float(G), float(dt), int(steps),
                                            prec, small, C.stream_handle(DEV))


def run_workspace(s, steps, precision):
    p, v, m = T(s.pos), T(s.vel), T(s.mass)
    nb.verlet_run(p, v, m, s.G, s.dt, steps, precision=precision)
    return H(p), H(v)


# (system, steps, precision): the calls run in this order, each on the same
# static scratch; the first is the largest
CASES = [(lambda: S.config(1), 101, "fp64"),
         (lambda: S.solar_system(61, 2969, n_moons=10, n_heavy=19), 40, "split"),
         (lambda: S.solar_system(62, 1969, n_moons=10, n_heavy=19), 7, "compensated"),
         (lambda: S.config(0), 50, "fp64"),
         (lambda: S.config(0), 33, "split")]


def test_static_run_matches_workspace_run():
    nb.reset_caches()
    for make, steps, precision in CASES:
        s = make()
        p, v, m = T(s.pos), T(s.vel), T(s.mass)
        assert run_static(p, v, m, s.G, s.dt, steps, precision) == C.NBODY_OK, C.last_error()
        got_p, got_v = H(p), H(v)
        want_p, want_v = run_workspace(s, steps, precision)
        print(f"n={s.n} {precision} {steps} steps: bitwise "
              f"{np.array_equal(got_p, want_p) and np.array_equal(got_v, want_v)}", flush=True)
        assert np.array_equal(got_p, want_p) and np.array_equal(got_v, want_v)
    # the last FP64 case against the oracle (positions within 1e-10 per body)
    s = S.config(0)
    p, v, m = T(s.pos), T(s.vel), T(s.mass)
    assert run_static(p, v, m, s.G, s.dt, 50, "fp64") == C.NBODY_OK
    pr, _ = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, 50)
    d = np.linalg.norm(H(p) - pr, axis=0)[1:] / np.linalg.norm(pr, axis=0)[1:]
    assert d.max() <= 1e-10
    nb.reset_caches()


def test_static_run_twice_then_smaller():
    """Two calls in a row on the 10,425-body system, then one on a smaller
    system: each equals the workspace entry point's result."""
    s = S.config(1)
    for steps in (64, 64):
        p, v, m = T(s.pos), T(s.vel), T(s.mass)
        assert run_static(p, v, m, s.G, s.dt, steps, "split") == C.NBODY_OK
        want_p, want_v = run_workspace(s, steps, "split")
        assert np.array_equal(H(p), want_p) and np.array_equal(H(v), want_v)
    small = S.solar_system(63, 500, n_major=30)
    p, v, m = T(small.pos), T(small.vel), T(small.mass)
    assert run_static(p, v, m, small.G, small.dt, 21, "split") == C.NBODY_OK
    want_p, want_v = run_workspace(small, 21, "split")
    assert np.array_equal(H(p), want_p) and np.array_equal(H(v), want_v)


def test_static_run_refuses_what_does_not_fit():
    s = S.solar_system(64, 40000 - 31, n_major=30)
    p, v, m = T(s.pos), T(s.vel), T(s.mass)
    st = run_static(p, v, m, s.G, s.dt, 3, "fp64")
    assert st == C.NBODY_EUNSUPPORTED and "static scratch" in C.last_error()
    assert np.array_equal(H(p), s.pos) and np.array_equal(H(v), s.vel)
