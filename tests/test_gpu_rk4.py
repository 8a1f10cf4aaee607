"""GPU fourth-order Runge-Kutta (the alternative integrator of Sec. 2)
against the oracle's, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import solar_ics as S

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2112_15079_amd")
DEV = "cuda:0"


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm(a - b, axis=0)
    r = np.linalg.norm(b, axis=0)
    return float(np.max(np.where(r > 0, d / np.where(r > 0, r, 1), d)))


@pytest.fixture(autouse=True)
def _fresh():
    nb.reset_caches()
    yield
    nb.reset_caches()


@pytest.mark.parametrize("steps", [1, 2, 17, 40, 365])
def test_rk4_workload0_matches_oracle(steps):
    """365 steps (36.5 days) of the 131-body system; 40 and 365 steps replay
    captured 16-step graphs plus a remainder."""
    s = S.config(0)
    pr, vr = oracle.rk4(s.pos, s.vel, s.mass, s.G, s.dt, steps)
    p, v = T(s.pos), T(s.vel)
    nb.rk4_run(p, v, T(s.mass), s.G, s.dt, steps)
    ep, ev = rel(H(p), pr), rel(H(v), vr)
    print(f"rk4 {steps} steps: pos {ep:.2e} vel {ev:.2e}", flush=True)
    assert ep <= 1e-10 and ev <= 1e-9


@pytest.mark.parametrize("tile", [None, (1, 1, 1, 0), (2, 4, 3, 0), (1, 2, 7, 1), (1, 4, 2, 2),
                                  (1, 16, 5, 3), (1, 8, 1, 4), (1, 4, 1, 5), (2, 2, 1, 5),
                                  (2, 4, 1, 5), (4, 4, 1, 5)])
@pytest.mark.parametrize("n", [1, 3, 65, 300, 1031])
def test_rk4_shapes_and_tiles(n, tile):
    """Ragged sizes over the force tiles; whole-step tiles (variants 3, 4)
    fall back to a force-only tile."""
    s = S.solar_system(80 + n, max(n - 31, 0), n_major=min(30, max(n - 1, 0)))
    if tile is not None:
        if tile[3] == 3 and n > 512:
            pytest.skip("the single-workgroup variant holds at most 512 bodies")
        nb.set_tile(0, "fp64", s.n, *tile)
    pr, vr = oracle.rk4(s.pos, s.vel, s.mass, s.G, 0.1, 20)
    p, v = T(s.pos), T(s.vel)
    nb.rk4_run(p, v, T(s.mass), s.G, 0.1, 20)
    assert rel(H(p), pr) <= 1e-12 and rel(H(v), vr) <= 1e-11


def test_rk4_split_matches_oracle():
    s = S.config(0)
    pr, vr = oracle.rk4(s.pos, s.vel, s.mass, s.G, s.dt, 100)
    p, v = T(s.pos), T(s.vel)
    nb.rk4_run(p, v, T(s.mass), s.G, s.dt, 100, precision="split")
    assert rel(H(p), pr) <= 1e-9 and rel(H(v), vr) <= 1e-8


def test_rk4_zero_steps_resume_and_determinism():
    s = S.config(0)
    m = T(s.mass)
    p, v = T(s.pos), T(s.vel)
    nb.rk4_run(p, v, m, s.G, s.dt, 0)
    assert np.array_equal(H(p), s.pos) and np.array_equal(H(v), s.vel)
    outs = []
    for split in ([100], [100], [33, 67], [1, 98, 1]):
        p, v = T(s.pos), T(s.vel)
        for k in split:
            nb.rk4_run(p, v, m, s.G, s.dt, k)
        outs.append((H(p), H(v)))
    for p, v in outs[1:]:
        assert np.array_equal(p, outs[0][0]) and np.array_equal(v, outs[0][1])


def test_rk4_fourth_order_on_the_gpu():
    """Halving dt divides the GPU run's error against a fine reference run by
    about 16 (the oracle pins the same property against Kepler)."""
    s = S.solar_system(97, 40, n_major=12)   # no moons: every orbit resolved at dt = 0.8
    m = T(s.mass)

    def run(dt, steps):
        p, v = T(s.pos), T(s.vel)
        nb.rk4_run(p, v, m, s.G, dt, steps)
        return H(p)

    ref = run(0.05, 800)
    errs = [np.abs(run(dt, int(round(40 / dt))) - ref).max() for dt in (0.8, 0.4, 0.2)]
    orders = [np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])]
    print(f"rk4 errors {errs}, orders {orders}", flush=True)
    assert all(3.5 <= o <= 4.6 for o in orders)


def test_rk4_nonfinite_flag():
    pos = np.array([[0.0, 1.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    nb.get_flags(DEV, clear=True)
    p, v = T(pos), T(np.zeros((3, 3)))
    nb.rk4_run(p, v, T(np.ones(3)), 1.0, 0.01, 2)
    assert nb.get_flags(DEV, clear=True) & 1


def test_rk4_10425_bodies_matches_oracle():
    """The 10,425-body workload, 5 RK4 steps with the default (each-pair-once)
    force pass, against the oracle's RK4."""
    s = S.config(1)
    pr, vr = oracle.rk4(s.pos, s.vel, s.mass, s.G, s.dt, 5)
    p, v = T(s.pos), T(s.vel)
    nb.rk4_run(p, v, T(s.mass), s.G, s.dt, 5)
    ep, ev = rel(H(p), pr), rel(H(v), vr)
    print(f"rk4 n={s.n} 5 steps: pos {ep:.2e} vel {ev:.2e}", flush=True)
    assert ep <= 1e-10 and ev <= 1e-9
