"""Accuracy against the step size (the study of Sec. 4 on synthetic data).

The analysis in bench.py (orbital energy of a body about its parent, errors
against a small-step reference run, log2 ratios between step sizes) is run
with the oracle as the stepper on the CPU, where velocity Verlet must show
its second order (Sec. 2), and with the GPU as the stepper, where every
figure must agree with the oracle's."""
import numpy as np
import pytest

import bench
import oracle
import solar_ics as S


def oracle_stepper(s, integrator="verlet"):
    run = oracle.verlet if integrator == "verlet" else oracle.rk4

    def start(dt):
        state = [s.pos.copy(), s.vel.copy()]

        def step(k):
            if k:
                state[0], state[1] = run(state[0], state[1], s.mass, s.G, dt, k)
            return state[0], state[1], oracle.energy(state[0], state[1], s.mass, s.G)[2]
        return step
    return start


SYSTEM = dict(n=80, seed=21, n_moons=8, n_heavy=5)
SCAN = dict(dts=[0.2, 0.1, 0.05], days=40.0, sample_days=4.0, dt_ref=0.003125)


def test_moons_are_bound_to_their_parents():
    s = bench.dt_scan_system(S, **SYSTEM)
    first_moon = 1 + s.counts["major"]
    moons = np.arange(first_moon, first_moon + s.counts["moons"])
    par = s.parent
    assert (par[moons] >= 1).all() and (par[moons] <= s.counts["major"]).all()
    assert (par[np.setdiff1d(np.arange(s.n), moons)] == 0).all()
    # negative two-body orbital energy about the parent
    eps = bench.orbit_energy(s.pos, s.vel, s.mass, s.G, moons, par[moons])
    assert (eps < 0).all()


def test_dt_scan_oracle_is_second_order():
    s = bench.dt_scan_system(S, **SYSTEM)
    res = bench.dt_scan(oracle_stepper(s), s, **SCAN)
    o = res["orders_log2_ratio"]
    # halving dt divides the errors by about four
    for key in ("dE_over_E_max", "inner_major_orbit_energy_err", "inner_major_pos_err_au"):
        assert all(1.7 <= x <= 2.3 for x in o[key]), (key, o[key])
    assert o["moon_orbit_energy_err"][-1] >= 1.7, o["moon_orbit_energy_err"]
    assert res["rows"][-1]["dE_over_E_max"] < res["rows"][0]["dE_over_E_max"]


def test_dt_scan_oracle_rk4_is_fourth_order():
    """Positions converge at fourth order; the orbital and total energy errors
    of these near-Keplerian orbits converge at least as fast (about fifth
    order here).  Smaller steps would reach roundoff."""
    s = bench.dt_scan_system(S, **SYSTEM)
    res = bench.dt_scan(oracle_stepper(s, "rk4"), s, [0.4, 0.2, 0.1], 40.0, 4.0, 0.0125)
    o = res["orders_log2_ratio"]
    for key in ("inner_major_pos_err_au", "moon_pos_err_au"):
        assert all(3.7 <= x <= 4.8 for x in o[key]), (key, o[key])
    assert all(x >= 3.7 for x in o["inner_major_pos_err_au"] + o["dE_over_E_max"]
               + o["inner_major_orbit_energy_err"] + o["moon_orbit_energy_err"]), o


def test_dt_scan_rejects_a_step_that_does_not_divide_the_sampling():
    s = bench.dt_scan_system(S, **SYSTEM)
    with pytest.raises(ValueError):
        bench.dt_scan(oracle_stepper(s), s, [0.3], 4.0, 4.0, 0.1)


@pytest.mark.gpu
@pytest.mark.parametrize("integrator", ["verlet", "rk4"])
def test_dt_scan_gpu_matches_oracle(integrator):
    torch = pytest.importorskip("torch")
    nb = pytest.importorskip("paper_2112_15079_amd")
    s = bench.dt_scan_system(S, **SYSTEM)
    scan = SCAN if integrator == "verlet" else dict(dts=[0.4, 0.2, 0.1], days=40.0,
                                                    sample_days=4.0, dt_ref=0.0125)
    ref = bench.dt_scan(oracle_stepper(s, integrator), s, **scan)
    got = bench.dt_scan(bench.gpu_stepper(nb, torch, "cuda:0", s, integrator=integrator), s,
                        **scan)
    assert got["bodies"] == ref["bodies"]
    for a, b in zip(got["rows"], ref["rows"]):
        for key in ("dE_over_E_max", "inner_major_orbit_energy_err", "moon_orbit_energy_err",
                    "inner_major_pos_err_au", "moon_pos_err_au"):
            # the errors are differences of trajectories that agree to ~1e-13
            assert abs(a[key] - b[key]) <= 1e-6 * abs(b[key]) + 1e-12, (a["dt"], key, a[key], b[key])
