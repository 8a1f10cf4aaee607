"""Pins for the CPU oracle: each test checks it against something other than
itself (a closed form, an invariant of Eq. (1), a published orbit, a
derivative taken by a different method).  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
import solar_ics as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0))


def _rand_rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q


# ---------------------------------------------------------------------------
# Eq. (1)
# ---------------------------------------------------------------------------

def _potential_complex(pos, mass, G):
    """U = -sum_{i<j} G m_i m_j / |r_i - r_j| for complex positions."""
    n = mass.shape[0]
    U = 0.0 + 0.0j
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[:, j] - pos[:, i]
            U = U - G * mass[i] * mass[j] / np.sqrt(np.sum(d * d))
    return U


def _accel_from_potential(pos, mass, G, h=1e-30):
    """a_p = -(1/m_p) dU/dr_p by complex-step differentiation (exact to
    rounding, no subtraction), an independent route to Eq. (1)."""
    n = mass.shape[0]
    acc = np.zeros((3, n))
    for p in range(n):
        for k in range(3):
            z = pos.astype(np.complex128)
            z[k, p] += 1j * h
            acc[k, p] = -_potential_complex(z, mass, G).imag / h / mass[p]
    return acc


@pytest.mark.parametrize("seed,n", [(0, 2), (1, 3), (2, 5), (3, 8)])
def test_accel_is_gradient_of_potential(seed, n):
    pos, _, mass = S.random_cluster(seed, n)
    a = oracle.accel(pos, mass, 0.7)
    ref = _accel_from_potential(pos, mass, 0.7)
    assert _rel(a, ref) < 1e-14


@pytest.mark.parametrize("seed,n", [(4, 4), (5, 8)])
def test_accel_naive_double_loop(seed, n):
    """A textbook pair loop over unordered pairs, applying Newton's third law."""
    pos, _, mass = S.random_cluster(seed, n)
    G = 1.3
    ref = np.zeros((3, n))
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[:, j] - pos[:, i]
            f = G / np.linalg.norm(d) ** 3 * d      # field factor without masses
            ref[:, i] += mass[j] * f
            ref[:, j] -= mass[i] * f
    assert _rel(oracle.accel(pos, mass, G), ref) < 1e-14


def test_two_body_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(20):
        d = rng.normal(size=3) * 10 ** rng.uniform(-3, 2)
        r1 = rng.normal(size=3)
        pos = np.stack([r1, r1 + d], axis=1)
        mass = np.array([rng.uniform(0.1, 2.0), rng.uniform(1e-12, 1.0)])
        G = 2.9591220828e-4
        a = oracle.accel(pos, mass, G)
        d = pos[:, 1] - pos[:, 0]          # the separation as stored
        dn = np.linalg.norm(d)
        want1 = G * mass[1] / dn ** 2 * d / dn
        want2 = -G * mass[0] / dn ** 2 * d / dn
        assert np.linalg.norm(a[:, 0] - want1) <= 2e-15 * np.linalg.norm(want1)
        assert np.linalg.norm(a[:, 1] - want2) <= 2e-15 * np.linalg.norm(want2)
        # antisymmetry of the pair force: m1 a1 + m2 a2 = 0
        f = mass[0] * a[:, 0] + mass[1] * a[:, 1]
        assert np.linalg.norm(f) <= 8 * 2.2e-16 * mass[0] * np.linalg.norm(a[:, 0])


def test_lagrange_equilateral_triangle():
    """Three equal masses at the corners of a triangle of side s: each
    acceleration has magnitude sqrt(3) G m / s^2 and points at the centroid."""
    rng = np.random.default_rng(3)
    s, m, G = 0.37, 0.8, 1.9
    tri = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3) / 2, 0.0], [-0.5, -np.sqrt(3) / 2, 0.0]]).T
    tri *= s / np.sqrt(3)
    R = _rand_rot(rng)
    c = rng.normal(size=(3, 1))
    pos = R @ tri + c
    a = oracle.accel(pos, np.full(3, m), G)
    mag = np.sqrt(3) * G * m / s ** 2
    for p in range(3):
        want = mag * (c[:, 0] - pos[:, p]) / np.linalg.norm(c[:, 0] - pos[:, p])
        assert np.linalg.norm(a[:, p] - want) <= 4e-15 * mag


def test_total_force_vanishes():
    pos, _, mass = S.random_cluster(7, 300)
    a = oracle.accel(pos, mass, 1.0)
    F = (mass * a).sum(axis=1)
    scale = np.abs(mass * a).sum()
    assert np.linalg.norm(F) <= 1e-14 * scale


def test_accel_non_finite_for_coincident_bodies():
    """No softening: two distinct bodies at one point give non-finite values,
    while a third body elsewhere stays finite."""
    pos = np.array([[0.0, 1.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    a = oracle.accel(pos, np.ones(3), 1.0)
    assert np.isfinite(a[:, 0]).all()
    assert not np.isfinite(a[:, 1]).all() and not np.isfinite(a[:, 2]).all()


def test_accel_threads_do_not_change_result():
    s = S.config(0)
    t = oracle.get_threads()
    try:
        oracle.set_threads(1)
        a1 = oracle.accel(s.pos, s.mass, s.G)
        oracle.set_threads(max(2, t))
        a2 = oracle.accel(s.pos, s.mass, s.G)
    finally:
        oracle.set_threads(t)
    assert np.array_equal(a1, a2)


# ---------------------------------------------------------------------------
# Eqs. (3)-(4)
# ---------------------------------------------------------------------------

def _circular_pair(m1, m2, a, G, rng):
    """Two bodies on a circular orbit of separation a, centre-of-mass frame,
    in a random plane.  Returns pos, vel, mass, omega."""
    M = m1 + m2
    w = np.sqrt(G * M / a ** 3)
    R = _rand_rot(rng)
    d = R[:, 0] * a
    vrel = R[:, 1] * w * a
    pos = np.stack([-m2 / M * d, m1 / M * d], axis=1)
    vel = np.stack([-m2 / M * vrel, m1 / M * vrel], axis=1)
    return pos, vel, np.array([m1, m2]), w


def test_circular_orbit_closes_with_second_order_error():
    """After one period the orbit closes to (2 pi / 3)(omega dt)^2 a
    (leading-order phase lag of velocity Verlet on a circular orbit), and the
    error falls as dt^2."""
    rng = np.random.default_rng(21)
    G = 2.9591220828e-4
    errs = []
    for nstep in (500, 1000, 2000):
        pos, vel, mass, w = _circular_pair(1.0, 3e-6, 1.0, G, rng)
        T = 2 * np.pi / w
        dt = T / nstep
        p, v = oracle.verlet(pos, vel, mass, G, dt, nstep)
        e = np.linalg.norm((p[:, 1] - p[:, 0]) - (pos[:, 1] - pos[:, 0]))
        bound = (2 * np.pi / 3) * (w * dt) ** 2
        assert e <= 1.05 * bound
        assert e >= 0.95 * bound
        errs.append(e)
    order = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert all(abs(o - 2.0) < 0.05 for o in order)


def test_gaussian_year():
    """A massless body at 1 AU about 1 Msun with G = k^2 returns to its start
    after 2 pi / k days, within the second-order bound above."""
    g = json.load(open(os.path.join(GOLD, "gaussian_year.json")))
    k, G, T = g["k"], g["G"], g["gaussian_year_days"]
    assert abs(k * k - G) < 1e-14
    assert abs(2 * np.pi / k - T) < 1e-6
    nstep = 3653
    dt = T / nstep
    pos = np.array([[0.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    vel = np.array([[0.0, 0.0], [0.0, k], [0.0, 0.0]])
    p, v = oracle.verlet(pos, vel, np.array([1.0, 0.0]), G, dt, nstep)
    err = np.linalg.norm(p[:, 1] - pos[:, 1])
    assert err <= 1.05 * (2 * np.pi / 3) * (k * dt) ** 2 + 1e-9
    assert np.array_equal(p[:, 0], pos[:, 0])    # the Sun feels no massless body


def test_figure_eight_closes():
    g = json.load(open(os.path.join(GOLD, "figure_eight.json")))
    pos = np.array(g["pos"]).T
    vel = np.array(g["vel"]).T
    mass = np.array(g["mass"])
    nstep = 21000
    dt = g["period"] / nstep
    p, v = oracle.verlet(pos, vel, mass, g["G"], dt, nstep)
    # 8-digit initial data and an O(dt^2) scheme: closure to about 1e-6
    assert np.max(np.abs(p - pos)) < 2e-6
    assert np.max(np.abs(v - vel)) < 2e-6
    # a choreography: after a third of the period the bodies have moved on
    # to one another's starting points
    p3, _ = oracle.verlet(pos, vel, mass, g["G"], dt, nstep // 3)
    assert np.max(np.abs(p3 - pos[:, [2, 0, 1]])) < 2e-6


def test_time_reversibility():
    s = S.config(0)
    p, v = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, 3650)
    p2, v2 = oracle.verlet(p, -v, s.mass, s.G, s.dt, 3650)
    rel = np.linalg.norm(p2 - s.pos, axis=0)[1:] / np.linalg.norm(s.pos, axis=0)[1:]
    assert rel.max() < 1e-11
    assert np.linalg.norm(p2[:, 0]) < 1e-11


def test_momenta_conserved():
    s = S.config(0)
    P0, L0 = oracle.momenta(s.pos, s.vel, s.mass)
    p, v = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, 3650)
    P1, L1 = oracle.momenta(p, v, s.mass)
    scaleP = np.sum(s.mass * np.linalg.norm(s.vel, axis=0))
    scaleL = np.sum(s.mass * np.linalg.norm(np.cross(s.pos.T, s.vel.T), axis=1))
    assert np.linalg.norm(P1 - P0) <= 1e-12 * scaleP
    assert np.linalg.norm(L1 - L0) <= 1e-12 * scaleL


def _energy_series(s, dt, days, every_days):
    E0 = oracle.energy(s.pos, s.vel, s.mass, s.G)[2]
    p, v = s.pos, s.vel
    k = int(round(every_days / dt))
    out = []
    for _ in range(int(round(days / every_days))):
        p, v = oracle.verlet(p, v, s.mass, s.G, dt, k)
        out.append((oracle.energy(p, v, s.mass, s.G)[2] - E0) / abs(E0))
    return np.array(out)


def test_energy_bounded_not_secular():
    """Sec. 2 / Sec. 4: Verlet's energy error at dt = 0.1 day oscillates with
    bounded amplitude over 10 years; explicit Euler drifts by orders of
    magnitude more within one year."""
    s = S.config(0)
    err = _energy_series(s, 0.1, 3650.0, 36.5)
    first, second = np.abs(err[:50]).max(), np.abs(err[50:]).max()
    assert second <= 2.0 * first
    assert np.abs(err).max() < 1e-5
    assert err.min() < 0.5 * err.max()        # it swings, it does not only grow
    pe, ve = oracle.euler(s.pos, s.vel, s.mass, s.G, 0.1, 3650)
    E0 = oracle.energy(s.pos, s.vel, s.mass, s.G)[2]
    eul = abs(oracle.energy(pe, ve, s.mass, s.G)[2] - E0) / abs(E0)
    assert eul >= 1e3 * np.abs(err[:10]).max()


def test_energy_error_second_order():
    s = S.config(0)
    amp = [np.abs(_energy_series(s, dt, 365.0, 18.25)).max() for dt in (0.2, 0.1, 0.05)]
    r1, r2 = amp[0] / amp[1], amp[1] / amp[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5


def test_energy_closed_form_circular():
    rng = np.random.default_rng(5)
    G = 2.9591220828e-4
    pos, vel, mass, _ = _circular_pair(1.0, 1e-3, 5.2, G, rng)
    K, U, E = oracle.energy(pos, vel, mass, G)
    want = -G * mass[0] * mass[1] / (2 * 5.2)
    assert abs(E - want) <= 1e-14 * abs(want)
    assert abs(U + G * mass[0] * mass[1] / 5.2) <= 1e-15 * abs(U)


def test_kdk_form_matches_literal_form():
    """Kick-drift-kick with one force pass per step equals Eqs. (3)-(4) in
    exact arithmetic; in FP64 the two agree to roundoff over a year."""
    s = S.config(0)
    dt, steps = s.dt, 3650
    p, v = s.pos.copy(), s.vel.copy()
    a = oracle.accel(p, s.mass, s.G)
    for _ in range(steps):
        v = v + 0.5 * dt * a
        p = p + dt * v
        a = oracle.accel(p, s.mass, s.G)
        v = v + 0.5 * dt * a
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, dt, steps)
    rel = np.linalg.norm(p - pr, axis=0) / np.linalg.norm(pr, axis=0)
    assert rel.max() < 1e-12


# ---------------------------------------------------------------------------
# Derivatives
# ---------------------------------------------------------------------------

def _accel_complex(pos, mass, G):
    """Eq. (1) in complex arithmetic, vectorised (for complex-step JVPs)."""
    d = pos[:, None, :] - pos[:, :, None]           # d[:, p, j] = r_j - r_p
    r2 = np.sum(d * d, axis=0)
    n = mass.shape[0]
    r2 = r2 + np.eye(n)                             # self-pair placeholder
    w = G * mass[None, :] / (r2 * np.sqrt(r2))
    w = w * (1 - np.eye(n))
    return np.sum(w[None] * d, axis=2)


def test_vjp_against_complex_step_jvp():
    rng = np.random.default_rng(8)
    n, G = 7, 1.1
    pos, _, mass = S.random_cluster(8, n)
    u = rng.normal(size=(3, n))
    jr, jm = oracle.vjp(pos, mass, u, G)
    h = 1e-30
    for _ in range(4):
        dr = rng.normal(size=(3, n))
        dm = rng.normal(size=n)
        jvp_r = _accel_complex(pos + 1j * h * dr, mass.astype(complex), G).imag / h
        jvp_m = _accel_complex(pos.astype(complex), mass + 1j * h * dm, G).imag / h
        lhs_r, rhs_r = np.sum(u * jvp_r), np.sum(jr * dr)
        lhs_m, rhs_m = np.sum(u * jvp_m), np.sum(jm * dm)
        assert abs(lhs_r - rhs_r) <= 1e-13 * np.sum(np.abs(u * jvp_r)) + 1e-300
        assert abs(lhs_m - rhs_m) <= 1e-13 * np.sum(np.abs(u * jvp_m)) + 1e-300


def test_vjp_invariants():
    rng = np.random.default_rng(9)
    n, G = 40, 0.9
    pos, _, mass = S.random_cluster(9, n)
    u = rng.normal(size=(3, n))
    jr, jm = oracle.vjp(pos, mass, u, G)
    # translation invariance: sum_q (J^T u)_q = 0
    assert np.linalg.norm(jr.sum(axis=1)) <= 1e-13 * np.abs(jr).sum()
    # Eq. (1) is homogeneous of degree 1 in the masses: sum_q m_q dm_q = u . a
    a = oracle.accel(pos, mass, G)
    assert abs(np.sum(mass * jm) - np.sum(u * a)) <= 1e-13 * np.sum(np.abs(u * a))


def test_tangent_against_finite_differences():
    rng = np.random.default_rng(12)
    s = S.solar_system(12, 2, n_major=2)
    n, G, dt, steps = s.n, s.G, 0.1, 200
    pos, vel, mass = s.pos, s.vel, s.mass
    dr, dv, dm = rng.normal(size=(3, n)), rng.normal(size=(3, n)) * 0.01, rng.normal(size=n) * mass
    p, v, tp, tv = oracle.tangent(pos, vel, mass, G, dt, steps, dr, dv, dm)
    pr, vr = oracle.verlet(pos, vel, mass, G, dt, steps)
    assert np.array_equal(p, pr) or np.max(np.abs(p - pr)) < 1e-13
    h = 1e-6
    pp, vp = oracle.verlet(pos + h * dr, vel + h * dv, mass + h * dm, G, dt, steps)
    pm, vm = oracle.verlet(pos - h * dr, vel - h * dv, mass - h * dm, G, dt, steps)
    fd_p, fd_v = (pp - pm) / (2 * h), (vp - vm) / (2 * h)
    assert np.max(np.abs(fd_p - tp)) <= 1e-6 * np.max(np.abs(tp))
    assert np.max(np.abs(fd_v - tv)) <= 1e-6 * np.max(np.abs(tv))


def test_adjoint_dot_product_with_tangent():
    """<lambda_n, dx_n> = <lambda_0, dx_0> for every direction: the reverse
    sweep is the exact transpose of the forward-mode derivative."""
    rng = np.random.default_rng(13)
    s = S.solar_system(13, 2, n_major=2)
    n, G, dt, steps = s.n, s.G, 0.1, 200
    pos, vel, mass = s.pos, s.vel, s.mass
    lr, lv = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    gr, gv, gm = oracle.adjoint(pos, vel, mass, G, dt, steps, lr, lv)
    for _ in range(6):
        dr, dv, dm = rng.normal(size=(3, n)), rng.normal(size=(3, n)), rng.normal(size=n)
        _, _, tp, tv = oracle.tangent(pos, vel, mass, G, dt, steps, dr, dv, dm)
        lhs = np.sum(lr * tp) + np.sum(lv * tv)
        rhs = np.sum(gr * dr) + np.sum(gv * dv) + np.sum(gm * dm)
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sum(np.abs(gr * dr)) + np.sum(np.abs(gv * dv)))


def test_adjoint_against_finite_differences_solar():
    """Sum of squared final asteroid offsets from a shifted target run.

    Central differences resolve only entries whose effect on the final state
    is far above FP64 roundoff: asteroid positions and velocities and the
    heaviest major body's mass.  (A 1e20 kg body's mass moves the final
    positions by less than one ulp; for such entries the dot-product test
    against the forward-mode tangent is the pin.)"""
    s = S.solar_system(31, 12, n_major=4, steps=200)
    steps = 200
    tgt, _ = oracle.verlet(s.pos + 1e-3, s.vel, s.mass, s.G, s.dt, steps)
    first = 5

    def loss(p0, v0, m):
        p, _ = oracle.verlet(p0, v0, m, s.G, s.dt, steps)
        return np.sum((p[:, first:] - tgt[:, first:]) ** 2)

    p, v = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, steps)
    lam_r = np.zeros_like(p)
    lam_r[:, first:] = 2 * (p[:, first:] - tgt[:, first:])
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, s.dt, steps, lam_r, np.zeros_like(p))
    for (k, q) in [(0, 6), (1, 9), (2, 15), (0, 12)]:
        h = 1e-6 * max(abs(s.pos[k, q]), 1.0)
        e = np.zeros_like(s.pos)
        e[k, q] = h
        fd = (loss(s.pos + e, s.vel, s.mass) - loss(s.pos - e, s.vel, s.mass)) / (2 * h)
        assert abs(fd - gr[k, q]) <= 1e-6 * abs(fd)
        hv = 1e-6 * max(abs(s.vel[k, q]), 0.01)
        ev = np.zeros_like(s.vel)
        ev[k, q] = hv
        fdv = (loss(s.pos, s.vel + ev, s.mass) - loss(s.pos, s.vel - ev, s.mass)) / (2 * hv)
        assert abs(fdv - gv[k, q]) <= 1e-6 * abs(fdv)
    q = int(np.argmax(s.mass[1:])) + 1
    hm = 1e-4 * s.mass[q]
    em = np.zeros_like(s.mass)
    em[q] = hm
    fdm = (loss(s.pos, s.vel, s.mass + em) - loss(s.pos, s.vel, s.mass - em)) / (2 * hm)
    assert abs(fdm - gm[q]) <= 1e-5 * abs(fdm)


def test_accel_against_extended_precision():
    """Eq. (1) is an exact sum: the oracle must sit within a few ulp of it
    even for a moon whose parent's term dominates 10^4 tiny asteroid terms.
    The reference re-evaluates the sum in x87 80-bit extended precision."""
    s = S.config(1)
    if np.finfo(np.longdouble).nmant < 63:
        pytest.skip("no extended precision long double on this platform")
    rng = np.random.default_rng(2)
    idx = np.unique(np.concatenate([[0, 1, 30], np.arange(31, 131), [131, 149, s.n - 1],
                                    rng.choice(s.n, 40, replace=False)]))
    got = oracle.accel_targets(s.pos, s.mass, s.G, idx)
    pos = s.pos.astype(np.longdouble)
    m = s.mass.astype(np.longdouble)
    G = np.longdouble(s.G)
    worst = 0.0
    for k, p in enumerate(idx):
        d = pos - pos[:, p:p + 1]
        r2 = np.sum(d * d, axis=0)
        r2[p] = 1
        w = G * m / (r2 * np.sqrt(r2))
        w[p] = 0
        a = (w * d).sum(axis=1)
        worst = max(worst, float(np.linalg.norm(got[:, k] - a.astype(np.float64))
                                 / np.linalg.norm(a.astype(np.float64))))
    assert worst <= 2e-15


# ---------------------------------------------------------------------------
# The classical fourth-order Runge-Kutta method (the higher-order alternative
# of Sec. 2), pinned to exact two-body solutions.

def test_rk4_circular_orbit_fourth_order():
    """After one period the circular orbit closes up to an error that falls
    as dt^4 (halving dt divides it by 16)."""
    rng = np.random.default_rng(23)
    G = 2.9591220828e-4
    errs = []
    for nstep in (200, 400, 800):
        pos, vel, mass, w = _circular_pair(1.0, 3e-6, 1.0, G, rng)
        T = 2 * np.pi / w
        p, v = oracle.rk4(pos, vel, mass, G, T / nstep, nstep)
        errs.append(np.linalg.norm((p[:, 1] - p[:, 0]) - (pos[:, 1] - pos[:, 0])))
    order = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    # (the next term still shows at these steps: 4.11, then 4.05)
    assert all(abs(o - 4.0) < 0.15 for o in order), order
    assert errs[-1] < 1e-8


def _kepler_relative(a, e, M, mu):
    """Relative position and velocity of a Kepler orbit (fixed orientation)."""
    r, v = S.elements_to_cartesian(np.array([a]), np.array([e]), 0.3, 1.1, 0.7,
                                   np.array([M]), mu)
    return r.reshape(3, 1), v.reshape(3, 1)


def test_rk4_eccentric_orbit_against_kepler():
    """An e = 0.5 orbit integrated for 1.3 periods agrees with the Kepler
    solution (mean anomaly advancing at n = sqrt(mu / a^3)) to O(dt^4)."""
    G = 2.9591220828e-4
    m1, m2, a, e = 1.0, 1e-3, 1.5, 0.5
    mu = G * (m1 + m2)
    nmean = np.sqrt(mu / a ** 3)
    t_end = 1.3 * 2 * np.pi / nmean
    r0, v0 = _kepler_relative(a, e, 0.4, mu)
    r1, v1 = _kepler_relative(a, e, 0.4 + nmean * t_end, mu)
    M = m1 + m2
    pos = np.concatenate([-m2 / M * r0, m1 / M * r0], axis=1)
    vel = np.concatenate([-m2 / M * v0, m1 / M * v0], axis=1)
    errs = []
    for nstep in (1000, 2000, 4000):
        p, v = oracle.rk4(pos, vel, np.array([m1, m2]), G, t_end / nstep, nstep)
        errs.append(np.linalg.norm((p[:, 1] - p[:, 0]) - r1[:, 0]) / a)
    order = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert all(abs(o - 4.0) < 0.2 for o in order), (errs, order)
    assert errs[-1] < 1e-9
    # velocity Verlet at the same step is second order: much larger error
    p2, _ = oracle.verlet(pos, vel, np.array([m1, m2]), G, t_end / 4000, 4000)
    assert np.linalg.norm((p2[:, 1] - p2[:, 0]) - r1[:, 0]) / a > 100 * errs[-1]


def test_rk4_conserves_momentum():
    """Each stage's accelerations are antisymmetric pair sums, so the total
    momentum of a random cluster is conserved to roundoff."""
    pos, vel, mass = S.random_cluster(8, 12, spread=5.0)
    p, v = oracle.rk4(pos, vel, mass, 0.5, 1e-3, 200)
    P0 = (mass * vel).sum(axis=1)
    P1 = (mass * v).sum(axis=1)
    assert np.linalg.norm(P1 - P0) <= 1e-13 * np.abs(mass * vel).sum()
