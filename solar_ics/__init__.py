"""Seeded synthetic Solar-System initial conditions.

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark. It holds none of the method's arithmetic (no forces, no
integration): it only draws random orbital elements and converts them to
heliocentric Cartesian states.

Workload shape (Sec. 2 of the paper): the Sun, 30 major bodies heavier than
1e19 kg, main-belt asteroids between Mars and Jupiter with masses uniform in
1e12-3e17 kg plus 19 heavier ones, and over 100 minor moons below 1e19 kg
orbiting massive planets. The paper's JPL HORIZONS ephemerides are not
available, so Kepler elements drawn from the distributions below stand in for
them.

Units: AU, day, solar mass.  G = k^2 with k the Gaussian gravitational constant.

Layout of every returned state: structure-of-arrays float64,
``pos[3, n]`` (x row, y row, z row), ``vel[3, n]``, ``mass[n]``.
Body order: Sun, major bodies, minor moons, heavy asteroids, small asteroids.

Draw order (fixed; the SHA-256 test pins it): ``numpy.random.default_rng(seed)``;
for each population in body order one ``rng.random((count, 7))`` (moons: 8)
matrix whose columns are mass, a, e, i, Omega, omega, M (moons: then parent).
The ensemble draws its asteroid count first with ``rng.integers``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

#: Gaussian gravitational constant squared, AU^3 Msun^-1 day^-2.
G_AU_DAY_MSUN = 2.9591220828e-4
#: Nominal solar mass in kg, used to convert the kg mass ranges.
MSUN_KG = 1.98847e30
#: Small-body class boundary (kg); sources lighter than this are "small".
SMALL_MASS_KG = 3e17
SMALL_MASS_MSUN = SMALL_MASS_KG / MSUN_KG

DEG = np.pi / 180.0


@dataclass
class System:
    """One initial state plus its description."""

    pos: np.ndarray            # (3, n) float64, AU
    vel: np.ndarray            # (3, n) float64, AU/day
    mass: np.ndarray           # (n,) float64, Msun
    G: float = G_AU_DAY_MSUN
    dt: float = 0.1
    steps: int = 0
    counts: dict = field(default_factory=dict)
    name: str = ""
    parent: np.ndarray | None = None   # (n,) body each body was placed about (0: the Sun)

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.pos, self.vel, self.mass):
            h.update(np.ascontiguousarray(a, dtype="<f8").tobytes())
        return h.hexdigest()


# ----------------------------------------------------------------------------
# Kepler elements -> Cartesian state
# ----------------------------------------------------------------------------

def solve_kepler(M: np.ndarray, e: np.ndarray, tol: float = 1e-15, maxit: int = 50) -> np.ndarray:
    """Eccentric anomaly E with E - e sin E = M, by Newton iteration."""
    M = np.asarray(M, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(maxit):
        f = E - e * np.sin(E) - M
        d = f / (1.0 - e * np.cos(E))
        E = E - d
        if np.all(np.abs(d) < tol):
            break
    return E


def elements_to_cartesian(a, e, inc, Omega, omega, M, mu):
    """Heliocentric (or parent-centric) position and velocity, each (3, k).

    Perifocal coordinates from the eccentric anomaly, rotated to the reference
    frame by R_z(Omega) R_x(inc) R_z(omega).
    """
    a = np.asarray(a, np.float64)
    e = np.asarray(e, np.float64)
    E = solve_kepler(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    xp = a * (cE - e)
    yp = a * b * sE
    r = a * (1.0 - e * cE)
    f = np.sqrt(mu * a) / r
    vxp = -f * sE
    vyp = f * b * cE
    cO, sO = np.cos(Omega), np.sin(Omega)
    ci, si = np.cos(inc), np.sin(inc)
    cw, sw = np.cos(omega), np.sin(omega)
    # Columns of R = R_z(Omega) R_x(inc) R_z(omega) applied to (xp, yp, 0).
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si])
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si])
    pos = P * xp + Q * yp
    vel = P * vxp + Q * vyp
    return pos, vel


def cartesian_to_elements(pos, vel, mu):
    """Inverse of :func:`elements_to_cartesian` (used by the round-trip test)."""
    pos = np.asarray(pos, np.float64)
    vel = np.asarray(vel, np.float64)
    r = np.linalg.norm(pos, axis=0)
    v2 = np.sum(vel * vel, axis=0)
    h = np.cross(pos.T, vel.T).T
    hn = np.linalg.norm(h, axis=0)
    inc = np.arccos(np.clip(h[2] / hn, -1, 1))
    Omega = np.mod(np.arctan2(h[0], -h[1]), 2 * np.pi)
    evec = (np.cross(vel.T, h.T).T / mu) - pos / r
    e = np.linalg.norm(evec, axis=0)
    a = 1.0 / (2.0 / r - v2 / mu)
    nvec = np.stack([np.cos(Omega), np.sin(Omega), np.zeros_like(Omega)])
    # argument of periapsis measured in the orbital plane from the node
    hx = h / hn
    ny = np.cross(hx.T, nvec.T).T
    omega = np.mod(np.arctan2(np.sum(evec * ny, 0), np.sum(evec * nvec, 0)), 2 * np.pi)
    # true anomaly -> eccentric -> mean
    nu = np.arctan2(np.sum(np.cross(evec.T, pos.T).T * hx, 0) / (e * r + 1e-300),
                    np.sum(evec * pos, 0) / (e * r + 1e-300))
    E = 2 * np.arctan2(np.sqrt(1 - e) * np.sin(nu / 2), np.sqrt(1 + e) * np.cos(nu / 2))
    M = np.mod(E - e * np.sin(E), 2 * np.pi)
    return a, e, inc, Omega, omega, M


# ----------------------------------------------------------------------------
# Populations
# ----------------------------------------------------------------------------

def _loguniform(u, lo, hi):
    return 10.0 ** (np.log10(lo) + u * (np.log10(hi) - np.log10(lo)))


def _uniform(u, lo, hi):
    return lo + u * (hi - lo)


def _heliocentric(u, m_kg, a, e, inc, G):
    m = m_kg / MSUN_KG
    Om = _uniform(u[:, 4], 0.0, 2 * np.pi)
    om = _uniform(u[:, 5], 0.0, 2 * np.pi)
    M = _uniform(u[:, 6], 0.0, 2 * np.pi)
    mu = G * (1.0 + m)
    p, v = elements_to_cartesian(a, e, inc, Om, om, M, mu)
    return p, v, m


def _major(rng, count, G):
    u = rng.random((count, 7))
    m_kg = _loguniform(u[:, 0], 1e19, 2e27)
    a = _loguniform(u[:, 1], 0.39, 40.0)
    e = _uniform(u[:, 2], 0.0, 0.1)
    inc = _uniform(u[:, 3], 0.0, 7.0) * DEG
    return _heliocentric(u, m_kg, a, e, inc, G)


def _belt(rng, count, G, m_lo, m_hi, log_mass):
    u = rng.random((count, 7))
    m_kg = (_loguniform if log_mass else _uniform)(u[:, 0], m_lo, m_hi)
    a = _uniform(u[:, 1], 2.1, 3.3)
    e = _uniform(u[:, 2], 0.0, 0.2)
    inc = _uniform(u[:, 3], 0.0, 20.0) * DEG
    return _heliocentric(u, m_kg, a, e, inc, G)


def _moons(rng, count, G, maj_pos, maj_vel, maj_mass):
    """Minor moons on Kepler orbits about one of the 4 most massive majors.

    Inclination is isotropic (cos i uniform in [-1, 1]); the remaining angles
    are uniform in [0, 2 pi); mu = G (m_parent + m_moon).
    """
    u = rng.random((count, 8))
    m = _uniform(u[:, 0], 1e14, 1e19) / MSUN_KG
    a = _uniform(u[:, 1], 0.005, 0.1)
    e = _uniform(u[:, 2], 0.0, 0.05)
    inc = np.arccos(_uniform(u[:, 3], -1.0, 1.0))
    Om = _uniform(u[:, 4], 0.0, 2 * np.pi)
    om = _uniform(u[:, 5], 0.0, 2 * np.pi)
    M = _uniform(u[:, 6], 0.0, 2 * np.pi)
    top4 = np.argsort(-maj_mass, kind="stable")[:4]
    parent = top4[np.minimum((u[:, 7] * 4).astype(np.int64), 3)]
    mu = G * (maj_mass[parent] + m)
    p, v = elements_to_cartesian(a, e, inc, Om, om, M, mu)
    return p + maj_pos[:, parent], v + maj_vel[:, parent], m, parent


def _assemble(parts, G, dt, steps, name, counts, parent=None):
    pos = np.concatenate([p[0] for p in parts], axis=1)
    vel = np.concatenate([p[1] for p in parts], axis=1)
    mass = np.concatenate([p[2] for p in parts])
    return System(np.ascontiguousarray(pos), np.ascontiguousarray(vel),
                  np.ascontiguousarray(mass), G=G, dt=dt, steps=steps,
                  counts=counts, name=name, parent=parent)


def _sun():
    return np.zeros((3, 1)), np.zeros((3, 1)), np.ones(1)


def solar_system(seed: int, n_small: int, n_moons: int = 0, n_heavy: int = 0,
                 n_major: int = 30, dt: float = 0.1, steps: int = 0,
                 G: float = G_AU_DAY_MSUN, name: str = "") -> System:
    """Sun + majors + moons + heavy asteroids + small asteroids (body order)."""
    rng = np.random.default_rng(seed)
    parts = [_sun()]
    maj = _major(rng, n_major, G)
    parts.append(maj)
    counts = {"sun": 1, "major": n_major}
    n = 1 + n_major + n_moons + n_heavy + n_small
    body_parent = np.zeros(n, dtype=np.int64)
    if n_moons:
        p, v, m, parent = _moons(rng, n_moons, G, maj[0], maj[1], maj[2])
        parts.append((p, v, m))
        counts["moons"] = n_moons
        body_parent[1 + n_major:1 + n_major + n_moons] = 1 + parent
    if n_heavy:
        parts.append(_belt(rng, n_heavy, G, 1e18, 1e21, log_mass=True))
        counts["heavy"] = n_heavy
    parts.append(_belt(rng, n_small, G, 1e12, 3e17, log_mass=False))
    counts["small"] = n_small
    return _assemble(parts, G, dt, steps, name, counts, body_parent)


# ----------------------------------------------------------------------------
# The named workloads
# ----------------------------------------------------------------------------

def config(k: int, system: int = 0) -> System:
    """Workload ``k`` (0..4); for the ensemble (k=3) ``system`` picks one of 512.

    0: N = 131 (Sun, 30 majors, 100 asteroids), seed 0, 3650 steps.
    1: N = 10,425 (Sun, 30 majors, 100 moons, 19 heavy, 10,275 small), seed 1,
       10,000 steps.
    2: N = 131,072 (Sun, 30 majors, 100 moons, 19 heavy, 130,922 small), seed 2,
       1000 steps.
    3: ensemble member ``system``: seed 100+system, Sun, 30 majors and a count
       drawn uniformly from the integers 100..8192 of asteroids, 1000 steps.
    4: N = 2079 (Sun, 30 majors, 2048 asteroids), seed 3, 36,500 steps.
    """
    if k == 0:
        return solar_system(0, 100, steps=3650, name="solar-131")
    if k == 1:
        return solar_system(1, 10275, n_moons=100, n_heavy=19, steps=10000,
                            name="solar-10425")
    if k == 2:
        return solar_system(2, 130922, n_moons=100, n_heavy=19, steps=1000,
                            name="solar-131072")
    if k == 3:
        seed = 100 + system
        rng = np.random.default_rng(seed)
        n_ast = int(rng.integers(100, 8193))
        # the body draws continue from the same generator stream
        parts = [_sun(), _major(rng, 30, G_AU_DAY_MSUN),
                 _belt(rng, n_ast, G_AU_DAY_MSUN, 1e12, 3e17, log_mass=False)]
        return _assemble(parts, G_AU_DAY_MSUN, 0.1, 1000, f"ensemble-{system}",
                         {"sun": 1, "major": 30, "small": n_ast})
    if k == 4:
        return solar_system(3, 2048, steps=36500, name="solar-2079")
    raise ValueError(f"unknown workload {k}")


def ensemble(count: int = 512):
    """The ensemble's member systems and their concatenation offsets."""
    systems = [config(3, s) for s in range(count)]
    offsets = np.zeros(count + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([s.n for s in systems])
    return systems, offsets


def adjoint_target_perturbation(sys: System, seed: int = 4, sigma: float = 1e-8) -> np.ndarray:
    """Perturbed initial positions of the adjoint workload's target run.

    Only asteroid positions (bodies after the Sun and majors) move, by
    N(0, sigma^2) AU per coordinate.
    """
    rng = np.random.default_rng(seed)
    pos = sys.pos.copy()
    first = 1 + sys.counts.get("major", 0)
    pos[:, first:] += rng.normal(0.0, sigma, size=(3, sys.n - first))
    return pos


def fd_coordinates(sys: System, count: int = 64, seed: int = 5, n_mass: int = 30):
    """Indices of gradient entries checked by finite differences.

    The gradient vector is laid out as [pos (3n), vel (3n), mass of the
    ``n_mass`` majors]; returns sorted distinct flat indices.
    """
    rng = np.random.default_rng(seed)
    total = 6 * sys.n + n_mass
    return np.sort(rng.choice(total, size=count, replace=False))


def small_mass_threshold() -> float:
    """3e17 kg in solar masses."""
    return SMALL_MASS_MSUN


def random_cluster(seed: int, n: int, spread: float = 1.0, mass_lo: float = 0.1,
                   mass_hi: float = 1.0, vscale: float = 0.1):
    """A generic random system (for invariants and small-case tests)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-spread, spread, size=(3, n))
    vel = rng.normal(0.0, vscale, size=(3, n))
    mass = rng.uniform(mass_lo, mass_hi, size=n)
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), np.ascontiguousarray(mass)
