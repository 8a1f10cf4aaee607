"""The oracle's adjoint over a long horizon, taken segment by segment (test
infrastructure: calls the oracle only).

The oracle's adjoint keeps its whole forward trajectory, so a long run is cut
into segments: the oracle's forward run gives the state at each segment
boundary, then its adjoint over each segment, last to first, maps the
cotangent of the segment's end state to that of its start state and adds the
segment's mass gradient.  This is the chain rule over a composition of maps,
exact up to rounding."""
import time

import numpy as np

import oracle


def adjoint_segmented(pos, vel, mass, G, dt, steps, lam_r, lam_v, seg=500, log=print):
    """(dL/dr0, dL/dv0, dL/dm, (r_T, v_T)) for dL/dr_T = lam_r, dL/dv_T = lam_v."""
    bounds = list(range(0, steps, seg)) + [steps]
    states = [(pos, vel)]
    t0 = time.perf_counter()
    for a, b in zip(bounds[:-1], bounds[1:]):
        states.append(oracle.verlet(*states[-1], mass, G, dt, b - a))
        if len(states) % 20 == 0:
            log(f"oracle forward: step {b} ({time.perf_counter() - t0:.1f} s)")
    log(f"oracle forward: {steps} steps in {time.perf_counter() - t0:.1f} s")
    gm = np.zeros(len(mass))
    for c in range(len(bounds) - 2, -1, -1):
        r, v = states[c]
        lam_r, lam_v, g = oracle.adjoint(r, v, mass, G, dt, bounds[c + 1] - bounds[c], lam_r, lam_v)
        gm += g
        log(f"oracle reverse: steps {bounds[c]}..{bounds[c + 1]} done "
            f"({time.perf_counter() - t0:.1f} s)")
    return lam_r, lam_v, gm, states[-1]


def workload_cotangent(s):
    """The cotangent both whole-horizon tests use: N(0, (1e-8)^2) on the
    asteroids' final positions (seed 250), zero on velocities."""
    first = 1 + s.counts["major"]
    rng = np.random.default_rng(250)
    lr = np.zeros((3, s.n))
    lr[:, first:] = rng.normal(size=(3, s.n - first)) * 1e-8
    return lr, np.zeros((3, s.n))


def nrel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
