"""The adjoint workload over its whole horizon (2,079 bodies, 36,500 steps of
0.1 day, checkpoints every 100 steps) against the oracle's reverse sweep,
taken segment by segment (about 6.5 minutes of oracle time on 16 host
cores), so the test runs only when NBODY_LONG_CHECKS=1 is set; it prints one
line per oracle segment.

Tolerance: over ten years this system amplifies rounding differences.
Perturbing the initial state by 1e-15 relative moves the oracle's own final
state by 1.7e-13 (r) to 3.4e-13 (v) and its gradients by 1.1e-11 to 2.6e-11
(tests/test_oracle_adjoint_conditioning.py).  The GPU and the oracle round
differently at every step (different summation orders, the kick-drift-kick
form against Eqs. (3)-(4) as written), so the gradients are held to 1e-9
relative in norm, forty times the single-perturbation change, with the
median relative error of a position-gradient entry held to 1e-11; the final
states to 1e-10 as in the shorter runs."""
import os

import numpy as np
import pytest
import torch

import solar_ics as S
from oracle_segments import adjoint_segmented, nrel, workload_cotangent

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(
    os.environ.get("NBODY_LONG_CHECKS") != "1",
    reason="several minutes of oracle time; set NBODY_LONG_CHECKS=1")]

nb = pytest.importorskip("paper_2112_15079_amd")
DEV = "cuda:0"


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def log(msg):
    print(msg, flush=True)


def test_adjoint_whole_horizon_matches_oracle():
    s = S.config(4)
    assert s.steps == 36500 and s.n == 2079
    lr, lv = workload_cotangent(s)
    nb.reset_caches()
    Gr, Gv, Gm, pT, vT = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, s.dt, s.steps,
                                           100, T(lr), T(lv))
    Gr, Gv, Gm, pT, vT = (H(x) for x in (Gr, Gv, Gm, pT, vT))
    log("GPU adjoint done")
    gr, gv, gm, (pr, vr) = adjoint_segmented(s.pos, s.vel, s.mass, s.G, s.dt, s.steps, lr, lv,
                                             log=log)
    es, ev_ = nrel(pT, pr), nrel(vT, vr)
    er, ev, em = nrel(Gr, gr), nrel(Gv, gv), nrel(Gm[1:31], gm[1:31])
    med = float(np.median(np.abs(Gr - gr) / np.maximum(np.abs(gr), 1e-300)))
    log(f"final state rel diff: r {es:.2e} v {ev_:.2e}; gradient rel err: r0 {er:.2e} "
        f"v0 {ev:.2e} major masses {em:.2e}; per-entry median (r0) {med:.2e}")
    assert es <= 1e-10 and ev_ <= 1e-10
    assert er <= 1e-9 and ev <= 1e-9 and em <= 1e-9
    assert med <= 1e-11
