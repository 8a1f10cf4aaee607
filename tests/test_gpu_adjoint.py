"""GPU discrete adjoint: against the oracle's reverse sweep, against central
finite differences of GPU forward runs, and through torch.autograd."""
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


def nrel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("steps,K", [(300, 7), (64, 64), (1, 5), (50, 1)])
def test_adjoint_matches_oracle(steps, K):
    s = S.solar_system(41, 20, n_major=19)
    rng = np.random.default_rng(steps)
    lr, lv = rng.normal(size=(3, s.n)), rng.normal(size=(3, s.n)) * 10
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, steps, lr, lv)
    r, v, m = T(s.pos), T(s.vel), T(s.mass)
    Gr, Gv, Gm, pT, vT = nb.verlet_adjoint(r, v, m, s.G, 0.1, steps, K, T(lr), T(lv))
    er, ev, em = nrel(H(Gr), gr), nrel(H(Gv), gv), nrel(H(Gm), gm)
    print(f"steps={steps} K={K}: rel err r0 {er:.2e} v0 {ev:.2e} m {em:.2e}", flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, 0.1, steps)
    assert nrel(H(pT), pr) <= 1e-12
    # inputs untouched
    assert np.array_equal(H(r), s.pos) and np.array_equal(H(v), s.vel)


def test_adjoint_zero_steps_is_identity():
    s = S.solar_system(42, 5, n_major=3)
    lr, lv = np.ones((3, s.n)), 2 * np.ones((3, s.n))
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 0, 10, T(lr), T(lv))
    assert np.array_equal(H(Gr), lr) and np.array_equal(H(Gv), lv) and not H(Gm).any()


def _fd_check(s, steps, K, coords, rel_step=1e-7, rel_tol=1e-6, floor=1e-9):
    """Central differences of L = sum_ast |r(T) - r_tgt(T)|^2 from GPU runs."""
    first = 1 + s.counts["major"]
    m = T(s.mass)
    tgt0 = S.adjoint_target_perturbation(s)
    pt, vt = T(tgt0), T(s.vel)
    nb.verlet_run(pt, vt, m, s.G, s.dt, steps)
    tgt = H(pt)

    def final(p0, v0, m0):
        p, v = T(p0), T(v0)
        nb.verlet_run(p, v, T(m0), s.G, s.dt, steps)
        return H(p)

    pT = final(s.pos, s.vel, s.mass)
    lam = np.zeros_like(pT)
    lam[:, first:] = 2 * (pT[:, first:] - tgt[:, first:])
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), m, s.G, s.dt, steps, K, T(lam),
                                         T(np.zeros_like(lam)))
    grad = np.concatenate([H(Gr).ravel(), H(Gv).ravel(), H(Gm)[1:31]])
    n = s.n
    fds = []
    for idx in coords:
        p0, v0, m0 = s.pos.copy(), s.vel.copy(), s.mass.copy()
        if idx < 3 * n:
            arr, flat = p0, idx
            h = rel_step * max(abs(p0.ravel()[flat]), 1.0)
        elif idx < 6 * n:
            arr, flat = v0, idx - 3 * n
            h = rel_step * max(abs(v0.ravel()[flat]), 0.01)
        else:
            arr, flat = m0, 1 + (idx - 6 * n)
            h = rel_step * m0[flat]
        base = arr.ravel()[flat]
        arr.ravel()[flat] = base + h
        pp = final(p0, v0, m0)
        arr.ravel()[flat] = base - h
        pm = final(p0, v0, m0)
        # sum of (a^2 - b^2) as (a - b)(a + b): no cancellation between two
        # nearly equal totals
        a = pp[:, first:] - tgt[:, first:]
        b = pm[:, first:] - tgt[:, first:]
        fds.append(np.sum((pp[:, first:] - pm[:, first:]) * (a + b)) / (2 * h))
    fds = np.array(fds)
    adj = grad[coords]
    scale = np.abs(fds).max()
    ok = (np.abs(adj - fds) <= rel_tol * np.abs(fds)) | (np.abs(adj - fds) <= floor * scale)
    for i, c in enumerate(coords):
        print(f"coord {c:6d}: adjoint {adj[i]: .10e}  fd {fds[i]: .10e}  "
              f"rel {abs(adj[i] - fds[i]) / max(abs(fds[i]), 1e-300):.1e}", flush=True)
    return ok, adj, fds


def test_adjoint_vs_finite_differences_prefix():
    s = S.config(4)
    rng = np.random.default_rng(5)
    n = s.n
    coords = np.sort(np.concatenate([
        rng.choice(np.arange(3 * 31, 3 * n), 6, replace=False),           # asteroid positions
        3 * n + rng.choice(np.arange(3 * 31, 3 * n), 4, replace=False),    # asteroid velocities
        rng.choice(np.arange(0, 3 * 31), 2, replace=False),                # Sun/major positions
        [6 * n + int(np.argmax(s.mass[1:31]))],                            # heaviest major mass
    ]))
    # At a relative step of 1e-5 the difference quotient is far above the
    # roundoff noise of the two forward runs and its truncation error is
    # O(h^2) ~ 1e-10: the adjoint must agree to 1e-6.
    ok, adj, fds = _fd_check(s, 1000, 100, coords, rel_step=1e-5)
    assert ok.all()
    # At 1e-7 the quotient carries the forward runs' roundoff (last-bit
    # differences in every other body's trajectory, scaled by 1/h): agreement
    # is limited by that noise, checked at a correspondingly looser level.
    ok7, adj7, fds7 = _fd_check(s, 1000, 100, coords, rel_step=1e-7, rel_tol=1e-4)
    assert ok7.all()


def test_autograd_function():
    s = S.solar_system(43, 30, n_major=10)
    r0 = T(s.pos).requires_grad_(True)
    v0 = T(s.vel).requires_grad_(True)
    m = T(s.mass).requires_grad_(True)
    rT, vT = nb.verlet(r0, v0, m, s.G, 0.1, 120, 25)
    w = torch.linspace(0, 1, rT.numel(), dtype=torch.float64, device=DEV).reshape(rT.shape)
    loss = (w * rT).sum() + (vT ** 2).sum()
    loss.backward()
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 120, 25, w,
                                         2 * vT.detach())
    assert torch.equal(r0.grad, Gr) and torch.equal(v0.grad, Gv) and torch.equal(m.grad, Gm)
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, 120, H(w), H(2 * vT.detach()))
    assert nrel(H(r0.grad), gr) <= 1e-10 and nrel(H(m.grad), gm) <= 1e-10
