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


# forward tile: None = default for n = 40 (one workgroup running whole
# steps); (1, 1, 2, 1) = the multi-workgroup force pass and step epilogue
@pytest.mark.parametrize("tile", [None, (1, 1, 2, 1)])
@pytest.mark.parametrize("steps,K", [(300, 7), (64, 64), (1, 5), (50, 1), (9, 2)])
def test_adjoint_matches_oracle(steps, K, tile):
    nb.reset_caches()
    s = S.solar_system(41, 20, n_major=19)
    if tile is not None:
        nb.set_tile(0, "fp64", s.n, *tile)
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
    # the forward half of the adjoint is the plain run, bit for bit
    p, vv = T(s.pos), T(s.vel)
    nb.verlet_run(p, vv, m, s.G, 0.1, steps)
    assert np.array_equal(H(p), H(pT)) and np.array_equal(H(vv), H(vT))
    nb.reset_caches()


def test_adjoint_pipelined_segments_bitwise():
    """The reverse sweep recomputes segment c - 1 on a second stream while it
    sweeps segment c.  Segments chain bit for bit and the transpose products
    run in the same order for any checkpoint spacing, so the gradients of the
    2,079-body workload over 120 steps are identical whether the run is one
    segment (K = 120) or eleven pipelined ones (K = 11, the last ragged), on a
    warm and on a cleared graph cache."""
    s = S.config(4)
    rng = np.random.default_rng(8)
    lr, lv = T(rng.normal(size=(3, s.n))), T(rng.normal(size=(3, s.n)))
    r, v, m = T(s.pos), T(s.vel), T(s.mass)
    outs = []
    for K, reset in [(120, False), (11, False), (11, False), (11, True)]:
        if reset:
            nb.reset_caches()
        outs.append([H(x) for x in nb.verlet_adjoint(r, v, m, s.G, s.dt, 120, K, lr, lv)])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("vtile", [(1, 1, 1, 0), (2, 1, 3, 0), (1, 4, 5, 0), (2, 2, 64, 0),
                                   (1, 1, 64, 0), (1, 2, 17, 0), (1, 1, 1, 1), (2, 1, 3, 1),
                                   (1, 4, 5, 1), (1, 1, 64, 1), (2, 2, 17, 1)])
@pytest.mark.parametrize("n_small", [20, 150])
def test_adjoint_transpose_pass_tiles(vtile, n_small):
    """The transpose-Jacobian pass over tile shapes and source chunkings
    (chunks of multiples of 8 sources, partly used LDS tiles)."""
    nb.reset_caches()
    s = S.solar_system(43, n_small, n_major=19)
    nb.set_tile(1, "fp64", s.n, *vtile)
    rng = np.random.default_rng(n_small)
    lr, lv = rng.normal(size=(3, s.n)), rng.normal(size=(3, s.n)) * 10
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, 30, lr, lv)
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 30, 7, T(lr), T(lv))
    er, ev, em = nrel(H(Gr), gr), nrel(H(Gv), gv), nrel(H(Gm), gm)
    print(f"n={s.n} vtile={vtile}: rel err r0 {er:.2e} v0 {ev:.2e} m {em:.2e}", flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10
    nb.reset_caches()


@pytest.mark.parametrize("shape", [(1, 4), (2, 2), (2, 4), (4, 4)])
@pytest.mark.parametrize("n_small", [20, 150, 300, 1100])
def test_adjoint_transpose_pass_each_pair_once(shape, n_small):
    """The transpose-Jacobian pass with each unordered pair once (tile
    variant 5): one range (20 and 150 small bodies), two and five ranges with
    a ragged last block (300, 1100), every workgroup shape."""
    nb.reset_caches()
    s = S.solar_system(44, n_small, n_major=19)
    nb.set_tile(1, "fp64", s.n, shape[0], shape[1], 1, 5)
    assert nb.get_tile(1, "fp64", s.n)["variant"] == 5
    rng = np.random.default_rng(n_small + shape[0])
    lr, lv = rng.normal(size=(3, s.n)), rng.normal(size=(3, s.n)) * 10
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, 30, lr, lv)
    args = (T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 30, 7, T(lr), T(lv))
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(*args)
    er, ev, em = nrel(H(Gr), gr), nrel(H(Gv), gv), nrel(H(Gm), gm)
    print(f"n={s.n} shape={shape}: rel err r0 {er:.2e} v0 {ev:.2e} m {em:.2e}", flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10
    again = nb.verlet_adjoint(*args)
    assert all(torch.equal(a, b) for a, b in zip(again[:3], (Gr, Gv, Gm)))
    nb.reset_caches()


def test_adjoint_each_pair_once_at_10425_bodies():
    """The 10,425-body workload, three steps, the pair-once pass in its
    default (4, 4) shape against the oracle's reverse sweep."""
    nb.reset_caches()
    s = S.config(1)
    assert nb.get_tile(1, "fp64", s.n) == {"targets_per_lane": 4, "waves": 4, "chunks": 1,
                                           "variant": 5}
    rng = np.random.default_rng(7)
    lr, lv = rng.normal(size=(3, s.n)) * 1e-8, rng.normal(size=(3, s.n)) * 1e-6
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, s.dt, 3, lr, lv)
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, s.dt, 3, 2,
                                         T(lr), T(lv))
    er, ev, em = nrel(H(Gr), gr), nrel(H(Gv), gv), nrel(H(Gm), gm)
    print(f"n={s.n}: rel err r0 {er:.2e} v0 {ev:.2e} m {em:.2e}", flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10
    nb.reset_caches()


def test_adjoint_pipelined_segments_with_split_last_round_bitwise():
    """The pipelined reverse sweep at 8,192 bodies, where the default
    transpose-Jacobian pass is each pair once with its last round of range
    pairs run as sub-phase halves: 24 steps in one segment (K = 24) and in
    five pipelined ones (K = 5, the last ragged) give identical gradients,
    and those match the oracle's reverse sweep."""
    nb.reset_caches()
    s = S.solar_system(49, 8192 - 31, n_major=30)
    assert nb.get_tile(1, "fp64", s.n)["variant"] == 5
    rng = np.random.default_rng(24)
    lr, lv = rng.normal(size=(3, s.n)) * 1e-8, rng.normal(size=(3, s.n)) * 1e-6
    r, v, m = T(s.pos), T(s.vel), T(s.mass)
    outs = [[H(x) for x in nb.verlet_adjoint(r, v, m, s.G, 0.1, 24, K, T(lr), T(lv))[:3]]
            for K in (24, 5)]
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, 24, lr, lv)
    er, ev, em = nrel(outs[0][0], gr), nrel(outs[0][1], gv), nrel(outs[0][2], gm)
    print(f"n={s.n} 24 steps pipelined: rel err r0 {er:.2e} v0 {ev:.2e} m {em:.2e}", flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10
    nb.reset_caches()


@pytest.mark.parametrize("n", [8192, 9990, 13056])
def test_adjoint_each_pair_once_split_last_round(n):
    """The pair-once transpose-Jacobian pass, shape (4, 4), at sizes whose
    last round of range pairs runs as halves by sub-phases (the second
    halves' sums and reactions in extra slots, the unused ones zero-filled):
    two steps against the oracle's reverse sweep, and a repeat bitwise."""
    nb.reset_caches()
    s = S.solar_system(45 + n, n - 31, n_major=30)
    nb.set_tile(1, "fp64", s.n, 4, 4, 1, 5)
    rng = np.random.default_rng(n)
    lr, lv = rng.normal(size=(3, s.n)) * 1e-8, rng.normal(size=(3, s.n)) * 1e-6
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, 2, lr, lv)
    args = (T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 2, 1, T(lr), T(lv))
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(*args)
    er, ev, em = nrel(H(Gr), gr), nrel(H(Gv), gv), nrel(H(Gm), gm)
    print(f"n={s.n} split last round: rel err r0 {er:.2e} v0 {ev:.2e} m {em:.2e}", flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10
    again = nb.verlet_adjoint(*args)
    assert all(torch.equal(a, b) for a, b in zip(again[:3], (Gr, Gv, Gm)))
    nb.reset_caches()


@pytest.mark.parametrize("n,variant", [(4499, 1), (4500, 5)])
def test_adjoint_default_tile_at_the_pair_once_boundary(n, variant):
    """The transpose-Jacobian pass's default tile on either side of the size
    where it switches to each pair once: two steps against the oracle's
    reverse sweep."""
    nb.reset_caches()
    s = S.solar_system(48 + n, n - 31, n_major=30)
    assert nb.get_tile(1, "fp64", s.n)["variant"] == variant
    rng = np.random.default_rng(n)
    lr, lv = rng.normal(size=(3, s.n)) * 1e-8, rng.normal(size=(3, s.n)) * 1e-6
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, 2, lr, lv)
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 2, 1,
                                         T(lr), T(lv))
    er, ev, em = nrel(H(Gr), gr), nrel(H(Gv), gv), nrel(H(Gm), gm)
    print(f"n={s.n} default variant {variant}: rel err r0 {er:.2e} v0 {ev:.2e} m {em:.2e}",
          flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10
    nb.reset_caches()


def test_adjoint_autotune_then_parity():
    """The autotuner over the transpose-Jacobian pass's tiles (LDS-staged and
    scalar-operand sources) keeps a supported tile for the size class, and the
    adjoint run with it matches the oracle."""
    nb.reset_caches()
    s = S.solar_system(47, 300, n_major=19)
    tile, ms = nb.autotune(T(s.pos), T(s.mass), s.G, kind=1)
    print(f"autotune adjoint pass n={s.n}: {tile} {ms:.4f} ms", flush=True)
    assert tile == nb.get_tile(1, "fp64", s.n) and tile["variant"] in (0, 1, 5) and ms > 0
    rng = np.random.default_rng(9)
    lr, lv = rng.normal(size=(3, s.n)), rng.normal(size=(3, s.n)) * 10
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, 0.1, 30, lr, lv)
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 30, 7, T(lr), T(lv))
    assert nrel(H(Gr), gr) <= 1e-10 and nrel(H(Gv), gv) <= 1e-10 and nrel(H(Gm), gm) <= 1e-10
    nb.reset_caches()


@pytest.mark.parametrize("steps", [150, 1000])
def test_adjoint_full_size_prefix_matches_oracle(steps):
    """The 2,079-body adjoint workload at full size in the benchmark's launch
    configuration (default tiles, checkpoints every 100 steps; a ragged last
    segment at 150 steps), over a 150- and a 1000-step prefix, against the
    oracle's reverse sweep."""
    nb.reset_caches()
    s = S.config(4)
    first = 1 + s.counts["major"]
    rng = np.random.default_rng(250)
    lr = np.zeros((3, s.n))
    lr[:, first:] = rng.normal(size=(3, s.n - first)) * 1e-8
    lv = np.zeros((3, s.n))
    gr, gv, gm = oracle.adjoint(s.pos, s.vel, s.mass, s.G, s.dt, steps, lr, lv)
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, s.dt, steps, 100,
                                         T(lr), T(lv))
    er, ev, em = nrel(H(Gr), gr), nrel(H(Gv), gv), nrel(H(Gm)[1:31], gm[1:31])
    print(f"n={s.n}, {steps} steps: rel err r0 {er:.2e} v0 {ev:.2e} major masses {em:.2e}",
          flush=True)
    assert er <= 1e-10 and ev <= 1e-10 and em <= 1e-10


def test_adjoint_zero_steps_is_identity():
    s = S.solar_system(42, 5, n_major=3)
    lr, lv = np.ones((3, s.n)), 2 * np.ones((3, s.n))
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), T(s.mass), s.G, 0.1, 0, 10, T(lr), T(lv))
    assert np.array_equal(H(Gr), lr) and np.array_equal(H(Gv), lv) and not H(Gm).any()


def fd_rows(s, steps, K, coords, rel_step=1e-7):
    """Central finite differences of the adjoint workload's loss
    L = sum_asteroids |delta|^2, delta = r(T) - r_tgt(T), from GPU forward
    runs at x0 and x0 +- h, x0 +- 2h, x0 +- h/2 for each coordinate
    (h = rel_step * scale; scales: max(|x|, 1 AU) for positions,
    max(|v|, 0.01 AU/day) for velocities, m for masses), beside the
    adjoint's entry g.  Per coordinate:
        fd_loss  = (L(x + h) - L(x - h)) / 2h           (two-point FD of L)
        J(k)     = (delta(x + k) - delta(x - k)) / 2k   (two-point FD of delta)
        fd_state = 2 delta0 . J(h)                      (dL/dr_T applied to J)
        curv     = h^2 J(h) . (delta(x+h) - 2 delta0 + delta(x-h)) / h^2
        bound    = |2 delta0 . J(2h) - fd_state| + |2 delta0 . J(h/2) - fd_state|
    fd_loss = fd_state + curv exactly: for a quadratic loss the two-point
    quotient of L carries the curvature term h^2 J . H, which does not
    shrink with the target offset while the gradient does.  `bound`
    estimates fd_state's own error from how much the same quotient moves
    when its step is doubled and halved: its truncation term grows as h^2
    (3 c h^2 from h to 2h) and the runs' rounding noise divided by the step
    enters each quotient independently."""
    first = 1 + s.counts["major"]
    m = T(s.mass)
    pt, vt = T(S.adjoint_target_perturbation(s)), T(s.vel)
    nb.verlet_run(pt, vt, m, s.G, s.dt, steps)
    tgt = H(pt)[:, first:]

    def delta(p0, v0, m0):
        p, v = T(p0), T(v0)
        nb.verlet_run(p, v, T(m0), s.G, s.dt, steps)
        return H(p)[:, first:] - tgt

    d0 = delta(s.pos, s.vel, s.mass)
    lam = np.zeros((3, s.n))
    lam[:, first:] = 2 * d0
    Gr, Gv, Gm, _, _ = nb.verlet_adjoint(T(s.pos), T(s.vel), m, s.G, s.dt, steps, K, T(lam),
                                         T(np.zeros_like(lam)))
    grad = np.concatenate([H(Gr).ravel(), H(Gv).ravel(), H(Gm)[1:31]])
    n = s.n
    rows = []
    for idx in coords:
        p0, v0, m0 = s.pos.copy(), s.vel.copy(), s.mass.copy()
        if idx < 3 * n:
            arr, flat = p0, idx
            scale = max(abs(p0.ravel()[flat]), 1.0)
        elif idx < 6 * n:
            arr, flat = v0, idx - 3 * n
            scale = max(abs(v0.ravel()[flat]), 0.01)
        else:
            arr, flat = m0, 1 + (idx - 6 * n)
            scale = m0[flat]
        h = rel_step * scale
        base = arr.ravel()[flat]

        def pair(k):
            arr.ravel()[flat] = base + k
            a = delta(p0, v0, m0)
            arr.ravel()[flat] = base - k
            b = delta(p0, v0, m0)
            arr.ravel()[flat] = base
            return a, b

        dp, dm = pair(h)
        J = (dp - dm) / (2 * h)
        fd_state = float(2 * np.sum(d0 * J))
        curv = float(np.sum(J * ((dp - d0) + (dm - d0))))
        fd_loss = float(np.sum((dp - dm) * (dp + dm)) / (2 * h))
        fd_k = []
        for k in (2 * h, 0.5 * h):
            a, b = pair(k)
            fd_k.append(float(2 * np.sum(d0 * (a - b)) / (2 * k)))
        bound = abs(fd_k[0] - fd_state) + abs(fd_k[1] - fd_state)
        rows.append((int(idx), float(grad[idx]), fd_state, fd_loss, curv, bound))
    return rows


def test_adjoint_vs_finite_differences_prefix():
    """The adjoint workload over a 1000-step prefix, 64 coordinates (the
    benchmark's draw), central differences at relative step 1e-7.

    The adjoint must agree with fd_state (the two-point difference of the
    final state applied to dL/dr_T) within 1e-6 relative plus that
    quotient's own error bound (`bound`, fd_rows: how far it moves when its
    step is doubled and halved), and within 1e-6 outright wherever that
    bound is below 1e-7 of the gradient; the median disagreement must stay
    below 1e-7.  The two-point quotient of the loss, fd_loss, equals
    fd_state plus its curvature term (checked to rounding) and agrees with
    the adjoint to the same bound once that term is added.  Entries below
    1e-9 of the largest sampled gradient are negligible."""
    s = S.config(4)
    coords = S.fd_coordinates(s, 64)
    rows = fd_rows(s, 1000, 100, coords)
    g, fs, fl, cv, bd = (np.array([r[i] for r in rows]) for i in range(1, 6))
    floor = 1e-9 * np.abs(fs).max()
    for (c, gi, a, b, k, e) in rows:
        print(f"coord {c:6d}: adjoint {gi: .10e} fd_state {a: .10e} "
              f"(rel {abs(gi - a) / max(abs(a), 1e-300):.1e}; fd error bound "
              f"{e / max(abs(a), 1e-300):.1e}) fd_loss {b: .10e} curvature {k: .3e}", flush=True)
    # the identity fd_loss = fd_state + curv (rounding only)
    assert np.all(np.abs(fl - (fs + cv)) <= 1e-9 * np.maximum(np.abs(fl), np.abs(cv)) + 1e-30)
    err = np.abs(g - fs)
    negligible = err <= floor
    strict = (err <= 1e-6 * np.abs(fs)) | negligible
    ok = strict | (err <= 1e-6 * np.abs(fs) + bd)
    assert ok.all(), [(int(c), float(e / abs(f)), float(b / abs(f)))
                      for c, e, f, b in zip(coords[~ok], err[~ok], fs[~ok], bd[~ok])]
    sharp = bd <= 1e-7 * np.abs(fs)
    assert strict[sharp].all()
    big = np.abs(fs) > floor
    assert np.median(err[big] / np.abs(fs[big])) <= 1e-7
    errl = np.abs(g - fl)
    okl = (errl <= 1e-6 * np.abs(fl) + np.abs(cv) * (1 + 1e-6) + bd) | (errl <= floor + np.abs(cv))
    assert okl.all()
    print(f"{int(strict.sum())} of {len(rows)} within 1e-6 of fd_state ({int(sharp.sum())} with a "
          f"finite-difference error bound below 1e-7); median rel err "
          f"{np.median(err[big] / np.abs(fs[big])):.2e}; median |curvature| / |fd_loss| "
          f"{np.median(np.abs(cv)[big] / np.abs(fl[big])):.2e}", flush=True)


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


@pytest.mark.parametrize("steps,K", [(120, 11), (100, 100), (7, 3), (0, 5)])
def test_checkpoints_then_reverse_equals_adjoint(steps, K):
    """nbody_verlet_checkpoints followed by nbody_verlet_adjoint_from_checkpoints
    gives nbody_verlet_adjoint's gradients and final state bit for bit, and
    the checkpoints are the plain run's states (record k = state after kK
    steps, the last one the final state)."""
    nb.reset_caches()
    s = S.config(4) if steps >= 100 else S.solar_system(44, 300, n_major=30)
    rng = np.random.default_rng(steps + K)
    lr, lv = T(rng.normal(size=(3, s.n))), T(rng.normal(size=(3, s.n)))
    r, v, m = T(s.pos), T(s.vel), T(s.mass)
    want = [H(x) for x in nb.verlet_adjoint(r, v, m, s.G, s.dt, steps, K, lr, lv)]
    pT, vT, ck = nb.verlet_checkpoints(r, v, m, s.G, s.dt, steps, K)
    got = [H(x) for x in nb.verlet_adjoint_from_checkpoints(ck, m, s.G, s.dt, steps, K, lr, lv)]
    for a, b in zip(got, want[:3]):
        assert np.array_equal(a, b)
    assert np.array_equal(H(pT), want[3]) and np.array_equal(H(vT), want[4])
    C = H(ck)
    assert C.shape == ((steps + K - 1) // K + 1, 6, s.n)
    for k in range(C.shape[0]):
        p, vv = T(s.pos), T(s.vel)
        nb.verlet_run(p, vv, m, s.G, s.dt, min(k * K, steps))
        assert np.array_equal(C[k, :3], H(p)) and np.array_equal(C[k, 3:], H(vv))
    assert np.array_equal(H(r), s.pos) and np.array_equal(H(v), s.vel)
