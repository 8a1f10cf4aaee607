"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Tolerances: FP64 accelerations within 1e-13 relative per body; positions
within 1e-10 relative per body after the run; the split form's errors are
reported and bounded.  All calls go through the C ABI (the Python binding
only marshals arguments)."""
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
    """max over bodies of |a_p - b_p| / |b_p| (absolute where b_p = 0)."""
    d = np.linalg.norm(a - b, axis=0)
    r = np.linalg.norm(b, axis=0)
    return float(np.max(np.where(r > 0, d / np.where(r > 0, r, 1), d)))


def log(msg):
    print(msg, flush=True)


@pytest.fixture(autouse=True)
def _fresh_tiles():
    nb.reset_caches()
    yield
    nb.reset_caches()


# ---------------------------------------------------------------------------
# Eq. (1)

TILES = [(1, 1, 1, 0), (2, 1, 3, 0), (4, 1, 2, 0), (1, 2, 5, 0), (2, 4, 2, 0), (4, 8, 1, 0),
         (1, 8, 64, 0), (4, 2, 9, 0), (1, 1, 1, 1), (2, 1, 3, 1), (4, 2, 5, 1), (1, 4, 7, 1),
         (2, 8, 2, 1), (1, 2, 64, 1), (1, 2, 1, 2), (2, 4, 3, 2), (4, 2, 5, 2), (1, 8, 9, 2)]
# one workgroup running whole steps (n <= 512): source slices per target
SMALL_TILES = [(1, 16, 1, 3), (1, 16, 3, 3), (1, 16, 7, 3), (1, 16, 64, 3)]
# each unordered pair once (FP64): T target blocks per wave, W waves; with
# T * W = 8 or 16 two or four waves share each target set and split the
# source blocks
MUTUAL = [(1, 4, 1, 5), (2, 2, 1, 5), (2, 4, 1, 5), (4, 4, 1, 5)]


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 131, 257, 1000, 2049])
def test_accel_fp64_shapes(n):
    s = S.solar_system(50 + n, max(n - 31, 0), n_major=min(30, max(n - 1, 0)))
    pos, mass = s.pos[:, :n], s.mass[:n]
    ref = oracle.accel(pos, mass, s.G)
    for tile in TILES + (SMALL_TILES if n <= 512 else []) + MUTUAL:
        nb.set_tile(0, "fp64", n, *tile)
        got = H(nb.accel(T(pos), T(mass), s.G))
        e = rel(got, ref)
        log(f"n={n} tile={tile} rel={e:.2e}")
        assert e <= 1e-13


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("n", [3, 200, 1031])
def test_accel_split_shapes(n, variant):
    """Split form on ragged sizes with the class boundary inside a group/tile."""
    if variant == 3 and n > 512:
        pytest.skip("the single-workgroup variant holds at most 512 bodies")
    s = S.solar_system(70 + n, max(n - 31, 0), n_major=min(30, n - 1))
    ref = oracle.accel(s.pos, s.mass, s.G)
    shapes = ([(1, 16, 1), (1, 16, 2), (1, 16, 5)] if variant == 3 else
              [t[:3] for t in MUTUAL] if variant == 5 else [(1, 1, 1), (2, 2, 3), (4, 1, 2)])
    for tile in shapes:
        nb.set_tile(0, "split", n, *tile, variant)
        got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision="split"))
        e = rel(got, ref)
        log(f"split n={n} tile={tile} variant={variant} rel={e:.2e}")
        assert e <= 2e-12


def test_accel_fp64_random_cluster():
    pos, _, mass = S.random_cluster(3, 777, spread=10.0)
    ref = oracle.accel(pos, mass, 0.37)
    got = H(nb.accel(T(pos), T(mass), 0.37))
    assert rel(got, ref) <= 1e-13


@pytest.mark.parametrize("k", [0, 1])
def test_accel_fp64_workloads(k):
    s = S.config(k)
    ref = oracle.accel(s.pos, s.mass, s.G)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G))
    e = rel(got, ref)
    log(f"workload {k} n={s.n} accel rel={e:.2e}")
    assert e <= 1e-13


def test_accel_fp64_131072_sampled():
    s = S.config(2)
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([[0, 1, 30, 31, 130, 149, 150, s.n - 1],
                                    rng.choice(s.n, 248, replace=False)]))
    ref = oracle.accel_targets(s.pos, s.mass, s.G, idx)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G))[:, idx]
    e = rel(got, ref)
    log(f"n=131072 sampled {idx.size} rel={e:.2e}")
    assert e <= 1e-13


# ---------------------------------------------------------------------------
# Eqs. (3)-(4)

_ORACLE_RUNS = {}


def _oracle_workload0():
    if "w0" not in _ORACLE_RUNS:
        s = S.config(0)
        _ORACLE_RUNS["w0"] = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, s.steps)
    return _ORACLE_RUNS["w0"]


# None: the default shape for n = 131 (one workgroup running whole steps);
# the others force the multi-workgroup force pass + step epilogue.
@pytest.mark.parametrize("tile", [None, (1, 1, 2, 1), (2, 1, 1, 0), (1, 16, 3, 3)])
def test_verlet_workload0_one_year(tile):
    s = S.config(0)
    pr, vr = _oracle_workload0()
    if tile is not None:
        nb.set_tile(0, "fp64", s.n, *tile)
    log(f"workload 0 tile={nb.get_tile(0, 'fp64', s.n)}")
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, T(s.mass), s.G, s.dt, s.steps)
    ep, ev = rel(H(p), pr), rel(H(v), vr)
    log(f"workload 0, {s.steps} steps, tile={tile}: pos rel={ep:.2e} vel rel={ev:.2e}")
    assert ep <= 1e-10
    assert ev <= 1e-9


def test_verlet_workload1_100_steps():
    s = S.config(1)
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, 100)
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, T(s.mass), s.G, s.dt, 100)
    ep, ev = rel(H(p), pr), rel(H(v), vr)
    log(f"workload 1, 100 steps: pos rel={ep:.2e} vel rel={ev:.2e}")
    assert ep <= 1e-10
    assert ev <= 1e-9


@pytest.mark.parametrize("steps", [1, 2, 3, 130, 131])
def test_verlet_step_counts(steps):
    s = S.solar_system(9, 60, n_major=10)
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, 0.1, steps)
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, T(s.mass), s.G, 0.1, steps)
    assert rel(H(p), pr) <= 1e-12
    assert rel(H(v), vr) <= 1e-11


def test_single_workgroup_run_across_launch_segments():
    """Runs longer than one launch of the single-workgroup kernel (4096
    launch indices) hand the state on through global memory: same results as
    the oracle, and resuming at any step is bitwise identical."""
    s = S.solar_system(11, 30, n_major=8)
    steps = 4096 + 37
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, 0.1, steps)
    m = T(s.mass)
    assert nb.get_tile(0, "fp64", s.n)["variant"] == 3
    outs = []
    for split in ([steps], [4095, 1, steps - 4096], [17, steps - 17]):
        p, v = T(s.pos), T(s.vel)
        for k in split:
            nb.verlet_run(p, v, m, s.G, 0.1, k)
        outs.append((H(p), H(v)))
    assert rel(outs[0][0], pr) <= 1e-10 and rel(outs[0][1], vr) <= 1e-9
    for p, v in outs[1:]:
        assert np.array_equal(p, outs[0][0]) and np.array_equal(v, outs[0][1])


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_single_workgroup_matches_multi_workgroup(precision):
    """The two paths for one small system agree to the parity tolerance."""
    s = S.config(0)
    m = T(s.mass)
    res = []
    for tile in [(1, 16, 7, 3), (1, 1, 2, 1)]:
        nb.set_tile(0, precision, s.n, *tile)
        p, v = T(s.pos), T(s.vel)
        nb.verlet_run(p, v, m, s.G, s.dt, 500, precision=precision)
        res.append(H(p))
    assert rel(res[0], res[1]) <= 1e-11


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("n,slices", [(342, 2), (500, 2), (512, 1)])
def test_single_workgroup_two_elements_per_lane(n, slices, precision):
    """Above 341 bodies each lane of the single-workgroup kernel carries two
    of the 3n (body, component) velocities through the steps."""
    s = S.solar_system(90 + n, n - 31, n_major=30)
    nb.set_tile(0, precision, n, 1, 16, slices, 3)
    steps = 40
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, 0.1, steps)
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, T(s.mass), s.G, 0.1, steps, precision=precision)
    tol = 1e-12 if precision == "fp64" else 1e-10
    assert rel(H(p), pr) <= tol and rel(H(v), vr) <= 10 * tol
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision=precision))
    assert rel(got, oracle.accel(s.pos, s.mass, s.G)) <= (1e-13 if precision == "fp64" else 2e-12)


@pytest.mark.parametrize("tile", [(1, 16, 7, 3), (1, 1, 2, 1), (1, 1, 1, 0), (4, 4, 1, 5),
                                  (1, 4, 1, 5)])
@pytest.mark.parametrize("threshold,tol_sun,tol", [(0.0, 2e-12, 2e-12), (0.5, 2e-6, 1e-9),
                                                   (2.0, 2e-6, 2e-6)])
def test_split_class_boundaries(threshold, tol_sun, tol, tile):
    """Split form with every body in the FP64 class (threshold 0), only the
    Sun in it (0.5 Msun: the Sun's own acceleration is then made of FP32
    terms only, and the planets' pulls, ~1e-3 of the Sun's, on the other
    bodies) and none (2 Msun: every term in FP32, so the error is FP32's), for
    the single-workgroup and the multi-workgroup kernels."""
    s = S.config(0)
    ref = oracle.accel(s.pos, s.mass, s.G)
    nb.set_tile(0, "split", s.n, *tile)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision="split", small_mass=threshold))
    e_sun, e = rel(got[:, :1], ref[:, :1]), rel(got[:, 1:], ref[:, 1:])
    log(f"split threshold {threshold} tile {tile}: rel Sun {e_sun:.2e}, others {e:.2e}")
    assert np.isfinite(got).all() and e_sun <= tol_sun and e <= tol
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, T(s.mass), s.G, s.dt, 100, precision="split", small_mass=threshold)
    pr, _ = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, 100)
    P = H(p)
    sun_tol, run_tol = {0.0: (1e-10, 1e-10), 0.5: (1e-6, 1e-8), 2.0: (1e-5, 1e-5)}[threshold]
    assert rel(P[:, :1], pr[:, :1]) <= sun_tol and rel(P[:, 1:], pr[:, 1:]) <= run_tol


FUSED_TILES = [(1, 2, 1, 4), (1, 8, 1, 4), (2, 4, 1, 4), (2, 8, 1, 4)]


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("n", [1, 3, 65, 300, 1031])
def test_fused_step_matches_oracle_and_shared_variant(n, precision):
    """Force pass and step in one kernel (variant 4): against the oracle, and
    bit for bit against the shared-target variant with one source chunk
    followed by the step epilogue (the same sums in the same order)."""
    s = S.solar_system(60 + n, max(n - 31, 0), n_major=min(30, max(n - 1, 0)))
    m = T(s.mass)
    aref = oracle.accel(s.pos, s.mass, s.G)
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, 0.1, 30)
    atol, ptol = (1e-13, 1e-12) if precision == "fp64" else (2e-12, 1e-10)
    for t, w, _, _ in FUSED_TILES:
        out = {}
        for variant in (4, 2):
            nb.reset_caches()
            nb.set_tile(0, precision, s.n, t, w, 1, variant)
            a = H(nb.accel(T(s.pos), m, s.G, precision=precision))
            p, v = T(s.pos), T(s.vel)
            nb.verlet_run(p, v, m, s.G, 0.1, 30, precision=precision)
            out[variant] = (a, H(p), H(v))
        a, p, v = out[4]
        log(f"fused n={s.n} {precision} T={t} W={w}: accel {rel(a, aref):.2e} pos {rel(p, pr):.2e}")
        assert rel(a, aref) <= atol and rel(p, pr) <= ptol and rel(v, vr) <= 10 * ptol
        for x, y in zip(out[4], out[2]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("tile", MUTUAL)
@pytest.mark.parametrize("k", [0, 1])
def test_mutual_pairs_workloads(k, tile):
    """Each unordered pair once (Newton's third law) on the two workloads:
    accelerations against the oracle, a run against the oracle and bitwise
    repeatable (every partial slot is written once per pass, summed in a
    fixed order)."""
    s = S.config(k)
    nb.set_tile(0, "fp64", s.n, *tile)
    m = T(s.mass)
    a = H(nb.accel(T(s.pos), m, s.G))
    ea = rel(a, oracle.accel(s.pos, s.mass, s.G))
    steps = 100
    pr, vr = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, steps)
    outs = []
    for _ in range(2):
        p, v = T(s.pos), T(s.vel)
        nb.verlet_run(p, v, m, s.G, s.dt, steps)
        outs.append((H(p), H(v)))
    ep = rel(outs[0][0], pr)
    log(f"mutual {tile} workload {k} n={s.n}: accel {ea:.2e}, {steps} steps pos {ep:.2e}")
    assert ea <= 1e-13 and ep <= 1e-10 and rel(outs[0][1], vr) <= 1e-9
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    # momentum: the pair terms cancel up to the products' rounding
    P0 = H(nb.momenta(T(s.pos), T(s.vel), m))[:3]
    P1 = H(nb.momenta(T(outs[0][0]), T(outs[0][1]), m))[:3]
    assert np.linalg.norm(P1 - P0) <= 1e-12 * np.sum(s.mass * np.linalg.norm(s.vel, axis=0))


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_mutual_pairs_more_than_64_ranges(precision):
    """Each pair once with 79 ranges of partials (more than the one-way
    passes' 64 chunks): sampled accelerations against the oracle, and 130
    steps (graph replays) bitwise equal to 65 + 65."""
    s = S.solar_system(919, 20000 - 150, n_major=30)
    assert s.n > 64 * 256
    nb.set_tile(0, precision, s.n, 4, 4, 1, 5)
    m = T(s.mass)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([[0, 1, 150, s.n - 1], rng.choice(s.n, 60, replace=False)]))
    got = H(nb.accel(T(s.pos), m, s.G, precision=precision))[:, idx]
    e = rel(got, oracle.accel_targets(s.pos, s.mass, s.G, idx))
    log(f"mutual {precision} n={s.n}: sampled accel {e:.2e}")
    assert e <= (1e-13 if precision == "fp64" else 2e-12)
    p1, v1 = T(s.pos), T(s.vel)
    nb.verlet_run(p1, v1, m, s.G, 0.1, 130, precision=precision)
    p2, v2 = T(s.pos), T(s.vel)
    nb.verlet_run(p2, v2, m, s.G, 0.1, 65, precision=precision)
    nb.verlet_run(p2, v2, m, s.G, 0.1, 65, precision=precision)
    assert np.array_equal(H(p1), H(p2)) and np.array_equal(H(v1), H(v2))


@pytest.mark.parametrize("tile", [(4, 4, 1, 5), (2, 4, 1, 5)])
@pytest.mark.parametrize("k", [0, 1])
def test_mutual_pairs_split_workloads(k, tile):
    """Split form with each pair once: FP32 light-light tiles, FP64 tiles for
    the heavy bodies' target blocks.  Accelerations within the split bar,
    energy within 1e-10 of the FP64 run's after 200 steps, bitwise repeat."""
    s = S.config(k)
    nb.set_tile(0, "split", s.n, *tile)
    m = T(s.mass)
    a = H(nb.accel(T(s.pos), m, s.G, precision="split"))
    ea = rel(a, oracle.accel(s.pos, s.mass, s.G))
    steps = 200
    outs = []
    for _ in range(2):
        p, v = T(s.pos), T(s.vel)
        nb.verlet_run(p, v, m, s.G, s.dt, steps, precision="split")
        outs.append((p, v))
    p1, v1 = T(s.pos), T(s.vel)
    nb.verlet_run(p1, v1, m, s.G, s.dt, steps)
    E0 = H(nb.energy(T(s.pos), T(s.vel), m, s.G))[2]
    d = abs(H(nb.energy(*outs[0], m, s.G))[2] - H(nb.energy(p1, v1, m, s.G))[2]) / abs(E0)
    log(f"mutual split {tile} workload {k} n={s.n}: accel {ea:.2e}, |E_split - E_fp64|/|E0| {d:.2e}")
    assert ea <= 2e-12 and d <= 1e-10
    assert np.array_equal(H(outs[0][0]), H(outs[1][0])) and np.array_equal(H(outs[0][1]), H(outs[1][1]))


@pytest.mark.parametrize("precision,n,variant", [("fp64", 4095, 1), ("fp64", 4096, 5),
                                                   ("split", 7999, 0), ("split", 8000, 5)])
def test_default_tiles_at_the_pair_once_boundaries(precision, n, variant):
    """The default tiles on either side of the sizes where the pass switches
    between one-way and each-pair-once: the expected variant, accelerations
    against the oracle, and a 20-step run equal to 10 + 10."""
    nb.reset_caches()
    s = S.solar_system(47 + n, n - 31, n_major=30)
    assert nb.get_tile(0, precision, n)["variant"] == variant
    m = T(s.mass)
    tol = 1e-13 if precision == "fp64" else 2e-12
    e = rel(H(nb.accel(T(s.pos), m, s.G, precision=precision)), oracle.accel(s.pos, s.mass, s.G))
    log(f"default tile {precision} n={n} variant {variant}: rel {e:.2e}")
    assert e <= tol
    p1, v1 = T(s.pos), T(s.vel)
    nb.verlet_run(p1, v1, m, s.G, 0.1, 20, precision=precision)
    p2, v2 = T(s.pos), T(s.vel)
    nb.verlet_run(p2, v2, m, s.G, 0.1, 10, precision=precision)
    nb.verlet_run(p2, v2, m, s.G, 0.1, 10, precision=precision)
    assert np.array_equal(H(p1), H(p2)) and np.array_equal(H(v1), H(v2))


@pytest.mark.parametrize("n", [8192, 9990, 10240, 13056, 30000, 45500])
def test_mutual_pairs_split_last_round(n):
    """Each pair once, shape (4, 4), at sizes whose last round of range pairs
    is split into halves by sub-phases (one to three super-diagonals of split
    pairs, the second halves' target sums and reactions in extra slots, the
    unused extra slots zero-filled by the diagonal workgroups): FP64 and split
    accelerations against the oracle, and 30 steps bitwise equal to 15 + 15."""
    s = S.solar_system(41 + n, n - 31, n_major=30)
    ref = oracle.accel(s.pos, s.mass, s.G)
    m = T(s.mass)
    for precision, tol in (("fp64", 1e-13), ("split", 2e-12)):
        nb.set_tile(0, precision, n, 4, 4, 1, 5)
        e = rel(H(nb.accel(T(s.pos), m, s.G, precision=precision)), ref)
        log(f"mutual split round {precision} n={n}: rel {e:.2e}")
        assert e <= tol
        p1, v1 = T(s.pos), T(s.vel)
        nb.verlet_run(p1, v1, m, s.G, 0.1, 30, precision=precision)
        p2, v2 = T(s.pos), T(s.vel)
        nb.verlet_run(p2, v2, m, s.G, 0.1, 15, precision=precision)
        nb.verlet_run(p2, v2, m, s.G, 0.1, 15, precision=precision)
        assert np.array_equal(H(p1), H(p2)) and np.array_equal(H(v1), H(v2))


def test_beyond_the_pair_once_limit_sampled():
    """160,000 bodies, past the each-pair-once pass's 131,072: the default
    one-way tiles, FP64 and split, on 256 sampled targets against the
    oracle, and a 4-step run equal to 2 + 2 steps."""
    nb.reset_caches()
    s = S.solar_system(90, 160000 - 31, n_major=30)
    assert nb.get_tile(0, "fp64", s.n)["variant"] in (0, 1, 2)
    rng = np.random.default_rng(160)
    idx = np.unique(np.concatenate([[0, s.n - 1], rng.choice(s.n, 254, replace=False)]))
    ref = oracle.accel_targets(s.pos, s.mass, s.G, idx)
    m = T(s.mass)
    for precision, tol in (("fp64", 1e-13), ("split", 2e-12)):
        e = rel(H(nb.accel(T(s.pos), m, s.G, precision=precision))[:, idx], ref)
        log(f"n={s.n} {precision}: sampled rel err {e:.2e}")
        assert e <= tol
        p1, v1 = T(s.pos), T(s.vel)
        nb.verlet_run(p1, v1, m, s.G, 0.1, 4, precision=precision)
        p2, v2 = T(s.pos), T(s.vel)
        nb.verlet_run(p2, v2, m, s.G, 0.1, 2, precision=precision)
        nb.verlet_run(p2, v2, m, s.G, 0.1, 2, precision=precision)
        assert np.array_equal(H(p1), H(p2)) and np.array_equal(H(v1), H(v2))


def test_mutual_pairs_rejected_where_unsupported():
    for tile in MUTUAL:   # beyond 131,072 bodies (512 ranges of partials)
        for precision in ("fp64", "split"):
            with pytest.raises(ValueError):
                nb.set_tile(0, precision, 131073, *tile)


def test_graph_cache_eviction():
    """More distinct buffer sets than the library keeps step graphs for (64):
    older graphs are dropped and recaptured, results stay bit-identical."""
    s = S.solar_system(17, 269, n_major=30)   # n = 300: graph-replayed steps
    m = T(s.mass)
    steps = 2 * 64 + 3                        # at least one graph replay per run
    keep, outs = [], []
    for k in range(70):
        p, v = T(s.pos), T(s.vel)             # new buffers each time: a new graph key
        nb.verlet_run(p, v, m, s.G, 0.1, steps)
        keep.append((p, v))
        if k in (0, 69):
            outs.append(H(p))
    p, v = keep[0]
    p.copy_(T(s.pos))
    v.copy_(T(s.vel))
    nb.verlet_run(p, v, m, s.G, 0.1, steps)   # its graph was evicted: recaptured
    outs.append(H(p))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    pr, _ = oracle.verlet(s.pos, s.vel, s.mass, s.G, 0.1, steps)
    assert rel(outs[0], pr) <= 1e-12


def test_runs_on_two_streams_use_separate_workspaces():
    """Calls made on two streams at once get a workspace each from the
    binding (device, stream): two overlapping runs of different systems give
    the same bits as each run made alone."""
    a = S.solar_system(71, 2969, n_major=30)
    b = S.solar_system(72, 5969, n_major=30)
    want = []
    for x in (a, b):
        p, v = T(x.pos), T(x.vel)
        nb.verlet_run(p, v, T(x.mass), x.G, 0.1, 150)
        want.append((H(p), H(v)))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    bufs = []
    torch.cuda.synchronize()
    for st, x in ((s1, a), (s2, b)):
        with torch.cuda.stream(st):
            p, v, m = T(x.pos), T(x.vel), T(x.mass)
            nb.verlet_run(p, v, m, x.G, 0.1, 150)
            bufs.append((p, v, m))
    torch.cuda.synchronize()
    for (p, v, _), (wp, wv) in zip(bufs, want):
        assert np.array_equal(H(p), wp) and np.array_equal(H(v), wv)


def test_verlet_zero_steps_is_noop():
    s = S.config(0)
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, T(s.mass), s.G, 0.1, 0)
    assert np.array_equal(H(p), s.pos) and np.array_equal(H(v), s.vel)


def test_determinism_and_resume():
    s = S.config(0)
    m = T(s.mass)
    runs = []
    for split in ([300], [300], [150, 150], [1, 298, 1], [200, 100]):
        p, v = T(s.pos), T(s.vel)
        for k in split:
            nb.verlet_run(p, v, m, s.G, s.dt, k)
        runs.append((H(p), H(v)))
    for p, v in runs[1:]:
        assert np.array_equal(p, runs[0][0]) and np.array_equal(v, runs[0][1])


def test_momenta_conserved_on_gpu():
    s = S.config(0)
    p, v, m = T(s.pos), T(s.vel), T(s.mass)
    P0 = H(nb.momenta(p, v, m))
    nb.verlet_run(p, v, m, s.G, s.dt, s.steps)
    P1 = H(nb.momenta(p, v, m))
    scaleP = np.sum(s.mass * np.linalg.norm(s.vel, axis=0))
    scaleL = np.sum(s.mass * np.linalg.norm(np.cross(s.pos.T, s.vel.T), axis=1))
    assert np.linalg.norm(P1[:3] - P0[:3]) <= 1e-12 * scaleP
    assert np.linalg.norm(P1[3:] - P0[3:]) <= 1e-12 * scaleL


# ---------------------------------------------------------------------------
# diagnostics

@pytest.mark.parametrize("k", [0, 1])
def test_energy_and_momenta_vs_oracle(k):
    s = S.config(k)
    E = H(nb.energy(T(s.pos), T(s.vel), T(s.mass), s.G))
    Er = oracle.energy(s.pos, s.vel, s.mass, s.G)
    for a, b in zip(E, Er):
        assert abs(a - b) <= 1e-13 * abs(b)
    PL = H(nb.momenta(T(s.pos), T(s.vel), T(s.mass)))
    P, L = oracle.momenta(s.pos, s.vel, s.mass)
    assert np.allclose(PL[:3], P, rtol=1e-13, atol=1e-13 * np.abs(P).max())
    assert np.allclose(PL[3:], L, rtol=1e-13, atol=1e-13 * np.abs(L).max())


def test_nonfinite_flag():
    pos = np.array([[0.0, 1.0, 1.0, 2.0], [0.0, 0.0, 0.0, 1.0], [0.0, 0.0, 0.0, 0.0]])
    mass = np.ones(4)
    nb.get_flags(DEV, clear=True)
    p, v = T(pos), T(np.zeros((3, 4)))
    nb.verlet_run(p, v, T(mass), 1.0, 0.01, 3)
    assert nb.get_flags(DEV, clear=True) & 1
    ref = oracle.accel(pos, mass, 1.0)
    assert not np.isfinite(ref[:, 1]).all()
    s = S.config(0)
    nb.verlet_run(T(s.pos), T(s.vel), T(s.mass), s.G, s.dt, 10)
    assert nb.get_flags(DEV, clear=True) == 0


# ---------------------------------------------------------------------------
# split precision

@pytest.mark.parametrize("k", [0, 1])
def test_split_accel_error(k):
    s = S.config(k)
    ref = oracle.accel(s.pos, s.mass, s.G)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision="split"))
    e = rel(got, ref)
    log(f"split accel workload {k}: max rel err {e:.2e}")
    assert e <= 2e-12


def test_split_all_major_is_one_newton_step():
    s = S.config(1)
    ref = oracle.accel(s.pos, s.mass, s.G)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision="split", small_mass=0.0))
    e = rel(got, ref)
    # one Newton step leaves -3/2 e0^2 in 1/r, about 3x that in 1/r^3
    assert e <= 2e-12


def test_many_partials_step_bitwise():
    """65,600 bodies: the each-pair-once pass writes 257 partial slots, which
    the step epilogue adds with one thread per element.  Sampled
    accelerations against the oracle, and 4 steps bitwise equal to 2 + 2."""
    s = S.solar_system(65, 65600 - 31, n_major=30)
    m = T(s.mass)
    idx = np.unique(np.concatenate([[0, 1, 30, 31, s.n - 1],
                                    np.random.default_rng(2).choice(s.n, 40, replace=False)]))
    e = rel(H(nb.accel(T(s.pos), m, s.G))[:, idx], oracle.accel_targets(s.pos, s.mass, s.G, idx))
    log(f"n={s.n} sampled accel rel={e:.2e}")
    assert e <= 1e-13
    p1, v1 = T(s.pos), T(s.vel)
    nb.verlet_run(p1, v1, m, s.G, 0.1, 4)
    p2, v2 = T(s.pos), T(s.vel)
    nb.verlet_run(p2, v2, m, s.G, 0.1, 2)
    nb.verlet_run(p2, v2, m, s.G, 0.1, 2)
    assert np.array_equal(H(p1), H(p2)) and np.array_equal(H(v1), H(v2))


def test_split_131072_sampled_error():
    s = S.config(2)
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([[0, 1, 150, s.n - 1], rng.choice(s.n, 124, replace=False)]))
    ref = oracle.accel_targets(s.pos, s.mass, s.G, idx)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision="split"))[:, idx]
    e = rel(got, ref)
    log(f"split accel n=131072 sampled: max rel err {e:.2e}")
    assert e <= 2e-12


def test_split_vs_fp64_131072_full_run():
    """The 131,072-body workload run for its full 1000 steps in FP64 and in
    the split form from the same state: the final energies agree to 1e-10 of
    |E(0)|, and the split form's per-step accelerations (at the initial
    state and at its own final state) are within 2e-12 of the oracle on 258
    sampled targets, the FP64 form's within 1e-13."""
    s = S.config(2)
    assert s.n == 131072
    m = T(s.mass)
    E0 = H(nb.energy(T(s.pos), T(s.vel), m, s.G))[2]
    runs = {}
    for prec in ("fp64", "split"):
        p, v = T(s.pos), T(s.vel)
        nb.verlet_run(p, v, m, s.G, s.dt, 1000, precision=prec)
        runs[prec] = (p, v, H(nb.energy(p, v, m, s.G))[2])
    d = abs(runs["split"][2] - runs["fp64"][2]) / abs(E0)
    log(f"n=131072, 1000 steps: |E_split - E_fp64|/|E0| = {d:.2e}, "
        f"fp64 dE/E = {(runs['fp64'][2] - E0) / abs(E0):.2e}")
    assert d <= 1e-10
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([[0, 1, 30, 149, 150, s.n - 1],
                                    rng.choice(s.n, 252, replace=False)]))
    assert idx.size >= 256
    for label, pos in (("initial", s.pos), ("final", H(runs["split"][0]))):
        ref = oracle.accel_targets(pos, s.mass, s.G, idx)
        e64 = rel(H(nb.accel(T(pos), m, s.G))[:, idx], ref)
        esp = rel(H(nb.accel(T(pos), m, s.G, precision="split"))[:, idx], ref)
        log(f"n=131072 {label} state: sampled accel rel err fp64 {e64:.2e}, split {esp:.2e}")
        assert e64 <= 1e-13 and esp <= 2e-12


@pytest.mark.parametrize("k,steps", [(0, 3650), (1, 200), (1, 10000)])
def test_split_energy_matches_fp64(k, steps):
    s = S.config(k)
    m = T(s.mass)
    E0 = H(nb.energy(T(s.pos), T(s.vel), m, s.G))[2]
    p1, v1 = T(s.pos), T(s.vel)
    nb.verlet_run(p1, v1, m, s.G, s.dt, steps)
    p2, v2 = T(s.pos), T(s.vel)
    nb.verlet_run(p2, v2, m, s.G, s.dt, steps, precision="split")
    E1 = H(nb.energy(p1, v1, m, s.G))[2]
    E2 = H(nb.energy(p2, v2, m, s.G))[2]
    d = abs(E2 - E1) / abs(E0)
    log(f"split vs fp64 workload {k}, {steps} steps: |dE|/|E0| = {d:.2e}, "
        f"fp64 dE/E = {(E1 - E0) / abs(E0):.2e}")
    assert d <= 1e-10


# ---------------------------------------------------------------------------
# batched ensemble

def _small_ensemble(count=6, steps=40):
    rng = np.random.default_rng(7)
    systems = [S.solar_system(200 + k, int(rng.integers(1, 700)), n_major=int(rng.integers(1, 31)))
               for k in range(count)]
    systems.append(S.solar_system(300, 0, n_major=0))        # a lone Sun
    offs = np.zeros(len(systems) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([x.n for x in systems])
    cat = lambda f: np.ascontiguousarray(np.concatenate([f(x) for x in systems], axis=-1))
    return systems, offs, cat(lambda x: x.pos), cat(lambda x: x.vel), cat(lambda x: x.mass)


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_batched_matches_oracle(precision, variant):
    systems, offs, pos, vel, mass = _small_ensemble()
    steps = 40
    nb.set_tile(2, precision, 0, 2, 4 if variant == 2 else 1, 16, variant)
    p, v = T(pos), T(vel)
    nb.verlet_run_batched(p, v, T(mass), offs, S.G_AU_DAY_MSUN, 0.1, steps, precision=precision)
    P, V = H(p), H(v)
    for k, x in enumerate(systems):
        a, b = offs[k], offs[k + 1]
        pr, vr = oracle.verlet(x.pos, x.vel, x.mass, x.G, 0.1, steps)
        e = rel(P[:, a:b], pr)
        tol = 1e-12 if precision == "fp64" else 1e-10
        assert e <= tol, (k, x.n, e)


def _mixed_ensemble():
    """Systems of 12 ranges of 256 bodies and of one or two, and a lone Sun."""
    systems = [S.solar_system(401, 3000, n_major=30), S.solar_system(402, 600, n_major=12),
               S.solar_system(403, 40, n_major=3), S.solar_system(404, 0, n_major=0)]
    offs = np.zeros(len(systems) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([x.n for x in systems])
    cat = lambda f: np.ascontiguousarray(np.concatenate([f(x) for x in systems], axis=-1))
    return systems, offs, cat(lambda x: x.pos), cat(lambda x: x.vel), cat(lambda x: x.mass)


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("tile", [(4, 4, 1, 5), (2, 4, 1, 5)])
def test_batched_mutual_matches_oracle(precision, tile):
    """The ensemble with each pair once: one workgroup per (system, g, r),
    per-body partial counts equal to the system's ranges; every system
    against the oracle after 40 steps, and a bitwise repeat."""
    systems, offs, pos, vel, mass = _mixed_ensemble()
    nb.set_tile(2, precision, 0, *tile)
    outs = []
    for _ in range(2):
        p, v = T(pos), T(vel)
        nb.verlet_run_batched(p, v, T(mass), offs, S.G_AU_DAY_MSUN, 0.1, 40, precision=precision)
        outs.append((H(p), H(v)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    for k, x in enumerate(systems):
        a, b = offs[k], offs[k + 1]
        pr, vr = oracle.verlet(x.pos, x.vel, x.mass, x.G, 0.1, 40)
        e = rel(outs[0][0][:, a:b], pr)
        log(f"ensemble mutual {precision} {tile} system {k} (n={x.n}): pos {e:.2e}")
        assert e <= (1e-12 if precision == "fp64" else 1e-10), (k, x.n, e)
        assert rel(outs[0][1][:, a:b], vr) <= (1e-11 if precision == "fp64" else 1e-9)


def test_batched_mutual_falls_back_beyond_40_ranges():
    """A system of more than 10,240 bodies (41 ranges) exceeds the ensemble
    workspace's partial slots: the each-pair-once tile gives way to the
    heuristic one and the results still match the oracle."""
    systems = [S.solar_system(405, 10300, n_major=30), S.solar_system(406, 200, n_major=8)]
    assert systems[0].n > 40 * 256
    offs = np.zeros(3, dtype=np.int64)
    offs[1:] = np.cumsum([x.n for x in systems])
    cat = lambda f: np.ascontiguousarray(np.concatenate([f(x) for x in systems], axis=-1))
    nb.set_tile(2, "fp64", 0, 4, 4, 1, 5)
    p, v = T(cat(lambda x: x.pos)), T(cat(lambda x: x.vel))
    nb.verlet_run_batched(p, v, T(cat(lambda x: x.mass)), offs, S.G_AU_DAY_MSUN, 0.1, 2)
    P = H(p)
    for k, x in enumerate(systems):
        pr, _ = oracle.verlet(x.pos, x.vel, x.mass, x.G, 0.1, 2)
        assert rel(P[:, offs[k]:offs[k + 1]], pr) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_batched_autotune_then_parity(precision):
    systems, offs, pos, vel, mass = _small_ensemble(count=5)
    tile, ms = nb.autotune_batched(T(pos), T(mass), offs, S.G_AU_DAY_MSUN, precision)
    log(f"ensemble autotune {precision}: {tile} {ms:.4f} ms")
    assert tile == nb.get_tile(2, precision, 0)
    p, v = T(pos), T(vel)
    nb.verlet_run_batched(p, v, T(mass), offs, S.G_AU_DAY_MSUN, 0.1, 20, precision=precision)
    P = H(p)
    for k, x in enumerate(systems):
        pr, _ = oracle.verlet(x.pos, x.vel, x.mass, x.G, 0.1, 20)
        assert rel(P[:, offs[k]:offs[k + 1]], pr) <= (1e-12 if precision == "fp64" else 1e-10)


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("how", ["autotune", "mutual", "one-way"])
def test_batched_full_ensemble_sampled(precision, how):
    """The 512-system ensemble at full size, in the launch configuration the
    benchmark times (autotuned tile, one batched launch per step), and with
    the each-pair-once and the one-way tiles forced, against the oracle on
    the smallest, the largest and two random member systems."""
    systems, offs = S.ensemble(512)
    cat = lambda f: np.ascontiguousarray(np.concatenate([f(x) for x in systems], axis=-1))
    pos, vel, mass = cat(lambda x: x.pos), cat(lambda x: x.vel), cat(lambda x: x.mass)
    p, v, m = T(pos), T(vel), T(mass)
    if how == "autotune":
        tile, _ = nb.autotune_batched(p, m, offs, S.G_AU_DAY_MSUN, precision)
    else:
        tile = (4, 4, 1, 5) if how == "mutual" else (4, 1, 16, 0)
        nb.set_tile(2, precision, 0, *tile)
    steps = 3
    nb.verlet_run_batched(p, v, m, offs, S.G_AU_DAY_MSUN, 0.1, steps, precision=precision)
    P, V = H(p), H(v)
    sizes = np.diff(offs)
    rng = np.random.default_rng(11)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *rng.choice(512, 2, replace=False)})
    for k in pick:
        x = systems[k]
        pr, vr = oracle.verlet(x.pos, x.vel, x.mass, x.G, 0.1, steps)
        a, b = offs[k], offs[k + 1]
        ep, ev = rel(P[:, a:b], pr), rel(V[:, a:b], vr)
        log(f"ensemble {precision} tile {tile} system {k} (n={x.n}): pos {ep:.2e} vel {ev:.2e}")
        assert ep <= (1e-12 if precision == "fp64" else 1e-10)
        assert ev <= (1e-11 if precision == "fp64" else 1e-9)


def test_batched_graph_replay_deterministic():
    systems, offs, pos, vel, mass = _small_ensemble(count=4)
    outs = []
    for _ in range(2):
        p, v = T(pos), T(vel)
        nb.verlet_run_batched(p, v, T(mass), offs, S.G_AU_DAY_MSUN, 0.1, 300)
        outs.append(H(p))
    assert np.array_equal(outs[0], outs[1])
    x = systems[2]
    pr, _ = oracle.verlet(x.pos, x.vel, x.mass, x.G, 0.1, 300)
    assert rel(outs[0][:, offs[2]:offs[3]], pr) <= 1e-11


# ---------------------------------------------------------------------------
# autotuner

@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_autotune_small_system_then_parity(precision):
    """At n = 131 the candidates include the single-workgroup variant."""
    s = S.config(0)
    tile, ms = nb.autotune(T(s.pos), T(s.mass), s.G, precision=precision)
    log(f"autotune n=131 {precision}: {tile} {ms:.4f} ms/pass")
    assert tile == nb.get_tile(0, precision, s.n)
    ref = oracle.accel(s.pos, s.mass, s.G)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision=precision))
    assert rel(got, ref) <= (1e-13 if precision == "fp64" else 2e-12)
    pr, _ = _oracle_workload0()
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, T(s.mass), s.G, s.dt, s.steps, precision=precision)
    assert rel(H(p), pr) <= (1e-10 if precision == "fp64" else 1e-8)


def test_tuning_cache_round_trip(tmp_path):
    """Autotuned tile shapes saved as JSON and installed in a fresh table."""
    s = S.config(0)
    tiles = {prec: nb.autotune(T(s.pos), T(s.mass), s.G, precision=prec)[0]
             for prec in ("fp64", "split")}
    path = tmp_path / "tuning.json"
    nb.save_tuning(path)
    nb.reset_caches()
    assert nb.load_tuning(path) == 2
    for prec, tile in tiles.items():
        assert nb.get_tile(0, prec, s.n) == tile
    # a file from another device is ignored unless asked for
    import json
    doc = json.loads(path.read_text())
    doc["device"] = "another device"
    path.write_text(json.dumps(doc))
    nb.reset_caches()
    assert nb.load_tuning(path) == 0
    assert nb.load_tuning(path, strict_device=False) == 2


def test_autotune_then_parity():
    s = S.config(1)
    tile, ms = nb.autotune(T(s.pos), T(s.mass), s.G)
    log(f"autotune n=10425 fp64: {tile} {ms:.4f} ms/pass")
    assert tile == nb.get_tile(0, "fp64", s.n)
    ref = oracle.accel(s.pos, s.mass, s.G)
    assert rel(H(nb.accel(T(s.pos), T(s.mass), s.G)), ref) <= 1e-13
