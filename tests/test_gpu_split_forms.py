"""The two split-precision forms against the FP64 oracle.

"split" (precision 1) is the library's fast form; "compensated" (precision
2) is the split form as specified: FP64 displacement and squared distance,
1/|r|^3 from the FP32 reciprocal square root refined by one FP64 Newton step
for every pair, heavy sources' terms in FP64 and light sources' terms rounded
to FP32 and added to FP32 Kahan sums.

Pin of the compensated FP32 sums (all sources light: the threshold above
every mass).  Each term x = float(G m f) * float(d) differs from the exact
term t by at most about 2u|t| (two roundings to FP32, u = 2^-24; the FP64
displacement and the Newton-refined factor are exact to ~1e-12 relative);
Kahan's compensated sum of the x is within (2u + O(n u^2)) sum |x| of their
exact sum (Higham, Accuracy and Stability of Numerical Algorithms, on
compensated summation); the per-workgroup sums are then added in FP64.  Per
body and component:
    |a_gpu - a_oracle| <= (2u + n u^2 + 3u) sum_j |t_j|  (+ FP64 roundoff).
The split form's FP32 tiles form every term in FP32 (FP32 displacement,
squared distance, v_rsq_f32 with relative error <= 2^-23.1 as measured, the
cube, the product with float(G m)): about 18u per term; and sum blocks of 16
terms by FMA (<= 15u sum |t| for a block), each block added in FP64:
    |a_gpu - a_oracle| <= 34u sum_j |t_j|.
sum_j |t_j| is computed here in FP64 with NumPy."""
import numpy as np
import pytest
import torch

import oracle
import solar_ics as S

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2112_15079_amd")
from paper_2112_15079_amd import _capi as C  # noqa: E402

DEV = "cuda:0"
U = 2.0 ** -24


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
def _fresh_tiles():
    nb.reset_caches()
    yield
    nb.reset_caches()


def abs_term_sums(pos, mass, G, block=256):
    """S[k, p] = sum_{j != p} |G m_j (r_j - r_p)_k| / |r_j - r_p|^3 (FP64)."""
    n = mass.shape[0]
    out = np.empty((3, n))
    for p0 in range(0, n, block):
        p1 = min(n, p0 + block)
        d = pos[:, None, :] - pos[:, p0:p1, None]            # (3, b, n): r_j - r_p
        r2 = np.einsum("kbn,kbn->bn", d, d)
        r2[np.arange(p1 - p0), np.arange(p0, p1)] = np.inf   # the self pair
        w = G * mass[None, :] / (r2 * np.sqrt(r2))
        out[:, p0:p1] = np.einsum("kbn,bn->kb", np.abs(d), w)
    return out


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("precision,coef", [("compensated", None), ("split", 34.0)])
def test_all_light_error_bound(k, precision, coef):
    """Every source light (threshold 2 Msun, the Sun included): per body and
    component the error against the oracle stays within the bound of the
    form's arithmetic (see the module docstring)."""
    s = S.config(k)
    ref = oracle.accel(s.pos, s.mass, s.G)
    if precision == "split":
        nb.set_tile(0, "split", s.n, 4, 4, 1, 5)   # the FP32 tiles of the pair-once pass
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision=precision, small_mass=2.0))
    Sabs = abs_term_sums(s.pos, s.mass, s.G)
    c = (5.0 + s.n * U) if coef is None else coef
    bound = c * U * Sabs + 8 * 2.0 ** -53 * Sabs
    err = np.abs(got - ref)
    ratio = float(np.max(err / bound))
    print(f"{precision} k={k} n={s.n}: max err / bound = {ratio:.3f}, "
          f"max err / (u sum|t|) = {float(np.max(err / (U * Sabs))):.2f}", flush=True)
    assert ratio <= 1.0


@pytest.mark.parametrize("k", [0, 1])
def test_compensated_matches_oracle(k):
    """Workloads with the usual threshold (3e17 kg): accelerations within 2e-12
    of the oracle per body, and a 100-step run within 1e-10 in position."""
    s = S.config(k)
    m = T(s.mass)
    ref = oracle.accel(s.pos, s.mass, s.G)
    e = rel(H(nb.accel(T(s.pos), m, s.G, precision="compensated")), ref)
    p, v = T(s.pos), T(s.vel)
    nb.verlet_run(p, v, m, s.G, s.dt, 100, precision="compensated")
    pr, _ = oracle.verlet(s.pos, s.vel, s.mass, s.G, s.dt, 100)
    P = H(p)
    ep = float(np.max(np.linalg.norm(P - pr, axis=0)[1:] / np.linalg.norm(pr, axis=0)[1:]))
    print(f"compensated k={k}: accel rel err {e:.2e}, 100-step position rel err {ep:.2e}",
          flush=True)
    assert e <= 2e-12 and ep <= 1e-10


def test_compensated_all_heavy_is_one_newton_step():
    """Threshold 0: every term in FP64 with the one-Newton-step factor, whose
    relative error is at most about 3/2 e0^2 in 1/r (e0 <= 2^-23.1), about
    three times that in 1/r^3."""
    s = S.config(1)
    ref = oracle.accel(s.pos, s.mass, s.G)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision="compensated", small_mass=0.0))
    assert rel(got, ref) <= 2e-12


def test_compensated_131072_sampled():
    s = S.config(2)
    rng = np.random.default_rng(12)
    idx = np.unique(np.concatenate([[0, 1, 149, 150, s.n - 1], rng.choice(s.n, 251, replace=False)]))
    ref = oracle.accel_targets(s.pos, s.mass, s.G, idx)
    got = H(nb.accel(T(s.pos), T(s.mass), s.G, precision="compensated"))[:, idx]
    e = rel(got, ref)
    print(f"compensated n=131072 sampled: max rel err {e:.2e}", flush=True)
    assert e <= 2e-12


def test_compensated_energy_and_determinism():
    """1000 steps of the 10,425-body workload: the compensated run's energy
    within 1e-10 of |E(0)| of the FP64 run's, bitwise repeatable, and a run
    of 600 + 400 steps equals one of 1000."""
    s = S.config(1)
    m = T(s.mass)
    E0 = H(nb.energy(T(s.pos), T(s.vel), m, s.G))[2]
    p1, v1 = T(s.pos), T(s.vel)
    nb.verlet_run(p1, v1, m, s.G, s.dt, 1000)
    outs = []
    for split in ([1000], [1000], [600, 400]):
        p, v = T(s.pos), T(s.vel)
        for k in split:
            nb.verlet_run(p, v, m, s.G, s.dt, k, precision="compensated")
        outs.append((H(p), H(v), p, v))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    E1 = H(nb.energy(p1, v1, m, s.G))[2]
    E2 = H(nb.energy(outs[0][2], outs[0][3], m, s.G))[2]
    d = abs(E2 - E1) / abs(E0)
    print(f"compensated vs fp64 after 1000 steps: |dE|/|E0| = {d:.2e}", flush=True)
    assert d <= 1e-10


def test_compensated_ensemble_matches_oracle():
    rng = np.random.default_rng(13)
    systems = [S.solar_system(300 + k, int(rng.integers(1, 900)), n_major=int(rng.integers(1, 31)))
               for k in range(5)]
    offs = np.concatenate([[0], np.cumsum([x.n for x in systems])])
    cat = lambda f: np.ascontiguousarray(np.concatenate([f(x) for x in systems], axis=-1))
    p, v, m = T(cat(lambda x: x.pos)), T(cat(lambda x: x.vel)), T(cat(lambda x: x.mass))
    nb.verlet_run_batched(p, v, m, offs, systems[0].G, 0.1, 30, precision="compensated")
    P = H(p)
    for k, x in enumerate(systems):
        pr, _ = oracle.verlet(x.pos, x.vel, x.mass, x.G, 0.1, 30)
        got = P[:, offs[k]:offs[k + 1]]
        e = np.linalg.norm(got - pr, axis=0)[1:] / np.linalg.norm(pr, axis=0)[1:]
        assert e.size == 0 or e.max() <= 1e-10, (k, x.n, e.max())


def test_compensated_refuses_more_than_131072_bodies():
    s = S.solar_system(65, 131073 - 31, n_major=30)
    with pytest.raises(C.NBodyError, match="compensated"):
        nb.accel(T(s.pos), T(s.mass), s.G, precision="compensated")
