"""One GPU's share of the force pass (nbody_accel_shard): the FP64
accelerations of a contiguous range of targets from all sources, against the
oracle at 1e-13 relative per body, for single bodies, ragged and unaligned
ranges, whole systems, the eight shares of the 10,425-body workload and two
of the eight shares of the 131,072-body workload (sampled)."""
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


def shares(n, g):
    w = -(-n // g)
    return [(k * w, min(w, n - k * w)) for k in range(g) if k * w < n]


@pytest.mark.parametrize("n_small,t0,nt", [
    (200, 0, 231), (200, 0, 1), (200, 230, 1), (200, 37, 100), (200, 64, 64),
    (3000, 0, 3031), (3000, 1000, 1), (3000, 255, 258), (3000, 2900, 131),
    (40000, 0, 40031), (40000, 12345, 6789), (40000, 40030, 1),
])
def test_share_matches_oracle(n_small, t0, nt):
    s = S.solar_system(60 + n_small % 97, n_small, n_major=30)
    assert t0 + nt <= s.n
    print(f"n={s.n} targets [{t0}, {t0 + nt})", flush=True)
    got = H(nb.accel_shard(T(s.pos), T(s.mass), s.G, t0, nt))
    idx = np.arange(t0, t0 + nt)
    if len(idx) > 512:   # the oracle on a sample of the range, its ends included
        rng = np.random.default_rng(nt)
        pick = np.unique(np.concatenate([[0, nt - 1], rng.choice(nt, 254, replace=False)]))
        idx, got = idx[pick], got[:, pick]
    ref = oracle.accel_targets(s.pos, s.mass, s.G, idx)
    assert rel(got, ref) <= 1e-13


def test_eight_shares_of_10425_body_workload():
    """The eight shares together give the whole pass: each within 1e-13 of
    the oracle; their concatenation within 1e-13 of nbody_accel."""
    s = S.config(1)
    pos, m = T(s.pos), T(s.mass)
    ref = oracle.accel(s.pos, s.mass, s.G)
    parts = []
    for t0, nt in shares(s.n, 8):
        got = H(nb.accel_shard(pos, m, s.G, t0, nt))
        e = rel(got, ref[:, t0:t0 + nt])
        print(f"share [{t0}, {t0 + nt}): rel err {e:.2e}", flush=True)
        assert e <= 1e-13
        parts.append(got)
    whole = np.concatenate(parts, axis=1)
    assert whole.shape == (3, s.n)
    assert rel(whole, H(nb.accel(pos, m, s.G))) <= 1e-13


def test_shares_of_131072_body_workload_sampled_and_repeatable():
    s = S.config(2)
    pos, m = T(s.pos), T(s.mass)
    for t0, nt in (shares(s.n, 8)[0], shares(s.n, 8)[-1]):
        a = nb.accel_shard(pos, m, s.G, t0, nt)
        b = nb.accel_shard(pos, m, s.G, t0, nt)
        assert torch.equal(a, b)
        rng = np.random.default_rng(t0)
        pick = np.unique(np.concatenate([[0, nt - 1], rng.choice(nt, 254, replace=False)]))
        ref = oracle.accel_targets(s.pos, s.mass, s.G, t0 + pick)
        e = rel(H(a)[:, pick], ref)
        print(f"share [{t0}, {t0 + nt}): rel err {e:.2e} on {len(pick)} targets", flush=True)
        assert e <= 1e-13


def test_share_rejects_ranges_outside_the_system():
    s = S.solar_system(61, 20, n_major=3)
    pos, m = T(s.pos), T(s.mass)
    for t0, nt in ((-1, 3), (0, 0), (s.n - 1, 2)):
        with pytest.raises(Exception):
            nb.accel_shard(pos, m, s.G, t0, nt)
