"""The far-tile claim of the FP32C force over the radial order (force_algo 4).

Bodies of a system are ordered by distance from the star and cut into tiles of
64.  Per tile the device keeps, from the FP32 (high, low) split of every
position, the least and greatest |x_hi| (rounded down and up), the greatest
|x_lo| (rounded up) and the largest widened rc^2.  A pair of tiles is taken
from the high parts alone when the gap between their shells is at least 2^21
times the sum of their largest low-part norms and its square exceeds both rc^2
bounds.  The claim: for every i, j of two such tiles the high parts' difference
is within 2^-21 of its length of the true difference (|lo_i| + |lo_j| <= gap /
2^21 <= |xh_j - xh_i| / 2^21), and |x_j - x_i| exceeds both critical radii
(weight 1, no changeover pair).  The test emulates the device's FP32
arithmetic for the bounds and the test (numpy float32, rounding to nearest)
and checks the claim pair by pair in FP64, on random shells (0.01 to 50 AU, and
annuli of 0.5-5 and 0.9-1.1 AU) and on records placed at the threshold.
"""
import numpy as np

F = np.float32
KFAR = F(2.0 ** 21)


def tile_bounds(xh, xl, rc2):
    """One record per tile, as the pass that writes the FP32C records writes it."""
    r = np.sqrt((xh.astype(np.float64) ** 2).sum(1))
    lam = np.sqrt((xl.astype(np.float64) ** 2).sum(1))
    return np.array([F(r.min() * (1 - 2.0 ** -22)), F(r.max() * (1 + 2.0 ** -22)),
                     F(lam.max() * (1 + 2.0 ** -22)), rc2.max()], dtype=np.float32)


def far_tiles(a, b):
    """The device's test, operation by operation in float32."""
    gap = F(max(F(b[0] - a[1]), F(a[0] - b[1])) * F(1 - 2.0 ** -20))
    lhs = F(F(KFAR * F(a[2] + b[2])) * F(1 + 2.0 ** -20))
    rc = F(max(a[3], b[3]) * F(1 + 2.0 ** -18))
    return bool(gap >= lhs and F(gap * gap) >= rc)


def _system(rng, n, lo=0.01, hi=50.0):
    r = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    u = rng.normal(size=(n, 3))
    u[:, 2] *= rng.uniform(0.0, 1.0)
    u /= np.linalg.norm(u, axis=1)[:, None]
    x = r[:, None] * u
    rc = r * rng.uniform(1e-4, 3e-2, n)
    return x, rc


def test_far_tiles_hold_pair_by_pair():
    rng = np.random.default_rng(11)
    n_far = n_near = 0
    worst_pos = worst_rc = 0.0
    for trial in range(6):
        # wide shells, then annuli like the planetesimal disks (0.5-5 AU, 0.9-1.1 AU)
        x, rc = _system(rng, 2048, *[(0.01, 50.0), (0.5, 5.0), (0.9, 1.1)][trial % 3])
        order = np.argsort(np.linalg.norm(x, axis=1), kind="stable")
        x, rc = x[order], rc[order]
        xh = x.astype(np.float32)
        xl = (x - xh.astype(np.float64)).astype(np.float32)
        rc2 = (rc ** 2 * (1 + 2.0 ** -20)).astype(np.float32)
        nt = len(x) // 64
        recs = [tile_bounds(xh[64 * t:64 * t + 64], xl[64 * t:64 * t + 64], rc2[64 * t:64 * t + 64])
                for t in range(nt)]
        for ta in range(nt):
            for tb in range(ta + 1, nt):
                if not far_tiles(recs[ta], recs[tb]):
                    n_near += 1
                    continue
                n_far += 1
                A, B = slice(64 * ta, 64 * ta + 64), slice(64 * tb, 64 * tb + 64)
                dh = xh[B].astype(np.float64)[None, :, :] - xh[A].astype(np.float64)[:, None, :]
                dx = x[B][None, :, :] - x[A][:, None, :]
                err = np.linalg.norm(dh - dx, axis=2) / np.linalg.norm(dh, axis=2)
                worst_pos = max(worst_pos, err.max())
                assert err.max() <= 2.0 ** -21, (trial, ta, tb, err.max())
                d = np.linalg.norm(dx, axis=2)
                rcm = np.maximum(rc[A][:, None], rc[B][None, :])
                worst_rc = max(worst_rc, (rcm / d).max())
                assert np.all(d > rcm), (trial, ta, tb)
    # both outcomes occur in numbers, and the position bound is approached
    assert n_far > 1500 and n_near > 1000, (n_far, n_near)
    assert worst_pos > 2.0 ** -25, worst_pos


def test_threshold_records():
    """Records placed at the thresholds: whatever the float32 test passes meets
    the exact conditions (gap >= 2^21 (lam_a + lam_b), gap^2 >= rc^2)."""
    rng = np.random.default_rng(12)
    passed = failed = 0
    for _ in range(200000):
        lam = rng.uniform(1e-9, 1e-6, 2)
        rc2 = rng.uniform(1e-8, 1e-2, 2)
        need = max(2.0 ** 21 * lam.sum(), np.sqrt(rc2.max()))
        gap = need * (1 + rng.uniform(-4e-6, 4e-6))
        rmax_a = rng.uniform(0.1, 40.0)
        a = np.array([rmax_a * rng.uniform(0.5, 1.0), rmax_a, lam[0], rc2[0]], dtype=np.float32)
        b = np.array([float(a[1]) + gap, float(a[1]) + gap + 1.0, lam[1], rc2[1]], dtype=np.float32)
        if rng.uniform() < 0.5:
            a, b = b, a
        if far_tiles(a, b):
            passed += 1
            g = max(float(b[0]) - float(a[1]), float(a[0]) - float(b[1]))
            assert g >= 2.0 ** 21 * (float(a[2]) + float(b[2]))
            assert g * g > max(float(a[3]), float(b[3]))
        else:
            failed += 1
    assert passed > 10000 and failed > 10000, (passed, failed)


def test_tile_bounds_enclose_the_tile():
    rng = np.random.default_rng(13)
    for _ in range(200):
        x, rc = _system(rng, 64)
        xh = x.astype(np.float32)
        xl = (x - xh.astype(np.float64)).astype(np.float32)
        rc2 = (rc ** 2).astype(np.float32)
        rec = tile_bounds(xh, xl, rc2)
        r = np.sqrt((xh.astype(np.float64) ** 2).sum(1))
        lam = np.sqrt((xl.astype(np.float64) ** 2).sum(1))
        assert float(rec[0]) <= r.min() and float(rec[1]) >= r.max()
        assert float(rec[2]) >= lam.max() and rec[3] == rc2.max()
