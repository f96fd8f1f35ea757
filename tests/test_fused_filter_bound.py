"""The FP32 midpoint-reach filter of the force pass with the encounter test in
it keeps every pair that the FP64 reach filter keeps.

The FP64 filter keeps a pair when |M_j - M_i| <= R_i + R_j (chord midpoints M,
reaches R, both from the drift; the reach bound itself is checked against the
oracle's exact minimum in test_reach_bound.py).  The fused pass evaluates it
in FP32 from M rounded to FP32 and a reach widened to
    R' = fl32((R + 2^-21 |M|_1) (1 + 2^-18)),
comparing fl(D^2) <= fl(fl(R'_i + R'_j)^2) with D^2 summed by fused
multiply-adds.  The widening covers the rounding of M (2^-24 |M| per
component), of the differences, of the squares and sums, and of R' itself.
Here pairs are placed at and just inside the FP64 reach, at heliocentric
distances up to 50 AU and reaches from 1e-6 to 1 AU, and the FP32 filter
(emulated in numpy, once with fused and once with separate roundings) must
keep every one of them.
"""
import numpy as np


def _widened(M, R):
    w = (R + 2.0 ** -21 * np.abs(M).sum(axis=-1)) * (1.0 + 2.0 ** -18)
    return w.astype(np.float32)


def _fmaf(a, b, c):
    # fl32(a b + c): the product of two floats is exact in FP64
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _keeps(Mi, Mj, Ri, Rj, fused):
    mi, mj = Mi.astype(np.float32), Mj.astype(np.float32)
    e = mj - mi                                   # FP32 differences
    if fused:
        d2 = _fmaf(e[:, 2], e[:, 2], _fmaf(e[:, 1], e[:, 1], e[:, 0] * e[:, 0]))
    else:
        d2 = (e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2]
    s = _widened(Mj, Rj) + _widened(Mi, Ri)
    return d2 <= s * s


def test_fp32_filter_keeps_every_pair_the_fp64_reach_keeps():
    rng = np.random.default_rng(7)
    n = 400000
    r = 10.0 ** rng.uniform(-1, np.log10(50.0), n)
    u = rng.normal(size=(n, 3))
    Mi = u / np.linalg.norm(u, axis=1)[:, None] * r[:, None]
    Ri = 10.0 ** rng.uniform(-6, 0, n)
    Rj = 10.0 ** rng.uniform(-6, 0, n)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    # separations at the reach, just inside it, and well inside
    f = rng.choice([1.0, 1.0 - 1e-15, 1.0 - 1e-9, 0.999, 0.5], n)
    Mj = Mi + d * ((Ri + Rj) * f)[:, None]
    D = np.linalg.norm(Mj - Mi, axis=1)
    inside = D <= Ri + Rj                         # what the FP64 filter keeps
    assert inside.mean() > 0.6
    for fused in (True, False):
        keep = _keeps(Mi, Mj, Ri, Rj, fused)
        missed = inside & ~keep
        assert not missed.any(), (fused, np.flatnonzero(missed)[:5])


def test_fp32_filter_still_drops_distant_pairs():
    """The widening is small: pairs 1 % beyond the reach are dropped."""
    rng = np.random.default_rng(8)
    n = 100000
    Mi = rng.uniform(-5, 5, (n, 3))
    Ri = 10.0 ** rng.uniform(-3, -1, n)
    Rj = 10.0 ** rng.uniform(-3, -1, n)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    Mj = Mi + d * (1.01 * (Ri + Rj))[:, None]
    assert not _keeps(Mi, Mj, Ri, Rj, True).any()
