"""The FP32 relative-chord filter (of the sorted encounter check, and of the
force pass with the encounter test in it) keeps every pair that can be flagged.

The encounter predicate's Hermite data split around the relative chord
dc = c_j - c_i give, for a pair whose chord midpoints are D apart,
f(s) > rc_ij^2 whenever D > |dc| + bb, bb = 3/4 (eps_i + eps_j) + rc_ij (the
argument of the encounter kernels, checked on the oracle in
test_reach_bound.py).  So a flagged pair has D <= |dc| + bb.  The filter
tests, in FP32, fl(D^2) <= fl(fl(|dc|^2) + S^2) * 2 (1 + 2^-18) with
S = fl(fl(b'_i + b'_j) + max(rc'_i, rc'_j)) and per body
    b' = fl32((3/4 eps + 2^-21 (|M|_1 + |c|_1)) (1 + 2^-18)),
    rc' = fl32(rc (1 + 2^-20)),
from the midpoints M and chords c rounded to FP32.  As (x + y)^2 <= 2 x^2 + 2 y^2
the test keeps every pair with D <= |dc| + bb once the widening covers the
rounding of M, c, their differences, the squares and sums.  Here pairs are
placed at and just inside D = |dc| + bb, at heliocentric distances up to 50 AU,
chords up to 1 AU and bounds from 1e-6 to 1 AU, and the FP32 filter (emulated
in numpy, once with fused and once with separate roundings) must keep every
one of them; pairs beyond the widened bound are dropped.
"""
import numpy as np

F32 = np.float32


def _bound(M, c, e34):
    w = (e34 + 2.0 ** -21 * (np.abs(M).sum(axis=-1) + np.abs(c).sum(axis=-1))) * (1.0 + 2.0 ** -18)
    return w.astype(F32)


def _rc32(rc):
    return (rc * (1.0 + 2.0 ** -20)).astype(F32)


def _fmaf(a, b, c):
    # fl32(a b + c): the product of two floats is exact in FP64
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def _norm2(e, fused):
    if fused:
        return _fmaf(e[:, 2], e[:, 2], _fmaf(e[:, 1], e[:, 1], e[:, 0] * e[:, 0]))
    return (e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2]


def _keeps(Mi, Mj, ci, cj, bi, bj, rci, rcj, fused):
    D2 = _norm2(Mj.astype(F32) - Mi.astype(F32), fused)
    C2 = _norm2(cj.astype(F32) - ci.astype(F32), fused)
    S = (bj + bi) + np.maximum(rci, rcj)
    rhs = (_fmaf(S, S, C2) if fused else C2 + S * S) * F32(2.0 * (1.0 + 2.0 ** -18))
    return D2 <= rhs


def _pairs(rng, n):
    r = 10.0 ** rng.uniform(-1, np.log10(50.0), n)
    u = rng.normal(size=(n, 3))
    Mi = u / np.linalg.norm(u, axis=1)[:, None] * r[:, None]
    ci = rng.normal(size=(n, 3)) * 10.0 ** rng.uniform(-4, 0, n)[:, None]
    cj = ci + rng.normal(size=(n, 3)) * 10.0 ** rng.uniform(-6, 0, n)[:, None]
    e34 = 10.0 ** rng.uniform(-7, -1, (2, n))
    rc = 10.0 ** rng.uniform(-6, -1, (2, n))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    bb = e34[0] + e34[1] + np.maximum(rc[0], rc[1])
    C = np.linalg.norm(cj - ci, axis=1)
    return Mi, ci, cj, e34, rc, d, C + bb


def test_fp32_filter_keeps_every_pair_that_can_be_flagged():
    rng = np.random.default_rng(7)
    n = 400000
    Mi, ci, cj, e34, rc, d, lim = _pairs(rng, n)
    f = rng.choice([1.0, 1.0 - 1e-15, 1.0 - 1e-9, 0.999, 0.5], n)
    Mj = Mi + d * (lim * f)[:, None]
    inside = np.linalg.norm(Mj - Mi, axis=1) <= lim
    assert inside.mean() > 0.6
    bi = _bound(Mi, ci, e34[0])
    bj = _bound(Mj, cj, e34[1])
    rci, rcj = _rc32(rc[0]), _rc32(rc[1])
    for fused in (True, False):
        keep = _keeps(Mi, Mj, ci, cj, bi, bj, rci, rcj, fused)
        missed = inside & ~keep
        assert not missed.any(), (fused, np.flatnonzero(missed)[:5])


def test_fp32_filter_drops_pairs_beyond_the_widened_bound():
    """The filter is no looser than its stated form where the bounds exceed the
    FP32 rounding of the positions (heliocentric distances to 5 AU, bounds from
    1e-4 AU): pairs 1 % beyond sqrt(2 |dc|^2 + 2 S^2) are dropped."""
    rng = np.random.default_rng(8)
    n = 100000
    Mi = rng.uniform(-5, 5, (n, 3))
    ci = rng.normal(size=(n, 3)) * 10.0 ** rng.uniform(-3, -1, n)[:, None]
    cj = ci + rng.normal(size=(n, 3)) * 10.0 ** rng.uniform(-3, -1, n)[:, None]
    e34 = 10.0 ** rng.uniform(-4, -1, (2, n))
    rc = 10.0 ** rng.uniform(-4, -1, (2, n))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    C = np.linalg.norm(cj - ci, axis=1)
    bi = _bound(Mi, ci, e34[0]).astype(np.float64)
    bj = _bound(Mi, cj, e34[1]).astype(np.float64)
    rci, rcj = _rc32(rc[0]), _rc32(rc[1])
    S = bi + bj + np.maximum(rci, rcj).astype(np.float64)
    lim = np.sqrt(2 * C ** 2 + 2 * S ** 2)
    Mj = Mi + d * (1.01 * lim)[:, None]
    assert not _keeps(Mi, Mj, ci, cj, _bound(Mi, ci, e34[0]), _bound(Mj, cj, e34[1]), rci, rcj, True).any()

