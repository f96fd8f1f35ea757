"""The encounter prefilter's claim, checked against the oracle's predicate.

The device encounter check skips a pair when the chord midpoints of the two
bodies are farther apart than R_i + R_j, with R = 2 rho + 3 eps/4 + rc
(rho: half the chord Q1 - Q0; eps: the larger of |dt V0 - c|, |dt V1 - c|).
The argument: the Hermite data split into the straight-chord quadratic
|dQ0 + s dc|^2 >= (D - rho_i - rho_j)^2 plus the velocity deviations weighted
by h10(s), h11(s) with |h10| + |h11| = s(1-s) <= 1/4.  Here the claim is
tested on arbitrary (non-physical) Hermite data placed just outside the reach,
and on Kepler arcs, with the oracle's exact minimum as the reference.
"""
import numpy as np

import oracle
import workloads


def reach(q0, v0, q1, v1, rc, dt):
    c = q1 - q0
    rho = 0.5 * np.linalg.norm(c)
    eps = max(np.linalg.norm(dt * v0 - c), np.linalg.norm(dt * v1 - c))
    return 2 * rho + 0.75 * eps + rc, 0.5 * (q0 + q1)


def _body(rng, scale):
    q0 = rng.normal(size=3) * scale
    v0 = rng.normal(size=3)
    q1 = q0 + rng.normal(size=3) * scale * rng.uniform(0, 2)
    v1 = rng.normal(size=3) * rng.uniform(0, 3)
    return q0, v0, q1, v1


def test_bound_holds_just_outside_the_reach():
    rng = np.random.default_rng(2024)
    worst = np.inf
    for trial in range(20000):
        dt = rng.uniform(0.01, 2.0) * rng.choice([-1, 1])
        bi = _body(rng, rng.uniform(0.01, 1))
        bj = list(_body(rng, rng.uniform(0.01, 1)))
        rci, rcj = rng.uniform(0, 0.5, 2)
        Ri, Mi = reach(*bi, rci, dt)
        Rj, Mj = reach(*bj, rcj, dt)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        target = Mi + u * (Ri + Rj) * (1 + rng.uniform(1e-9, 0.05))
        shift = target - Mj
        bj[0] = bj[0] + shift
        bj[2] = bj[2] + shift
        d2 = oracle.pair_min_d2(dt, *bi, *bj)
        thr = max(rci, rcj) ** 2
        assert d2 > thr, (trial, d2, thr)
        worst = min(worst, (d2 - thr) / max(thr, 1e-300))
    assert worst > 0


def test_bound_on_kepler_arcs_of_a_dense_ring():
    """Every flagged pair of a dense ring lies within the reach sum."""
    w = workloads.ring(400, m=1e-7)
    Q0, V0 = oracle.helio_to_dh(1.0, w.m, w.x, w.v)
    rc = oracle.rcrit(1.0, w.m, Q0)
    for dt in (0.04, 0.2, -0.1):
        Q1, V1, _ = oracle.drift(w.G, dt, Q0, V0)
        out = oracle.encounters(dt, Q0, V0, Q1, V1, rc)
        R = np.empty(400); M = np.empty((400, 3))
        for i in range(400):
            R[i], M[i] = reach(Q0[i], V0[i], Q1[i], V1[i], rc[i], dt)
        for i, j in zip(out["ice"], out["jce"]):
            assert np.linalg.norm(M[j] - M[i]) <= R[i] + R[j]
        assert out["nce"] > 0


def _tile(rng, k, center_scale, spread, dt):
    """k bodies whose midpoints, chords and velocity deviations cluster."""
    base_q = rng.normal(size=3) * center_scale
    base_c = rng.normal(size=3) * spread * rng.uniform(0.5, 5)
    out = []
    for _ in range(k):
        q0 = base_q + rng.normal(size=3) * spread
        c = base_c + rng.normal(size=3) * spread * 0.3
        q1 = q0 + c
        v0 = (c + rng.normal(size=3) * spread * 0.2) / dt
        v1 = (c + rng.normal(size=3) * spread * 0.2) / dt
        out.append((q0, v0, q1, v1))
    return out


def tile_bounds(bodies, rcs, dt):
    """Centre/spread of chord midpoints M, chords c and velocity deviations e."""
    M = np.array([0.5 * (b[0] + b[2]) for b in bodies])
    C = np.array([b[2] - b[0] for b in bodies])
    e0 = np.array([dt * b[1] - (b[2] - b[0]) for b in bodies])
    e1 = np.array([dt * b[3] - (b[2] - b[0]) for b in bodies])
    eb, se = 0.5 * (e0 + e1), 0.5 * np.linalg.norm(e0 - e1, axis=1)
    CM, Cc, Ce = M.mean(0), C.mean(0), eb.mean(0)
    return (CM, np.max(np.linalg.norm(M - CM, axis=1)), Cc, np.max(np.linalg.norm(C - Cc, axis=1)),
            Ce, np.max(np.linalg.norm(eb - Ce, axis=1) + se), max(rcs))


def tiles_may_meet(A, B):
    """False only if no pair (i in A, j in B) can be flagged:
    |L(s)| >= D - S_M - C_m/2 = Lmin, |dQ| <= D + S_M + C_m/2 = Qmax,
    |de| <= E_m, f >= Lmin^2 - Qmax E_m / 2 (basis weights |h10| + |h11| <= 1/4)."""
    D = np.linalg.norm(B[0] - A[0])
    Cm = np.linalg.norm(B[2] - A[2]) + A[3] + B[3]
    Em = np.linalg.norm(B[4] - A[4]) + A[5] + B[5]
    Lmin = D - A[1] - B[1] - 0.5 * Cm
    Qmax = D + A[1] + B[1] + 0.5 * Cm
    RC = max(A[6], B[6])
    return not (Lmin > 0 and Lmin * Lmin - 0.5 * Qmax * Em > RC * RC)


def test_tile_pair_bound_never_drops_a_flagged_pair():
    rng = np.random.default_rng(77)
    checked = culled = 0
    for trial in range(400):
        dt = rng.uniform(0.01, 0.2)
        spread = 10 ** rng.uniform(-3, -1)
        A = _tile(rng, 6, 1.0, spread, dt)
        B = _tile(rng, 6, 1.0, spread, dt)
        # pull B towards A so that many tile pairs are near the cull boundary
        shift = (np.mean([b[0] for b in A], 0) - np.mean([b[0] for b in B], 0)) * rng.uniform(0.5, 1.0)
        B = [(q0 + shift, v0, q1 + shift, v1) for q0, v0, q1, v1 in B]
        rca = rng.uniform(0, 3 * spread, 6)
        rcb = rng.uniform(0, 3 * spread, 6)
        ok = tiles_may_meet(tile_bounds(A, rca, dt), tile_bounds(B, rcb, dt))
        culled += not ok
        for a, ra in zip(A, rca):
            for b, rb in zip(B, rcb):
                d2 = oracle.pair_min_d2(dt, *a, *b)
                if d2 <= max(ra, rb) ** 2:
                    assert ok, trial
                checked += 1
    assert culled > 50 and checked == 400 * 36



def lane_ball(body, rc, dt):
    """One body as a tile of the tile-pair test, from its FP32 records as the
    sorted check stores them: midpoint M, chord c and mean endpoint deviation eb
    rounded to FP32, each a ball of 2^-23 of its norm; the deviation radius se
    and rc rounded to FP32 after a 2^-20 relative increase."""
    q0, v0, q1, v1 = body
    c = q1 - q0
    M = q0 + 0.5 * c
    e0, e1 = dt * v0 - c, dt * v1 - c
    eb, se = 0.5 * (e0 + e1), 0.5 * np.linalg.norm(e0 - e1)
    f = np.float32
    M32, c32, eb32 = (x.astype(f).astype(np.float64) for x in (M, c, eb))
    se32 = float(f(se * (1 + 2.0 ** -20)))
    rc32 = float(f(rc * (1 + 2.0 ** -20)))
    n = np.linalg.norm
    return (M32, 2.0 ** -23 * n(M32), c32, 2.0 ** -23 * n(c32), eb32, se32 + 2.0 ** -23 * n(eb32), rc32)


def test_lane_ball_against_a_tile_never_drops_a_flagged_pair():
    """The sorted check's lane test: a target body, from its rounded FP32 records,
    against the bounds of a source tile.  Lanes pulled toward the tile so that
    many sit near the cull boundary; whenever the oracle flags the lane with a
    body of the tile, the test keeps the lane."""
    rng = np.random.default_rng(99)
    checked = culled = 0
    for trial in range(3000):
        dt = rng.uniform(0.01, 0.2)
        spread = 10 ** rng.uniform(-3, -1)
        B = _tile(rng, 8, 1.0, spread, dt)
        a = _tile(rng, 1, 1.0, spread, dt)[0]
        shift = (np.mean([b[0] for b in B], 0) - a[0]) * rng.uniform(0.6, 1.0)
        a = (a[0] + shift, a[1], a[2] + shift, a[3])
        rca = rng.uniform(0, 3 * spread)
        rcb = rng.uniform(0, 3 * spread, 8)
        ok = tiles_may_meet(lane_ball(a, rca, dt), tile_bounds(B, rcb, dt))
        culled += not ok
        for b, rb in zip(B, rcb):
            d2 = oracle.pair_min_d2(dt, *a, *b)
            if d2 <= max(rca, rb) ** 2:
                assert ok, trial
                checked += 1
    assert culled > 300 and checked > 300


def relative_bound_culls(bi, bj, rci, rcj, dt):
    """The pair filter on relative chords: with dM the midpoint difference, dc
    the chord difference, E = eps_i + eps_j and b = 3E/4 + max(rc_i, rc_j), a pair
    with |dM|^2 > 2 |dc|^2 + 2 b^2 cannot be flagged.  (Hermite data = relative
    chord quadratic, >= (D - |dc|/2)^2, plus deviations weighted by
    |h10| + |h11| <= 1/4; D > |dc| + 3E/4 + rc suffices, and
    (|dc| + b)^2 <= 2 |dc|^2 + 2 b^2.)"""
    def parts(q0, v0, q1, v1):
        c = q1 - q0
        eps = max(np.linalg.norm(dt * v0 - c), np.linalg.norm(dt * v1 - c))
        return 0.5 * (q0 + q1), c, eps
    Mi, ci, ei = parts(*bi)
    Mj, cj, ej = parts(*bj)
    D2 = np.sum((Mj - Mi) ** 2)
    C2 = np.sum((cj - ci) ** 2)
    b = 0.75 * (ei + ej) + max(rci, rcj)
    return D2 > 2 * C2 + 2 * b * b


def test_relative_chord_bound_holds_just_outside():
    rng = np.random.default_rng(4242)
    for trial in range(20000):
        dt = rng.uniform(0.01, 2.0) * rng.choice([-1, 1])
        bi = _body(rng, rng.uniform(0.01, 1))
        bj = list(_body(rng, rng.uniform(0.01, 1)))
        # often co-moving: j's chord close to i's
        if rng.uniform() < 0.5:
            bj[2] = bj[0] + (bi[2] - bi[0]) + rng.normal(size=3) * 1e-3
        rci, rcj = rng.uniform(0, 0.5, 2)
        # put j's midpoint just beyond the filter radius along a random direction
        c_i, c_j = bi[2] - bi[0], bj[2] - bj[0]
        eps = lambda b: max(np.linalg.norm(dt * b[1] - (b[2] - b[0])), np.linalg.norm(dt * b[3] - (b[2] - b[0])))
        b = 0.75 * (eps(bi) + eps(bj)) + max(rci, rcj)
        radius = np.sqrt(2 * np.sum((c_j - c_i) ** 2) + 2 * b * b) * (1 + rng.uniform(1e-9, 0.05))
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        Mi = 0.5 * (bi[0] + bi[2])
        shift = Mi + u * radius - 0.5 * (bj[0] + bj[2])
        bj[0] = bj[0] + shift
        bj[2] = bj[2] + shift
        assert relative_bound_culls(bi, bj, rci, rcj, dt)
        d2 = oracle.pair_min_d2(dt, *bi, *bj)
        assert d2 > max(rci, rcj) ** 2, (trial, d2)


def test_relative_chord_bound_on_ring_arcs():
    """Every flagged pair of a dense ring passes the relative filter, and the
    filter keeps far fewer pairs than the per-body reach."""
    w = workloads.ring(400, m=1e-7)
    Q0, V0 = oracle.helio_to_dh(1.0, w.m, w.x, w.v)
    rc = oracle.rcrit(1.0, w.m, Q0)
    for dt in (0.04, 0.2):
        Q1, V1, _ = oracle.drift(w.G, dt, Q0, V0)
        out = oracle.encounters(dt, Q0, V0, Q1, V1, rc)
        for i, j in zip(out["ice"], out["jce"]):
            assert not relative_bound_culls((Q0[i], V0[i], Q1[i], V1[i]), (Q0[j], V0[j], Q1[j], V1[j]),
                                            rc[i], rc[j], dt)
        if dt != 0.04:
            continue                # at dt = 0.2 a chord spans the ring: both keep every pair
        kept_rel = kept_reach = 0
        R = np.empty(400); M = np.empty((400, 3))
        for i in range(400):
            R[i], M[i] = reach(Q0[i], V0[i], Q1[i], V1[i], rc[i], dt)
        for i in range(0, 400, 7):
            for j in range(i + 1, 400):
                kept_reach += np.linalg.norm(M[j] - M[i]) <= R[i] + R[j]
                kept_rel += not relative_bound_culls((Q0[i], V0[i], Q1[i], V1[i]), (Q0[j], V0[j], Q1[j], V1[j]),
                                                     rc[i], rc[j], dt)
        assert kept_rel < 0.5 * kept_reach, (kept_rel, kept_reach)
