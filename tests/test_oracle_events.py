"""Pins of the oracle's collisions, star impacts, ejections and compaction
(Sec. 2.1.1: physical radii, removal of lost bodies; Sec. 2.1.2: planet-planet
and planet-star collisions, ejections beyond 400 AU checked every 200 yr).

The paper names these events, not their arithmetic (readings in the oracle's
header).  What fixes them here, from outside the routines:
  * the physical radius inverts the sphere's mass 4/3 pi R^3 rho;
  * the closest approach to the star on a drift arc equals the classical
    pericentre distance a (1 - e) of the elements the orbit was generated from
    (an independent elements-to-Cartesian conversion) when the arc passes the
    pericentre, a dense sampling of the arc otherwise bounds it, and without a
    pericentre passage it is the nearer end;
  * a star impact conserves mass and leaves the system barycentre and the
    others' barycentric velocities where they were;
  * mergers conserve mass, momentum and the centre of mass, a chain of
    colliding pairs becomes one body at its smallest index, and a pair whose
    paths cross inside the step collides although both ends are apart;
  * an ejection removes exactly the bodies beyond r_eject and leaves the
    others' heliocentric positions and velocities unchanged;
  * compaction keeps the order of the kept bodies (against numpy masking).
"""
import numpy as np

import oracle
import workloads

G = workloads.G_AU_MSUN_YR
U = 2.0 ** -53


def _circ(r, th, z=0.0, mu=G):
    v = np.sqrt(mu / r)
    return np.array([r * np.cos(th), r * np.sin(th), z]), np.array([-v * np.sin(th), v * np.cos(th), 0.0])


def test_physical_radius_inverts_sphere_mass():
    rng = np.random.default_rng(1)
    m = 10 ** rng.uniform(-12, -3, 200)
    for rho in (3.37e6, 1.0, 1e-3):
        R = oracle.phys_radius(m, rho)
        # cbrt within an ulp (3 ulp once cubed) plus the roundings of this check
        assert np.max(np.abs(4.0 / 3.0 * np.pi * R ** 3 * rho / m - 1.0)) <= 16 * U


def test_star_min_at_pericentre_passage():
    rng = np.random.default_rng(2)
    for _ in range(200):
        a, e = rng.uniform(0.3, 5.0), rng.uniform(0.0, 0.99)
        inc, node, peri = rng.uniform(0, 3), rng.uniform(0, 6), rng.uniform(0, 6)
        dM = rng.uniform(1e-3, 0.5)
        mu = np.array([G])
        x0, v0 = workloads.elements_to_cartesian(mu, [a], [e], [inc], [node], [peri], [-dM])
        x1, v1 = workloads.elements_to_cartesian(mu, [a], [e], [inc], [node], [peri], [dM])
        tau = 2 * dM / np.sqrt(G / a ** 3)
        got = oracle.star_min(G, tau, x0[0], v0[0], x1[0], v1[0])
        assert abs(got - a * (1 - e)) <= 1e-12 * a, (a, e, got)


def test_star_min_against_dense_arc():
    rng = np.random.default_rng(3)
    for _ in range(40):
        a, e = rng.uniform(0.5, 3.0), rng.uniform(0.0, 0.95)
        M0 = rng.uniform(-np.pi, np.pi)
        x0, v0 = workloads.elements_to_cartesian(np.array([G]), [a], [e], [0.3], [1.0], [2.0], [M0])
        tau = rng.uniform(0.01, 0.6) * 2 * np.pi * np.sqrt(a ** 3 / G)
        q1, w1, _ = oracle.drift(G, tau, x0, v0)
        got = oracle.star_min(G, tau, x0[0], v0[0], q1[0], w1[0])
        # the arc sampled densely by the oracle's own Kepler flow
        ts = np.linspace(0.0, tau, 4001)
        qs = np.array([oracle.drift(G, t, x0, v0)[0][0] for t in ts])
        rs = np.linalg.norm(qs, axis=1)
        assert got <= rs.min() * (1 + 1e-12)
        assert got >= rs.min() * (1 - 1e-5)
        # no pericentre in the arc: the nearer end (mean anomaly from M0 over n tau)
        n = np.sqrt(G / a ** 3)
        Ma, Mb = M0, M0 + n * tau
        if np.floor(Mb / (2 * np.pi)) * 2 * np.pi < Ma:
            assert got == min(np.linalg.norm(x0[0]), np.linalg.norm(q1[0]))


def _arcs(Q0, V0, tau, mu=G):
    Q1, V1, fl = oracle.drift(mu, tau, Q0, V0)
    assert not fl.any()
    return Q1, V1


def test_star_impact_conserves_mass_and_barycentre():
    tau = 0.01
    bodies = [_circ(1.0 + 0.1 * k, 0.7 * k) for k in range(5)]
    mu = np.array([G])
    # a plunging body at pericentre (q = 0.002 AU) in the middle of the step
    P = 2 * np.pi * np.sqrt(1.0 / G)
    dM = np.pi * tau / P
    xp, vp = workloads.elements_to_cartesian(mu, [1.0], [0.998], [0.1], [0.2], [0.3], [-dM])
    Q0 = np.array([b[0] for b in bodies] + [xp[0]])
    V0 = np.array([b[1] for b in bodies] + [vp[0]])
    m = np.array([1e-6, 2e-6, 3e-7, 5e-6, 1e-7, 4e-6])
    Q1, V1 = _arcs(Q0, V0, tau)
    assert oracle.star_min(G, tau, Q0[5], V0[5], Q1[5], V1[5]) < 0.0021
    m0 = 1.0
    m0n, mn, Qn, Vn, lost, ev = oracle.events(G, m0, m, Q1, V1, Q0, V0, Q1, V1, tau, [], [], 1.0, 0.005)
    assert ev == (1, 0, 0, 0) and list(lost) == [0, 0, 0, 0, 0, 1]
    assert mn[5] == 0.0 and abs(m0n - (m0 + m[5])) <= 2 * U
    Mt = m0 + m.sum()
    bary = (m[:, None] * Q1).sum(0) / Mt                    # the star at the origin before
    s = m[5] * Q1[5] / m0n                                   # the merged star's displacement
    bary_after = (m0n * s + (mn[:5, None] * (Qn[:5] + s)).sum(0)) / Mt
    assert np.max(np.abs(bary_after - bary)) <= 1e-15
    assert np.array_equal(Vn[:5], V1[:5])


def test_collisions_merge_components_and_conserve():
    tau = 0.01
    m = np.array([1e-6, 2e-6, 1.5e-6, 1e-6, 3e-6, 2e-6])
    rho = 1.0                                                # R ~ 0.006 AU, below rc ~ 0.02 AU
    R = oracle.phys_radius(m, rho)
    x, v = _circ(1.0, 0.0)
    ex = np.array([1.0, 0.0, 0.0])
    Q0 = np.array([x, x + 0.8 * (R[0] + R[1]) * ex, x + (0.8 * (R[0] + R[1]) + 0.8 * (R[1] + R[2])) * ex,
                   x + 0.2 * ex, x + 0.2 * ex + 2.0 * (R[3] + R[4]) * np.array([0, 0, 1.0]),
                   x + 0.5 * ex])
    V0 = np.array([v] * 6)
    # body 5 runs through body 3 two thirds into the step (apart at both ends)
    # and stops short of the chain 0-1-2
    V0[5] = v + (Q0[3] - Q0[5]) * 1.5 / tau
    Q1, V1 = _arcs(Q0, V0, tau)
    rc = oracle.rcrit(1.0, m, Q0)
    enc = oracle.encounters(tau, Q0, V0, Q1, V1, rc)
    pairs = set(zip(enc["ice"].tolist(), enc["jce"].tolist()))
    assert {(0, 1), (1, 2), (3, 4), (3, 5)} <= pairs
    assert np.linalg.norm(Q1[5] - Q1[3]) > 5 * (R[3] + R[5]) and np.linalg.norm(Q0[5] - Q0[3]) > 5 * (R[3] + R[5])
    m0n, mn, Qn, Vn, lost, ev = oracle.events(G, 1.0, m, Q1, V1, Q0, V0, Q1, V1, tau, enc["ice"], enc["jce"],
                                              rho, 0.005)
    assert m0n == 1.0
    # {0, 1, 2} chain -> body 0; {3, 5} crossing -> body 3; 4 is 2 (R3 + R4) away: kept
    assert list(lost) == [0, 2, 2, 0, 0, 2]
    assert ev[0] == 0 and ev[2] == 3 and ev[1] >= 3
    for root, mem in ((0, [0, 1, 2]), (3, [3, 5])):
        M = m[mem].sum()
        assert abs(mn[root] - M) <= 4 * U * M
        assert np.max(np.abs(mn[root] * Qn[root] - (m[mem, None] * Q1[mem]).sum(0))) <= 1e-15 * M
        assert np.max(np.abs(mn[root] * Vn[root] - (m[mem, None] * V1[mem]).sum(0))) <= 1e-14 * M
    assert np.all(mn[[1, 2, 5]] == 0.0)
    assert np.array_equal(Qn[4], Q1[4]) and np.array_equal(Vn[4], V1[4])


def test_ejection_removes_far_bodies_and_keeps_heliocentric_motion():
    tau = 0.05
    m = np.array([1e-6, 3e-6, 2e-6, 1e-9])
    Q0 = np.array([_circ(1.0, 0.1)[0], _circ(399.0, 1.0)[0], _circ(401.0, 2.0)[0], _circ(500.0, 3.0)[0]])
    V0 = np.array([_circ(1.0, 0.1)[1], _circ(399.0, 1.0)[1], _circ(401.0, 2.0)[1], _circ(500.0, 3.0)[1]])
    V0[2] += [0.05, -0.02, 0.01]
    Q1, V1 = _arcs(Q0, V0, tau)
    m0 = 1.0
    for r_ej, want in ((400.0, [0, 0, 3, 3]), (0.0, [0, 0, 0, 0])):
        m0n, mn, Qn, Vn, lost, ev = oracle.events(G, m0, m, Q1, V1, Q0, V0, Q1, V1, tau, [], [], 3.37e6, 0.005,
                                                  r_ej)
        assert list(lost) == want and ev[3] == sum(1 for w in want if w)
        keep = np.array(want) == 0
        xh0, vh0 = oracle.dh_to_helio(m0, m, Q1, V1)
        xh1, vh1 = oracle.dh_to_helio(m0n, mn, Qn, Vn)
        assert np.array_equal(xh1[keep], xh0[keep])
        assert np.max(np.abs(vh1[keep] - vh0[keep])) <= 1e-15 * np.max(np.abs(vh0))
        assert abs(m0n + mn.sum() - (m0 + m[keep].sum())) <= 4 * U


def test_compaction_keeps_order():
    rng = np.random.default_rng(7)
    for n in (0, 1, 17, 300):
        lost = rng.integers(0, 4, n) * (rng.uniform(size=n) < 0.3)
        m = rng.uniform(size=n); Q = rng.normal(size=(n, 3)); V = rng.normal(size=(n, 3))
        mk, Qk, Vk, ik = oracle.compact(lost, m, Q, V)
        keep = lost == 0
        assert np.array_equal(ik, np.flatnonzero(keep))
        assert np.array_equal(mk, m[keep]) and np.array_equal(Qk, Q[keep]) and np.array_equal(Vk, V[keep])


def test_state_events_then_compacted_state():
    """Three systems stepped by the oracle; a plunging body, a colliding pair
    and a far body are placed in them; after the events the compacted state
    holds the kept bodies in order, offsets and big counts follow, and its
    force is the oracle's force of the kept bodies."""
    w = workloads.batch([40, 30, 25], cfg_id=41)
    x, v, m = w.x.copy(), w.v.copy(), w.m.copy()
    m[:] = 1e-6
    tau = 0.01
    # system 0, body 7: a plunging orbit with its pericentre at mid-step
    P = 2 * np.pi * np.sqrt(1.0 / G)
    xp, vp = workloads.elements_to_cartesian(np.array([G]), [1.0], [0.998], [0.0], [0.0], [0.0],
                                             [-np.pi * tau / P])
    x[7], v[7] = xp[0], vp[0]
    # system 1: bodies 40 + 3 and 40 + 4 on top of each other
    x[44] = x[43] + [2e-4, 0.0, 0.0]; v[44] = v[43]
    # system 2: body 70 + 5 beyond 400 AU
    x[75], v[75] = _circ(450.0, 0.3)
    st = oracle.State(w.off, w.m0, m, x, v)
    st.step(tau)
    ev = st.events(tau, rho=1.0, r_star=0.005, r_eject=400.0)
    assert ev[0] == 1 and ev[2] >= 1 and ev[3] == 1
    assert st.lost[7] == 1 and st.lost[44] == 2 and st.lost[75] == 3
    new, idx = st.compacted()
    keep = np.flatnonzero(st.lost == 0)
    assert np.array_equal(idx, keep)
    assert list(np.diff(new.off)) == [39, 29, 24]
    assert np.array_equal(new.Q, st.Q[keep]) and np.array_equal(new.V, st.V[keep])
    for s, (a, b) in enumerate(new.systems()):
        rc = oracle.rcrit(new.m0[s], new.m[a:b], new.Q[a:b])
        assert np.array_equal(new.a[a:b], oracle.force(new.m[a:b], new.Q[a:b], rc, G))
    assert new.m0[0] > 1.0 and new.m0[1] == 1.0
