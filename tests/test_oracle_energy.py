"""Pins for the oracle's energy/momentum diagnostics and coordinate transforms.

Sec. 2.1.1: Mercury-Arxes works in democratic-heliocentric coordinates
(heliocentric positions, barycentric velocities) and reports total energy and
momentum.  Pins: the DH energy and angular momentum equal the explicit
barycentric-frame sums over star and bodies; the transforms match the
barycentre definition and invert each other; an N = 1 analytic case.
"""
import math

import numpy as np

import workloads

U = 2.0 ** -53
G = workloads.G_AU_MSUN_YR


def _barycentric(m0, m, xh, vh):
    """Explicit barycentric state of star + bodies from heliocentric input."""
    M = m0 + m.sum()
    Xs = -(m[:, None] * xh).sum(0) / M
    Vs = -(m[:, None] * vh).sum(0) / M
    return Xs, Vs, xh + Xs, vh + Vs


def test_helio_to_dh_is_barycentric_velocity(orc):
    w = workloads.c1(50)
    Q, V = orc.helio_to_dh(w.m0[0], w.m, w.x, w.v)
    Xs, Vs, X, Vb = _barycentric(w.m0[0], w.m, w.x, w.v)
    assert np.all(Q == w.x)
    assert np.max(np.abs(V - Vb)) <= 8 * U * np.max(np.abs(Vb))
    # total barycentric momentum (star included) vanishes
    ptot = w.m0[0] * Vs + (w.m[:, None] * V).sum(0)
    assert np.max(np.abs(ptot)) <= 64 * U * np.sum(w.m * np.linalg.norm(V, axis=1))
    xh, vh = orc.dh_to_helio(w.m0[0], w.m, Q, V)
    assert np.all(xh == w.x)
    assert np.max(np.abs(vh - w.v)) <= 8 * U * np.max(np.abs(w.v))


def test_energy_and_L_match_barycentric_sums(orc):
    import mpmath as mp
    mp.mp.dps = 40
    w = workloads.c1(30)
    m0, m = w.m0[0], w.m
    m = m * 1e3  # heavier bodies so pair terms matter
    Q, V = orc.helio_to_dh(m0, m, w.x, w.v)
    rc = orc.rcrit(m0, m, Q)
    out = orc.energy(G, m0, m, Q, V, rc)
    Xs, Vs, X, Vb = _barycentric(m0, m, w.x, w.v)
    # exact barycentric energy of star + bodies, evaluated in 40 digits
    pos = [Xs] + list(X)
    vel = [Vs] + list(Vb)
    mass = [m0] + list(m)
    mpv = lambda a: [mp.mpf(float(t)) for t in a]
    E = mp.mpf(0)
    Lb = [mp.mpf(0)] * 3
    for a in range(len(mass)):
        va = mpv(vel[a]); xa = mpv(pos[a])
        E += mp.mpf(mass[a]) * sum(t * t for t in va) / 2
        Lb[0] += mp.mpf(mass[a]) * (xa[1] * va[2] - xa[2] * va[1])
        Lb[1] += mp.mpf(mass[a]) * (xa[2] * va[0] - xa[0] * va[2])
        Lb[2] += mp.mpf(mass[a]) * (xa[0] * va[1] - xa[1] * va[0])
        for b in range(a + 1, len(mass)):
            d = [x - y for x, y in zip(mpv(pos[a]), mpv(pos[b]))]
            E -= mp.mpf(G) * mp.mpf(mass[a]) * mp.mpf(mass[b]) / mp.sqrt(sum(t * t for t in d))
    # the barycentric state was built from the same heliocentric input in FP64,
    # so allow the FP64 rounding of that construction
    assert abs(out["E"] - float(E)) <= 1e-13 * abs(float(E))
    Lref = np.array([float(t) for t in Lb])
    assert np.max(np.abs(out["L"] - Lref)) <= 1e-13 * np.linalg.norm(Lref)
    # P = sum m V is minus the star's barycentric momentum
    assert np.max(np.abs(out["P"] + m0 * Vs)) <= 1e-13 * np.linalg.norm(m0 * Vs)


def test_energy_split_EK(orc):
    """EK weights each pair by K: equal to E when no pair is inside rc, and the
    difference equals the K-1 weighted pair terms otherwise."""
    m0 = 1.0
    m = np.array([1e-6, 1e-6, 1e-6])
    Q = np.array([[1.0, 0, 0], [1.0 + 0.004, 0, 0], [-2.0, 0.5, 0]])
    V = np.zeros((3, 3))
    rc = np.array([0.01, 0.01, 0.01])
    out = orc.energy(G, m0, m, Q, V, rc)
    r = Q[1, 0] - Q[0, 0]
    K, _ = orc.changeover(r, 0.01)
    want = -(K - 1.0) * G * m[0] * m[1] / r
    # the difference of two totals carries their rounding (a few u |E|)
    assert abs((out["EK"] - out["E"]) - want) <= 8 * U * abs(out["E"])
    out2 = orc.energy(G, m0, m, Q, V, np.zeros(3))
    assert out2["EK"] == out2["E"]


def test_single_body_analytic(orc):
    """N = 1 at rest relative to the barycentre frame: E = -G m0 m1/r plus the
    DH kinetic terms, all closed form."""
    m0, m1 = 1.0, 1e-3
    x = np.array([[2.0, 0.0, 0.0]])
    v = np.array([[0.0, 4.0, 0.0]])
    Q, V = orc.helio_to_dh(m0, [m1], x, v)
    out = orc.energy(G, m0, [m1], Q, V, [0.0])
    # barycentric speeds: body v m0/(m0+m1), star -v m1/(m0+m1)
    M = m0 + m1
    kin = 0.5 * m1 * (4.0 * m0 / M) ** 2 + 0.5 * m0 * (4.0 * m1 / M) ** 2
    E = kin - G * m0 * m1 / 2.0
    assert abs(out["E"] - E) <= 8 * U * abs(E)
    assert abs(out["L"][2] - m1 * 2.0 * 4.0 * m0 / M) <= 8 * U * m1 * 8.0
