"""Pins for the oracle's interaction force, changeover function and critical radius.

The force block of Sec. 3.1 sums, for every target body, pair accelerations
over all source bodies; Sec. 2.1.1 restricts the symplectic interaction part to
pairs outside the critical radius (a multiple of the Hill radius).  Nothing in
the paper prints a value, so the pins are closed forms (two-body Newton,
equilateral triangle), invariants (Newton's third law, zero net torque,
translation), the finite-difference gradient of the oracle's own energy routine
(a different code path), and the rc -> 0 limit against a textbook Newtonian sum.
"""
import math

import numpy as np
import pytest

U = 2.0 ** -53
G = (0.01720209895 * 365.25) ** 2


def _scale(m, Q, G):
    """A_i = sum_j G m_j / r_ij^2 (the tolerance scale)."""
    d = Q[None, :, :] - Q[:, None, :]
    r2 = np.sum(d * d, axis=-1)
    np.fill_diagonal(r2, np.inf)
    return np.sum(G * m[None, :] / r2, axis=1)


def test_two_body_closed_form(orc):
    m = np.array([3e-6, 1e-3])
    Q = np.array([[1.0, 0.2, -0.1], [-2.0, 1.5, 0.3]])
    rc = np.array([1e-3, 1e-2])
    a = orc.force(m, Q, rc, G)
    d = Q[1] - Q[0]
    r = math.sqrt(float(d @ d))
    want0 = G * m[1] / r ** 2 * d / r
    want1 = -G * m[0] / r ** 2 * d / r
    assert np.max(np.abs(a[0] - want0)) <= 4 * U * G * m[1] / r ** 2
    assert np.max(np.abs(a[1] - want1)) <= 4 * U * G * m[0] / r ** 2


def test_equilateral_triangle(orc):
    s = 0.7
    m = np.full(3, 2e-7)
    ang = np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3]) + 0.3
    c = np.array([1.3, -0.4, 0.05])
    R = s / math.sqrt(3.0)
    Q = c + R * np.stack([np.cos(ang), np.sin(ang), np.zeros(3)], axis=1)
    a = orc.force(m, Q, np.zeros(3), G)
    mag = math.sqrt(3.0) * G * m[0] / s ** 2
    for i in range(3):
        u = (c - Q[i]) / np.linalg.norm(c - Q[i])
        assert np.max(np.abs(a[i] - mag * u)) <= 16 * U * mag


def _random_cluster(n, seed, close_pairs=5):
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(n, 3)) * [2.0, 2.0, 0.05] + [3.0, 0.0, 0.0]
    m = 10.0 ** rng.uniform(-10, -7, n)
    rc = rng.uniform(1e-4, 3e-2, n)
    # place some pairs inside the changeover zone and one pair coincident
    for k in range(close_pairs):
        i, j = 2 * k, 2 * k + 1
        rcij = max(rc[i], rc[j])
        dirv = rng.normal(size=3)
        dirv /= np.linalg.norm(dirv)
        Q[j] = Q[i] + dirv * rcij * rng.uniform(0.05, 1.2)
    return m, Q, rc


def test_newton_third_law(orc):
    m, Q, rc = _random_cluster(60, 1)
    a = orc.force(m, Q, rc, G)
    tot = np.sum(m[:, None] * a, axis=0)
    scale = np.sum(m * np.linalg.norm(a, axis=1))
    assert np.max(np.abs(tot)) <= 10 * U * scale


def test_zero_net_torque(orc):
    m, Q, rc = _random_cluster(60, 2)
    a = orc.force(m, Q, rc, G)
    tq = np.sum(m[:, None] * np.cross(Q, a), axis=0)
    scale = np.sum(m * np.linalg.norm(Q, axis=1) * np.linalg.norm(a, axis=1))
    assert np.max(np.abs(tq)) <= 20 * U * scale


def test_translation_invariance(orc):
    m, Q, rc = _random_cluster(40, 3)
    a = orc.force(m, Q, rc, G)
    b = orc.force(m, Q + np.array([0.5, -0.25, 0.125]), rc, G)
    A = _scale(m, Q, G)
    assert np.all(np.max(np.abs(a - b), axis=1) <= 64 * U * A + 1e-300)


def test_permutation_invariance(orc):
    m, Q, rc = _random_cluster(40, 4)
    p = np.random.default_rng(9).permutation(40)
    a = orc.force(m, Q, rc, G)
    b = orc.force(m[p], Q[p], rc[p], G)
    A = _scale(m, Q, G)
    assert np.all(np.max(np.abs(a[p] - b), axis=1) <= 8 * U * A[p])


def test_rc_zero_is_plain_newton(orc):
    """With rc = 0 every pair is outside the zone: the textbook Newtonian sum."""
    m, Q, _ = _random_cluster(30, 5, close_pairs=0)
    a = orc.force(m, Q, np.zeros(30), G)
    import mpmath as mp
    mp.mp.dps = 40
    for i in range(30):
        acc = [mp.mpf(0)] * 3
        for j in range(30):
            if j == i:
                continue
            d = [mp.mpf(Q[j, k]) - mp.mpf(Q[i, k]) for k in range(3)]
            r = mp.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
            for k in range(3):
                acc[k] += mp.mpf(G) * mp.mpf(m[j]) * d[k] / r ** 3
        A = float(sum(mp.mpf(G) * mp.mpf(m[j]) / ((mp.mpf(Q[j, 0]) - mp.mpf(Q[i, 0])) ** 2 +
                                                    (mp.mpf(Q[j, 1]) - mp.mpf(Q[i, 1])) ** 2 +
                                                    (mp.mpf(Q[j, 2]) - mp.mpf(Q[i, 2])) ** 2)
                      for j in range(30) if j != i))
        err = max(abs(float(acc[k]) - a[i, k]) for k in range(3))
        assert err <= 8 * U * A


def test_force_is_gradient_of_weighted_potential(orc):
    """m_i a_i = -grad_i U_K where U_K = -sum_{i<j} G m_i m_j K(r_ij)/r_ij is the
    K-weighted pair energy from the oracle's energy routine (rc held fixed)."""
    m, Q, rc = _random_cluster(12, 6, close_pairs=5)
    a = orc.force(m, Q, rc, G)
    V = np.zeros_like(Q)

    def UK(Qp):
        return orc.energy(G, 1e-300, m, Qp, V, rc)["EK"]

    D = np.linalg.norm(Q[:, None, :] - Q[None, :, :], axis=-1)
    np.fill_diagonal(D, np.inf)
    for i in range(10):
        for k in range(3):
            h = 1e-5 * np.min(D[i])
            Qp = Q.copy(); Qp[i, k] += h
            Qm = Q.copy(); Qm[i, k] -= h
            grad = (UK(Qp) - UK(Qm)) / (2 * h)
            F = m[i] * a[i, k]
            scale = m[i] * _scale(m, Q, G)[i]
            assert abs(F + grad) <= 1e-7 * scale, (i, k, F, -grad)


def test_changeover_function_properties(orc):
    rc, f = 2.0, 0.1
    assert orc.changeover(f * rc, rc, f) == (0.0, 0.0)
    assert orc.changeover(rc, rc, f) == (1.0, 0.0)
    assert orc.changeover(0.0, rc, f)[0] == 0.0
    assert orc.changeover(5 * rc, rc, f)[0] == 1.0
    ys = np.linspace(0.01, 0.99, 99)
    r = f * rc + ys * (1 - f) * rc
    K = np.array([orc.changeover(x, rc, f)[0] for x in r])
    assert np.all(np.diff(K) > 0)                       # monotone
    Kr = np.array([orc.changeover(f * rc + (1 - y) * (1 - f) * rc, rc, f)[0] for y in ys])
    assert np.max(np.abs(K + Kr - 1.0)) <= 4 * U         # K(y) + K(1-y) = 1
    # dK/dr against central differences of K, and C1 continuity at both edges
    for x in np.linspace(f * rc + 1e-3, rc - 1e-3, 17):
        h = 1e-6
        fd = (orc.changeover(x + h, rc, f)[0] - orc.changeover(x - h, rc, f)[0]) / (2 * h)
        assert abs(fd - orc.changeover(x, rc, f)[1]) <= 1e-8
    eps = 1e-7
    assert orc.changeover(f * rc + eps, rc, f)[1] < 1e-5
    assert orc.changeover(rc - eps, rc, f)[1] < 1e-5


def test_coincident_and_zone_interior(orc):
    """Coincident distinct bodies and pairs inside 0.1 rc contribute nothing."""
    m = np.array([1e-9, 2e-9, 3e-9])
    Q = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [1.0 + 0.05 * 0.01, 0.0, 0.0]])
    rc = np.array([0.01, 0.01, 0.01])
    a = orc.force(m, Q, rc, G)
    assert np.all(a == 0.0)


def test_rcrit_hill_radius(orc):
    """rc = n_H |Q| (m/(3 m0))^(1/3): the Hill radius at the current distance."""
    m = np.array([M := 9.547919e-4, 1e-9])
    Q = np.array([[5.2, 0.0, 0.0], [0.0, 3.0, 4.0]])
    rc = orc.rcrit(1.0, m, Q, 3.0)
    assert abs(rc[0] - 3 * 5.2 * (M / 3) ** (1 / 3)) <= 4 * U * rc[0]
    assert abs(rc[1] - 3 * 5.0 * (1e-9 / 3) ** (1 / 3)) <= 4 * U * rc[1]
    # Jupiter at 5.2 AU: about 1.07 AU for three Hill radii
    assert 1.0 < rc[0] < 1.1
