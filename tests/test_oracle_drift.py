"""Pins for the oracle's Kepler drift and Stumpff functions.

Sec. 2.1 and 3.1 of the paper: every body is propagated on its Kepler orbit
about the star for the full step (the drift block, one call per body, with a
failure flag).  The oracle uses universal variables; these tests check it
against an independent method -- the classical elliptic and hyperbolic Kepler
equations solved in 40-digit arithmetic -- and against the invariants of the
two-body flow (energy, angular momentum, Laplace-Runge-Lenz vector,
time reversal and the group property).
"""
import math

import mpmath as mp
import numpy as np
import pytest

U = 2.0 ** -53
G = (0.01720209895 * 365.25) ** 2
MU = G * 1.0


def classical_drift(mu, tau, q, v):
    """Two-body propagation by the classical Kepler equation (mpmath)."""
    mp.mp.dps = 40
    q = [mp.mpf(float(t)) for t in q]
    v = [mp.mpf(float(t)) for t in v]
    mu = mp.mpf(mu); tau = mp.mpf(tau)
    r0 = mp.sqrt(sum(t * t for t in q))
    v2 = sum(t * t for t in v)
    eta = sum(a * b for a, b in zip(q, v))
    a = 1 / (2 / r0 - v2 / mu)
    if a > 0:
        n = mp.sqrt(mu / a ** 3)
        ecE = 1 - r0 / a
        esE = eta / mp.sqrt(mu * a)
        E0 = mp.atan2(esE, ecE)
        e = mp.sqrt(ecE ** 2 + esE ** 2)
        M0 = E0 - e * mp.sin(E0)
        M1 = M0 + n * tau
        E1 = E0 + n * tau
        for _ in range(200):
            d = (E1 - e * mp.sin(E1) - M1) / (1 - e * mp.cos(E1))
            E1 -= d
            if abs(d) < mp.mpf(10) ** -35:
                break
        dE = E1 - E0
        r = a * (1 - e * mp.cos(E1))
        f = 1 - a / r0 * (1 - mp.cos(dE))
        g = tau - (dE - mp.sin(dE)) / n
        fd = -mp.sqrt(mu * a) * mp.sin(dE) / (r * r0)
        gd = 1 - a / r * (1 - mp.cos(dE))
    else:
        n = mp.sqrt(mu / (-a) ** 3)
        echF = 1 - r0 / a
        eshF = eta / mp.sqrt(-mu * a)
        e = mp.sqrt(echF ** 2 - eshF ** 2)
        F0 = mp.asinh(eshF / e)
        M0 = e * mp.sinh(F0) - F0
        M1 = M0 + n * tau
        F1 = F0 + mp.asinh(n * tau / e) if e > 0 else F0
        for _ in range(400):
            d = (e * mp.sinh(F1) - F1 - M1) / (e * mp.cosh(F1) - 1)
            F1 -= d
            if abs(d) < mp.mpf(10) ** -35:
                break
        dF = F1 - F0
        r = a * (1 - e * mp.cosh(F1))
        f = 1 - a / r0 * (1 - mp.cosh(dF))
        g = tau - (mp.sinh(dF) - dF) / n
        fd = -mp.sqrt(-mu * a) * mp.sinh(dF) / (r * r0)
        gd = 1 - a / r * (1 - mp.cosh(dF))
    qn = np.array([float(f * q[k] + g * v[k]) for k in range(3)])
    vn = np.array([float(fd * q[k] + gd * v[k]) for k in range(3)])
    return qn, vn


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def test_stumpff_closed_forms_and_recurrence(orc):
    for z in list(np.linspace(-2.0, -0.5, 7)) + list(np.linspace(0.5, 2.0, 7)) + [1e-3, -1e-3, 0.999, 1.001, 25.0, -25.0]:
        c = orc.stumpff(z)
        if z > 0:
            x = math.sqrt(z)
            ref = [math.cos(x), math.sin(x) / x]
        else:
            x = math.sqrt(-z)
            ref = [math.cosh(x), math.sinh(x) / x]
        assert abs(c[0] - ref[0]) <= 8 * U * max(1.0, abs(ref[0]))
        assert abs(c[1] - ref[1]) <= 8 * U * max(1.0, abs(ref[1]))
        # c_k(z) = 1/k! - z c_{k+2}(z)
        assert abs(c[0] - (1.0 - z * c[2])) <= 16 * U * max(1.0, abs(c[0]))
        assert abs(c[1] - (1.0 - z * c[3])) <= 16 * U * max(1.0, abs(c[1]))
    # high-precision values of c2 and c3 from their series
    mp.mp.dps = 40
    for z in [0.3, -0.7, 0.95, 1.5, -1.7, 4.0]:
        zz = mp.mpf(z)
        c2 = mp.nsum(lambda k: (-zz) ** k / mp.factorial(2 * k + 2), [0, mp.inf])
        c3 = mp.nsum(lambda k: (-zz) ** k / mp.factorial(2 * k + 3), [0, mp.inf])
        c = orc.stumpff(z)
        assert abs(c[2] - float(c2)) <= 32 * U * abs(float(c2))
        assert abs(c[3] - float(c3)) <= 64 * U * abs(float(c3))


def _state(a, e, inc, node, peri, M, mu=MU):
    import workloads
    x, v = workloads.elements_to_cartesian([mu], [a], [e], [inc], [node], [peri], [M])
    return x[0], v[0]


@pytest.mark.parametrize("a,e,frac", [(1.0, 0.01, 0.05), (5.2, 0.22, 0.01), (2.0, 0.6, 0.37),
                                      (0.5, 0.95, 0.05), (3.0, 0.0, 1.7), (1.5, 0.3, 12.3)])
def test_drift_matches_classical_elliptic(orc, a, e, frac):
    q, v = _state(a, e, 0.3, 1.1, 2.2, 0.7)
    P = 2 * math.pi * math.sqrt(a ** 3 / MU)
    for tau in (frac * P, -frac * P):
        Q, V, fl = orc.drift(MU, tau, q[None], v[None])
        assert fl[0] == 0
        qe, ve = classical_drift(MU, tau, q, v)
        assert _rel(Q[0], qe) <= 1e-13, (tau, _rel(Q[0], qe))
        assert _rel(V[0], ve) <= 1e-13, (tau, _rel(V[0], ve))


@pytest.mark.parametrize("speed,tau", [(1.5, 0.3), (3.0, 2.0), (10.0, 0.05), (1.5, -0.4)])
def test_drift_matches_classical_hyperbolic(orc, speed, tau):
    q = np.array([0.8, -0.3, 0.1])
    vesc = math.sqrt(2 * MU / np.linalg.norm(q))
    v = np.array([0.2, 1.0, 0.05])
    v = v / np.linalg.norm(v) * vesc * speed
    Q, V, fl = orc.drift(MU, tau, q[None], v[None])
    assert fl[0] == 0
    qe, ve = classical_drift(MU, tau, q, v)
    assert _rel(Q[0], qe) <= 1e-13
    assert _rel(V[0], ve) <= 1e-13


def _invariants(q, v, mu=MU):
    r = np.linalg.norm(q)
    eps = 0.5 * v @ v - mu / r
    h = np.cross(q, v)
    A = np.cross(v, h) - mu * q / r
    return eps, h, A


def test_drift_invariants_reversal_and_group(orc):
    rng = np.random.default_rng(11)
    for _ in range(20):
        a = rng.uniform(0.5, 10); e = rng.uniform(0, 0.8)
        q, v = _state(a, e, rng.uniform(0, 1), rng.uniform(0, 6), rng.uniform(0, 6), rng.uniform(0, 6))
        P = 2 * math.pi * math.sqrt(a ** 3 / MU)
        t1, t2 = rng.uniform(-0.3, 0.3) * P, rng.uniform(-0.3, 0.3) * P
        Q1, V1, _ = orc.drift(MU, t1, q[None], v[None])
        e0, h0, A0 = _invariants(q, v)
        e1, h1, A1 = _invariants(Q1[0], V1[0])
        assert abs(e1 - e0) <= 1e-14 * abs(e0) * 8
        assert np.max(np.abs(h1 - h0)) <= 1e-14 * np.linalg.norm(h0) * 8
        assert np.max(np.abs(A1 - A0)) <= 1e-13 * MU
        Qb, Vb, _ = orc.drift(MU, -t1, Q1, V1)
        assert _rel(Qb[0], q) <= 1e-14 * 8 and _rel(Vb[0], v) <= 1e-14 * 8
        Q12, V12, _ = orc.drift(MU, t2, Q1, V1)
        Qs, Vs, _ = orc.drift(MU, t1 + t2, q[None], v[None])
        assert _rel(Q12[0], Qs[0]) <= 1e-14 * 8 and _rel(V12[0], Vs[0]) <= 1e-14 * 8


def test_many_periods_of_short_drifts(orc):
    """1000 orbits in steps of P/20: the accumulated drift stays on the exact orbit."""
    q, v = _state(1.0, 0.05, 0.1, 0.2, 0.3, 0.4)
    P = 2 * math.pi * math.sqrt(1.0 / MU)
    tau = P / 20
    Q, V = q[None].copy(), v[None].copy()
    nsteps = 20000
    for _ in range(nsteps):
        Q, V, fl = orc.drift(MU, tau, Q, V)
    qe, ve = classical_drift(MU, nsteps * tau, q, v)
    # Roundoff makes the orbital energy random-walk (about sqrt(N) u); the
    # mean-motion error 1.5 de/e then integrates into an along-track phase
    # error of order 1.5 n T de/e.
    e0, h0, _ = _invariants(q, v)
    e1, h1, _ = _invariants(Q[0], V[0])
    de = abs(e1 - e0) / abs(e0)
    assert de <= 8 * U * math.sqrt(nsteps)
    assert np.linalg.norm(h1 - h0) <= 8 * U * math.sqrt(nsteps) * np.linalg.norm(h0)
    nT = 2 * math.pi * nsteps / 20
    assert _rel(Q[0], qe) <= 1.5 * nT * 8 * U * math.sqrt(nsteps)


def test_drift_failure_leaves_body_unchanged(orc):
    q = np.array([[1.0, 0.0, 0.0], [np.nan, 0.0, 0.0], [0.0, 0.0, 0.0]])
    v = np.array([[0.0, 6.0, 0.0], [0.0, 6.0, 0.0], [1.0, 0.0, 0.0]])
    Q, V, fl = orc.drift(MU, 0.01, q, v)
    assert list(fl) == [0, 1, 1]
    assert np.isnan(Q[1, 0]) and np.all(Q[2] == q[2]) and np.all(V[2] == v[2])
    assert not np.all(Q[0] == q[0])


def test_drift_zero_time_is_identity(orc):
    q, v = _state(1.3, 0.1, 0.2, 0.3, 0.4, 0.5)
    Q, V, fl = orc.drift(MU, 0.0, q[None], v[None])
    assert np.all(Q[0] == q) and np.all(V[0] == v)
