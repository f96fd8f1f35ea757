"""Pins of the oracle's close-encounter resolver (full hybrid method).

Inside the critical radius the full method restores the flagged bodies to
their pre-drift state and advances them by Bulirsch-Stoer under the Kepler
part plus the (1 - K)-weighted pair part of the Hamiltonian (Sec. 2.1.1,
footnote on the critical radius; Sec. 3 and 3.2 keep that integration on the
host).  The pins below reach the resolver from outside its own arithmetic:
the Kepler flow of a lone body (the oracle drift, itself pinned to Kepler's
equation), the relative Kepler orbit of a bound pair with a negligible star,
conservation of H0, time reversal, the grouping of pairs into connected
components, and the second-order convergence of the full step to an
independent Newtonian integration (scipy's DOP853) through a close encounter,
which hot-path-only steps do not reach.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle

G = oracle.Params().G


def _elliptic(a, e, mu, phase=0.3, inc=0.2):
    # position/velocity at true anomaly `phase` of an orbit with pericentre on x
    p = a * (1 - e * e)
    r = p / (1 + e * np.cos(phase))
    x = np.array([r * np.cos(phase), r * np.sin(phase), 0.0])
    v = np.sqrt(mu / p) * np.array([-np.sin(phase), e + np.cos(phase), 0.0])
    c, s = np.cos(inc), np.sin(inc)
    R = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    return R @ x, R @ v


@pytest.mark.parametrize("a,e,tau", [(1.0, 0.05, 0.05), (1.0, 0.6, 0.9), (2.0, 0.3, -1.7), (1.0, 1.8, 0.4)])
def test_lone_body_follows_the_kepler_flow(a, e, tau):
    q, v = _elliptic(a if e < 1 else -a, e, G)
    Q, V, steps = oracle.bs_h0(G, 1.0, [1e-9], [0.0], q[None], v[None], tau)
    Qk, Vk, f = oracle.drift(G, tau, q[None], v[None])
    assert f[0] == 0 and steps >= 1
    assert np.linalg.norm(Q - Qk) <= 1e-10 * np.linalg.norm(Qk)
    assert np.linalg.norm(V - Vk) <= 1e-10 * np.linalg.norm(Vk)


def test_bound_pair_without_star_is_a_relative_kepler_orbit():
    """m0 negligible, r << 0.1 rc (K = 0): H0 is the Newtonian two-body
    problem, so the separation follows Kepler with mu = G (m1 + m2) and the
    centre of mass moves uniformly."""
    m = np.array([3e-6, 1e-6])
    mu = G * m.sum()
    qrel, vrel = _elliptic(0.002, 0.4, mu, phase=1.1, inc=0.5)
    cm_q, cm_v = np.array([1.0, 0.2, -0.1]), np.array([0.05, -0.02, 0.01])
    Q = np.array([cm_q - m[1] / m.sum() * qrel, cm_q + m[0] / m.sum() * qrel])
    V = np.array([cm_v - m[1] / m.sum() * vrel, cm_v + m[0] / m.sum() * vrel])
    tau = 0.37
    Q1, V1, _ = oracle.bs_h0(G, 1e-30, m, [10.0, 10.0], Q, V, tau)
    qk, vk, f = oracle.drift(mu, tau, qrel[None], vrel[None])
    assert f[0] == 0
    # the step control holds each body's error near tol |Q_i| (|Q_i| ~ 1 AU here,
    # 500 times the separation) per step, over ~8 relative orbits / ~100 steps
    assert np.linalg.norm((Q1[1] - Q1[0]) - qk[0]) <= 1e-10
    assert np.linalg.norm((V1[1] - V1[0]) - vk[0]) <= 2e-8 * np.linalg.norm(vk)
    cm1 = (m[:, None] * Q1).sum(0) / m.sum()
    assert np.linalg.norm(cm1 - (cm_q + tau * cm_v)) <= 1e-12


def _h0_energy(m0, m, rc, Q, V, inner=0.1):
    E = 0.5 * np.sum(m * np.sum(V * V, 1)) - np.sum(G * m0 * m / np.linalg.norm(Q, axis=1))
    for i in range(len(m)):
        for j in range(i + 1, len(m)):
            r = np.linalg.norm(Q[j] - Q[i])
            K, _ = oracle.changeover(r, max(rc[i], rc[j]), inner)
            E -= G * m[i] * m[j] * (1 - K) / r
    return E


def _cluster():
    """Three bodies inside each other's changeover zones near 1 AU."""
    m = np.array([3e-6, 1e-6, 2e-6])
    Q = np.array([[1.0, 0.0, 0.0], [1.012, 0.006, 0.001], [0.995, -0.009, -0.002]])
    V = np.array([[0.0, 6.28, 0.0], [0.02, 6.2, 0.01], [-0.03, 6.33, 0.0]])
    rc = 3 * np.linalg.norm(Q, axis=1) * (m / 3) ** (1 / 3)
    return m, rc, Q, V


def test_h0_energy_is_conserved():
    m, rc, Q, V = _cluster()
    E0 = _h0_energy(1.0, m, rc, Q, V)
    Q1, V1, steps = oracle.bs_h0(G, 1.0, m, rc, Q, V, 0.2)
    assert steps > 3                      # the encounter forces several steps
    # the pair part is a sizeable share of H0 here, so a wrong pair force shows
    assert abs(_h0_energy(1.0, m, rc, Q, V) - _h0_energy(1.0, m, np.zeros(3), Q, V)) > 1e-4 * abs(E0)
    assert abs(_h0_energy(1.0, m, rc, Q1, V1) - E0) <= 1e-11 * abs(E0)


def test_pair_part_changes_the_motion():
    """With rc = 0 every K is 1, so H0 is pure Kepler; with the cluster's rc
    the (1 - K) pairs deflect the bodies measurably."""
    m, rc, Q, V = _cluster()
    Qa, _, _ = oracle.bs_h0(G, 1.0, m, rc, Q, V, 0.2)
    Qb, _, _ = oracle.bs_h0(G, 1.0, m, np.zeros(3), Q, V, 0.2)
    Qk, _, _ = oracle.drift(G, 0.2, Q, V)
    assert np.max(np.abs(Qb - Qk)) <= 1e-10
    assert np.max(np.abs(Qa - Qk)) > 1e-5


def test_time_reversal():
    m, rc, Q, V = _cluster()
    Q1, V1, _ = oracle.bs_h0(G, 1.0, m, rc, Q, V, 0.15)
    Q2, V2, _ = oracle.bs_h0(G, 1.0, m, rc, Q1, V1, -0.15)
    assert np.max(np.abs(Q2 - Q)) <= 1e-10
    assert np.max(np.abs(V2 - V)) <= 1e-9


def test_groups_are_connected_components():
    n = 9
    rng = np.random.default_rng(5)
    Q0 = rng.normal(size=(n, 3)) + np.array([3.0, 0, 0]); V0 = rng.normal(size=(n, 3)) * 0.1 + np.array([0, 3.0, 0])
    Q = Q0 + 0.01; V = V0 - 0.01
    m = np.full(n, 1e-9); rc = np.full(n, 1e-4)
    ice = np.array([0, 3, 2], np.int32); jce = np.array([3, 7, 5], np.int32)
    Q1, V1, comp, nf, ng, _ = oracle.resolve(G, 1.0, m, rc, 0.1, Q0, V0, ice, jce, Q, V)
    assert nf == 0 and ng == 2
    assert comp.tolist() == [0, -1, 2, 0, -1, 2, -1, 0, -1]
    out = [1, 4, 6, 8]
    assert np.array_equal(Q1[out], Q[out]) and np.array_equal(V1[out], V[out])
    for members in ([0, 3, 7], [2, 5]):
        Qg, Vg, _ = oracle.bs_h0(G, 1.0, m[members], rc[members], Q0[members], V0[members], 0.1)
        assert np.array_equal(Q1[members], Qg) and np.array_equal(V1[members], Vg)


def _encounter_setup():
    m0 = 1.0
    m = np.array([3e-6, 1e-7])

    def circ(r, th):
        v = np.sqrt(G * m0 / r)
        return np.array([r * np.cos(th), r * np.sin(th), 0.0]), np.array([-v * np.sin(th), v * np.cos(th), 0.0])
    xa, va = circ(1.0, 0.0)
    xb, vb = circ(1.02, 0.06)
    return m0, m, np.array([xa, xb]), np.array([va, vb])


def _newton_reference(m0, m, x, v, T):
    def rhs(t, y):
        X = y[:6].reshape(2, 3); Vv = y[6:].reshape(2, 3)
        A = np.zeros((2, 3))
        for i in range(2):
            A[i] -= G * (m0 + m[i]) * X[i] / np.linalg.norm(X[i]) ** 3
            j = 1 - i
            d = X[j] - X[i]
            A[i] += G * m[j] * (d / np.linalg.norm(d) ** 3 - X[j] / np.linalg.norm(X[j]) ** 3)
        return np.concatenate([Vv.ravel(), A.ravel()])
    ref = solve_ivp(rhs, (0, T), np.concatenate([x.ravel(), v.ravel()]), method="DOP853", rtol=1e-13, atol=1e-16)
    sep = np.min(np.linalg.norm(ref.y[3:6] - ref.y[0:3], axis=0))
    return ref.y[:6, -1].reshape(2, 3), sep


def test_full_step_converges_through_a_close_encounter():
    """A planetesimal passes within 4e-4 AU of an Earth-mass body (critical
    radius 0.03 AU).  Full steps converge at second order to the Newtonian
    solution; hot-path-only steps (encounters flagged, not resolved) do not."""
    m0, m, x, v = _encounter_setup()
    T = 0.6
    xr, sep = _newton_reference(m0, m, x, v, T)
    assert sep < 1e-3
    errs = {}
    for full in (True, False):
        errs[full] = []
        for nst in (30, 60, 120):
            st = oracle.State(np.array([0, 2]), np.array([m0]), m, x, v)
            groups = 0
            for _ in range(nst):
                st.step(T / nst, full=full)
                groups += st.ngroups if full else 0
            if full:
                assert groups > nst // 2
            xh, _ = st.helio()
            errs[full].append(np.max(np.linalg.norm(xh - xr, axis=1)))
    e = errs[True]
    assert e[0] / e[1] > 3.0 and e[1] / e[2] > 3.0, e
    assert e[2] < 2e-5, e
    assert min(errs[False]) > 100 * e[2], errs
