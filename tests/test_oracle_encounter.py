"""Pins for the oracle's close-encounter predicate (Sec. 3.1, encounter block).

The paper flags every unordered pair i<j whose minimum separation over the step
is at or below the critical distance, appends it to (ice, jce) and sets both
bodies' flags to 2.  The reading used: the squared separation over the step is
the cubic Hermite interpolant of its end values and end slopes.  Pins: for
straight-line relative motion that interpolant is exact, so the minimum has a
closed form; on random data the minimum must equal a dense sampling of the
Hermite basis form (a representation the oracle does not use); endpoint and
i<->j symmetry invariants; the flag/list bookkeeping on a constructed set.
"""
import numpy as np
import pytest


def _straight(rng, tau):
    q0i, q0j = rng.normal(size=3), rng.normal(size=3)
    vi, vj = rng.normal(size=3), rng.normal(size=3)
    return q0i, vi, q0i + tau * vi, vi, q0j, vj, q0j + tau * vj, vj


def test_straight_line_closed_form(orc):
    rng = np.random.default_rng(3)
    for _ in range(500):
        tau = rng.uniform(0.01, 2.0) * rng.choice([-1, 1])
        args = _straight(rng, tau)
        d0 = args[4] - args[0]
        dv = args[5] - args[1]
        # min over t in [0, tau] of |d0 + t dv|^2 (t measured along the step)
        ts = -float(d0 @ dv) / float(dv @ dv)
        s = ts / tau
        if 0 < s < 1:
            want = float(d0 @ d0) - float(d0 @ dv) ** 2 / float(dv @ dv)
        else:
            d1 = d0 + tau * dv
            want = min(float(d0 @ d0), float(d1 @ d1))
        got = orc.pair_min_d2(tau, *args)
        assert abs(got - want) <= 1e-12 * max(float(d0 @ d0), 1e-300)


def _hermite_dense(tau, q0i, v0i, q1i, v1i, q0j, v0j, q1j, v1j, n=100001):
    d0, d1 = q0j - q0i, q1j - q1i
    e0, e1 = v0j - v0i, v1j - v1i
    f0, f1 = d0 @ d0, d1 @ d1
    g0, g1 = 2 * tau * (d0 @ e0), 2 * tau * (d1 @ e1)
    s = np.linspace(0, 1, n)
    h00 = 2 * s ** 3 - 3 * s ** 2 + 1
    h10 = s ** 3 - 2 * s ** 2 + s
    h01 = -2 * s ** 3 + 3 * s ** 2
    h11 = s ** 3 - s ** 2
    return max(float(np.min(h00 * f0 + h10 * g0 + h01 * f1 + h11 * g1)), 0.0), f0, f1, abs(g0), abs(g1)


def test_dense_sampling_of_hermite(orc):
    rng = np.random.default_rng(5)
    for _ in range(300):
        tau = rng.uniform(0.01, 1.0)
        args = [rng.normal(size=3) for _ in range(8)]
        got = orc.pair_min_d2(tau, *args)
        ref, f0, f1, g0, g1 = _hermite_dense(tau, *args)
        scale = f0 + f1 + g0 + g1
        # sampling can only overestimate the minimum; quadratic in the step
        assert got <= ref + 1e-12 * scale
        assert ref - got <= 1e-8 * scale


def test_swap_and_endpoint_invariants(orc):
    rng = np.random.default_rng(6)
    for _ in range(200):
        tau = rng.uniform(-1.0, 1.0)
        a = [rng.normal(size=3) for _ in range(8)]
        x = orc.pair_min_d2(tau, *a)
        y = orc.pair_min_d2(tau, *a[4:], *a[:4])
        assert abs(x - y) <= 1e-13 * (1 + abs(x))
        d0, d1 = a[4] - a[0], a[6] - a[2]
        assert x <= min(d0 @ d0, d1 @ d1) * (1 + 1e-15)
        assert x >= 0.0


def test_lower_bound_lemma(orc):
    """min f >= min(f0, f1) - (4/27)(max(0,-g0) + max(0,g1)): the bound a
    conservative prefilter may use (h10 in [0,4/27], h11 in [-4/27,0])."""
    rng = np.random.default_rng(7)
    for _ in range(500):
        tau = rng.uniform(-1.0, 1.0)
        a = [rng.normal(size=3) for _ in range(8)]
        x = orc.pair_min_d2(tau, *a)
        d0, d1 = a[4] - a[0], a[6] - a[2]
        g0 = 2 * tau * (d0 @ (a[5] - a[1]))
        g1 = 2 * tau * (d1 @ (a[7] - a[3]))
        lb = min(d0 @ d0, d1 @ d1) - 4.0 / 27.0 * (max(0.0, -g0) + max(0.0, g1))
        assert x >= lb - 1e-14 * (abs(lb) + abs(g0) + abs(g1))


def test_flag_list_and_ce(orc):
    """A constructed system: pairs (0,3) cross, (1,2) end inside rc, others far."""
    tau = 0.1
    n = 6
    Q0 = np.array([[1, 0, 0], [2, 0, 0], [2.05, 0, 0], [1.0, 0.2, 0], [5, 5, 0], [-5, 2, 0]], float)
    V0 = np.zeros((n, 3))
    V0[0] = [0, 1.0, 0]
    V0[3] = [0, -1.0, 0]
    Q1 = Q0 + tau * V0
    Q1[2] = [2.005, 0, 0]
    V1 = V0.copy()
    rc = np.array([0.01, 0.01, 0.01, 0.01, 0.5, 0.5])
    out = orc.encounters(tau, Q0, V0, Q1, V1, rc)
    assert out["nce"] == 2
    assert list(zip(out["ice"], out["jce"])) == [(0, 3), (1, 2)]
    assert list(out["ce"]) == [2, 2, 2, 2, 0, 0]
    # capacity smaller than the count: true count still reported
    out = orc.encounters(tau, Q0, V0, Q1, V1, rc, cap=1)
    assert out["nce"] == 2 and len(out["ice"]) == 1


def test_threshold_is_inclusive(orc):
    """Flag iff min separation <= rc_ij (the paper's .le. test)."""
    Q0 = np.array([[0.0, 0, 0], [0.5, 0, 0]])
    V0 = np.zeros((2, 3))
    rc = np.array([0.5, 0.25])
    out = orc.encounters(0.1, Q0, V0, Q0, V0, rc)
    assert out["nce"] == 1
    out = orc.encounters(0.1, Q0, V0, Q0, V0, np.array([0.25, 0.4999999]))
    assert out["nce"] == 0
