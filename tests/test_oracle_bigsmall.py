"""Pins of the oracle's big/small split (Sec. 2.1: only big bodies are gravity
sources; small bodies are massless, feel the big ones and do not interact with
each other).

Checked from outside the formulas: massless sources change no sum (the split
force equals the all-pairs force bit for bit when small masses are 0); the big
bodies' motion does not see the small ones; each small body moves exactly as it
would alone with the big bodies; two coincident small bodies are not an
encounter, while a small body close to a big one is.
"""
import numpy as np

import oracle
import workloads


def _system(nbig=6, nsmall=40, seed=3):
    rng = np.random.default_rng(seed)
    n = nbig + nsmall
    w = workloads.batch([n], cfg_id=11)
    m = w.m.copy()
    m[:nbig] = 10 ** rng.uniform(-7, -5, nbig)
    m[nbig:] = 0.0
    return w, m


def test_split_force_equals_all_pairs_force_with_massless_small_bodies():
    w, m = _system()
    Q, V = oracle.helio_to_dh(1.0, m, w.x, w.v)
    rc = oracle.rcrit(1.0, m, Q)
    a_split = oracle.force(m, Q, rc, w.G, nbig=6)
    a_all = oracle.force(m, Q, rc, w.G)
    assert np.array_equal(a_split, a_all)
    # a small target with one big source far away: the Newtonian pull of that source
    a1 = oracle.force(m[[0, 10]], Q[[0, 10]], rc[[0, 10]], w.G, nbig=1)
    d = Q[0] - Q[10]
    r = np.linalg.norm(d)
    assert r > rc[0]
    assert np.allclose(a1[1], w.G * m[0] * d / r ** 3, rtol=1e-15, atol=0)
    assert np.all(a1[0] == 0.0)


def test_big_bodies_do_not_see_small_bodies():
    w, m = _system()
    st = oracle.State(np.array([0, 46]), np.array([1.0]), m, w.x, w.v, nbig=[6])
    big = oracle.State(np.array([0, 6]), np.array([1.0]), m[:6], w.x[:6], w.v[:6])
    for _ in range(20):
        st.step(0.05)
        big.step(0.05)
    assert np.array_equal(st.Q[:6], big.Q) and np.array_equal(st.V[:6], big.V)


def test_each_small_body_moves_as_if_alone_with_the_big_ones():
    w, m = _system()
    st = oracle.State(np.array([0, 46]), np.array([1.0]), m, w.x, w.v, nbig=[6])
    for _ in range(20):
        st.step(0.05)
    for k in (6, 23, 45):
        idx = list(range(6)) + [k]
        one = oracle.State(np.array([0, 7]), np.array([1.0]), m[idx], w.x[idx], w.v[idx], nbig=[6])
        for _ in range(20):
            one.step(0.05)
        assert np.array_equal(one.Q[6], st.Q[k]) and np.array_equal(one.V[6], st.V[k])


def test_small_pairs_are_not_encounters():
    w, m = _system(nbig=2, nsmall=3)
    Q0, V0 = oracle.helio_to_dh(1.0, m, w.x, w.v)
    # body 4 (small) sits on body 3 (small); body 2 (small) next to body 0 (big)
    Q0[4] = Q0[3]; V0[4] = V0[3]
    rc = oracle.rcrit(1.0, m, Q0)
    Q0[2] = Q0[0] + np.array([0.3, 0.0, 0.0]) * rc[0]; V0[2] = V0[0]
    Q1, V1, _ = oracle.drift(w.G, 0.01, Q0, V0)
    split = oracle.encounters(0.01, Q0, V0, Q1, V1, rc, nbig=2)
    full = oracle.encounters(0.01, Q0, V0, Q1, V1, rc)
    pairs_split = set(zip(split["ice"].tolist(), split["jce"].tolist()))
    pairs_full = set(zip(full["ice"].tolist(), full["jce"].tolist()))
    assert (3, 4) in pairs_full and (3, 4) not in pairs_split
    assert (0, 2) in pairs_split
    assert pairs_split == {p for p in pairs_full if p[0] < 2}
    f, _ = oracle.pair_scan(0.01, Q0, V0, Q1, V1, rc, 3, nbig=2)
    assert not f[4]
