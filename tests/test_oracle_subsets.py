"""Pins of the oracle's sampled-check routines against its pinned full routines.

The full-size GPU checks (16384 and 131072 bodies, the benchmark's error
figure) cannot afford the oracle's O(N^2) force or pair list, so they use two
per-body routines: ``force_subset`` (the force sum of chosen targets, Sec. 3.1
force block, loop 2) and ``pair_scan`` (one body against every other body under
the encounter predicate, Sec. 3.1 encounter block).  Each is tied here to the
full routine whose own pins (closed forms, invariants, brute force) live in
``test_oracle_force.py`` and ``test_oracle_encounter.py``:

* ``force_subset(idx)`` equals ``force()[idx]`` bit for bit, on clustered
  systems with many pairs inside the changeover zone, on a big/small system
  (only the first nbig bodies are sources) and for every target of a small
  system, so a wrong index, a dropped changeover term or an ignored nbig fails;
* the rows of ``pair_scan`` over every body of a dense ring, with pairs placed
  on the threshold (the tie band), reproduce the flagged set, the per-body
  flags and the tie set of ``encounters`` exactly;
* the OpenMP build of the oracle (the threaded CPU baseline) gives the same
  bits as the serial build for force, drift, pair list and whole steps.
"""
import numpy as np

import oracle
import workloads


def _clustered(n=240, nclust=6, seed=11):
    """Bodies in tight clusters: many pairs inside the changeover zone."""
    rng = np.random.default_rng(seed)
    w = workloads.batch([n], cfg_id=12)
    m = 10 ** rng.uniform(-8, -6, n)
    Q, _ = oracle.helio_to_dh(1.0, m, w.x, w.v)
    rc = oracle.rcrit(1.0, m, Q)
    centres = Q[rng.choice(n, nclust, replace=False)]
    k = rng.integers(0, nclust, n)
    # offsets from 0.02 to 3 critical radii around a cluster centre
    d = rng.normal(size=(n, 3))
    d *= (rng.uniform(0.02, 3.0, n) * rc / np.linalg.norm(d, axis=1))[:, None]
    Q = centres[k] + d
    rc = oracle.rcrit(1.0, m, Q)
    return m, Q, rc, w.G


def _zone_pairs(Q, rc, idx, inner=0.1):
    """Number of (target in idx, source) pairs inside the changeover zone."""
    c = 0
    for i in idx:
        r = np.linalg.norm(Q - Q[i], axis=1)
        rcij = np.maximum(rc, rc[i])
        c += int(np.sum((r > inner * rcij) & (r < rcij)))
    return c


def test_force_subset_is_force_rows_on_clusters():
    m, Q, rc, G = _clustered()
    full = oracle.force(m, Q, rc, G)
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(len(m), 60, replace=False))
    assert _zone_pairs(Q, rc, idx) > 100
    sub = oracle.force_subset(m, Q, rc, G, idx)
    assert np.array_equal(sub, full[idx])
    # every target, in reverse order and with repeats
    idx2 = np.concatenate([np.arange(len(m))[::-1], idx[:5]])
    assert np.array_equal(oracle.force_subset(m, Q, rc, G, idx2), full[idx2])


def test_force_subset_honours_big_bodies():
    m, Q, rc, G = _clustered(n=120, seed=5)
    nbig = 17
    full = oracle.force(m, Q, rc, G, nbig=nbig)
    idx = np.array([0, 3, 16, 17, 18, 60, 119], dtype=np.int32)
    sub = oracle.force_subset(m, Q, rc, G, idx, nbig=nbig)
    assert np.array_equal(sub, full[idx])
    # sources past nbig contribute nothing: the all-pairs rows differ
    all_pairs = oracle.force_subset(m, Q, rc, G, idx)
    assert not np.array_equal(all_pairs, sub)
    # a big target sees only the other big bodies: force on the big subsystem
    big = oracle.force(m[:nbig], Q[:nbig], rc[:nbig], G)
    assert np.array_equal(sub[:3], big[[0, 3, 16]])


def _dense_ring(n=300, seed=4, tau=0.04):
    # a narrow ring of heavy bodies: wide critical radii, many flagged pairs
    w = workloads.ring(n, seed_sys=seed, m=1e-6, a_lo=0.99, a_hi=1.01)
    m = w.m.copy()
    Q0, V0 = oracle.helio_to_dh(1.0, m, w.x, w.v)
    rc = oracle.rcrit(1.0, m, Q0)
    Q1, V1, _ = oracle.drift(w.G, tau, Q0, V0)
    # pairs placed on the threshold: body j rides along with body i at exactly
    # rc_ij (no relative motion, so the minimum separation is |d|), the critical
    # radii being an input of the check
    for i, j in ((3, 40), (77, 78), (150, n - 1)):
        d = max(rc[i], rc[j]) * np.array([0.6, 0.0, 0.8])
        Q0[j], V0[j] = Q0[i] + d, V0[i]
        Q1[j], V1[j] = Q1[i] + d, V1[i]
    return m, Q0, V0, Q1, V1, rc, tau


def test_pair_scan_rows_reproduce_the_encounter_list():
    m, Q0, V0, Q1, V1, rc, tau = _dense_ring()
    n = len(m)
    tie = 1e-6            # a wide tie band, so that it holds pairs
    ref = oracle.encounters(tau, Q0, V0, Q1, V1, rc, tie=tie)
    pairs = set(zip(ref["ice"].tolist(), ref["jce"].tolist()))
    assert len(pairs) > 50 and ref["ntie"] >= 3
    got, got_tie = set(), set()
    ce = np.zeros(n, np.int32)
    for i in range(n):
        f, t = oracle.pair_scan(tau, Q0, V0, Q1, V1, rc, i, tie=tie)
        assert not f[i] and not t[i]
        for j in np.flatnonzero(f):
            got.add((min(i, j), max(i, j)))
            ce[i] = 2
        for j in np.flatnonzero(t):
            got_tie.add((min(i, j), max(i, j)))
    assert got == pairs
    assert got_tie == ref["tie"]
    assert np.array_equal(ce, ref["ce"])


def test_pair_scan_rows_with_small_bodies():
    m, Q0, V0, Q1, V1, rc, tau = _dense_ring(n=200, seed=6)
    nbig = 30
    ref = oracle.encounters(tau, Q0, V0, Q1, V1, rc, nbig=nbig)
    pairs = set(zip(ref["ice"].tolist(), ref["jce"].tolist()))
    got = set()
    for i in range(len(m)):
        f, _ = oracle.pair_scan(tau, Q0, V0, Q1, V1, rc, i, nbig=nbig)
        got |= {(min(i, j), max(i, j)) for j in np.flatnonzero(f)}
    assert got == pairs and len(pairs) > 5
    assert all(i < nbig for i, _ in pairs)


def test_openmp_build_gives_the_serial_bits():
    serial, threaded = oracle.lib(), oracle.lib(threads=True)
    m, Q, rc, G = _clustered(n=500, seed=8)
    p = lambda a: a.ctypes.data_as(oracle.ctypes.c_void_p)  # noqa: E731
    a1, a2 = np.empty((500, 3)), np.empty((500, 3))
    serial.orc_force_nb(500, 500, G, 0.1, p(m), p(Q), p(rc), p(a1))
    threaded.orc_force_nb(500, 500, G, 0.1, p(m), p(Q), p(rc), p(a2))
    assert np.array_equal(a1, a2)
    w = workloads.batch([700, 300, 1], cfg_id=13)
    s1 = oracle.State.from_workload(w)
    s2 = oracle.State.from_workload(w, threads=True)
    for _ in range(3):
        s1.step(0.05)
        s2.step(0.05)
    assert np.array_equal(s1.Q, s2.Q) and np.array_equal(s1.V, s2.V) and np.array_equal(s1.a, s2.a)
    for (n1, i1, j1), (n2, i2, j2) in zip(s1.enc, s2.enc):
        assert n1 == n2 and np.array_equal(i1, i2) and np.array_equal(j1, j2)
