"""GPU parity: every call of the C ABI against the CPU oracle on the same
seeded inputs (element by element), at sizes that span several tiles and
splits with ragged tails, plus edge cases.

Tolerances (relative, see the design notes): FP64 force 1e-12 of
A_i = sum_j G m_j / r_ij^2; drift 1e-13 per body; kick, stellar drift and
transforms a few ulp; encounter sets equal outside a 1e-10 rc^2 tie band;
diagnostics 1e-13.  FP32C force errors are measured and bounded at 1e-6 A_i.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import (U, accel_error, ctx_for, enc_compare, oracle_dh, pair_scale, rel_rows,
                        systems)

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2601_19654_amd.nb")


def _cases():
    return {
        "c1_n100": lambda: workloads.c1(100),
        "ring_n700": lambda: workloads.ring(700, m=3e-8),        # many changeover pairs
        "batch_ragged": lambda: workloads.batch([1, 2, 3, 17, 0, 257, 600, 1031]),
        "single_n1537": lambda: workloads.batch([1537], cfg_id=7),
    }


CASES = _cases()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    w = CASES[request.param]()
    return request.param, w, oracle_dh(w)


# ---------------------------------------------------------------- force
@pytest.mark.parametrize("r,jchunk", [(2, 0), (1, 256), (4, 512)])
@pytest.mark.parametrize("force_algo", [1, 2])
def test_force_fp64(case, r, jchunk, force_algo):
    """force_algo 1: every ordered pair; 2: each unordered pair once, applied to
    both bodies (tile pairs of 64 r bodies, ragged tails, diagonal tiles)."""
    name, w, (Q, V, rc, a_ref) = case
    c = ctx_for(w, mode=nb.NB_FP64, force_r=r, force_jchunk=jchunk, force_algo=force_algo)
    a = c.accel()
    assert np.all(np.isfinite(a)), name
    rc_g = c.rcrit()
    # cbrt and sqrt differ between the device library and glibc by about an ulp each
    assert np.all(np.abs(rc_g - rc) <= 16 * U * np.abs(rc))
    for s, lo, hi in systems(w):
        if hi - lo < 2:
            assert np.all(a[lo:hi] == 0.0)
            continue
        A = pair_scale(w.m[lo:hi], Q[lo:hi], w.G)
        err = accel_error(a[lo:hi], a_ref[lo:hi], A)
        assert err <= 1e-12, (name, s, err)


@pytest.mark.parametrize("r,jchunk", [(2, 0), (1, 256), (4, 512)])
@pytest.mark.parametrize("force_algo", [1, 2, 4])
def test_force_fp32c(case, r, jchunk, force_algo):
    name, w, (Q, V, rc, a_ref) = case
    c = ctx_for(w, mode=nb.NB_FP32C, force_r=r, force_jchunk=jchunk, force_algo=force_algo)
    a = c.accel()
    assert np.all(np.isfinite(a)), name
    worst = 0.0
    for s, lo, hi in systems(w):
        if hi - lo < 2:
            continue
        A = pair_scale(w.m[lo:hi], Q[lo:hi], w.G)
        err = accel_error(a[lo:hi], a_ref[lo:hi], A)
        worst = err if not (err <= worst) else worst      # a NaN error is kept
    print(f"FP32C force error {name} r={r} j={jchunk} algo={force_algo}: {worst:.3e} A_i")
    assert worst <= 1e-6, (name, worst)


def _far_fraction(w, R):
    """Fraction of the off-diagonal tile pairs (wave rows of 64 R targets
    against source tiles of 64) that the radial order's far test takes from
    the high parts, emulated on the host from the DH positions' FP32 split
    (the test of the far-tile pin)."""
    from test_far_tiles import far_tiles, tile_bounds
    Q, _, rc, _ = oracle_dh(w)
    far = tot = 0
    for s, lo, hi in systems(w):
        n = hi - lo
        if n < 2 * 64 * R:
            continue
        order = np.lexsort((np.arange(n), np.einsum("ij,ij->i", Q[lo:hi], Q[lo:hi])))
        q = Q[lo:hi][order]
        xh = q.astype(np.float32)
        xl = (q - xh.astype(np.float64)).astype(np.float32)
        rc2 = (rc[lo:hi][order] ** 2).astype(np.float32)
        recs = [tile_bounds(xh[b:b + 64], xl[b:b + 64], rc2[b:b + 64]) for b in range(0, n, 64)]
        nrow = n // (64 * R)
        for i in range(nrow):
            for t in range(len(recs)):
                if t // R <= i:
                    continue
                tot += 1
                far += all(far_tiles(recs[i * R + r], recs[t]) for r in range(R))
    return far / max(tot, 1)


@pytest.mark.parametrize("r,g", [(2, 1), (1, 2), (4, 1), (2, 4)])
def test_force_radial_order(r, g):
    """force_algo 4: the symmetric FP32C force over the bodies of every system
    by distance from the star, tile pairs proven far apart from the FP32 high
    parts alone.  A 0.5-5 AU annulus (where most tile pairs are far) and a
    ragged batch, against the oracle at the FP32C bar, and against the same
    force over the index order (force_algo 2)."""
    for w in (workloads.c3(n=4000), workloads.batch([1, 2, 300, 0, 1031, 2600], cfg_id=31, a_lo=0.5,
                                                    a_hi=5.0)):
        Q, V, rc, a_ref = oracle_dh(w)
        frac = _far_fraction(w, r)
        c = ctx_for(w, mode=nb.NB_FP32C, force_r=r, force_g=g, force_algo=4)
        ch = c.choices()
        assert ch["force_algo"] == 4 and ch["force_g"] == g, ch
        a = c.accel()
        a2 = ctx_for(w, mode=nb.NB_FP32C, force_r=r, force_g=g, force_algo=2).accel()
        worst = worst2 = 0.0
        for s, lo, hi in systems(w):
            if hi - lo < 2:
                assert np.all(a[lo:hi] == 0.0)
                continue
            A = pair_scale(w.m[lo:hi], Q[lo:hi], w.G)
            worst = max(worst, accel_error(a[lo:hi], a_ref[lo:hi], A))
            worst2 = max(worst2, accel_error(a2[lo:hi], a_ref[lo:hi], A))
        print(f"radial order {w.name} r={r} g={g}: far tile pairs {frac:.2f}, error {worst:.3e} A_i "
              f"(index order {worst2:.3e})", flush=True)
        assert frac > 0.3
        assert worst <= 1e-6 and worst <= 4 * worst2 + 1e-7


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("r", [1, 2, 4])
@pytest.mark.parametrize("g", [1, 2, 4])
def test_force_super_tiles(case, mode, r, g):
    """Symmetric force with super-tiles of g tiles of 64 r bodies (one
    workgroup of g waves per super-tile pair, rotating over the source tiles):
    ragged super-tiles with empty tiles, diagonal super-tiles, every width and
    tile size, both precisions."""
    name, w, (Q, V, rc, a_ref) = case
    c = ctx_for(w, mode=mode, force_r=r, force_algo=2, force_g=g)
    ch = c.choices()
    assert ch["force_algo"] == 2 and ch["force_g"] == g, ch
    a = c.accel()
    assert np.all(np.isfinite(a)), name
    bar = 1e-12 if mode == 0 else 1e-6
    for s, lo, hi in systems(w):
        if hi - lo < 2:
            assert np.all(a[lo:hi] == 0.0)
            continue
        A = pair_scale(w.m[lo:hi], Q[lo:hi], w.G)
        err = accel_error(a[lo:hi], a_ref[lo:hi], A)
        assert err <= bar, (name, s, mode, r, g, err)


# ---------------------------------------------------------------- O(N) phases
def test_transforms_kick_sun_drift(case):
    name, w, (Q, V, rc, a_ref) = case
    c = ctx_for(w)
    x, v = c.download(nb.NB_DH)
    assert np.all(x == Q)
    assert rel_rows(v, V) <= 8 * U
    xh, vh = c.download(nb.NB_HELIO)
    assert np.all(xh == w.x)
    assert rel_rows(vh, w.v) <= 8 * U
    h = 0.5 * w.dt
    a = c.accel()
    c.kick(h)
    _, v1 = c.download(nb.NB_DH)
    ref = oracle.kick(h, a, V)          # same a on both sides isolates the kick
    assert rel_rows(v1, ref) <= 4 * U
    c.sun_drift(h)
    x2, _ = c.download(nb.NB_DH)
    for s, lo, hi in systems(w):
        if hi == lo:
            continue
        qref = oracle.sun_drift(h, w.m0[s], w.m[lo:hi], ref[lo:hi], Q[lo:hi])
        assert rel_rows(x2[lo:hi], qref) <= 4 * U, (name, s)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_kepler_drift(case, sign):
    name, w, (Q, V, rc, a_ref) = case
    c = ctx_for(w)
    dt = sign * w.dt
    assert c.drift(dt) == 0
    x, v = c.download(nb.NB_DH)
    for s, lo, hi in systems(w):
        if hi == lo:
            continue
        q1, v1, fl = oracle.drift(w.G * w.m0[s], dt, Q[lo:hi], V[lo:hi])
        assert not fl.any()
        assert rel_rows(x[lo:hi], q1) <= 1e-13, (name, s, rel_rows(x[lo:hi], q1))
        assert rel_rows(v[lo:hi], v1) <= 1e-13, (name, s)


def test_drift_long_steps_and_eccentric():
    """Steps of many orbits and high eccentricity exercise the closed-form
    Stumpff branches and the bracketed Newton iteration."""
    mu = workloads.G_AU_MSUN_YR
    n = 300
    rng = np.random.default_rng(3)
    x, v = workloads.elements_to_cartesian(mu * np.ones(n), rng.uniform(0.3, 20, n),
                                           rng.uniform(0, 0.97, n), rng.uniform(0, 3, n),
                                           rng.uniform(0, 6, n), rng.uniform(0, 6, n),
                                           rng.uniform(0, 6, n))
    m = np.zeros(n)
    w = workloads.Workload("ecc", np.array([0, n], np.int32), np.array([1.0]), m, x, v, 7.3, 1)
    c = ctx_for(w)
    for dt in (7.3, -3.1, 0.013):
        c.upload(w.m0, m, x, v)
        assert c.drift(dt) == 0
        xg, vg = c.download(nb.NB_DH)
        q1, v1, fl = oracle.drift(mu, dt, x, v)
        assert not fl.any()
        assert rel_rows(xg, q1) <= 1e-12 and rel_rows(vg, v1) <= 1e-12, dt


# ---------------------------------------------------------------- encounters
def _oracle_encounters(w, Q, V, rc, dt):
    pairs, tie, ce = [], [], np.zeros(w.ntot, np.int32)
    for s, lo, hi in systems(w):
        if hi - lo < 2:
            continue
        q1, v1, _ = oracle.drift(w.G * w.m0[s], dt, Q[lo:hi], V[lo:hi])
        out = oracle.encounters(dt, Q[lo:hi], V[lo:hi], q1, v1, rc[lo:hi])
        pairs += [(int(i) + lo, int(j) + lo) for i, j in zip(out["ice"], out["jce"])]
        tie += [(i + lo, j + lo) for i, j in out["tie"]]
        ce[lo:hi] = out["ce"]
    return pairs, tie, ce


@pytest.mark.parametrize("algo", [1, 2])
@pytest.mark.parametrize("wname", ["ring_n700", "batch_ragged", "ring_dense"])
def test_encounter_set(wname, algo):
    w = workloads.ring(900, m=1e-7) if wname == "ring_dense" else CASES[wname]()
    Q, V, rc, _ = oracle_dh(w)
    pairs, tie, ce = _oracle_encounters(w, Q, V, rc, w.dt)
    c = ctx_for(w, enc_algo=algo)
    c.drift(w.dt)
    e = c.encounters()
    got = list(zip(e.ice.tolist(), e.jce.tolist()))
    assert got == sorted(got), "list must be sorted by (i, j)"
    assert all(i < j for i, j in got)
    assert not enc_compare(got, pairs, tie), (wname, len(got), len(pairs))
    flagged = {i for p in got for i in p}
    assert set(np.nonzero(e.ce == 2)[0].tolist()) == flagged
    assert set(np.unique(e.ce).tolist()) <= {0, 2}
    print(f"{wname}: {e.nce} flagged pairs, {len(tie)} in the tie band")
    if wname == "ring_dense":
        assert e.nce > 10


@pytest.mark.parametrize("dt", [0.04, 0.2, -0.1])
def test_encounter_algorithms_agree(dt):
    """All-pairs and sorted-tile checks give the same list on dense rings and
    on a ragged batch (both apply the same exact predicate)."""
    for w in (workloads.ring(5000, m=3e-8), workloads.batch([3, 1500, 64, 65, 1, 900, 2000])):
        outs = []
        for algo in (1, 2):
            c = ctx_for(w, enc_algo=algo, enc_cap=1 << 18)
            c.drift(dt)
            e = c.encounters()
            outs.append(e)
            c.close()
        assert outs[0].nce == outs[1].nce
        assert np.array_equal(outs[0].ice, outs[1].ice) and np.array_equal(outs[0].jce, outs[1].jce)
        assert np.array_equal(outs[0].ce, outs[1].ce)
        print(f"{w.name} dt={dt}: {outs[0].nce} pairs")


def test_encounter_capacity_overflow():
    w = workloads.ring(900, m=1e-7)
    c = ctx_for(w, enc_cap=4)
    c.drift(w.dt)
    with pytest.raises(nb.NbError) as ei:
        c.encounters()
    assert ei.value.code == nb.NB_E_CAPACITY
    e = c.encounters(allow_overflow=True)
    assert e.nce > 4 and len(e.ice) == 4          # true count still reported


# ---------------------------------------------------------------- diagnostics
def test_diagnostics(case):
    name, w, (Q, V, rc, a_ref) = case
    c = ctx_for(w)
    d = c.diagnostics()
    for s, lo, hi in systems(w):
        if hi == lo:
            continue
        ref = oracle.energy(w.G, w.m0[s], w.m[lo:hi], Q[lo:hi], V[lo:hi], rc[lo:hi])
        assert abs(d["E"][s] - ref["E"]) <= 1e-13 * abs(ref["E"]), (name, s)
        assert abs(d["EK"][s] - ref["EK"]) <= 1e-13 * abs(ref["EK"]), (name, s)
        assert np.max(np.abs(d["L"][s] - ref["L"])) <= 1e-13 * np.linalg.norm(ref["L"])
        Pscale = np.sum(w.m[lo:hi] * np.linalg.norm(V[lo:hi], axis=1))
        assert np.max(np.abs(d["P"][s] - ref["P"])) <= 64 * U * Pscale


# ---------------------------------------------------------------- full steps
@pytest.mark.parametrize("mode,algo,step_algo,force_algo", [(0, 1, 1, 0), (1, 1, 1, 0), (0, 2, 1, 0),
                                                            (0, 0, 2, 0), (0, 1, 1, 1), (1, 2, 1, 4)])
def test_steps_match_oracle(case, mode, algo, step_algo, force_algo):
    name, w, _ = case
    k = 5
    c = ctx_for(w, mode=mode, enc_algo=algo, step_algo=step_algo, force_algo=force_algo)
    st = oracle.State.from_workload(w)
    stats = c.step(w.dt, k)
    total = 0
    for _ in range(k):
        st.step(w.dt)
        total += sum(e[0] for e in st.enc)
    x, v = c.download(nb.NB_DH)
    tol = 1e-11 if mode == 0 else 1e-7
    assert rel_rows(x, st.Q) <= tol, (name, rel_rows(x, st.Q))
    assert rel_rows(v, st.V) <= tol * 10, (name, rel_rows(v, st.V))
    if mode == 0:
        assert stats["total_nce"] == total
        e = c.last_encounters()
        ref = [(int(i), int(j)) for (_, ii, jj) in st.enc for i, j in zip(ii, jj)]
        got = list(zip(e.ice.tolist(), e.jce.tolist()))
        # the last step's list, put in (i, j) order when it is read
        assert got == sorted(got)
        assert got == sorted(ref)


@pytest.mark.parametrize("step_algo", [1, 2])
def test_step_with_drag(step_algo):
    w = workloads.c2(400)
    c = ctx_for(w, step_algo=step_algo)
    st = oracle.State.from_workload(w)
    c.step(w.dt, 3)
    for _ in range(3):
        st.step(w.dt)
    x, v = c.download(nb.NB_DH)
    assert rel_rows(x, st.Q) <= 1e-11
    assert rel_rows(v, st.V) <= 1e-10


def test_step_launches_agree():
    """The per-phase launches and the persistent launch follow the same step
    with different summation orders: equal to rounding over 40 steps, same
    encounter statistics."""
    w = workloads.batch([5, 300, 1700, 64, 1, 2048, 900])
    outs = []
    for step_algo in (1, 2):
        c = ctx_for(w, step_algo=step_algo)
        st = c.step(w.dt, 40)
        x, v = c.download(nb.NB_DH)
        e = c.last_encounters()
        outs.append((x, v, st, e))
        c.close()
    assert rel_rows(outs[0][0], outs[1][0]) <= 1e-11
    assert rel_rows(outs[0][1], outs[1][1]) <= 1e-10
    assert outs[0][2]["total_nce"] == outs[1][2]["total_nce"]
    assert outs[0][2]["max_nce"] == outs[1][2]["max_nce"]
    assert np.array_equal(outs[0][3].ice, outs[1][3].ice) and np.array_equal(outs[0][3].jce, outs[1][3].jce)


@pytest.mark.parametrize("step_algo", [1, 2])
def test_graph_replays_match_direct_steps(step_algo):
    """nb_step replays a captured graph; chunks of steps must equal one call."""
    w = workloads.batch([300, 700, 41])
    a = ctx_for(w, step_algo=step_algo)
    b = ctx_for(w, step_algo=step_algo)
    a.step(w.dt, 20)
    for _ in range(20):
        b.step(w.dt, 1)
    xa, va = a.download(nb.NB_DH)
    xb, vb = b.download(nb.NB_DH)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


@pytest.mark.parametrize("enc_algo", [1, 2])
def test_bitwise_determinism(enc_algo):
    w = workloads.ring(1200, m=3e-8)
    outs = []
    for _ in range(2):
        c = ctx_for(w, mode=nb.NB_FP32C, enc_algo=enc_algo)
        c.step(w.dt, 4)
        outs.append((*c.download(nb.NB_DH), c.accel(), c.last_encounters().ice))
        c.close()
    for u, v in zip(*outs):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("enc_algo", [1, 2])
def test_overlapped_encounter_branch_matches_serial_steps(enc_algo):
    """On a context with a stream the encounter check runs on a second stream
    beside S(h), the force and K(h) (graph branches); a context on the null
    stream runs every phase in order on one stream.  Same state, same lists,
    same statistics after 21 steps (graph replays plus a direct remainder)."""
    import torch
    w = workloads.ring(2000, m=3e-8)
    p = nb.default_params(G=w.G, enc_algo=enc_algo)
    serial = nb.Context(w.off, p, device="cuda:0", stream=torch.cuda.default_stream(torch.device("cuda:0")))
    serial.upload(w.m0, w.m, w.x, w.v)
    forked = ctx_for(w, enc_algo=enc_algo)
    outs = []
    for c in (serial, forked):
        st = c.step(w.dt, 21)
        e = c.last_encounters()
        outs.append((*c.download(nb.NB_DH), e.ice, e.jce, st["total_nce"], st["max_nce"]))
    assert outs[1][4] > 0
    for u, v in zip(*outs):
        assert np.array_equal(u, v)


# ---------------------------------------------------------------- edge cases
def test_nonfinite_upload_rejected():
    w = workloads.c1(50)
    c = ctx_for(w)
    x = w.x.copy()
    x[7, 1] = np.nan
    with pytest.raises(nb.NbError) as ei:
        c.upload(w.m0, w.m, x, w.v)
    assert ei.value.code == nb.NB_E_NONFINITE
    with pytest.raises(nb.NbError) as ei:
        c.upload(np.array([0.0]), w.m, w.x, w.v)
    assert ei.value.code == nb.NB_E_NONFINITE
    m = w.m.copy(); m[3] = -1.0
    with pytest.raises(nb.NbError):
        c.upload(w.m0, m, w.x, w.v)


def test_kepler_failure_flagged_and_body_kept():
    w = workloads.c1(40)
    x = w.x.copy(); v = w.v.copy()
    x[5] = 0.0                                  # a body at the star: no Kepler orbit
    c = ctx_for(w)
    c.upload(w.m0, w.m, x, v, frame=nb.NB_DH)
    with pytest.raises(nb.NbError) as ei:
        c.drift(w.dt)
    assert ei.value.code == nb.NB_E_KEPLER
    xg, vg = c.download(nb.NB_DH)
    assert np.all(xg[5] == 0.0) and np.all(vg[5] == v[5])
    q1, v1, fl = oracle.drift(w.G, w.dt, x, v)
    assert fl[5] == 1 and fl.sum() == 1
    keep = np.arange(40) != 5
    assert rel_rows(xg[keep], q1[keep]) <= 1e-13


def test_state_errors():
    w = workloads.c1(20)
    c = nb.Context(w.off, nb.default_params(), device="cuda:0")
    with pytest.raises(nb.NbError) as ei:
        c.step(0.1, 1)
    assert ei.value.code == nb.NB_E_NOT_READY
    c.upload(w.m0, w.m, w.x, w.v)
    with pytest.raises(nb.NbError) as ei:
        c.encounters()
    assert ei.value.code == nb.NB_E_NOT_READY


def test_device_pointer_upload_and_download():
    import torch
    w = workloads.batch([100, 33])
    c = ctx_for(w)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    c.upload(dev(w.m0), dev(w.m), dev(w.x.T), dev(w.v.T))
    xd = torch.empty((3, w.ntot), dtype=torch.float64, device="cuda:0")
    vd = torch.empty_like(xd)
    c.download_device(xd, vd, nb.NB_HELIO)
    torch.cuda.synchronize()
    assert np.array_equal(xd.cpu().numpy().T, w.x)
    assert rel_rows(vd.cpu().numpy().T, w.v) <= 8 * U


# ---------------------------------------------------------------- full hybrid method
def _oracle_full(w, steps, tol):
    st = oracle.State.from_workload(w)
    groups = bodies = 0
    for _ in range(steps):
        st.step(w.dt, full=True, tol=tol)
        groups += st.ngroups
        bodies += int(np.sum(st.groups >= 0))
    return st, groups, bodies


FULL_CASES = {
    "ring_n700": lambda: workloads.ring(700, m=3e-8),
    "batch_ragged": lambda: workloads.batch([1, 2, 3, 17, 0, 257, 600, 1031]),
    "ring_batch": lambda: workloads.batch([300, 5, 450], cfg_id=8, a_lo=0.98, a_hi=1.02),
}


@pytest.mark.parametrize("name", list(FULL_CASES))
@pytest.mark.parametrize("mode", [0, 1])
def test_full_steps_match_oracle(name, mode):
    """nb_step with resolve = 1 against the oracle's full step over 5 steps.
    Bar: the resolver's own global error (oracle at tol 1e-12 against 1e-14)
    plus the hot-path bar of the mode (1e-11 FP64, 1e-7 FP32C)."""
    w = FULL_CASES[name]()
    k = 5
    print(f"[full] {name} mode={mode}", flush=True)
    c = ctx_for(w, mode=mode, resolve=1)
    stats = c.step(w.dt, k)
    x, v = c.download(nb.NB_DH)
    st, groups, bodies = _oracle_full(w, k, 1e-12)
    st14, _, _ = _oracle_full(w, k, 1e-14)
    hot = 1e-11 if mode == 0 else 1e-7
    eq = rel_rows(st.Q, st14.Q) + hot
    ev = rel_rows(st.V, st14.V) + 10 * hot
    assert rel_rows(x, st.Q) <= 3 * eq, (name, rel_rows(x, st.Q), eq)
    assert rel_rows(v, st.V) <= 3 * ev, (name, rel_rows(v, st.V), ev)
    assert stats["bs_fail"] == 0
    if mode == 0:
        assert stats["resolved_groups"] == groups and stats["resolved_bodies"] == bodies
    if name != "batch_ragged":
        assert groups > 0


def test_full_steps_differ_from_hot_path_and_are_deterministic():
    w = FULL_CASES["ring_n700"]()
    outs = []
    for resolve in (1, 1, 0):
        c = ctx_for(w, resolve=resolve)
        st = c.step(w.dt, 5)
        outs.append((c.download(nb.NB_DH), st))
        c.close()
    (x1, v1), s1 = outs[0]
    (x2, v2), s2 = outs[1]
    (x0, v0), s0 = outs[2]
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
    assert s1["resolved_groups"] > 0 and s0["resolved_groups"] == 0
    assert rel_rows(x1, x0) > 1e-9


def test_full_mode_rejects_persistent_launch():
    w = workloads.c1(100)
    p = nb.default_params(G=w.G, resolve=1, step_algo=2)
    with pytest.raises(nb.NbError):
        nb.Context(w.off, p, device="cuda:0")


def test_full_mode_resolves_a_close_encounter():
    """Two bodies inside each other's changeover zone: the GPU full step and
    the oracle's full step agree through the encounter (20 steps)."""
    G = workloads.G_AU_MSUN_YR
    m = np.array([3e-6, 1e-7])

    def circ(r, th):
        vv = np.sqrt(G / r)
        return [r * np.cos(th), r * np.sin(th), 0.0], [-vv * np.sin(th), vv * np.cos(th), 0.0]
    xa, va = circ(1.0, 0.0)
    xb, vb = circ(1.02, 0.06)
    w = workloads.Workload("pair", np.array([0, 2], np.int32), np.array([1.0]), m, np.array([xa, xb]),
                           np.array([va, vb]), 0.02, 20)
    c = ctx_for(w, resolve=1)
    stats = c.step(w.dt, 20)
    x, v = c.download(nb.NB_DH)
    st, groups, _ = _oracle_full(w, 20, 1e-12)
    st14, _, _ = _oracle_full(w, 20, 1e-14)
    assert groups >= 10 and stats["resolved_groups"] == groups
    eq = rel_rows(st.Q, st14.Q) + 1e-11
    assert rel_rows(x, st.Q) <= 3 * eq, (rel_rows(x, st.Q), eq)


def test_resolved_choices():
    """nb_get_choices reports what the automatic choices resolved to."""
    ring = workloads.ring(2000, m=3e-8)
    c = ctx_for(ring)
    ch = c.choices()
    assert ch["force_algo"] == 2 and ch["enc_algo"] in (1, 2) and ch["step_algo"] in (1, 2)
    assert ctx_for(ring, force_algo=1).choices()["force_algo"] == 1
    # the radial order: FP32C only (FP64 takes the index order), not with the fused check
    assert ctx_for(ring, mode=1, force_algo=4).choices()["force_algo"] == 4
    assert ctx_for(ring, mode=0, force_algo=4).choices()["force_algo"] == 2
    assert ctx_for(ring, mode=1, force_algo=4, enc_algo=4).choices()["force_algo"] == 2
    assert ctx_for(ring, enc_algo=2).choices()["enc_algo"] == 2
    assert ctx_for(ring, resolve=1).choices()["step_algo"] == 1
    bs = workloads.bigsmall(50, 140000)
    chb = ctx_for(bs, force_r=1).choices()
    assert chb["force_algo"] == 3 and chb["enc_algo"] == 3      # few sources, few partners
    small = workloads.bigsmall(20, 3000)
    assert ctx_for(small).choices()["force_algo"] == 1           # too few target tiles
