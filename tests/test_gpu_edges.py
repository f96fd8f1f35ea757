"""GPU edge cases of the hot path against the CPU oracle, and call sequences.

* Coincident distinct bodies (r = 0): the changeover weight is zero there
  (Sec. 3.1 force block with the changeover reading), so they add nothing to
  each other; FP32C must route them to its FP64 branch and stay finite.
* Massless bodies inside an all-big system (sources with m = 0, rc = 0).
* Time reversal of whole steps (the paper's integration direction flag,
  Sec. 3.2): with every pair outside the changeover zone (K = 1) the step
  K S D S K is a symmetric composition of exact flows, so 20 steps forward
  and 20 back return to the start within rounding.
* Checkpoint and resume: download, upload into a fresh context, continue.
* Graph cache: runs of different lengths in any order equal single steps bit
  for bit, and the encounter check can be re-run on the last step's drift
  outputs after them; nb_prepare changes nothing.
* After persistent steps (no drift outputs kept) the encounter check cannot
  be re-timed on stale data.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import accel_error, ctx_for, oracle_dh, pair_scale, rel_rows

pytestmark = pytest.mark.gpu
nb = pytest.importorskip("paper_2601_19654_amd.nb")


def _coincident():
    """A 300-body batch with exact copies of some bodies (same Q and V), a
    massless copy pair and a massless body on a massive one."""
    w = workloads.batch([300], cfg_id=21)
    m, x, v = w.m.copy(), w.x.copy(), w.v.copy()
    for a, b in ((3, 150), (10, 11), (200, 299)):
        x[b], v[b] = x[a], v[a]
    m[[40, 41]] = 0.0
    x[41], v[41] = x[40], v[40]
    m[77] = 0.0
    x[77], v[77] = x[78], v[78]
    return workloads.Workload("coincident", w.off, w.m0, m, x, v, w.dt, 5)


def _massless_in_all_big():
    w = workloads.batch([700, 257], cfg_id=22)
    m = w.m.copy()
    m[::7] = 0.0
    return workloads.Workload("massless", w.off, w.m0, m, w.x, w.v, w.dt, 5)


@pytest.mark.parametrize("mode,tol", [(0, 1e-12), (1, 1e-6)])
@pytest.mark.parametrize("force_algo", [1, 2, 4])
@pytest.mark.parametrize("maker", [_coincident, _massless_in_all_big])
def test_degenerate_bodies_force_and_steps(maker, mode, tol, force_algo):
    w = maker()
    Q, V, rc, a_ref = oracle_dh(w)
    c = ctx_for(w, mode=mode, force_algo=force_algo)
    a = c.accel()
    assert np.all(np.isfinite(a))
    for s in range(w.nsys):
        lo, hi = int(w.off[s]), int(w.off[s + 1])
        A = pair_scale(w.m[lo:hi], Q[lo:hi], w.G)
        A = np.where(A > 0, A, np.max(A))
        err = accel_error(a[lo:hi], a_ref[lo:hi], A)
        print(f"{w.name} mode {mode} algo {force_algo} system {s}: {err:.3e} A_i", flush=True)
        assert err <= tol
    st = oracle.State.from_workload(w)
    c.step(w.dt, 3)
    for _ in range(3):
        st.step(w.dt)
    x, v = c.download(nb.NB_DH)
    qtol = 1e-11 if mode == 0 else 1e-7
    assert rel_rows(x, st.Q) <= qtol and rel_rows(v, st.V) <= 10 * qtol


@pytest.mark.parametrize("mode,tol", [(0, 1e-12), (1, 1e-9)])
def test_steps_reverse(mode, tol):
    """20 steps forward, 20 back, with critical radii too small for any pair to
    reach its changeover zone (K = 1 everywhere)."""
    w = workloads.batch([100, 301], cfg_id=23)
    c = ctx_for(w, mode=mode, n_hill=1e-9)
    x0, v0 = c.download(nb.NB_DH)
    st = c.step(w.dt, 20)
    assert st["near_pairs"] == 0 and st["total_nce"] == 0
    x1, _ = c.download(nb.NB_DH)
    assert rel_rows(x1, x0) > 1e-3            # it moved
    c.step(-w.dt, 20)
    x2, v2 = c.download(nb.NB_DH)
    eq, ev = rel_rows(x2, x0), rel_rows(v2, v0)
    print(f"reversal mode {mode}: Q {eq:.2e} V {ev:.2e}")
    assert eq <= tol and ev <= tol


@pytest.mark.parametrize("mode,step_algo", [(0, 1), (1, 1), (0, 2)])
def test_checkpoint_resume(mode, step_algo):
    """Per-phase launches (step_algo 1): a run resumed from a downloaded state
    equals, bit for bit, the straight run whose stellar momentum is summed again
    at the same point (a zero kick makes the next step sum it from V instead of
    carrying it over, which is what a fresh context does); against the
    uninterrupted run it differs only by the rounding of that sum.
    Persistent launch (step_algo 2): its force loop sums each target's sources
    in its own order, while nb_upload primes the force with the force kernel,
    so a resumed run starts from a force rounded differently; it stays within
    1e-12 of the straight run."""
    w = workloads.ring(1500, m=3e-8)
    a = ctx_for(w, mode=mode, step_algo=step_algo)
    b = ctx_for(w, mode=mode, step_algo=step_algo)
    u = ctx_for(w, mode=mode, step_algo=step_algo)
    assert a.choices()["step_algo"] == step_algo
    a.step(w.dt, 6)
    b.step(w.dt, 6)
    u.step(w.dt, 6)
    x, v = b.download(nb.NB_DH)
    b.close()
    r = ctx_for(w, mode=mode, step_algo=step_algo)
    r.upload(w.m0, w.m, x, v, frame=nb.NB_DH)
    a.kick(0.0)
    sa = a.step(w.dt, 7)
    sr = r.step(w.dt, 7)
    su = u.step(w.dt, 7)
    xa, va = a.download(nb.NB_DH)
    xr, vr = r.download(nb.NB_DH)
    xu, vu = u.download(nb.NB_DH)
    if step_algo == 1:
        assert np.array_equal(xa, xr) and np.array_equal(va, vr)
        assert np.array_equal(a.accel(), r.accel())
        assert sa["total_nce"] == sr["total_nce"] > 0
        assert np.array_equal(a.last_encounters().ice, r.last_encounters().ice)
    else:
        dq, dv = rel_rows(xr, xa), rel_rows(vr, va)
        print(f"resume persistent: vs straight run Q {dq:.2e} V {dv:.2e}")
        assert dq <= 1e-12 and dv <= 1e-12 and sa["total_nce"] == sr["total_nce"] > 0
    du = rel_rows(xr, xu)
    print(f"resume mode {mode} step_algo {step_algo}: vs uninterrupted run {du:.2e}")
    assert du <= 1e-12 and su["total_nce"] == sr["total_nce"]


@pytest.mark.parametrize("force_algo", [0, 4])
def test_graph_runs_of_mixed_lengths(force_algo):
    """Captured runs of any lengths give the bits of single steps; with the
    radial order too (it is set at upload, not by the runs)."""
    w = workloads.ring(2500, m=3e-8, a_lo=0.6, a_hi=1.4) if force_algo == 4 else workloads.ring(2500, m=3e-8)
    a = ctx_for(w, mode=1, force_algo=force_algo)
    b = ctx_for(w, mode=1, force_algo=force_algo)
    lists = []
    for k in (8, 3, 8, 5, 20, 1, 8):
        a.prepare(w.dt, k)
        a.step(w.dt, k)
        e = a.last_encounters()
        # re-running the check on the last step's drift outputs gives its list
        a.time_kernel(nb.NB_K_ENCOUNTER, reps=2)
        e2 = a.last_encounters()
        assert e.nce == e2.nce > 0
        assert np.array_equal(e.ice, e2.ice) and np.array_equal(e.jce, e2.jce)
        lists.append(e)
        for _ in range(k):
            b.step(w.dt, 1)
        eb = b.last_encounters()
        assert np.array_equal(e.ice, eb.ice) and np.array_equal(e.jce, eb.jce)
    xa, va = a.download(nb.NB_DH)
    xb, vb = b.download(nb.NB_DH)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_prepare_then_timed_steps():
    w = workloads.batch([800, 1200], cfg_id=24)
    a = ctx_for(w)
    b = ctx_for(w)
    a.prepare(w.dt, 21)
    xa0, _ = a.download(nb.NB_DH)
    xb0, _ = b.download(nb.NB_DH)
    assert np.array_equal(xa0, xb0)           # preparing runs no step
    ms = a.time_kernel(nb.NB_K_STEP, reps=21, dt=w.dt)
    b.step(w.dt, 1)
    b.step(w.dt, 21)
    xa, va = a.download(nb.NB_DH)
    xb, vb = b.download(nb.NB_DH)
    assert ms > 0
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_no_stale_check_after_persistent_steps():
    w = workloads.batch([300, 500], cfg_id=25)
    c = ctx_for(w, step_algo=2)
    assert c.choices()["step_algo"] == 2
    c.step(w.dt, 5)
    e = c.last_encounters()                   # the persistent launch's own list
    assert e.nce >= 0
    with pytest.raises(nb.NbError) as ei:
        c.time_kernel(nb.NB_K_ENCOUNTER, reps=1)
    assert ei.value.code == nb.NB_E_NOT_READY
    c.time_kernel(nb.NB_K_STEP, reps=2, dt=w.dt)
    with pytest.raises(nb.NbError) as ei:
        c.encounters()
    assert ei.value.code == nb.NB_E_NOT_READY
    with pytest.raises(nb.NbError) as ei:
        c.time_kernel(nb.NB_K_ENCOUNTER, reps=1)
    assert ei.value.code == nb.NB_E_NOT_READY
    # a drift provides fresh outputs again
    c.drift(w.dt)
    c.encounters()
    c.time_kernel(nb.NB_K_ENCOUNTER, reps=1)
