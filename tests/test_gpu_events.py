"""GPU collisions, star impacts, ejections and compaction (nb_events,
nb_compact) against the oracle's (Sec. 2.1.1: physical radii, removal of lost
bodies; Sec. 2.1.2: planet-planet and planet-star collisions, ejections).

Three systems (one with massless small bodies) get a plunging body whose
pericentre falls inside the step, a chain of three overlapping bodies, a
coincident pair, a body that runs through another inside the step (apart at
both ends), and bodies beyond the ejection radius.  After one step the event
flags and counts must equal the oracle's, the changed masses, positions and
velocities agree to rounding, and after the compaction the offsets, big-body
counts, kept indices, state and force agree; two further steps follow the
oracle's.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import pair_scale, rel_rows

pytestmark = pytest.mark.gpu
nb = pytest.importorskip("paper_2601_19654_amd.nb")

G = workloads.G_AU_MSUN_YR
TAU = 0.01
RHO = 1.0          # Msun / AU^3: R ~ 6e-3 AU for 1e-6 Msun, inside rc ~ 2e-2 AU
R_STAR = 0.005
R_EJECT = 400.0


def _circ(r, th):
    s = np.sqrt(G / r)
    return np.array([r * np.cos(th), r * np.sin(th), 0.0]), np.array([-s * np.sin(th), s * np.cos(th), 0.0])


def _events_workload(nbig_small=True):
    w = workloads.batch([300, 200, 150], cfg_id=43)
    x, v, m = w.x.copy(), w.v.copy(), w.m.copy()
    m[:] = 1e-6
    R = oracle.phys_radius(np.array([1e-6]), RHO)[0]
    ex = np.array([1.0, 0.0, 0.0])
    # system 0, body 7: pericentre 0.002 AU at mid-step
    P = 2 * np.pi * np.sqrt(1.0 / G)
    xp, vp = workloads.elements_to_cartesian(np.array([G]), [1.0], [0.998], [0.1], [0.2], [0.3],
                                             [-np.pi * TAU / P])
    x[7], v[7] = xp[0], vp[0]
    # system 0: a chain 20 - 21 - 22 (neighbours overlap, the ends do not)
    x[21] = x[20] + 1.6 * R * ex
    x[22] = x[21] + 1.6 * R * ex
    v[21] = v[20]
    v[22] = v[20]
    # system 1: 303 on top of 304; 310 runs through 305 two thirds into the step
    x[304] = x[303] + [2e-4, 0.0, 0.0]
    v[304] = v[303]
    x[310] = x[305] + 0.2 * ex
    v[310] = v[305] + (x[305] - x[310]) * 1.5 / TAU
    # system 2: two bodies beyond the ejection radius
    x[505], v[505] = _circ(450.0, 0.3)
    x[510], v[510] = _circ(420.0, 2.0)
    nbig = None
    if nbig_small:
        # system 1: its last 10 bodies are small (massless)
        nbig = np.array([300, 190, 150], np.int32)
        m[490:500] = 0.0
    return workloads.Workload("events", w.off, w.m0, m, x, v, TAU, 3, nbig=nbig)


def _ctx(w, mode):
    # the per-phase step launch: the persistent one keeps no drift arcs for nb_events
    p = nb.default_params(G=w.G, mode=mode, step_algo=1)
    c = nb.Context(w.off, p, enc_cap=1 << 12, device="cuda:0", nbig=w.nbig)
    c.upload(w.m0, w.m, w.x, w.v)
    return c


@pytest.mark.parametrize("mode,tol_a", [(0, 1e-12), (1, 1e-6)])
def test_events_and_compaction_match_oracle(mode, tol_a):
    w = _events_workload()
    c = _ctx(w, mode)
    # no step yet: no drift arcs, no list
    with pytest.raises(nb.NbError) as e:
        c.events(RHO, R_STAR, R_EJECT)
    assert e.value.code == nb.NB_E_NOT_READY
    st = oracle.State(w.off, w.m0, w.m, w.x, w.v, oracle.Params(G=w.G), nbig=w.nbig)
    print(f"[events] mode {mode}: one step of {w.ntot} bodies", flush=True)
    c.step(TAU, 1)
    st.step(TAU)
    cnt, lost = c.events(RHO, R_STAR, R_EJECT)
    ev = st.events(TAU, RHO, R_STAR, R_EJECT)
    print(f"[events] counts gpu {cnt} oracle {ev}", flush=True)
    assert (cnt["star"], cnt["collide"], cnt["merged"], cnt["ejected"]) == ev
    assert np.array_equal(lost, st.lost)
    # the planted events all happened
    assert lost[7] == 1 and lost[21] == 2 and lost[22] == 2 and lost[304] == 2 and lost[310] == 2
    assert lost[505] == 3 and lost[510] == 3
    x, v = c.download(nb.NB_DH)
    keep = lost == 0
    # the kept bodies after the events (star shift, mergers, ejection dv); one
    # step carries the force's error through two half kicks and the drift
    # (FP32C: far pairs in FP32, <= 1e-6 of A_i; changeover pairs in FP64;
    # measured 3e-13 relative)
    tol1 = 1e-13 if mode == 0 else 1e-10
    assert rel_rows(x[keep], st.Q[keep]) <= tol1
    assert rel_rows(v[keep], st.V[keep]) <= tol1
    # compaction
    idx = c.compact()
    new, idx_ref = st.compacted()
    assert np.array_equal(idx, idx_ref)
    assert np.array_equal(c.off, new.off.astype(np.int32))
    assert np.array_equal(c.nbig, new.nbig.astype(np.int32))
    x, v = c.download(nb.NB_DH)
    assert rel_rows(x, new.Q) <= tol1 and rel_rows(v, new.V) <= tol1
    a = c.accel()
    for s, (lo, hi) in enumerate(new.systems()):
        A = pair_scale(new.m[lo:hi], new.Q[lo:hi], G)
        A[A == 0] = 1.0
        err = np.max(np.max(np.abs(a[lo:hi] - new.a[lo:hi]), axis=1) / A)
        assert err <= tol_a, (s, err)
    # the smaller arrays step on like the oracle's
    c.step(TAU, 2)
    for _ in range(2):
        new.step(TAU)
    x, v = c.download(nb.NB_DH)
    tol = 1e-11 if mode == 0 else 1e-7
    assert rel_rows(x, new.Q) <= tol and rel_rows(v, new.V) <= tol
    c.close()


def test_events_without_losses_change_nothing():
    w = workloads.batch([400, 123], cfg_id=44)
    c = _ctx(w, 0)
    c.step(w.dt, 2)
    x0, v0 = c.download(nb.NB_DH)
    a0 = c.accel()
    cnt, lost = c.events(3.37e6, 0.0, 0.0)
    assert cnt == {"star": 0, "collide": 0, "merged": 0, "ejected": 0} and not lost.any()
    x1, v1 = c.download(nb.NB_DH)
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1) and np.array_equal(a0, c.accel())
    idx = c.compact()
    assert np.array_equal(idx, np.arange(w.ntot)) and np.array_equal(c.off, w.off)
    # the list of the last step is still there and steps continue
    c.step(w.dt, 1)
    c.close()
