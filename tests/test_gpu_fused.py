"""The encounter check inside the force pass (enc_algo 4; Sec. 3.1 force block
loop 2 and encounter block in one loop over spatially sorted tiles) against
the separate sorted check and the CPU oracle.

After one step from an uploaded state both contexts drift the same arcs (the
first kick uses the force nb_upload computed), so the flagged lists and flags
must be identical; the force of the fused pass (summed over the sorted order)
agrees with the oracle to the FP32C bar.  Over five steps the states follow
the oracle within the FP32C bars.  Runs are bit-reproducible (the order inside
a cell of the sort is the index order), and timing the fused pass leaves the
last step's list as it was.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import accel_error, ctx_for, oracle_dh, pair_scale, rel_rows, systems

pytestmark = pytest.mark.gpu
nb = pytest.importorskip("paper_2601_19654_amd.nb")

CASES = {
    "ring_n700": lambda: workloads.ring(700, m=3e-8),
    "batch_ragged": lambda: workloads.batch([1, 2, 3, 17, 0, 257, 600, 1031]),
    "ring_n3000": lambda: workloads.ring(3000, m=3e-8),
    "c4_like_12": lambda: workloads.c4(nsys=12),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    return request.param, CASES[request.param]()


@pytest.mark.parametrize("r,g", [(2, 0), (1, 2), (4, 1), (2, 4)])
def test_fused_list_equals_sorted_check(case, r, g):
    name, w = case
    a = ctx_for(w, mode=nb.NB_FP32C, enc_algo=4, force_r=r, force_g=g, force_algo=2)
    # the same tiles (the fused mode takes two targets per lane where four were asked)
    assert a.params.force_r == min(r, 2)
    b = ctx_for(w, mode=nb.NB_FP32C, enc_algo=2, force_r=a.params.force_r, force_g=a.choices()["force_g"],
                force_algo=2)
    assert a.choices()["enc_algo"] == 4 and b.choices()["enc_algo"] == 2
    sa, sb = a.step(w.dt, 1), b.step(w.dt, 1)
    ea, eb = a.last_encounters(), b.last_encounters()
    print(f"[fused] {name} r={r} g={g}: {sa['total_nce']} pairs (sorted check {sb['total_nce']})", flush=True)
    assert sa["total_nce"] == sb["total_nce"] == ea.nce
    assert np.array_equal(ea.ice, eb.ice) and np.array_equal(ea.jce, eb.jce)
    assert np.array_equal(ea.ce, eb.ce)
    # the force at the new state: sorted order against index order, both FP32C
    xa, _ = a.download(nb.NB_DH)
    xb, _ = b.download(nb.NB_DH)
    assert np.array_equal(xa, xb)
    aa, ab = a.accel(), b.accel()
    for s, lo, hi in systems(w):
        if hi - lo < 2:
            continue
        A = pair_scale(w.m[lo:hi], xa[lo:hi], w.G)
        ref = oracle.force(w.m[lo:hi], xa[lo:hi], a.rcrit()[lo:hi], w.G)
        assert accel_error(aa[lo:hi], ref, A) <= 1e-6, (name, s)
        assert accel_error(ab[lo:hi], ref, A) <= 1e-6, (name, s)


def test_fused_steps_match_oracle(case):
    name, w = case
    c = ctx_for(w, mode=nb.NB_FP32C, enc_algo=4)
    st = oracle.State.from_workload(w)
    stats = c.step(w.dt, 5)
    total = 0
    for _ in range(5):
        st.step(w.dt)
        total += sum(e[0] for e in st.enc)
    x, v = c.download(nb.NB_DH)
    eq, ev = rel_rows(x, st.Q), rel_rows(v, st.V)
    print(f"[fused] {name} 5 steps: Q {eq:.2e} V {ev:.2e}, {stats['total_nce']} pairs (oracle {total})",
          flush=True)
    assert eq <= 1e-7 and ev <= 1e-6
    assert stats["total_nce"] == total


def test_fused_bitwise_determinism():
    w = workloads.ring(2400, m=3e-8)
    outs = []
    for _ in range(2):
        c = ctx_for(w, mode=nb.NB_FP32C, enc_algo=4)
        c.step(w.dt, 6)
        e = c.last_encounters()
        outs.append((*c.download(nb.NB_DH), c.accel(), e.ice, e.jce, e.ce))
        c.close()
    assert len(outs[0][3]) > 0
    for u, v in zip(*outs):
        assert np.array_equal(u, v)


def test_fused_timing_keeps_the_list():
    w = workloads.ring(3000, m=3e-8)
    c = ctx_for(w, mode=nb.NB_FP32C, enc_algo=4)
    with pytest.raises(nb.NbError):
        c.time_kernel(nb.NB_K_FORCE_FUSED, reps=2)      # no step yet
    c.step(w.dt, 2)
    e0 = c.last_encounters()
    a0 = c.accel()
    ms = c.time_kernel(nb.NB_K_FORCE_FUSED, reps=5)
    e1 = c.last_encounters()
    assert ms > 0 and e0.nce == e1.nce > 0
    assert np.array_equal(e0.ice, e1.ice) and np.array_equal(e0.jce, e1.jce) and np.array_equal(e0.ce, e1.ce)
    assert np.array_equal(a0, c.accel())


def test_fused_falls_back_where_it_does_not_apply():
    w = workloads.ring(700, m=3e-8)
    assert ctx_for(w, mode=nb.NB_FP64, enc_algo=4).choices()["enc_algo"] == 2      # FP64
    assert ctx_for(w, mode=nb.NB_FP32C, enc_algo=4, force_algo=1).choices()["enc_algo"] == 2   # ordered
    assert ctx_for(w, mode=nb.NB_FP32C, enc_algo=4, resolve=1).choices()["enc_algo"] == 2      # full method
