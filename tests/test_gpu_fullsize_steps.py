"""Whole hybrid steps at full benchmark size, on the path the benchmark times,
against the CPU oracle body by body.

The timed step (``nb_step``: captured runs of steps replayed as HIP graphs,
the encounter check of a step on a second queue beside the next step, the
closing and opening kicks of consecutive steps merged into one launch, the
first stellar drift fused into the Kepler drift, the symmetric tile-pair force
kernels with their split partials) is compared with the oracle's step
K S D C S F K (Sec. 3.1: force, Hamiltonian, drift and encounter blocks) after
every one of three steps:

  * 16384-body annulus (the headline workload), FP64 and FP32C pair arithmetic
    (FP32C also with the force over the radial order, force_algo 4);
  * the first 64 systems of the 256-system batch (N_s from 200 to 4000, the
    largest system setting the split count, longest work first), FP32C.

Both FP32C cases also run with the encounter test inside the force pass over
the sorted order (enc_algo 4).

Bars: every body's Q and V within 1e-11 (FP64) or 1e-7 (FP32C) relative, the
accelerations within 1e-12 A_i (FP64) or 1e-6 A_i (FP32C), the flagged-pair
count of every step equal to the oracle's, and the last step's list equal to
the oracle's as a set.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import accel_error, ctx_for, pair_scale, rel_rows

pytestmark = pytest.mark.gpu
nb = pytest.importorskip("paper_2601_19654_amd.nb")

STEPS = 3


def _oracle_run(w):
    """The oracle's trajectory: (Q, V, a) after each step and the per-step lists."""
    st = oracle.State.from_workload(w, threads=True)
    out = []
    for k in range(STEPS):
        st.step(w.dt)
        pairs = set()
        for (nce, ii, jj) in st.enc:
            assert nce == len(ii)
            pairs |= set(zip(ii.tolist(), jj.tolist()))
        out.append((st.Q.copy(), st.V.copy(), st.a.copy(), pairs))
        print(f"[{w.name}] oracle step {k + 1}: {len(pairs)} flagged pairs", flush=True)
    return out


def _sampled_scale(w, Q, nsample=512, seed=3):
    """A_i of sampled bodies of every system (the force-error scale)."""
    rng = np.random.default_rng(seed)
    idx, A = [], []
    for s in range(w.nsys):
        lo, hi = int(w.off[s]), int(w.off[s + 1])
        k = min(hi - lo, max(4, nsample // w.nsys))
        ii = np.sort(rng.choice(hi - lo, k, replace=False))
        A.append(pair_scale(w.m[lo:hi], Q[lo:hi], w.G, ii))
        idx.append(ii + lo)
    return np.concatenate(idx), np.concatenate(A)


def _compare_steps(w, mode, ref, qtol, atol, enc_algo=0, force_algo=0):
    c = ctx_for(w, mode=mode, enc_cap=1 << 18, enc_algo=enc_algo, force_algo=force_algo)
    if force_algo == 4:
        assert c.choices()["force_algo"] == 4
    if enc_algo == 4:
        assert c.choices()["enc_algo"] == 4
    print(f"[{w.name}] mode {mode} choices {c.choices()} tiles {c.tiles}", flush=True)
    for k in range(STEPS):
        # one step per call: the run of one step is itself captured and replayed
        st = c.step(w.dt, 1)
        Q, V, a, pairs = ref[k]
        x, v = c.download(nb.NB_DH)
        eq, ev = rel_rows(x, Q), rel_rows(v, V)
        idx, A = _sampled_scale(w, Q)
        ea = accel_error(c.accel()[idx], a[idx], A)
        e = c.last_encounters()
        got = set(zip(e.ice.tolist(), e.jce.tolist()))
        print(f"[{w.name}] mode {mode} step {k + 1}: Q {eq:.2e} V {ev:.2e} a {ea:.2e} A_i, "
              f"{st['total_nce']} pairs (oracle {len(pairs)})", flush=True)
        assert eq <= qtol and ev <= qtol
        assert ea <= atol
        assert st["total_nce"] == len(pairs) and e.nce == len(pairs)
        assert got == pairs
    c.close()


def _compare_run(w, mode, ref, qtol, enc_algo=0, force_algo=0):
    """The same three steps as one nb_step call (a captured run of three steps)."""
    c = ctx_for(w, mode=mode, enc_cap=1 << 18, enc_algo=enc_algo, force_algo=force_algo)
    st = c.step(w.dt, STEPS)
    Q, V, _, pairs = ref[-1]
    x, v = c.download(nb.NB_DH)
    eq, ev = rel_rows(x, Q), rel_rows(v, V)
    total = sum(len(r[3]) for r in ref)
    print(f"[{w.name}] mode {mode} run of {STEPS}: Q {eq:.2e} V {ev:.2e}, {st['total_nce']} pairs "
          f"(oracle {total})", flush=True)
    assert eq <= qtol and ev <= qtol
    assert st["total_nce"] == total
    e = c.last_encounters()
    assert set(zip(e.ice.tolist(), e.jce.tolist())) == pairs
    c.close()


@pytest.fixture(scope="module")
def c3_ref():
    w = workloads.c3()
    return w, _oracle_run(w)


@pytest.mark.parametrize("mode,qtol,atol,enc_algo,force_algo", [(0, 1e-11, 1e-12, 0, 0), (1, 1e-7, 1e-6, 0, 0),
                                                                (1, 1e-7, 1e-6, 4, 0), (1, 1e-7, 1e-6, 0, 4)])
def test_c3_steps_match_oracle(c3_ref, mode, qtol, atol, enc_algo, force_algo):
    """enc_algo 4: the encounter test inside the force pass over the sorted
    order; force_algo 4: the symmetric force over the radial order."""
    w, ref = c3_ref
    _compare_steps(w, mode, ref, qtol, atol, enc_algo, force_algo)
    _compare_run(w, mode, ref, qtol, enc_algo, force_algo)


@pytest.fixture(scope="module")
def c4_ref():
    w = workloads.c4(nsys=64)
    return w, _oracle_run(w)


@pytest.mark.parametrize("enc_algo,force_algo", [(0, 0), (4, 0), (0, 4)])
def test_c4_batch_steps_match_oracle(c4_ref, enc_algo, force_algo):
    w, ref = c4_ref
    sizes = np.diff(w.off)
    assert w.nsys == 64 and sizes.min() >= 200 and sizes.max() <= 4000 and sizes.max() > 3500
    _compare_steps(w, 1, ref, 1e-7, 1e-6, enc_algo, force_algo)
    _compare_run(w, 1, ref, 1e-7, enc_algo, force_algo)
