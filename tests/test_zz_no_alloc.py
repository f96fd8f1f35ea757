"""The force entry point that allocates nothing (nb_force_noalloc) against the
context's nb_force + nb_get_accel on the same state and parameters: two calls
in a row, the second with a smaller system, each equal to the context's result
bit for bit (the same kernels and work items; the sums are taken in slot order
whatever the item order), and the oracle within the force bars."""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_common import accel_error, oracle_dh, pair_scale

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2601_19654_amd.nb")


def _context_accel(w, Q, mode, r, g):
    p = nb.default_params(G=w.G, mode=mode, force_r=r, force_g=g, force_algo=2)
    c = nb.Context(w.off, p, device="cuda:0", tuned=False)
    c.upload(w.m0, w.m, Q, np.zeros_like(Q), frame=nb.NB_DH)
    c.force()
    a = c.accel()
    used_g = c.choices()["force_g"]
    c.close()
    return a, used_g


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("r,g", [(2, 0), (1, 4), (4, 1)])
def test_noalloc_force_matches_context(mode, r, g):
    import torch
    bar = 1e-12 if mode == 0 else 1e-6
    for n, seed in ((5000, 11), (1203, 12)):            # the second call is smaller
        w = workloads.batch([n], cfg_id=seed)
        Q, _, _, a_ref = oracle_dh(w)
        a_ctx, used_g = _context_accel(w, Q, mode, r, g)
        p = nb.default_params(G=w.G, mode=mode, force_r=r, force_g=g, force_algo=2)
        dev = torch.device("cuda:0")
        m_d = torch.as_tensor(w.m, device=dev)
        x_d = torch.as_tensor(np.ascontiguousarray(Q.T), device=dev)     # plane-major
        a_d = torch.full((3, n), float("nan"), dtype=torch.float64, device=dev)
        print(f"nb_force_noalloc mode={mode} r={r} g={g} n={n}", flush=True)
        nb.force_noalloc(p, n, float(w.m0[0]), m_d, x_d, a_d)
        torch.cuda.synchronize()
        a = a_d.cpu().numpy().T
        assert np.array_equal(a, a_ctx), (mode, r, g, n, used_g)
        err = accel_error(a, a_ref, pair_scale(w.m, Q, w.G))
        assert err <= bar, (mode, r, g, n, err)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import torch
    p = nb.default_params(mode=0)
    dev = torch.device("cuda:0")
    n = nb.NOALLOC_MAX_N + 1
    m_d = torch.zeros(n, dtype=torch.float64, device=dev)
    x_d = torch.zeros(3 * n, dtype=torch.float64, device=dev)
    a_d = torch.zeros(3 * n, dtype=torch.float64, device=dev)
    assert nb.force_noalloc(p, n, 1.0, m_d, x_d, a_d, check=False) == nb.NB_E_WORKSPACE
    # a layout larger than the scratch (tiles of 64, one per super-tile) is refused too
    n = nb.NOALLOC_MAX_N
    p1 = nb.default_params(mode=0, force_r=1, force_g=1)
    assert nb.force_noalloc(p1, n, 1.0, m_d[:n], x_d[:3 * n], a_d[:3 * n], check=False) == nb.NB_E_WORKSPACE
