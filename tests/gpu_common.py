"""Shared helpers for the GPU parity tests (HIP library vs CPU oracle)."""
import numpy as np

import oracle
import workloads

U = 2.0 ** -53


def ctx_for(w, mode=0, enc_cap=1 << 16, **kw):
    from paper_2601_19654_amd import nb
    p = nb.default_params(G=w.G, mode=mode, drag=int(w.drag), **kw)
    c = nb.Context(w.off, p, enc_cap=enc_cap, device="cuda:0", nbig=getattr(w, "nbig", None))
    c.upload(w.m0, w.m, w.x, w.v)
    return c


def systems(w):
    for s in range(w.nsys):
        yield s, int(w.off[s]), int(w.off[s + 1])


def nbig_of(w, s):
    nb = getattr(w, "nbig", None)
    return int(w.off[s + 1] - w.off[s]) if nb is None else int(nb[s])


def oracle_dh(w):
    """DH state, critical radii and force of every system from the oracle."""
    Q = np.empty_like(w.x); V = np.empty_like(w.v); rc = np.empty(w.ntot); a = np.empty_like(w.x)
    for s, lo, hi in systems(w):
        if hi == lo:
            continue
        Q[lo:hi], V[lo:hi] = oracle.helio_to_dh(w.m0[s], w.m[lo:hi], w.x[lo:hi], w.v[lo:hi])
        rc[lo:hi] = oracle.rcrit(w.m0[s], w.m[lo:hi], Q[lo:hi])
        a[lo:hi] = oracle.force(w.m[lo:hi], Q[lo:hi], rc[lo:hi], w.G, nbig=nbig_of(w, s))
    return Q, V, rc, a


def pair_scale(m, Q, G, idx=None, chunk=2048):
    """A_i = sum_{j != i} G m_j / r_ij^2 for targets idx (tolerance scale)."""
    idx = np.arange(len(m)) if idx is None else np.asarray(idx)
    out = np.empty(len(idx))
    for a in range(0, len(idx), chunk):
        ii = idx[a:a + chunk]
        d = Q[None, :, :] - Q[ii, None, :]
        r2 = np.einsum("ijk,ijk->ij", d, d)
        r2[np.arange(len(ii)), ii] = np.inf
        r2[r2 == 0] = np.inf
        out[a:a + chunk] = np.sum(G * m[None, :] / r2, axis=1)
    return out


def accel_error(a_gpu, a_ref, A):
    """max over targets of max-component |error| / A_i (inf if any value is not finite)."""
    if not np.all(np.isfinite(a_gpu)):
        return float("inf")
    return float(np.max(np.max(np.abs(a_gpu - a_ref), axis=1) / A))


def rel_rows(x, ref):
    """max over bodies of |x_i - ref_i| / |ref_i| (vector rows)."""
    n = np.linalg.norm(ref, axis=1)
    n[n == 0] = 1.0
    return float(np.max(np.linalg.norm(x - ref, axis=1) / n)) if len(ref) else 0.0


def enc_compare(gpu_pairs, ref, tie):
    """Symmetric difference of two pair sets, excluding tie-band pairs."""
    g = set(gpu_pairs)
    r = set(ref)
    diff = (g ^ r) - set(tie)
    return diff
