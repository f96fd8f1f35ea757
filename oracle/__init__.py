"""CPU oracle for the hybrid symplectic N-body hot path (Mercury-Opal, arXiv 2601.19654).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` are the only callers.  The product path never
imports this package.

``nbody_oracle.c`` is a plain serial FP64 implementation written from the paper
(Sec. 2.1.1 for the integrator and its coordinates, Sec. 3.1 for the force,
Hamiltonian, drift and encounter blocks) and from the textbook definitions it
relies on; this module is argument marshalling around it (numpy, ctypes) plus a
multi-system driver that repeats the single-system C routines per system.

Parity status per function (pins live in ``tests/test_oracle_*.py``):
  force, changeover, rcrit   pinned (closed forms, Newton III, torque, FD gradient)
  Kepler drift, Stumpff      pinned (Kepler's equation, invariants, library trig)
  encounter predicate        pinned (straight-line closed form, dense sampling)
  energy / momenta           pinned (explicit barycentric formula, invariants)
  transforms                 pinned (barycentre definition, round trip)
  step                       pinned (2nd-order convergence, reversibility, E bound)
  big/small split            pinned (massless sources change no sum, big bodies
                             do not see small ones, each small body moves as if
                             alone with the big ones, small pairs never flagged)
  close-encounter resolver   pinned (Kepler flow for a lone body, relative Kepler
  (Bulirsch-Stoer on H0)     orbit of a bound pair, H0 energy, time reversal;
                             the full step converges at second order to an
                             independent Newtonian integration)
  collisions, star impacts,  pinned (sphere mass, pericentre distance of the
  ejections, compaction      generating elements and dense arc sampling, mass,
                             momentum and barycentre conservation, unchanged
                             heliocentric motion of the rest, order kept)
  sampled force / pair scan  pinned (bit-equal to the full routines' rows)
  gas drag                   parity unpinned by the paper (limits and closed form
                             of the chosen formula only)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with OpenMP (targets, bodies and encounter rows split over
# threads, results bit-identical): the threaded CPU baseline only
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99"]


def _stale(path: str) -> bool:
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, no contraction, no fast math),
    serial and with OpenMP."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or _stale(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB


_lib = None
_lib_omp = None


def lib(threads: bool = False):
    """The serial oracle (threads=True: the OpenMP build of the same source)."""
    global _lib, _lib_omp
    if threads:
        if _lib_omp is None:
            build(force=False)
            _lib_omp = _load(_LIB_OMP)
        return _lib_omp
    if _lib is None:
        build(force=False)
        _lib = _load(_LIB)
    return _lib


def _load(path):
    L = ctypes.CDLL(path)
    d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    sig = {
        "orc_changeover": (None, [d, d, d, p, p]),
        "orc_rcrit": (None, [i, d, p, p, d, p]),
        "orc_force": (None, [i, d, d, p, p, p, p]),
        "orc_force_nb": (None, [i, i, d, d, p, p, p, p]),
        "orc_force_subset": (None, [i, i, d, d, p, p, p, i, p, p]),
        "orc_kick": (None, [i, d, p, p]),
        "orc_momentum": (None, [i, p, p, p]),
        "orc_sun_drift": (None, [i, d, d, p, p, p]),
        "orc_helio_to_dh": (None, [i, d, p, p, p, p, p]),
        "orc_dh_to_helio": (None, [i, d, p, p, p, p, p]),
        "orc_stumpff": (None, [d, p]),
        "orc_kepler_drift": (i, [d, d, p, p]),
        "orc_drift": (i, [i, d, d, p, p, p]),
        "orc_pair_min_d2": (d, [d, p, p, p, p, p, p, p, p]),
        "orc_encounters": (None, [i, d, p, p, p, p, p, i, p, p, p, p, d, i, p, p, p]),
        "orc_encounters_nb": (None, [i, i, d, p, p, p, p, p, i, p, p, p, p, d, i, p, p, p]),
        "orc_pair_scan": (None, [i, i, d, p, p, p, p, p, i, d, p, p]),
        "orc_energy": (None, [i, d, d, d, p, p, p, p, p, p, p, p]),
        "orc_drag_accel": (None, [i, d, d, p, p, p, p, d, d, d, d, p]),
        "orc_kick_drag": (None, [i, d, d, d, p, p, p, p, d, d, d, d, p]),
        "orc_step": (i, [i, i, d, d, d, d, p, p, p, p, p, d, i, d, d, d, d, p, p, p, p, i, p, p, p, p]),
        "orc_bs_work_doubles": (i, [i]),
        "orc_resolve_work_doubles": (i, [i]),
        "orc_bs_h0": (i, [i, d, d, d, p, p, d, d, p, p, p]),
        "orc_resolve": (i, [i, d, d, d, p, p, d, d, p, p, i, p, p, p, p, p, p, p, p]),
        "orc_step_full": (i, [i, i, d, d, d, d, p, p, p, p, p, d, i, d, d, d, d, d, p, p, p, p, i, p,
                              p, p, p, p, p, p, p]),
        "orc_phys_radius": (None, [i, p, d, p]),
        "orc_star_min": (d, [d, d, p, p, p, p]),
        "orc_events": (None, [i, d, p, p, p, p, p, p, p, p, d, i, p, p, d, d, d, p, p]),
        "orc_compact": (i, [i, p, p, p, p, p, p, p, p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- constants
# Project constants (units AU, Msun, yr).  Written out here independently of
# the HIP library; the paper fixes none of them.
AU_CM = 1.495978707e13
MSUN_G = 1.98840987e33
RHO_UNIT = MSUN_G / AU_CM ** 3          # g/cm^3 per Msun/AU^3
SIGMA_UNIT = MSUN_G / AU_CM ** 2        # g/cm^2 per Msun/AU^2


@dataclass
class Params:
    G: float = (0.01720209895 * 365.25) ** 2
    n_hill: float = 3.0
    inner: float = 0.1
    drag: bool = False
    sigma0: float = 1000.0 / SIGMA_UNIT   # 1000 g/cm^2 at 1 AU
    h: float = 0.05
    cd: float = 1.0
    rho_p: float = 2.0 / RHO_UNIT         # 2 g/cm^3


# ---------------------------------------------------------------- single system
def changeover(r, rc, inner=0.1):
    K, dK = ctypes.c_double(), ctypes.c_double()
    lib().orc_changeover(float(r), float(rc), float(inner), ctypes.byref(K), ctypes.byref(dK))
    return K.value, dK.value


def rcrit(m0, m, Q, n_hill=3.0):
    m = _f64(m); Q = _f64(Q, (-1, 3)); rc = np.empty(len(m))
    lib().orc_rcrit(len(m), float(m0), _ptr(m), _ptr(Q), float(n_hill), _ptr(rc))
    return rc


def force(m, Q, rc, G, inner=0.1, nbig=None):
    """Interaction acceleration; with nbig, only the first nbig bodies are sources."""
    m = _f64(m); Q = _f64(Q, (-1, 3)); rc = _f64(rc); a = np.empty_like(Q)
    n = len(m)
    lib().orc_force_nb(n, n if nbig is None else int(nbig), float(G), float(inner), _ptr(m), _ptr(Q),
                       _ptr(rc), _ptr(a))
    return a


def force_subset(m, Q, rc, G, idx, inner=0.1, nbig=None):
    """Accelerations of the targets idx only (the same per-target sum as force)."""
    m = _f64(m); Q = _f64(Q, (-1, 3)); rc = _f64(rc)
    idx = np.ascontiguousarray(idx, dtype=np.int32); a = np.empty((len(idx), 3))
    n = len(m)
    if len(idx) and (idx.min() < 0 or idx.max() >= n):
        raise IndexError("force_subset: target index out of range")
    lib().orc_force_subset(n, n if nbig is None else int(nbig), float(G), float(inner), _ptr(m), _ptr(Q),
                           _ptr(rc), len(idx), _ptr(idx), _ptr(a))
    return a


def momentum(m, V):
    m = _f64(m); V = _f64(V, (-1, 3)); P = np.empty(3)
    lib().orc_momentum(len(m), _ptr(m), _ptr(V), _ptr(P))
    return P


def kick(h, a, V):
    a = _f64(a, (-1, 3)); V = _f64(V, (-1, 3)).copy()
    lib().orc_kick(len(V), float(h), _ptr(a), _ptr(V))
    return V


def sun_drift(h, m0, m, V, Q):
    m = _f64(m); V = _f64(V, (-1, 3)); Q = _f64(Q, (-1, 3)).copy()
    lib().orc_sun_drift(len(m), float(h), float(m0), _ptr(m), _ptr(V), _ptr(Q))
    return Q


def helio_to_dh(m0, m, xh, vh):
    m = _f64(m); xh = _f64(xh, (-1, 3)); vh = _f64(vh, (-1, 3))
    Q = np.empty_like(xh); V = np.empty_like(vh)
    lib().orc_helio_to_dh(len(m), float(m0), _ptr(m), _ptr(xh), _ptr(vh), _ptr(Q), _ptr(V))
    return Q, V


def dh_to_helio(m0, m, Q, V):
    m = _f64(m); Q = _f64(Q, (-1, 3)); V = _f64(V, (-1, 3))
    xh = np.empty_like(Q); vh = np.empty_like(V)
    lib().orc_dh_to_helio(len(m), float(m0), _ptr(m), _ptr(Q), _ptr(V), _ptr(xh), _ptr(vh))
    return xh, vh


def stumpff(z):
    c = np.empty(4)
    lib().orc_stumpff(float(z), _ptr(c))
    return c


def drift(mu, tau, Q, V):
    """Kepler-drift every body; returns (Q, V, flags)."""
    Q = _f64(Q, (-1, 3)).copy(); V = _f64(V, (-1, 3)).copy()
    flag = np.zeros(len(Q), dtype=np.int32)
    lib().orc_drift(len(Q), float(mu), float(tau), _ptr(Q), _ptr(V), _ptr(flag))
    return Q, V, flag


def pair_min_d2(tau, q0i, v0i, q1i, v1i, q0j, v0j, q1j, v1j):
    args = [_f64(t, (3,)) for t in (q0i, v0i, q1i, v1i, q0j, v0j, q1j, v1j)]
    return lib().orc_pair_min_d2(float(tau), *[_ptr(t) for t in args])


def encounters(tau, Q0, V0, Q1, V1, rc, cap=None, tie=1e-10, nbig=None):
    """Flagged pairs (i<j, lexicographic), per-body flags, tie-band pairs.
    With nbig, pairs of two small bodies (both >= nbig) are not tested."""
    Q0, V0, Q1, V1 = (_f64(t, (-1, 3)) for t in (Q0, V0, Q1, V1))
    rc = _f64(rc); n = len(rc)
    cap = n * (n - 1) // 2 if cap is None else cap
    cap_alloc = max(cap, 1)
    ice = np.zeros(cap_alloc, np.int32); jce = np.zeros(cap_alloc, np.int32)
    ce = np.zeros(max(n, 1), np.int32)
    tie_cap = 1 << 16
    ti = np.zeros(tie_cap, np.int32); tj = np.zeros(tie_cap, np.int32)
    nce = ctypes.c_int(); ntie = ctypes.c_int()
    lib().orc_encounters_nb(n, n if nbig is None else int(nbig), float(tau), _ptr(Q0), _ptr(V0), _ptr(Q1),
                            _ptr(V1), _ptr(rc), int(cap), _ptr(ice), _ptr(jce), _ptr(ce), ctypes.byref(nce),
                            float(tie), tie_cap, _ptr(ti), _ptr(tj), ctypes.byref(ntie))
    k = min(nce.value, cap)
    t = min(ntie.value, tie_cap)
    return {"nce": nce.value, "ice": ice[:k].copy(), "jce": jce[:k].copy(), "ce": ce[:n].copy(),
            "tie": set(zip(ti[:t].tolist(), tj[:t].tolist())), "ntie": ntie.value}


def pair_scan(tau, Q0, V0, Q1, V1, rc, i, tie=1e-10, nbig=None):
    """Flags of every pair (i, j) of one system under the encounter predicate."""
    Q0, V0, Q1, V1 = (_f64(t, (-1, 3)) for t in (Q0, V0, Q1, V1))
    rc = _f64(rc); n = len(rc)
    flag = np.zeros(n, np.int32); tflag = np.zeros(n, np.int32)
    lib().orc_pair_scan(n, n if nbig is None else int(nbig), float(tau), _ptr(Q0), _ptr(V0), _ptr(Q1),
                        _ptr(V1), _ptr(rc), int(i),
                        float(tie), _ptr(flag), _ptr(tflag))
    return flag.astype(bool), tflag.astype(bool)


def energy(G, m0, m, Q, V, rc, inner=0.1):
    m = _f64(m); Q = _f64(Q, (-1, 3)); V = _f64(V, (-1, 3)); rc = _f64(rc)
    E, EK = ctypes.c_double(), ctypes.c_double()
    L = np.empty(3); P = np.empty(3)
    lib().orc_energy(len(m), float(G), float(m0), float(inner), _ptr(m), _ptr(Q), _ptr(V), _ptr(rc),
                     ctypes.byref(E), ctypes.byref(EK), _ptr(L), _ptr(P))
    return {"E": E.value, "EK": EK.value, "L": L, "P": P}


def drag_accel(G, m0, m, Q, V, prm: Params):
    m = _f64(m); Q = _f64(Q, (-1, 3)); V = _f64(V, (-1, 3))
    P = momentum(m, V); ad = np.empty_like(Q)
    lib().orc_drag_accel(len(m), float(G), float(m0), _ptr(m), _ptr(Q), _ptr(V), _ptr(P),
                         prm.sigma0, prm.h, prm.cd, prm.rho_p, _ptr(ad))
    return ad


def bs_h0(G, m0, m, rc, Q, V, tau, tol=1e-12, inner=0.1):
    """Advance one group under H0 (Kepler + (1 - K) pair part) by tau.
    Returns (Q, V, steps); raises on failure."""
    m = _f64(m); rc = _f64(rc); k = len(m)
    y = np.empty((k, 6)); y[:, :3] = _f64(Q, (-1, 3)); y[:, 3:] = _f64(V, (-1, 3))
    y = np.ascontiguousarray(y)
    work = np.empty(max(lib().orc_bs_work_doubles(k), 1))
    st = ctypes.c_int()
    if lib().orc_bs_h0(k, float(G), float(m0), float(inner), _ptr(m), _ptr(rc), float(tau), float(tol),
                       _ptr(y), _ptr(work), ctypes.byref(st)):
        raise RuntimeError("Bulirsch-Stoer integration failed")
    return y[:, :3].copy(), y[:, 3:].copy(), st.value


def resolve(G, m0, m, rc, tau, Q0, V0, ice, jce, Q, V, tol=1e-12, inner=0.1):
    """Resolve the groups of one system's pair list (local indices).
    Returns (Q, V, comp, nfail, ngroups, max_steps)."""
    m = _f64(m); rc = _f64(rc); n = len(m)
    Q0 = _f64(Q0, (-1, 3)); V0 = _f64(V0, (-1, 3))
    Q = _f64(Q, (-1, 3)).copy(); V = _f64(V, (-1, 3)).copy()
    ice = np.ascontiguousarray(ice, dtype=np.int32); jce = np.ascontiguousarray(jce, dtype=np.int32)
    comp = np.empty(max(n, 1), np.int32)
    work = np.empty(max(lib().orc_resolve_work_doubles(n), 1))
    ng, ms = ctypes.c_int(), ctypes.c_int()
    nf = lib().orc_resolve(n, float(G), float(m0), float(inner), _ptr(m), _ptr(rc), float(tau), float(tol),
                           _ptr(Q0), _ptr(V0), len(ice), _ptr(ice), _ptr(jce), _ptr(Q), _ptr(V), _ptr(comp),
                           _ptr(work), ctypes.byref(ng), ctypes.byref(ms))
    return Q, V, comp[:n].copy(), nf, ng.value, ms.value


def phys_radius(m, rho):
    """Physical radii from mass and one bulk density."""
    m = _f64(m); R = np.empty(len(m))
    lib().orc_phys_radius(len(m), _ptr(m), float(rho), _ptr(R))
    return R


def star_min(mu, tau, q0, v0, q1, v1):
    """Closest approach to the star along one drift arc of duration tau."""
    a = [_f64(t, (3,)) for t in (q0, v0, q1, v1)]
    return lib().orc_star_min(float(mu), float(tau), *[_ptr(t) for t in a])


LOST_STAR, LOST_MERGED, LOST_EJECTED = 1, 2, 3


def events(G, m0, m, Q, V, Q0, V0, Q1, V1, tau, ice, jce, rho, r_star, r_eject=0.0):
    """Star impacts, collisions and ejections of one step of one system (local
    pair indices).  Returns (m0, m, Q, V, lost, counts) with counts = (star
    impacts, colliding pairs, bodies merged away, ejections)."""
    m = _f64(m).copy(); Q = _f64(Q, (-1, 3)).copy(); V = _f64(V, (-1, 3)).copy()
    Q0, V0, Q1, V1 = (_f64(t, (-1, 3)) for t in (Q0, V0, Q1, V1))
    ice = np.ascontiguousarray(ice, dtype=np.int32); jce = np.ascontiguousarray(jce, dtype=np.int32)
    n = len(m)
    mm0 = ctypes.c_double(float(m0))
    lost = np.zeros(max(n, 1), np.int32); ev = np.zeros(4, np.int32)
    lib().orc_events(n, float(G), ctypes.byref(mm0), _ptr(m), _ptr(Q), _ptr(V), _ptr(Q0), _ptr(V0), _ptr(Q1),
                     _ptr(V1), float(tau), len(ice), _ptr(ice), _ptr(jce), float(rho), float(r_star),
                     float(r_eject), _ptr(lost), _ptr(ev))
    return mm0.value, m, Q, V, lost[:n].copy(), tuple(int(e) for e in ev)


def compact(lost, m, Q, V):
    """The kept bodies (lost == 0) in order, and their old indices."""
    lost = np.ascontiguousarray(lost, dtype=np.int32); m = _f64(m)
    Q = _f64(Q, (-1, 3)); V = _f64(V, (-1, 3)); n = len(m)
    mo = np.empty(max(n, 1)); Qo = np.empty((max(n, 1), 3)); Vo = np.empty((max(n, 1), 3))
    idx = np.empty(max(n, 1), np.int32)
    k = lib().orc_compact(n, _ptr(lost), _ptr(m), _ptr(Q), _ptr(V), _ptr(mo), _ptr(Qo), _ptr(Vo), _ptr(idx))
    return mo[:k].copy(), Qo[:k].copy(), Vo[:k].copy(), idx[:k].copy()


# ---------------------------------------------------------------- multi-system driver
class State:
    """Oracle state of a batch of independent systems in DH coordinates.

    Mirrors the step order K(h) S(h) D(tau) C S(h) [rc, force] K(h) with the
    force primed at construction (first-same-as-last).
    """

    def __init__(self, off, m0, m, x, v, prm: Params | None = None, frame="helio", nbig=None,
                 threads: bool = False):
        self.prm = prm or Params()
        # threads: steps run in the OpenMP build of the oracle (same results)
        self.threads = bool(threads)
        self.off = np.asarray(off, dtype=np.int64)
        # per system: bodies [off[s], off[s] + nbig[s]) are big (gravity sources)
        self.nbig = (np.diff(self.off) if nbig is None else np.asarray(nbig, dtype=np.int64)).copy()
        self.m0 = _f64(m0).copy()
        self.m = _f64(m).copy()
        n = len(self.m)
        self.Q = np.empty((n, 3)); self.V = np.empty((n, 3))
        for s, (a, b) in enumerate(self.systems()):
            if frame == "helio":
                self.Q[a:b], self.V[a:b] = helio_to_dh(self.m0[s], self.m[a:b], x[a:b], v[a:b])
            else:
                self.Q[a:b] = x[a:b]; self.V[a:b] = v[a:b]
        self.rc = np.empty(n)
        self.a = np.empty((n, 3))
        self.Q0 = self.Q.copy(); self.V0 = self.V.copy()
        self.kflag = np.zeros(n, np.int32)
        self.ce = np.zeros(n, np.int32)
        self.enc = []
        self.prime()

    @classmethod
    def from_workload(cls, w, prm: Params | None = None, threads: bool = False):
        prm = prm or Params(G=w.G, drag=w.drag)
        return cls(w.off, w.m0, w.m, w.x, w.v, prm, nbig=getattr(w, "nbig", None), threads=threads)

    def systems(self):
        for s in range(len(self.m0)):
            yield int(self.off[s]), int(self.off[s + 1])

    def prime(self):
        p = self.prm
        L = lib(self.threads)
        for s, (a, b) in enumerate(self.systems()):
            self.rc[a:b] = rcrit(self.m0[s], self.m[a:b], self.Q[a:b], p.n_hill)
            m = np.ascontiguousarray(self.m[a:b]); Q = np.ascontiguousarray(self.Q[a:b])
            rc = np.ascontiguousarray(self.rc[a:b]); acc = np.empty((b - a, 3))
            L.orc_force_nb(b - a, int(self.nbig[s]), p.G, p.inner, _ptr(m), _ptr(Q), _ptr(rc), _ptr(acc))
            self.a[a:b] = acc

    def step(self, tau, cap=None, full=False, tol=1e-12):
        """One hybrid step of every system; returns the total Kepler failures
        (plus, with ``full``, the failed close-encounter groups).

        ``full`` resolves the flagged groups by Bulirsch-Stoer on H0 between
        the encounter check and the second stellar drift (the full hybrid
        method); ``self.groups`` then holds, per body, its group label (the
        smallest member, global index) or -1.  ``self.enc`` receives, per
        system, the flagged pair list in global indices."""
        p = self.prm
        L = lib(self.threads)
        nfail = 0
        self.enc = []
        if full:
            self.groups = np.full(len(self.m), -1, np.int64)
            self.ngroups = 0
        for s, (a, b) in enumerate(self.systems()):
            n = b - a
            Q = np.ascontiguousarray(self.Q[a:b]); V = np.ascontiguousarray(self.V[a:b])
            A = np.ascontiguousarray(self.a[a:b]); rc = np.ascontiguousarray(self.rc[a:b])
            m = np.ascontiguousarray(self.m[a:b])
            Q0 = np.empty_like(Q); V0 = np.empty_like(V)
            kf = np.zeros(n, np.int32); ce = np.zeros(max(n, 1), np.int32)
            scratch = np.empty_like(Q)
            nbs = int(self.nbig[s])
            # pairs with a big member: at most nbig (n - 1) - nbig (nbig - 1) / 2
            c = nbs * (n - 1) - nbs * (nbs - 1) // 2 if cap is None else cap
            ice = np.zeros(max(c, 1), np.int32); jce = np.zeros(max(c, 1), np.int32)
            nce = ctypes.c_int()
            if full:
                comp = np.empty(max(n, 1), np.int32)
                work = np.empty(max(L.orc_resolve_work_doubles(n), 1))
                bsf, ng = ctypes.c_int(), ctypes.c_int()
                nfail += L.orc_step_full(n, int(self.nbig[s]), p.G, float(self.m0[s]), p.n_hill, p.inner, _ptr(m), _ptr(Q),
                                         _ptr(V), _ptr(A), _ptr(rc), float(tau), int(p.drag), p.sigma0, p.h,
                                         p.cd, p.rho_p, float(tol), _ptr(Q0), _ptr(V0), _ptr(kf),
                                         _ptr(scratch), int(c), _ptr(ice), _ptr(jce), _ptr(ce),
                                         ctypes.byref(nce), _ptr(comp), _ptr(work), ctypes.byref(bsf),
                                         ctypes.byref(ng))
                g = comp[:n].astype(np.int64)
                self.groups[a:b] = np.where(g >= 0, g + a, -1)
                self.ngroups += ng.value
            else:
                nfail += L.orc_step(n, int(self.nbig[s]), p.G, float(self.m0[s]), p.n_hill, p.inner, _ptr(m), _ptr(Q), _ptr(V),
                                    _ptr(A), _ptr(rc), float(tau), int(p.drag), p.sigma0, p.h, p.cd, p.rho_p,
                                    _ptr(Q0), _ptr(V0), _ptr(kf), _ptr(scratch), int(c), _ptr(ice), _ptr(jce),
                                    _ptr(ce), ctypes.byref(nce))
            self.Q[a:b] = Q; self.V[a:b] = V; self.a[a:b] = A; self.rc[a:b] = rc
            self.Q0[a:b] = Q0; self.V0[a:b] = V0; self.kflag[a:b] = kf; self.ce[a:b] = ce[:n]
            k = min(nce.value, c)
            self.enc.append((nce.value, ice[:k] + a, jce[:k] + a))
        return nfail

    def events(self, tau, rho, r_star, r_eject=0.0):
        """Star impacts, collisions and ejections after the last step (its
        drift arcs and flagged pairs), applied to every system in place
        (Sec. 2.1.1-2.1.2).  Sets self.lost (per body) and returns the summed
        counts (star impacts, colliding pairs, bodies merged away, ejections)."""
        self.lost = np.zeros(len(self.m), np.int32)
        tot = np.zeros(4, np.int64)
        for s, (a, b) in enumerate(self.systems()):
            if b == a:
                continue
            # the step's drift arc, recomputed by the same routine from its start
            q1, v1, _ = drift(self.prm.G * self.m0[s], tau, self.Q0[a:b], self.V0[a:b])
            nce, ii, jj = self.enc[s]
            m0, m, Q, V, lost, ev = events(self.prm.G, self.m0[s], self.m[a:b], self.Q[a:b], self.V[a:b],
                                           self.Q0[a:b], self.V0[a:b], q1, v1, tau, ii - a, jj - a, rho,
                                           r_star, r_eject)
            self.m0[s] = m0; self.m[a:b] = m; self.Q[a:b] = Q; self.V[a:b] = V; self.lost[a:b] = lost
            tot += ev
        return tuple(int(t) for t in tot)

    def compacted(self):
        """A new state without the lost bodies (mxx_elim), its critical radii
        and force computed again (mce_init).  Returns (state, old index of every
        kept body)."""
        off = [0]
        ms, Qs, Vs, idx, nbig = [], [], [], [], []
        for s, (a, b) in enumerate(self.systems()):
            mk, Qk, Vk, ik = compact(self.lost[a:b], self.m[a:b], self.Q[a:b], self.V[a:b])
            ms.append(mk); Qs.append(Qk); Vs.append(Vk); idx.append(ik + a)
            off.append(off[-1] + len(mk))
            # big bodies stay first: the kept ones among the first nbig
            nbig.append(int(np.sum(ik < self.nbig[s])))
        cat = lambda xs, shape: np.concatenate(xs) if xs else np.zeros(shape)  # noqa: E731
        st = State(np.array(off), self.m0, cat(ms, 0), cat(Qs, (0, 3)), cat(Vs, (0, 3)), self.prm, frame="dh",
                   nbig=nbig, threads=self.threads)
        return st, cat(idx, 0).astype(np.int64)

    def energy(self):
        p = self.prm
        out = []
        for s, (a, b) in enumerate(self.systems()):
            out.append(energy(p.G, self.m0[s], self.m[a:b], self.Q[a:b], self.V[a:b], self.rc[a:b], p.inner))
        return out

    def helio(self):
        xh = np.empty_like(self.Q); vh = np.empty_like(self.V)
        for s, (a, b) in enumerate(self.systems()):
            xh[a:b], vh[a:b] = dh_to_helio(self.m0[s], self.m[a:b], self.Q[a:b], self.V[a:b])
        return xh, vh
