"""Seeded synthetic workloads for the hybrid symplectic N-body hot path.

This module only draws initial conditions.  It holds none of the integrator's
arithmetic (no force, drift, transform, encounter or energy code), so the CPU
oracle under ``oracle/`` and the HIP library can both be fed from it without
sharing any of the method.

Units: AU, solar masses, Julian years.  The paper fixes none of the inputs of
its runs (its profiling runs in Sec. 2.1.2 use a star, four giant planets and
1e-2 Earth-mass bodies between 1 and 10 AU, with unpublished initial
conditions), so every workload here is a synthetic stand-in with the sizes and
orbital distributions of the five benchmark configurations:

  c1  star + 100 planetesimals, m log-uniform in [1e-10, 1e-8], a ~ U[1,3],
      e ~ Rayleigh(0.01), i ~ Rayleigh(0.005); dt = 0.05 yr, 1000 steps.
  c2  star + a Jupiter-mass body on a circular orbit at 5.2 AU + 1000 bodies of
      1e-9 with a ~ U[2,10], e ~ Rayleigh(0.02), i ~ Rayleigh(0.01), gas drag;
      dt = 0.1 yr, 1e4 steps.
  c3  star + 16384 equal-mass bodies totalling 10 Earth masses, a ~ U[0.5,5]
      (surface density ~ 1/r), e ~ Rayleigh(0.01), i ~ Rayleigh(0.005);
      dt = 0.0175 yr (about P(0.5 AU)/20) halved until an FP64 run of 1e4
      steps keeps the changeover-weighted energy within 1e-9: three halvings,
      dt = 0.0021875 yr.
  c4  256 independent systems, N_s ~ U{200..4000}, c1 distributions;
      dt = 0.05 yr, 5000 steps.
  c5  star + 131072 bodies of 1e-11 in a 0.9-1.1 AU ring, e ~ Rayleigh(0.005),
      i ~ Rayleigh(0.0025); dt = 0.04 yr, 2000 steps.

Big and small bodies (Sec. 2.1: only big bodies are gravity sources; small
bodies are massless planetesimals; production runs have N_big of 1-100 and
N_small of 1e4-1e6): ``bigsmall`` draws N_big Mars-mass embryos (3.2e-7) and
N_small massless bodies, both with a ~ U[1,5], e ~ Rayleigh(0.01),
i ~ Rayleigh(0.005); dt = 0.05 yr.  The big bodies come first in each system.

Random stream: numpy ``default_rng(SeedSequence(20260119, spawn_key=(cfg, s)))``
per system s; draw order m, a, e, i, Omega, omega, M as length-N vectors.
Elements are converted with mu_i = G (m0 + m_i).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Gaussian gravitational constant k = 0.01720209895 AU^1.5 Msun^-0.5 day^-1;
# in AU^3 Msun^-1 yr^-2 (Julian year = 365.25 d) G = (k * 365.25)^2.
G_AU_MSUN_YR = (0.01720209895 * 365.25) ** 2
M_EARTH = 3.003489e-6      # Msun
M_JUPITER = 9.547919e-4    # Msun
SEED = 20260119

CONFIG_IDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}


@dataclass
class Workload:
    """A batch of independent systems in heliocentric Cartesian coordinates.

    Bodies of system s occupy rows off[s]:off[s+1] of ``m``, ``x`` and ``v``;
    the star of system s has mass ``m0[s]`` and is not stored as a body.
    """
    name: str
    off: np.ndarray          # int32, nsys+1
    m0: np.ndarray           # float64, nsys
    m: np.ndarray            # float64, ntot
    x: np.ndarray            # float64, (ntot, 3) heliocentric positions
    v: np.ndarray            # float64, (ntot, 3) heliocentric velocities
    dt: float
    steps: int
    G: float = G_AU_MSUN_YR
    drag: bool = False
    meta: dict = field(default_factory=dict)
    nbig: np.ndarray | None = None   # per system: the first nbig[s] bodies are big (None: all)

    @property
    def nsys(self) -> int:
        return len(self.m0)

    @property
    def ntot(self) -> int:
        return int(self.off[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.off)

    def pairs(self) -> int:
        """Ordered pair interactions per force evaluation: sum of N_s (N_s - 1),
        or with big bodies only as sources, sum of nbig_s (N_s - 1)."""
        n = self.sizes().astype(np.int64)
        nb = n if self.nbig is None else np.asarray(self.nbig, dtype=np.int64)
        return int(np.sum(nb * np.maximum(n - 1, 0)))


def _rng(cfg_id: int, sys_index: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(SEED, spawn_key=(cfg_id, sys_index)))


def _eccentric_anomaly(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Solve E - e sin E = M for elliptic orbits (vectorised Newton)."""
    E = M + e * np.sin(M)
    for _ in range(60):
        d = (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        E = E - d
        if np.all(np.abs(d) <= 4e-16 * np.maximum(1.0, np.abs(E))):
            break
    return E


def elements_to_cartesian(mu, a, e, inc, node, peri, M):
    """Osculating elliptic elements -> Cartesian position and velocity.

    ``mu`` is G times the sum of the two masses; angles in radians.  Returns
    (x, v) with shape (n, 3).
    """
    mu, a, e, inc, node, peri, M = (np.asarray(t, dtype=np.float64) for t in (mu, a, e, inc, node, peri, M))
    E = _eccentric_anomaly(np.mod(M, 2.0 * np.pi), e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    # perifocal frame
    px = a * (cE - e)
    py = a * b * sE
    nmean = np.sqrt(mu / a ** 3)
    dEdt = nmean / (1.0 - e * cE)
    pvx = -a * sE * dEdt
    pvy = a * b * cE * dEdt
    # rotation R3(node) R1(inc) R3(peri)
    cO, sO = np.cos(node), np.sin(node)
    ci, si = np.cos(inc), np.sin(inc)
    cw, sw = np.cos(peri), np.sin(peri)
    r11 = cO * cw - sO * sw * ci
    r12 = -cO * sw - sO * cw * ci
    r21 = sO * cw + cO * sw * ci
    r22 = -sO * sw + cO * cw * ci
    r31 = sw * si
    r32 = cw * si
    x = np.stack([r11 * px + r12 * py, r21 * px + r22 * py, r31 * px + r32 * py], axis=-1)
    v = np.stack([r11 * pvx + r12 * pvy, r21 * pvx + r22 * pvy, r31 * pvx + r32 * pvy], axis=-1)
    return x, v


def _disk(rng, n, mass, a_lo, a_hi, sig_e, sig_i, m0=1.0, G=G_AU_MSUN_YR):
    """Draw n bodies: masses (callable or scalar), then a, e, i, node, peri, M."""
    m = mass(rng, n) if callable(mass) else np.full(n, float(mass))
    a = rng.uniform(a_lo, a_hi, n)
    e = rng.rayleigh(sig_e, n)
    inc = rng.rayleigh(sig_i, n)
    node = rng.uniform(0.0, 2.0 * np.pi, n)
    peri = rng.uniform(0.0, 2.0 * np.pi, n)
    M = rng.uniform(0.0, 2.0 * np.pi, n)
    e = np.minimum(e, 0.9)  # Rayleigh tail guard; never reached at these sigmas
    x, v = elements_to_cartesian(G * (m0 + m), a, e, inc, node, peri, M)
    return m, x, v


def _loguniform(lo, hi):
    return lambda rng, n: 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), n)


def _pack(name, systems, dt, steps, drag=False, meta=None) -> Workload:
    sizes = [len(s[1]) for s in systems]
    off = np.zeros(len(systems) + 1, dtype=np.int32)
    off[1:] = np.cumsum(sizes)
    m0 = np.array([s[0] for s in systems], dtype=np.float64)
    m = np.concatenate([s[1] for s in systems]) if systems else np.zeros(0)
    x = np.concatenate([s[2] for s in systems]) if systems else np.zeros((0, 3))
    v = np.concatenate([s[3] for s in systems]) if systems else np.zeros((0, 3))
    return Workload(name, off, m0, np.ascontiguousarray(m), np.ascontiguousarray(x),
                    np.ascontiguousarray(v), dt, steps, drag=drag, meta=meta or {})


def c1(n: int = 100) -> Workload:
    rng = _rng(1, 0)
    m, x, v = _disk(rng, n, _loguniform(1e-10, 1e-8), 1.0, 3.0, 0.01, 0.005)
    return _pack("c1", [(1.0, m, x, v)], 0.05, 1000)


def c2(n_small: int = 1000) -> Workload:
    rng = _rng(2, 0)
    m, x, v = _disk(rng, n_small, 1e-9, 2.0, 10.0, 0.02, 0.01)
    xj, vj = elements_to_cartesian(G_AU_MSUN_YR * (1.0 + M_JUPITER), [5.2], [0.0], [0.0], [0.0], [0.0], [0.0])
    m = np.concatenate([[M_JUPITER], m])
    x = np.concatenate([xj, x])
    v = np.concatenate([vj, v])
    return _pack("c2", [(1.0, m, x, v)], 0.1, 10000, drag=True)


def c3(n: int = 16384, dt: float = 0.0175 / 8) -> Workload:
    rng = _rng(3, 0)
    m, x, v = _disk(rng, n, 10.0 * M_EARTH / n, 0.5, 5.0, 0.01, 0.005)
    return _pack("c3", [(1.0, m, x, v)], dt, 10000)


def c4(nsys: int = 256, n_lo: int = 200, n_hi: int = 4000) -> Workload:
    sizes = _rng(4, 1 << 20).integers(n_lo, n_hi + 1, nsys)
    systems = []
    for s in range(nsys):
        rng = _rng(4, s)
        m, x, v = _disk(rng, int(sizes[s]), _loguniform(1e-10, 1e-8), 1.0, 3.0, 0.01, 0.005)
        systems.append((1.0, m, x, v))
    return _pack("c4", systems, 0.05, 5000)


def c5(n: int = 131072) -> Workload:
    rng = _rng(5, 0)
    m, x, v = _disk(rng, n, 1e-11, 0.9, 1.1, 0.005, 0.0025)
    return _pack("c5", [(1.0, m, x, v)], 0.04, 2000)


def batch(sizes, cfg_id: int = 6, a_lo=1.0, a_hi=3.0) -> Workload:
    """A batch of independent c1-like systems of the given sizes (tests)."""
    systems = []
    for s, n in enumerate(sizes):
        rng = _rng(cfg_id, s)
        m, x, v = _disk(rng, int(n), _loguniform(1e-10, 1e-8), a_lo, a_hi, 0.01, 0.005)
        systems.append((1.0, m, x, v))
    return _pack(f"batch{list(sizes)}", systems, 0.05, 10)


M_MARS = 3.227151e-7       # Msun


def bigsmall(n_big: int = 100, n_small: int = 1 << 20, nsys: int = 1, cfg_id: int = 9,
             a_lo: float = 1.0, a_hi: float = 5.0, m_big: float = M_MARS) -> Workload:
    """Big embryos plus massless small bodies (nsys identical-size systems)."""
    systems, nbig = [], []
    for s in range(nsys):
        rng = _rng(cfg_id, s)
        mb, xb, vb = _disk(rng, n_big, m_big, a_lo, a_hi, 0.01, 0.005)
        ms, xs, vs = _disk(rng, n_small, 0.0, a_lo, a_hi, 0.01, 0.005)
        systems.append((1.0, np.concatenate([mb, ms]), np.concatenate([xb, xs]), np.concatenate([vb, vs])))
        nbig.append(n_big)
    w = _pack(f"bigsmall{n_big}x{n_small}", systems, 0.05, 1000)
    w.nbig = np.array(nbig, dtype=np.int32)
    return w


def ring(n: int, seed_sys: int = 0, m: float = 1e-11, a_lo=0.9, a_hi=1.1) -> Workload:
    """A c5-like dense ring of any size (encounter-rich tests)."""
    rng = _rng(5, 1000 + seed_sys)
    mm, x, v = _disk(rng, n, m, a_lo, a_hi, 0.005, 0.0025)
    return _pack(f"ring{n}", [(1.0, mm, x, v)], 0.04, 10)


def by_name(name: str) -> Workload:
    return {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5, "bigsmall": bigsmall}[name]()
