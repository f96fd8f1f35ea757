"""Checks of the oracle's gas-drag term.

PARITY UNPINNED BY THE PAPER: Sec. 2.1 says aerodynamic drag acts on every
body and Sec. 3.1 computes it per body in the force block, but the disk model
is in a companion paper that is not available.  These tests only pin limits
and geometric facts of the quadratic-drag formula chosen here: no gas, no drag;
drag opposes the velocity relative to the gas; the magnitude for a circular
coplanar orbit; energy decreases.
"""
import math

import numpy as np

import workloads

G = workloads.G_AU_MSUN_YR


def test_no_gas_no_drag(orc):
    w = workloads.c2(50)
    prm = orc.Params(G=G, drag=True, sigma0=0.0)
    Q, V = orc.helio_to_dh(1.0, w.m, w.x, w.v)
    assert np.all(orc.drag_accel(G, 1.0, w.m, Q, V, prm) == 0.0)


def test_circular_coplanar_orbit(orc):
    """A body on a circular Keplerian orbit in the midplane moves faster than the
    pressure-supported gas by (1 - sqrt(1 - 3 h^2)) v_K: the drag points along
    -phi_hat with magnitude k dv^2, k = 3 C_D rho_mid / (8 rho_p s)."""
    prm = orc.Params(G=G, drag=True)
    R, m = 3.0, 1e-9
    vk = math.sqrt(G * 1.0 / R)
    x = np.array([[0.0, R, 0.0]])
    v = np.array([[-vk, 0.0, 0.0]])
    Q, V = orc.helio_to_dh(1.0, [m], x, v)
    ad = orc.drag_accel(G, 1.0, [m], Q, V, prm)[0]
    dv = vk * (1 - math.sqrt(1 - 3 * prm.h ** 2))
    rho = prm.sigma0 / R / (math.sqrt(2 * math.pi) * prm.h * R)
    s = (3 * m / (4 * math.pi * prm.rho_p)) ** (1 / 3)
    k = 3 * prm.cd * rho / (8 * prm.rho_p * s)
    assert abs(ad[0] - k * dv * dv) <= 1e-12 * k * dv * dv
    assert abs(ad[1]) <= 1e-12 * k * dv * dv and ad[2] == 0.0


def test_drag_opposes_relative_velocity_and_dissipates(orc):
    w = workloads.c2(200)
    m, x, v = w.m[1:], w.x[1:], w.v[1:]               # planetesimals only
    off = [0, len(m)]
    prm = orc.Params(G=G, drag=True, sigma0=1e-2)   # strong gas to see it quickly
    st = orc.State(off, w.m0, m, x, v, prm)
    E = [st.energy()[0]["E"]]
    for _ in range(20):
        st.step(w.dt)
        E.append(st.energy()[0]["E"])
    prm0 = orc.Params(G=G, drag=False)
    st0 = orc.State(off, w.m0, m, x, v, prm0)
    E0 = [st0.energy()[0]["E"]]
    for _ in range(20):
        st0.step(w.dt)
        E0.append(st0.energy()[0]["E"])
    # with drag the energy falls monotonically, far below the drag-free envelope
    assert np.all(np.diff(E) < 0)
    assert E[-1] < E0[-1] - 100 * abs(max(E0) - min(E0))
