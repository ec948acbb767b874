"""Oracle with points that move between backward-Euler steps (the per-step re-integration of Sec. 1).

The per-point coefficients stay with the points while cells, functions and
blocks are rebuilt each step.  On the manufactured solution the scalar-flux
error then stays at the level of the fixed-point run (the coefficients only
move by the flow times the step), and a flow that vanishes reproduces the
fixed-point run exactly.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _run(n, amplitude, steps=4, dt=0.02, M=8):
    w = W.config(8, n)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    om, wq = oracle.angular_quadrature(2, M)
    psi = W.mms_sin_psi(x, om, 0.0)
    phi = psi @ wq
    for s in range(1, steps + 1):
        x = x + dt * W.cellular_flow(x, amplitude)
        g = oracle.geometry(x, R, w.lo, w.hi)
        it = oracle.integrate(g, 1)
        tr = oracle.Transport(it, om, wq, 1.0, 0.5, 1.0 / dt, dx)
        psi, phi, _ = tr.step(psi, W.mms_sin_source(x, om, s * dt, 1.0, 0.5), None, phi)
    pv = tr.point_values(phi)
    ex = W.mms_sin_phi(x, steps * dt)
    return np.abs(pv - ex).sum() / ex.sum(), psi


def test_cellular_flow_keeps_points_inside_and_is_divergence_free():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (2000, 2))
    u = W.cellular_flow(x, 0.7)
    h = 1e-6
    div = ((W.cellular_flow(x + [h, 0], 0.7)[:, 0] - W.cellular_flow(x - [h, 0], 0.7)[:, 0]) +
           (W.cellular_flow(x + [0, h], 0.7)[:, 1] - W.cellular_flow(x - [0, h], 0.7)[:, 1])) / (2 * h)
    assert np.abs(div).max() <= 1e-8
    edge = np.array([[0.0, 0.3], [1.0, 0.6], [0.4, 0.0], [0.8, 1.0]])
    un = W.cellular_flow(edge, 0.7)
    assert abs(un[0, 0]) + abs(un[1, 0]) + abs(un[2, 1]) + abs(un[3, 1]) <= 1e-15
    assert np.abs(u).max() <= 0.7 + 1e-15


def test_zero_flow_equals_fixed_points():
    """Rebuilding cells and blocks at unchanged positions every step gives the fixed-point run bit for bit."""
    e0, psi0 = _run(8, 0.0)
    w = W.config(8, 8)
    x, dx = W.points_for(w)
    g = oracle.geometry(x, W.radii_for(w, x, dx), w.lo, w.hi)
    it = oracle.integrate(g, 1)
    om, wq = oracle.angular_quadrature(2, 8)
    tr = oracle.Transport(it, om, wq, 1.0, 0.5, 1.0 / 0.02, dx)
    psi = W.mms_sin_psi(x, om, 0.0)
    phi = psi @ wq
    for s in range(1, 5):
        psi, phi, _ = tr.step(psi, W.mms_sin_source(x, om, s * 0.02, 1.0, 0.5), None, phi)
    assert np.array_equal(psi, psi0)


@pytest.mark.slow
def test_moving_points_keep_the_error_level():
    e_fixed, _ = _run(12, 0.0)
    e_moving, _ = _run(12, 0.5)
    assert e_moving <= 1.5 * e_fixed, (e_fixed, e_moving)
