"""Pins of the Lagrangian oracle: a uniform stream translates the node set
rigidly and leaves the fields untouched; the material rates are the Eulerian
right-hand side plus the convective terms; a Lagrangian Taylor-Green run
follows the analytic decay at the moved positions as closely as the Eulerian
run does at fixed ones. CPU only."""
import math

import numpy as np
import pytest

from oracle import labfm_oracle as O
from oracle import lagrangian_oracle as G
from paper_2102_02019_amd import inputs


def test_uniform_stream_translates_the_nodes():
    nodes = inputs.jittered_lattice(16, L=1.0, seed=4, m=4)
    n = nodes.n
    U, V = 0.3, -0.2
    prm = inputs.FlowParams(c2=25.0, mu=0.01)
    dt, steps = 0.01, 5
    x, y, l, u, v = G.lagrangian_run(nodes.x, nodes.y, np.zeros(n), np.full(n, U), np.full(n, V),
                                     nodes.h, nodes.s, nodes.m, nodes.box, prm, dt, steps)
    t = dt * steps
    dx = O.min_image(x - np.mod(nodes.x + U * t, 1.0), 1.0, True)
    dy = O.min_image(y - np.mod(nodes.y + V * t, 1.0), 1.0, True)
    assert np.max(np.abs(dx)) < 1e-14 and np.max(np.abs(dy)) < 1e-14
    assert np.all(u == U) and np.all(v == V) and np.all(l == 0.0)
    assert np.all((x >= 0) & (x < 1.0) & (y >= 0) & (y < 1.0))


def test_material_rates_are_eulerian_rates_plus_convection():
    """D phi/Dt = d phi/dt + u . grad phi with the same operators."""
    nodes = inputs.jittered_lattice(20, L=2.0 * math.pi, seed=6, m=6)
    W = G.weights_at(nodes.x, nodes.y, nodes.h, nodes.s, nodes.m, nodes.box)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y)
    pl, pu, pv = inputs.fourier_perturbation(nodes.x, nodes.y, seed=2, amp=0.05)
    l, u, v = np.log(rho) + pl, u + pu, v + pv
    prm = inputs.FlowParams(c2=100.0, mu=0.03, gx=0.1, gy=-0.2)
    lag = G.lagrangian_rates(l, u, v, W, prm)
    eul = O.ns_rhs(l, u, v, W, prm)
    rp, col, w = W["row_ptr"], W["col"], W["w"]
    for f, rl, re in zip((l, u, v), lag, eul):
        conv = u * O.apply_op(rp, col, w[O.OP_X], f) + v * O.apply_op(rp, col, w[O.OP_Y], f)
        np.testing.assert_allclose(rl, re + conv, atol=1e-10 * np.max(np.abs(re)))


@pytest.mark.slow
def test_lagrangian_taylor_green_tracks_the_analytic_decay():
    """24^2 nodes, m = 6, Re = 100, Ma = 0.1, 8 filtered steps: the velocity at
    the moved nodes against the analytic Taylor-Green field there, next to the
    Eulerian oracle run on the fixed nodes; the nodes have moved by about
    u dt per step."""
    wl = inputs.jittered_lattice(24, seed=8, m=6)
    prm = inputs.taylor_green_params()
    rho, u, v = inputs.taylor_green_state(wl.x, wl.y)
    l = np.log(rho)
    dt = O.time_step(wl.s, l, u, v, prm)
    steps = 8
    x1, y1, l1, u1, v1 = G.lagrangian_run(wl.x, wl.y, l, u, v, wl.h, wl.s, wl.m, wl.box, prm,
                                          dt, steps)
    t = dt * steps
    ua, va = G.taylor_green_decay(x1, y1, t, prm.mu)
    e_lag = math.sqrt(np.sum((u1 - ua) ** 2 + (v1 - va) ** 2) / np.sum(ua ** 2 + va ** 2))
    W = G.weights_at(wl.x, wl.y, wl.h, wl.s, wl.m, wl.box)
    le, ue, ve = O.rk_run(l, u, v, W, prm, dt, steps)
    ub, vb = G.taylor_green_decay(wl.x, wl.y, t, prm.mu)
    e_eul = math.sqrt(np.sum((ue - ub) ** 2 + (ve - vb) ** 2) / np.sum(ub ** 2 + vb ** 2))
    assert e_lag < 3.0 * e_eul + 1e-6, (e_lag, e_eul)
    disp = np.hypot(O.min_image(x1 - wl.x, wl.box.Lx, True), O.min_image(y1 - wl.y, wl.box.Ly, True))
    speed = np.hypot(u, v)
    np.testing.assert_allclose(disp, speed * t, rtol=0.05, atol=0.02 * t)
