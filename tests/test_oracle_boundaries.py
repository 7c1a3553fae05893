"""Pins of the boundary oracle (section "Boundaries", Appendix A, section
"Poiseuille flow"): finite-difference weights against their closed forms, 1D
LABFM against the finite differences it reduces to and the library Hermite
polynomials, the strip operators' polynomial exactness, the wall equation
against its closed form on smooth fields, the analytic start-up solution
against its PDE, and the Poiseuille convergence of the whole scheme. CPU only."""
import math

import numpy as np
import pytest

from oracle import boundaries_oracle as B
from oracle import labfm_oracle as O
from paper_2102_02019_amd import inputs


# ---------------------------------------------------------------------------
# finite differences along the strip columns
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("offsets,expected", [
    # one-sided, asymmetric and centred 5-point first differences (x 12)
    ((0, 1, 2, 3, 4), (-25, 48, -36, 16, -3)),
    ((-1, 0, 1, 2, 3), (-3, -10, 18, -6, 1)),
    ((-2, -1, 0, 1, 2), (1, -8, 0, 8, -1)),
])
def test_first_differences_match_the_textbook_coefficients(offsets, expected):
    w = B.fd_weights(offsets, 1)
    np.testing.assert_allclose(w * 12.0, expected, rtol=0, atol=1e-12)


def test_fourth_difference_is_the_binomial_stencil():
    np.testing.assert_allclose(B.fd_weights(range(5), 4), (1, -4, 6, -4, 1), atol=1e-11)


def test_fd_weights_exact_on_quartics_at_uneven_offsets():
    o = np.array([-1.3, -0.2, 0.0, 0.7, 2.1])
    for deriv in (1, 2):
        w = B.fd_weights(o, deriv)
        for k in range(5):
            exact = math.factorial(k) / math.factorial(k - deriv) * 0.0 ** (k - deriv) \
                if k >= deriv else 0.0
            assert abs(np.sum(w * o ** k) - exact) < 1e-12


def test_one_sided_fourth_difference_has_the_wrong_sign_at_the_filter_wavenumber():
    """Why the wall filter is tangential only: at k s = 2 pi / 3 the one-sided
    fourth difference responds with +4.5 / s^4 (exactly: phi = 0, 3/2, 3/2, 0,
    3/2), the derivative itself with -(2 pi/3)^4 / s^4."""
    r = B.one_sided_fourth_difference_response(2.0 * math.pi / 3.0)
    assert abs(r - 4.5) < 1e-12
    assert -(2.0 * math.pi / 3.0) ** 4 < 0.0


# ---------------------------------------------------------------------------
# Appendix A: one-dimensional LABFM
# ---------------------------------------------------------------------------

def test_1d_abfs_are_wendland_times_probabilists_hermite():
    """psi(|z|) H_q(z/sqrt2)/sqrt(2^q) = psi(|z|) He_q(z) (numpy's HermiteE)."""
    from numpy.polynomial import hermite_e

    z = np.linspace(-1.9, 1.9, 23)
    W = B.hermite_abfs_1d(z, 6)
    psi = O.wendland_c2(np.abs(z))
    for q in range(1, 7):
        c = np.zeros(q + 1)
        c[q] = 1.0
        np.testing.assert_allclose(W[:, q - 1], psi * hermite_e.hermeval(z, c), atol=1e-12)


def test_1d_labfm_with_m_neighbours_is_the_finite_difference():
    """With exactly m points the m moment conditions fix the weights, whatever
    the basis functions: 1D LABFM then equals the finite difference on those
    points plus the node itself."""
    eta = np.array([-0.11, -0.052, 0.047, 0.1])  # 4 neighbours, m = 4
    h = 0.06
    w1, w2 = B.labfm_1d_weights(eta, h, 4, derivs=(1, 2))
    pts = np.concatenate([[0.0], eta])
    for w, d in ((w1, 1), (w2, 2)):
        fd = B.fd_weights(pts, d)
        np.testing.assert_allclose(w, fd[1:], rtol=1e-9)


def test_1d_labfm_on_a_symmetric_row():
    """A symmetric row gives odd first-derivative and even fourth-derivative
    weights, exact on quartics and convergent on a sine."""
    s = 0.01
    eta = np.array([-4, -3, -2, -1, 1, 2, 3, 4], dtype=float) * s
    w1, w4 = B.labfm_1d_weights(eta, 2.1 * s, 4, derivs=(1, 4))
    np.testing.assert_allclose(w1, -w1[::-1], rtol=1e-10)
    np.testing.assert_allclose(w4, w4[::-1], rtol=1e-10)
    for k in range(1, 5):
        assert abs(np.sum(w1 * eta ** k) - (1.0 if k == 1 else 0.0)) < 1e-9
        assert abs(np.sum(w4 * eta ** k) - (24.0 if k == 4 else 0.0)) < 1e-6 * 24
    errs = []
    for s in (0.02, 0.01):
        eta = np.array([-4, -3, -2, -1, 1, 2, 3, 4], dtype=float) * s
        w1 = B.labfm_1d_weights(eta, 2.1 * s, 4)[0]
        errs.append(abs(np.sum(w1 * (np.sin(0.3 + eta) - np.sin(0.3))) - math.cos(0.3)))
    assert errs[1] < errs[0] / 12.0  # fourth order: the ratio is 2^4


# ---------------------------------------------------------------------------
# strip operators
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def open_channel():
    """A 24-wide channel cut open in x, so that polynomials are admissible
    fields; the strip columns in the middle have whole stencils."""
    nodes, strips = inputs.channel(24, seed=11)
    box = inputs.Box(nodes.box.Lx, nodes.box.Ly, False, False)
    nodes = inputs.NodeSet(nodes.x, nodes.y, nodes.s, nodes.h, nodes.m, box, nodes.meta)
    W = B.channel_weights(nodes, strips)
    return nodes, strips, W


def test_strip_operators_exact_on_quartics(open_channel):
    nodes, strips, W = open_channel
    x, y = nodes.x, nodes.y
    mid = np.abs(x[strips.column[:, 0]] - 0.5) < 0.2
    cols = strips.column[mid]
    rp, col, w = W["row_ptr"], W["col"], W["w"]
    worst = 0.0
    for a in range(5):
        for b in range(5 - a):
            f = (x - 0.5) ** a * (y - 0.5) ** b
            fx = a * (x - 0.5) ** max(a - 1, 0) * (y - 0.5) ** b if a else 0.0 * x
            fy = b * (x - 0.5) ** a * (y - 0.5) ** max(b - 1, 0) if b else 0.0 * x
            for q in range(3):
                i = cols[:, q]
                gx = O.apply_op(rp, col, w[O.OP_X], f)[i]
                gy = O.apply_op(rp, col, w[O.OP_Y], f)[i]
                worst = max(worst, np.max(np.abs(gx - fx[i])), np.max(np.abs(gy - fy[i])))
    assert worst < 1e-9


def test_strip_rows_and_columns_carry_the_weights(open_channel):
    """d/dy at a strip node uses only its column, d/dx only its strip row; a
    wall node has no second-derivative weights and a tangential filter."""
    nodes, strips, W = open_channel
    rp, col, w = W["row_ptr"], W["col"], W["w"]
    k = int(np.nonzero(np.abs(nodes.x[strips.column[:, 0]] - 0.5) < 0.05)[0][0])
    for q in range(3):
        i = strips.column[k, q]
        c = col[rp[i]:rp[i + 1]]
        on_col = np.isin(c, strips.column[k])
        same_row = np.abs(nodes.y[c] - nodes.y[i]) < 1e-12
        assert np.all(w[O.OP_Y, rp[i]:rp[i + 1]][~on_col] == 0.0)
        assert np.all(w[O.OP_X, rp[i]:rp[i + 1]][~same_row] == 0.0)
        assert np.count_nonzero(w[O.OP_Y, rp[i]:rp[i + 1]]) == 4  # the other column nodes
    i0 = strips.column[k, 0]
    for d in (O.OP_L, O.OP_XX, O.OP_XY):
        assert np.all(w[d, rp[i0]:rp[i0 + 1]] == 0.0)
    c = col[rp[i0]:rp[i0 + 1]]
    assert np.all(w[O.OP_HYP, rp[i0]:rp[i0 + 1]][nodes.y[c] != nodes.y[i0]] == 0.0)
    assert W["kappa"][i0] < 0.0  # a damping filter for the fourth derivative
    assert np.all(W["status"] == O.STATUS_OK)
    assert np.array_equal(np.nonzero(np.any(W["wall_normal"] != 0, axis=1))[0],
                          np.sort(strips.column[:, 0]))


# ---------------------------------------------------------------------------
# the wall equation (eq. lodilnro)
# ---------------------------------------------------------------------------

def test_wall_equation_matches_its_closed_form():
    """On smooth fields with u = v = 0 on both walls, the oracle's wall rate
    is c dl/dxi - d u_xi/dxi - 2 g.n/c, i.e. c l_y - v_y - 2 g_y/c on the
    bottom wall (n = +y) and -c l_y - v_y + 2 g_y/c on the top wall (n = -y),
    to the accuracy of the 5-point differences."""
    nodes, strips = inputs.channel(40, seed=5)
    W = B.channel_weights(nodes, strips)
    x, y = nodes.x, nodes.y
    tp = 2.0 * math.pi
    lnrho = 0.01 * np.cos(tp * x) * (1.0 + y + y * y)
    u = np.sin(tp * x) * y * (1.0 - y)
    v = np.cos(tp * x) * y * y * (1.0 - y) ** 2 + 0.3 * y * (1.0 - y)
    ly = 0.01 * np.cos(tp * x) * (1.0 + 2.0 * y)
    vy = np.cos(tp * x) * (2 * y * (1 - y) ** 2 - 2 * y * y * (1 - y)) + 0.3 * (1.0 - 2.0 * y)
    flow = inputs.FlowParams(c2=400.0, mu=0.1, gx=0.8, gy=-0.5)
    r_l, r_u, r_v = B.channel_rhs(lnrho, u, v, W, flow)
    c = 20.0
    bot, top = strips.column[strips.normal[:, 1] > 0, 0], strips.column[strips.normal[:, 1] < 0, 0]
    np.testing.assert_allclose(r_l[bot], c * ly[bot] - vy[bot] - 2 * flow.gy / c, atol=2e-4)
    np.testing.assert_allclose(r_l[top], -c * ly[top] - vy[top] + 2 * flow.gy / c, atol=2e-4)
    assert np.all(r_u[bot] == 0.0) and np.all(r_v[top] == 0.0)


def test_fluid_at_rest_stays_at_rest():
    nodes, strips = inputs.channel(16, seed=2)
    W = B.channel_weights(nodes, strips)
    z = np.zeros(nodes.n)
    flow = inputs.FlowParams(c2=400.0, mu=0.1)
    for r in B.channel_rhs(z + 0.25, z, z, W, flow):
        assert np.max(np.abs(r)) < 1e-10


# ---------------------------------------------------------------------------
# section "Poiseuille flow"
# ---------------------------------------------------------------------------

def test_startup_solution_solves_its_problem():
    """u_t = nu u_yy + g with u = 0 on the walls, from rest: checked by
    centred differences in t and y; u -> g y (H - y)/(2 nu); early on the
    core accelerates uniformly, u ~ g t."""
    H, nu, g = 1.0, 0.1, 0.8
    y = np.linspace(0.05, 0.95, 19)
    t, dt, dy = 0.7, 1e-4, 1e-3
    u = lambda yy, tt: B.poiseuille_startup(yy, tt, H, nu, g)  # noqa: E731
    ut = (u(y, t + dt) - u(y, t - dt)) / (2 * dt)
    uyy = (u(y + dy, t) - 2 * u(y, t) + u(y - dy, t)) / dy ** 2
    np.testing.assert_allclose(ut, nu * uyy + g, atol=1e-5)
    assert np.max(np.abs(u(np.array([0.0, H]), t))) < 1e-12
    np.testing.assert_allclose(u(y, 200.0), g * y * (H - y) / (2 * nu), rtol=1e-12)
    assert abs(u(np.array([0.5]), 1e-3)[0] - g * 1e-3) < 1e-6


def test_startup_series_agrees_with_the_benchmark_copy():
    """The benchmark keeps its own coding of the same series (the product
    package never calls the oracle); the two agree to rounding."""
    y = np.linspace(0.0, 1.0, 41)
    for t in (0.0, 0.05, 1.0, 30.0):
        a = B.poiseuille_startup(y, t, 1.0, 0.1, 0.8)
        b = inputs.poiseuille_startup(y, t, 1.0, 0.1, 0.8)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * 0.8 / (8 * 0.1))


@pytest.mark.slow
def test_poiseuille_converges_at_fourth_order():
    """Start-up to t* = 1 at Re = 10, Ma = 0.05 (the paper's case): the
    velocity error against the analytic solution falls at about fourth order
    (the paper reports ~4) between s = H/12 and H/20."""
    P = inputs.POISEUILLE
    flow = P.flow()
    errs = []
    for nx in (12, 20):
        nodes, strips = inputs.channel(nx)
        W = B.channel_weights(nodes, strips)
        dt, n = B.poiseuille_steps(nodes, P, flow, 1.0)
        z = np.zeros(nodes.n)
        _, u, v = B.channel_run(z, z, z, W, flow, dt, n)
        ua = B.poiseuille_startup(nodes.y, P.time(1.0), P.H, P.mu / P.rho0, P.gx)
        errs.append(B.velocity_error(u, v, ua))
    rate = math.log(errs[0] / errs[1]) / math.log(20 / 12)
    assert errs[1] < 5e-4
    assert 3.5 < rate < 6.5, (errs, rate)


def test_wall_equation_on_a_curved_wall():
    """On the cylinder (normals in every direction, g.n != 0) with u = v = 0
    on the wall, the oracle's wall rate is c n.grad(ln rho) - d u_xi/dxi
    - 2 g.n / c, with u_xi's normal derivative known in closed form, to the
    accuracy of the 5-point differences."""
    nodes, strips = inputs.cylinder(96, seed=4)
    W = B.channel_weights(nodes, strips)
    tp = 2.0 * math.pi
    x, y = nodes.x, nodes.y
    r = np.hypot(x - 0.5, y - 0.5)
    l = 0.01 * np.cos(tp * x) * np.sin(tp * y)
    u = 0.5 * (r - 0.2) * np.sin(tp * y)
    v = 0.5 * (r - 0.2) * np.cos(tp * x)
    wall = strips.column[:, 0]
    u[wall] = 0.0
    v[wall] = 0.0
    flow = inputs.FlowParams(c2=400.0, mu=0.05, gx=0.3, gy=0.1)
    r_l, r_u, r_v = B.channel_rhs(l, u, v, W, flow)
    nx_, ny_ = strips.normal[:, 0], strips.normal[:, 1]
    xw, yw = x[wall], y[wall]
    lx = -0.01 * tp * np.sin(tp * xw) * np.sin(tp * yw)
    ly = 0.01 * tp * np.cos(tp * xw) * np.cos(tp * yw)
    duxi = 0.5 * (nx_ * np.sin(tp * yw) + ny_ * np.cos(tp * xw))
    gn = flow.gx * nx_ + flow.gy * ny_
    expect = 20.0 * (nx_ * lx + ny_ * ly) - duxi - 2.0 * gn / 20.0
    np.testing.assert_allclose(r_l[wall], expect, atol=2e-3 * np.max(np.abs(expect)))
    assert np.all(r_u[wall] == 0.0) and np.all(r_v[wall] == 0.0)
