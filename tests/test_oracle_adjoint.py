"""Pins of the oracle's adjoint: exact transposes (dot-product tests) and
complex-step directional derivatives of the filtered RK loop (CPU only)."""
import numpy as np
import pytest

from oracle import labfm_oracle as O
from paper_2102_02019_amd import inputs


@pytest.fixture(scope="module")
def small():
    nodes = inputs.jittered_lattice(20, seed=5, m=4)
    rp, col = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
    W = O.weights_batched(nodes.x, nodes.y, nodes.h, nodes.s, 4, rp, col, nodes.box)
    W.update(row_ptr=rp, col=col)
    prm = inputs.taylor_green_params()
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y)
    l = np.log(rho) + 0.03 * np.sin(nodes.x - nodes.y)
    return nodes, W, prm, (l, u, v)


def test_operator_matrices_apply_the_operator(small):
    nodes, W, _, (l, u, v) = small
    mats = O.operator_matrices(W)
    for d in range(6):
        np.testing.assert_allclose(mats[d] @ u, O.apply_op(W["row_ptr"], W["col"], W["w"][d], u),
                                   rtol=1e-10, atol=1e-10 * np.abs(mats[d] @ u).max())


def test_rhs_vjp_matches_complex_step(small):
    """<Rbar, J_R d> by complex step equals <J_R^T Rbar, d>."""
    nodes, W, prm, q = small
    rng = np.random.default_rng(0)
    d = tuple(rng.standard_normal(nodes.n) for _ in range(3))
    rbar = tuple(rng.standard_normal(nodes.n) for _ in range(3))
    h = 1e-30
    qc = tuple(a + 1j * h * b for a, b in zip(q, d))
    R = O.ns_rhs(*qc, W, prm)
    lhs = sum(np.dot(rb, r.imag / h) for rb, r in zip(rbar, R))
    qb = O.ns_rhs_vjp(*q, W, prm, rbar)
    rhs = sum(np.dot(a, b) for a, b in zip(qb, d))
    assert lhs == pytest.approx(rhs, rel=1e-11)


@pytest.mark.parametrize("filt", [True, False])
def test_rk_adjoint_matches_complex_step(small, filt):
    nodes, W, prm, q = small
    dt = 0.5 * O.time_step(nodes.s, *q, prm)
    n_steps = 3
    rng = np.random.default_rng(1)
    qbar = tuple(rng.standard_normal(nodes.n) for _ in range(3))
    g = O.rk_adjoint(*q, W, prm, dt, n_steps, qbar, filt=filt)
    for trial in range(3):
        d = tuple(rng.standard_normal(nodes.n) for _ in range(3))
        h = 1e-30
        qc = tuple(a + 1j * h * b for a, b in zip(q, d))
        out = O.rk_run(*qc, W, prm, dt, n_steps, filt=filt)
        lhs = sum(np.dot(qb, o.imag / h) for qb, o in zip(qbar, out))
        rhs = sum(np.dot(a, b) for a, b in zip(g, d))
        assert lhs == pytest.approx(rhs, rel=1e-10)


def test_rk_adjoint_zero_for_zero_seed(small):
    nodes, W, prm, q = small
    z = tuple(np.zeros(nodes.n) for _ in range(3))
    g = O.rk_adjoint(*q, W, prm, 0.01, 2, z)
    assert all(np.all(a == 0) for a in g)
