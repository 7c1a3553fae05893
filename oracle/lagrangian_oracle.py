"""FP64 CPU oracle of LABFM in a Lagrangian frame (King & Lind, arXiv
2102.02019, section "Conclusions": node positions advanced by the same time
integration as the flow, which puts the evaluation and solution of every
node's consistency matrix on every time step).

TEST INFRASTRUCTURE ONLY: the product path never imports this module; the
tests, the smoke check and the benchmark's CPU-baseline leg do.

Readings (also listed in the design notes):

* The nodes move with the fluid, dr_i/dt = u_i, and the flow equations are
  eq. icns written for the material derivative, i.e. without the convective
  terms u . grad: D ln rho/Dt = -div u, Du/Dt = -c^2 grad ln rho +
  (mu/rho)(viscous terms) + g.
* The extended state (x, y, ln rho, u, v) is advanced by the same
  RK3(2)4[2R+]C two-register scheme; every stage evaluates its right-hand side
  with stencils and weights built at that stage's positions, so the scheme
  stays the consistent Runge-Kutta method of the extended system.
* The filter after each step uses weights built at the step's final
  positions; the first stage of the next step starts from those positions.
* Positions are folded into the periodic box [0, L) when the right-hand side
  and the filter use them; node spacings s_i, stencil scales h_i and orders
  travel with the nodes unchanged.
"""
from __future__ import annotations

import math

import numpy as np

from . import labfm_oracle as O


def fold(p: np.ndarray, L: float, periodic: bool) -> np.ndarray:
    """Coordinates folded into [0, L) on a periodic axis (one period at most)."""
    if not periodic:
        return p
    return np.where(p >= L, p - L, np.where(p < 0.0, p + L, p))


def weights_at(x, y, h, s, m, box) -> dict:
    """Stencils and operator weights of the nodes at positions (x, y)."""
    xf, yf = fold(x, box.Lx, box.periodic_x), fold(y, box.Ly, box.periodic_y)
    rp, col = O.neighbours(xf, yf, h, box)
    mm = np.broadcast_to(np.asarray(m), (xf.size,))
    if np.all(mm == mm[0]):
        W = O.weights_batched(xf, yf, h, s, int(mm[0]), rp, col, box)
    else:
        W = O.weights(xf, yf, h, s, mm, rp, col, box)
    W.update(row_ptr=rp, col=col)
    return W


def lagrangian_rates(lnrho, u, v, W: dict, prm) -> tuple:
    """Material rates of (ln rho, u, v): eq. icns without u . grad."""
    rp, col, w = W["row_ptr"], W["col"], W["w"]

    def L(d, f):
        return O.apply_op(rp, col, w[d], f)

    lx, ly = L(O.OP_X, lnrho), L(O.OP_Y, lnrho)
    ux, uy, uL, uxx, uxy = (L(d, u) for d in (O.OP_X, O.OP_Y, O.OP_L, O.OP_XX, O.OP_XY))
    vx, vy, vL, vxx, vxy = (L(d, v) for d in (O.OP_X, O.OP_Y, O.OP_L, O.OP_XX, O.OP_XY))
    nu = prm.mu / np.exp(lnrho)
    r_l = -(ux + vy)
    r_u = -prm.c2 * lx + nu * (4.0 / 3.0 * uxx + (uL - uxx) + 1.0 / 3.0 * vxy) + prm.gx
    r_v = -prm.c2 * ly + nu * (4.0 / 3.0 * (vL - vxx) + vxx + 1.0 / 3.0 * uxy) + prm.gy
    return r_l, r_u, r_v


def lagrangian_rhs(x, y, lnrho, u, v, h, s, m, box, prm) -> tuple:
    """Right-hand side of the extended system (dx/dt, dy/dt, Dln rho/Dt,
    Du/Dt, Dv/Dt) with weights built at (x, y)."""
    W = weights_at(x, y, h, s, m, box)
    r_l, r_u, r_v = lagrangian_rates(lnrho, u, v, W, prm)
    return u.copy(), v.copy(), r_l, r_u, r_v


def lagrangian_run(x, y, lnrho, u, v, h, s, m, box, prm, dt: float, n_steps: int,
                   filt: bool = True) -> tuple:
    """n_steps RK steps of the extended system, each followed by the filter
    (weights at the new positions) on ln rho, u and v. Returns
    (x, y, ln rho, u, v) with positions folded into the box."""
    def rhs(x_, y_, l_, u_, v_):
        return lagrangian_rhs(x_, y_, l_, u_, v_, h, s, m, box, prm)

    def post(q):
        xf = fold(q[0], box.Lx, box.periodic_x)
        yf = fold(q[1], box.Ly, box.periodic_y)
        if not filt:
            return (xf, yf) + tuple(q[2:])
        W = weights_at(xf, yf, h, s, m, box)
        return (xf, yf) + O.filter_fields(tuple(q[2:]), W)

    return O.rk_integrate((x, y, lnrho, u, v), rhs, dt, n_steps, post)


def taylor_green_decay(x, y, t: float, nu: float, L: float = 2.0 * math.pi) -> tuple:
    """Incompressible Taylor-Green velocity at (x, y) and time t:
    u = sin(kx) cos(ky) e^{-2 nu k^2 t}, v = -cos(kx) sin(ky) e^{-2 nu k^2 t}."""
    k = 2.0 * math.pi / L
    f = math.exp(-2.0 * nu * k * k * t)
    return np.sin(k * x) * np.cos(k * y) * f, -np.cos(k * x) * np.sin(k * y) * f
