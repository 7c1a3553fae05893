"""FP64 CPU oracle for LABFM's boundary scheme (section "Boundaries" and
Appendix A of King & Lind, arXiv 2102.02019) and the Poiseuille start-up.

TEST INFRASTRUCTURE ONLY: the product path never imports this module; the
tests, the smoke check and the benchmark's CPU-baseline leg do. It shares no
code with the HIP library.

What it computes (table tab:boundaries):

* Strip nodes i0, i1, i2 (levels 0..2 of the 5-node orthogonal strip): the
  boundary-normal derivative d/dxi by 5-point finite differences along the
  strip column (one-sided at i0, asymmetric at i1, centred at i2), the
  tangential derivative d/deta by one-dimensional LABFM along the node's own
  strip row (Appendix A), both turned into d/dx, d/dy by the Jacobian of the
  section (grad = n d/dxi + t d/deta with t = (-n_y, n_x)).
* Second derivatives and the filter operator at i1 and i2 are the
  two-dimensional LABFM operators of order 4 (the weight build of the main
  oracle with m = 4 there); i3, i4 and the bulk use LABFM throughout.
* Wall nodes (i0) of a no-slip wall: u = v = 0 is imposed and ln rho follows
  the characteristic (LODI) form eq. lodilnro with L2 = 0 and the incoming
  wave L4 = L1 + 2 rho c g.n.

Readings of the paper (also listed in the design notes):

* One-dimensional LABFM is solved in the scaled form used for two dimensions
  (monomials (eta/h)^k / k!, target h^-d e_d): the same weights as the
  printed unscaled system, better conditioned.
* A node's strip row B_i is the set of its stencil neighbours on the same
  strip level whose wall normals are within 60 degrees of its own.
* The filter at a wall node is tangential only: kappa L^hyp with L^hyp the
  one-dimensional LABFM d^4/deta^4 along the wall, kappa calibrated by the
  same rule as in the bulk. The one-sided 5-point fourth difference that the
  table's "FD" would add has a response of the wrong sign at the calibration
  wavenumber (``one_sided_fourth_difference_response``), which would make the
  wall filter amplify the normal modes it should damp.
* At wall nodes only ln rho is filtered (the velocity is imposed), and the
  second-derivative slots are zero: neither the imposed velocity nor the
  ln rho wall equation uses them.
* The wall's incoming wave is taken as printed, L4 = L1 + 2 rho c g.n. A fluid
  at rest in hydrostatic balance would need rho c g.n in place of
  2 rho c g.n; the Poiseuille flow has g.n = 0, so no test here can tell
  them apart.
"""
from __future__ import annotations

import math

import numpy as np

from . import labfm_oracle as O

STRIP_DEPTH = 5
TANGENT_ORDER = 4          # order of 1D LABFM along the strip rows
SAME_WALL_COS = 0.5        # B_i: neighbours whose normals are within 60 degrees


# ---------------------------------------------------------------------------
# Finite differences along a strip column
# ---------------------------------------------------------------------------

def fd_weights(offsets, deriv: int) -> np.ndarray:
    """Weights w_q of the P-point finite difference for the deriv-th
    derivative on the points at ``offsets`` (any units): the unique solution
    of sum_q w_q o_q^k / k! = [k == deriv] for k = 0..P-1 (Taylor table)."""
    o = np.asarray(offsets, dtype=np.float64)
    P = o.size
    A = np.array([[oq ** k / math.factorial(k) for oq in o] for k in range(P)])
    b = np.zeros(P)
    b[deriv] = 1.0
    return np.linalg.solve(A, b)


def one_sided_fourth_difference_response(k_s: float) -> float:
    """L(1 - cos(k xi)) at xi = 0 of the one-sided 5-point fourth difference
    on xi = 0, s, .., 4s, in units of 1/s^4, for k s = k_s. The exact fourth
    derivative gives -(k s)^4."""
    w = fd_weights(np.arange(5.0), 4)
    phi = 1.0 - np.cos(k_s * np.arange(5.0))
    return float(np.sum(w * (phi - phi[0])))


# ---------------------------------------------------------------------------
# Appendix A: one-dimensional LABFM
# ---------------------------------------------------------------------------

def hermite_abfs_1d(es: np.ndarray, m: int) -> np.ndarray:
    """W^q = psi(|eta|/h) H_q(eta/(h sqrt2)) / sqrt(2^q), q = 1..m, for the
    scaled offsets es = eta/h. Shape (K, m)."""
    psi = O.wendland_c2(np.abs(es))
    r2 = math.sqrt(2.0)
    return np.stack([psi * O.hermite_phys(q, es / r2) / math.sqrt(2.0 ** q)
                     for q in range(1, m + 1)], axis=-1)


def labfm_1d_weights(eta: np.ndarray, h: float, m: int, derivs=(1,)) -> np.ndarray:
    """Weights w^d_ji = W_ji . Psi^d of 1D LABFM (eq. general_do1d) for each
    derivative order d in ``derivs``, from the offsets eta_ji of B_i.

    M = sum_j H~_ji (outer) W_ji with H~_ji = ((eta/h)^k / k!)_{k=1..m},
    M Psi^d = C~^d with C~^d = h^-d e_d (eq. lsys1d, scaled). Returns
    (len(derivs), K); raises numpy.linalg.LinAlgError when M is singular."""
    es = np.asarray(eta, dtype=np.float64) / h
    Ht = np.stack([es ** k / math.factorial(k) for k in range(1, m + 1)], axis=-1)
    W = hermite_abfs_1d(es, m)
    M = Ht.T @ W
    C = np.zeros((m, len(derivs)))
    for c, d in enumerate(derivs):
        C[d - 1, c] = h ** (-d)
    Psi = np.linalg.solve(M, C)
    return (W @ Psi).T


# ---------------------------------------------------------------------------
# Boundary weights (table tab:boundaries)
# ---------------------------------------------------------------------------

def strip_maps(n: int, strips) -> tuple:
    """Per-node strip level (-1 off the strips), column index and normal."""
    level = np.full(n, -1, dtype=np.int64)
    colidx = np.full(n, -1, dtype=np.int64)
    normal = np.zeros((n, 2))
    for k in range(strips.column.shape[0]):
        for q in range(STRIP_DEPTH):
            i = int(strips.column[k, q])
            level[i] = q
            colidx[i] = k
            normal[i] = strips.normal[k]
    return level, colidx, normal


def boundary_weights(nodes, strips, row_ptr, col, W: dict, columns=None) -> dict:
    """Weights of the strip nodes i0..i2 written over the two-dimensional
    ones in W (a dict with w (6, nnz), kappa, status as from
    labfm_oracle.weights). Returns a new dict; also 'wall_normal' (n, 2),
    the inward normal at wall nodes and zero elsewhere. ``columns`` limits the
    work to those strip columns (their rows must be in the CSR); the strip
    levels of every column still decide the rows B_i."""
    x, y, h, s, box = nodes.x, nodes.y, nodes.h, nodes.s, nodes.box
    n = x.size
    level, colidx, normal = strip_maps(n, strips)
    w = W["w"].copy()
    kappa = W["kappa"].copy()
    status = W["status"].copy()
    wall_normal = np.zeros((n, 2))
    mp = O.filter_power(TANGENT_ORDER)
    for k in (range(strips.column.shape[0]) if columns is None else columns):
        nx_, ny_ = strips.normal[k]
        tx, ty = -ny_, nx_
        column = strips.column[k]
        for q in range(3):
            i = int(column[q])
            a, b = int(row_ptr[i]), int(row_ptr[i + 1])
            c = col[a:b]
            dx, dy = O.stencil_offsets(x, y, box, row_ptr, col, i)
            xi = dx * nx_ + dy * ny_
            eta = dx * tx + dy * ty
            # boundary-normal derivative: 5-point FD along the column
            w_xi = np.zeros(b - a)
            offs = np.zeros(STRIP_DEPTH)
            pos = np.zeros(STRIP_DEPTH, dtype=np.int64)
            for kk in range(STRIP_DEPTH):
                if kk == q:
                    continue
                hit = np.nonzero(c == column[kk])[0]
                if hit.size != 1:
                    raise ValueError(f"strip node {column[kk]} is not in the stencil of {i}")
                pos[kk] = hit[0]
                offs[kk] = xi[hit[0]]
            fd = fd_weights(offs, 1)
            for kk in range(STRIP_DEPTH):
                if kk != q:
                    w_xi[pos[kk]] = fd[kk]
            # tangential derivative: 1D LABFM along the strip row
            row = (level[c] == q) & (normal[c] @ strips.normal[k] > SAME_WALL_COS)
            derivs = (1, mp) if q == 0 else (1,)
            w_eta = np.zeros((len(derivs), b - a))
            st = O.STATUS_OK
            try:
                w_eta[:, row] = labfm_1d_weights(eta[row], float(h[i]), TANGENT_ORDER, derivs)
            except np.linalg.LinAlgError:
                w_eta[:] = np.nan
                st = O.STATUS_SINGULAR
            w[O.OP_X, a:b] = nx_ * w_xi + tx * w_eta[0]
            w[O.OP_Y, a:b] = ny_ * w_xi + ty * w_eta[0]
            if q == 0:
                for d in (O.OP_L, O.OP_XX, O.OP_XY):
                    w[d, a:b] = 0.0
                w[O.OP_HYP, a:b] = w_eta[1]
                kap, fst = O.filter_coefficient(dx, dy, float(s[i]), w_eta[1])
                kappa[i] = kap
                status[i] = st if st != O.STATUS_OK else fst
                wall_normal[i] = (nx_, ny_)
            elif st != O.STATUS_OK:
                status[i] = st
    return {"row_ptr": row_ptr, "col": col, "w": w, "kappa": kappa, "status": status,
            "wall_normal": wall_normal}


def channel_weights(nodes, strips) -> dict:
    """Neighbours, two-dimensional weights at every node's own order and the
    boundary weights of the strips, for a node set with wall strips."""
    rp, col = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
    W = O.weights(nodes.x, nodes.y, nodes.h, nodes.s, nodes.m, rp, col, nodes.box)
    return boundary_weights(nodes, strips, rp, col, W)


# ---------------------------------------------------------------------------
# Equations icns in the bulk and eq. lodilnro on no-slip walls
# ---------------------------------------------------------------------------

def wall_lnrho_rhs(lnrho, u, v, lx, ly, ux, uy, vx, vy, nrm, prm) -> np.ndarray:
    """d(ln rho)/dt at wall nodes from eq. lodilnro: the characteristic
    amplitudes of the normal direction xi (along the inward normal n),
        L1 = (u_xi - c)/2 (dp/dxi - rho c du_xi/dxi),  L2 = 0,
        L4 = L1 + 2 rho c g.n        (no-slip wall),
    and the tangential terms:
        dlnrho/dt = -(c^2 L2 + L4 + L1)/(rho c^2) - u_eta dlnrho/deta - du_eta/deta,
    with p = c^2 rho, so dp/dxi = c^2 rho dlnrho/dxi."""
    c2 = prm.c2
    c = math.sqrt(c2)
    rho = np.exp(lnrho)
    nx_, ny_ = nrm[:, 0], nrm[:, 1]
    tx, ty = -ny_, nx_
    l_xi = nx_ * lx + ny_ * ly
    l_eta = tx * lx + ty * ly
    u_xi = nx_ * u + ny_ * v
    u_eta = tx * u + ty * v
    duxi_dxi = nx_ * (nx_ * ux + ny_ * uy) + ny_ * (nx_ * vx + ny_ * vy)
    dueta_deta = tx * (tx * ux + ty * uy) + ty * (tx * vx + ty * vy)
    dp_dxi = c2 * rho * l_xi
    L1 = 0.5 * (u_xi - c) * (dp_dxi - rho * c * duxi_dxi)
    L2 = 0.0
    L4 = L1 + 2.0 * rho * c * (prm.gx * nx_ + prm.gy * ny_)
    return -(c2 * L2 + L4 + L1) / (rho * c2) - u_eta * l_eta - dueta_deta


def channel_rhs(lnrho, u, v, W: dict, prm) -> tuple:
    """Eq. icns at every node (labfm_oracle.ns_rhs, body force included), with
    the wall nodes' ln rho replaced by eq. lodilnro and their velocity held."""
    r_l, r_u, r_v = O.ns_rhs(lnrho, u, v, W, prm)
    wall = np.nonzero(np.any(W["wall_normal"] != 0.0, axis=1))[0]
    if wall.size:
        rp, col, w = W["row_ptr"], W["col"], W["w"]
        d = {}
        for name, f in (("l", lnrho), ("u", u), ("v", v)):
            d[name + "x"] = O.apply_op(rp, col, w[O.OP_X], f)[wall]
            d[name + "y"] = O.apply_op(rp, col, w[O.OP_Y], f)[wall]
        r_l = r_l.copy()
        r_u = r_u.copy()
        r_v = r_v.copy()
        r_l[wall] = wall_lnrho_rhs(lnrho[wall], u[wall], v[wall], d["lx"], d["ly"], d["ux"],
                                   d["uy"], d["vx"], d["vy"], W["wall_normal"][wall], prm)
        r_u[wall] = 0.0
        r_v[wall] = 0.0
    return r_l, r_u, r_v


def channel_filter(q: tuple, W: dict) -> tuple:
    """The filter of every node; wall nodes keep their (imposed) velocity."""
    l_, u_, v_ = O.filter_fields(q, W)
    wall = np.any(W["wall_normal"] != 0.0, axis=1)
    u_ = np.where(wall, q[1], u_)
    v_ = np.where(wall, q[2], v_)
    return l_, u_, v_


def channel_run(lnrho, u, v, W: dict, prm, dt: float, n_steps: int, filt: bool = True) -> tuple:
    """n_steps filtered RK steps of the channel equations."""
    rhs = lambda l_, u_, v_: channel_rhs(l_, u_, v_, W, prm)  # noqa: E731
    post = (lambda q: channel_filter(q, W)) if filt else None
    return O.rk_integrate((lnrho, u, v), rhs, dt, n_steps, post)


# ---------------------------------------------------------------------------
# Section "Poiseuille flow" (the analytic start-up itself is a reference field
# of the inputs module, pinned in the tests)
# ---------------------------------------------------------------------------

def velocity_error(u, v, u_exact) -> float:
    """Relative L2 norm of the velocity error, sqrt(sum |u - u_a|^2 / sum |u_a|^2)."""
    num = np.sum((u - u_exact) ** 2 + v * v)
    den = np.sum(u_exact * u_exact)
    return float(math.sqrt(num / den))


def poiseuille_steps(nodes, prm, flow, t_star: float, conv_coef: float = 1.0,
                     visc_coef: float = 0.4) -> tuple:
    """(dt, n_steps) reaching t* exactly with dt at most eq. dt's value on the
    state at rest."""
    z = np.zeros(nodes.n)
    dt_max = O.time_step(nodes.s, z, z, z, flow, conv_coef, visc_coef)
    t_end = prm.time(t_star)
    n_steps = max(1, int(math.ceil(t_end / dt_max - 1e-9)))
    return t_end / n_steps, n_steps


# ---------------------------------------------------------------------------
# Section "Poiseuille flow": the analytic start-up solution
# ---------------------------------------------------------------------------

def poiseuille_startup(y, t: float, H: float, nu: float, g: float,
                       n_modes: int = 400) -> np.ndarray:
    """u(y, t) of the flow between no-slip walls at y = 0 and y = H driven
    from rest by a uniform body force g: the solution of u_t = nu u_yy + g
    with u(0, t) = u(H, t) = 0 and u(y, 0) = 0 (uniform density, so the
    isothermal equations reduce to this diffusion problem).

    Separation of variables: the steady state is the parabola
    U(y) = g y (H - y) / (2 nu); the transient U - u solves the homogeneous
    heat equation with initial value U, whose sine coefficients on (0, H),
    (2/H) int_0^H U sin(k pi y/H) dy, are 4 g H^2 / (nu pi^3 k^3) for odd k
    (zero for even k), each decaying as exp(-nu (k pi / H)^2 t). The first n_modes odd modes are kept."""
    y = np.asarray(y, dtype=np.float64)
    steady = g / (2.0 * nu) * y * (H - y)
    transient = np.zeros_like(y)
    for j in range(n_modes):
        k = 2.0 * j + 1.0
        lam = nu * (k * math.pi / H) ** 2
        coef = 4.0 * g * H * H / (nu * math.pi ** 3 * k ** 3)
        transient += coef * math.exp(-lam * t) * np.sin(k * math.pi * y / H)
    return steady - transient
