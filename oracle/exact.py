"""The exact LABFM weights of a node, by a 40-digit solve (TEST
INFRASTRUCTURE ONLY, like the rest of ``oracle/``: never imported by the
product path).

The weights are defined as the solution of the node's linear system
(eqs. disc_form, lsys, w_abf and hermite of section "The Local Anisotropic
Basis Function Method" and "New ABFs"); the float64 solve of
``labfm_oracle.node_weights`` approximates that solution to within about
cond(M~) eps. This module evaluates the same definition in mpmath at 40
significant digits, with mpmath's own Hermite polynomials and LU solver, so
that the float64 oracle (and the GPU) can be measured against the exact
result where cond(M~) eps is far above 1e-12 (orders 9 and 10).
"""
from __future__ import annotations

import mpmath
import numpy as np

from . import labfm_oracle as O


def _system(dx, dy, h, m):
    ex = O.monomial_exponents(m)
    n = len(ex)
    hm = mpmath.mpf(h)
    K = dx.size
    Xt = mpmath.matrix(K, n)
    Wm = mpmath.matrix(K, n)
    for k in range(K):
        xs = mpmath.mpf(dx[k]) / hm
        ys = mpmath.mpf(dy[k]) / hm
        q = mpmath.sqrt(xs * xs + ys * ys)
        psi = (1 - q / 2) ** 4 * (1 + 2 * q) if q < 2 else mpmath.mpf(0)
        for c, (a, b) in enumerate(ex):
            Xt[k, c] = xs ** a * ys ** b / (mpmath.factorial(a) * mpmath.factorial(b))
            Wm[k, c] = (psi * mpmath.hermite(a, xs / mpmath.sqrt(2))
                        * mpmath.hermite(b, ys / mpmath.sqrt(2)) / mpmath.sqrt(2) ** (a + b))
    M = Xt.T * Wm
    C = O.target_vectors(m, 1.0)
    rhs = []
    for d in range(6):
        rhs.append(mpmath.matrix([mpmath.mpf(C[p, d]) / hm ** sum(ex[p]) for p in range(n)]))
    return M, Wm, rhs


def exact_node_weights(dx, dy, h: float, m: int, digits: int = 40) -> tuple:
    """Weights of the six operators (6, K), rounded to float64 from a
    `digits`-digit solve, and cond(M~) (2-norm, of the float64-rounded M~)."""
    with mpmath.workdps(digits):
        M, Wm, rhs = _system(dx, dy, h, m)
        K = dx.size
        out = np.zeros((6, K))
        for d in range(6):
            wd = Wm * mpmath.lu_solve(M, rhs[d])
            out[d] = [float(wd[k]) for k in range(K)]
        n = M.rows
        Mf = np.array([[float(M[r, c]) for c in range(n)] for r in range(n)])
    return out, float(np.linalg.cond(Mf))


def exact_node_outputs(dx, dy, h: float, m: int, dphis, digits: int = 40) -> np.ndarray:
    """L^d_i(phi) = sum_j (phi_j - phi_i) w^d_ji (eq. general_do) with the
    exact weights, for each array of differences phi_j - phi_i in `dphis`
    (float64 inputs, taken as exact), the sums in `digits` digits and rounded
    once. Returns (len(dphis), 6)."""
    with mpmath.workdps(digits):
        M, Wm, rhs = _system(dx, dy, h, m)
        K = dx.size
        out = np.zeros((len(dphis), 6))
        for d in range(6):
            wd = Wm * mpmath.lu_solve(M, rhs[d])
            for f, dphi in enumerate(dphis):
                out[f, d] = float(mpmath.fsum(mpmath.mpf(float(dphi[k])) * wd[k]
                                              for k in range(K)))
    return out
