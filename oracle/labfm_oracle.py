"""FP64 CPU oracle for the LABFM hot path (King & Lind, arXiv 2102.02019).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import or call this
module; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do. It shares no code, table or constant generator with the HIP
library: every routine here is written from the paper's equations.

The method has no cheaper closed form than its own definition, so each routine
restates the paper's steps in its order and notation, in float64, with LAPACK
``gesv`` (through ``numpy.linalg.solve``) for the local systems, as the paper
does. Loops are vectorised over nodes only where that changes no per-node
arithmetic.

Readings of silent or garbled passages (each one is also listed in the design
notes of the repository):

* Wendland C2 kernel (section "New ABFs", cited, not printed):
  psi(q) = (1 - q/2)^4 (1 + 2q) for q = |r|/h < 2, else 0 (support 2h, the
  stencil radius).
* The stencil excludes the node itself (it contributes exactly zero) and
  includes ties at |r_ji| = 2h (the paper writes <=).
* Operators beyond x, y, L needed by the momentum equation (xx, xy) come from
  other choices of C^d, as the filter section allows; yy = L - xx.
* The hyperviscous filter operator is nabla^m for even m and nabla^(m-1) for
  odd m; its C vector puts binom(m'/2, p) at the monomial x^(2p) y^(m'-2p).
* The filter is calibrated on the mode of wavenumber 2/3 of the Nyquist
  wavenumber pi/s (the printed phase would put it above Nyquist; see
  ``filter_coefficient``).
* The pressure term -(1/rho) dp/dx with p = c^2 rho is evaluated as
  -c^2 d(ln rho)/dx.
* The time step is evaluated once, on the initial state.
* RK3(2)4[2R+]C coefficients (named, not printed, in the paper) are those of
  Kennedy, Carpenter & Lewis (2000); they are pinned by the third-order
  conditions in the tests.

Parity of the Taylor-Green run is pinned by trends only (the paper prints
figures, not values); every other routine is pinned by closed forms,
invariants, library routines or brute force in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

OPS = ("x", "y", "L", "xx", "xy", "hyp")
OP_X, OP_Y, OP_L, OP_XX, OP_XY, OP_HYP = range(6)

STATUS_OK = 0
STATUS_SINGULAR = 1
STATUS_FEW_NEIGHBOURS = 2
STATUS_BAD_FILTER = 3


# ---------------------------------------------------------------------------
# Section "The Local Anisotropic Basis Function Method": index order
# ---------------------------------------------------------------------------

def n_moments(m: int) -> int:
    """Length of the monomial vector X for order m: (m^2 + 3m)/2."""
    return (m * m + 3 * m) // 2


def monomial_exponents(m: int) -> list:
    """(a, b) for each entry of X = [x, y, x^2/2, xy, y^2/2, x^3/6, ...]:
    ordered by total degree, then by decreasing power of x."""
    out = []
    for d in range(1, m + 1):
        for b in range(0, d + 1):
            out.append((d - b, b))
    return out


# ---------------------------------------------------------------------------
# Section "Stencil": neighbour sets
# ---------------------------------------------------------------------------

def min_image(d: np.ndarray, L: float, periodic: bool) -> np.ndarray:
    """Nearest periodic image of a coordinate difference."""
    if not periodic:
        return d
    half = 0.5 * L
    return np.where(d > half, d - L, np.where(d < -half, d + L, d))


def morton_permutation(x, y, box, cell: float) -> np.ndarray:
    """Z-order permutation of the nodes: cell (ix, iy) = floor(p / cell)
    clamped to 0..ceil(L/cell)-1; the key carries bit b of ix at position 2b
    and bit b of iy at 2b + 1; nodes in ascending key, equal keys in
    ascending index."""
    ncx = max(1, math.ceil(box.Lx / cell))
    ncy = max(1, math.ceil(box.Ly / cell))
    ix = np.clip(np.floor(x / cell), 0, ncx - 1).astype(np.int64)
    iy = np.clip(np.floor(y / cell), 0, ncy - 1).astype(np.int64)
    key = np.zeros(x.size, dtype=np.uint64)
    for b in range(21):
        key |= ((ix >> b) & 1).astype(np.uint64) << np.uint64(2 * b)
        key |= ((iy >> b) & 1).astype(np.uint64) << np.uint64(2 * b + 1)
    return np.argsort(key, kind="stable")


def in_stencil(dx: np.ndarray, dy: np.ndarray, h_i) -> np.ndarray:
    """|r_ji| <= 2 h_i evaluated as dx*dx + dy*dy <= (2h)*(2h), each product
    and the sum rounded separately (no fused multiply-add)."""
    d2 = np.multiply(dx, dx) + np.multiply(dy, dy)
    r = 2.0 * h_i
    return d2 <= r * r


def neighbours_bruteforce(x, y, h, box) -> tuple:
    """All j != i with |r_ji| <= 2 h_i, by testing every pair. Rows list j in
    ascending order. Returns CSR (row_ptr int64[N+1], col int64[nnz])."""
    n = x.size
    rows = []
    for i in range(n):
        dx = min_image(x - x[i], box.Lx, box.periodic_x)
        dy = min_image(y - y[i], box.Ly, box.periodic_y)
        sel = in_stencil(dx, dy, h[i])
        sel[i] = False
        rows.append(np.nonzero(sel)[0])
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([r.size for r in rows])
    col = np.concatenate(rows).astype(np.int64) if n else np.zeros(0, np.int64)
    return row_ptr, col


def neighbours(x, y, h, box, nodes=None) -> tuple:
    """Same set as ``neighbours_bruteforce``. Above a few thousand nodes (or
    for a range of rows) the candidates come from scipy's k-d tree with a
    slightly enlarged radius and every candidate is then tested with the
    exact predicate above. ``nodes``: a range of rows to compute (the CSR
    then has the other rows empty), for node sets split over processes."""
    n = x.size
    if n <= 4096 and nodes is None:
        return neighbours_bruteforce(x, y, h, box)
    from scipy.spatial import cKDTree

    rows_of = range(n) if nodes is None else nodes
    pts = np.stack([x, y], axis=1)
    boxsize = None
    if box.periodic_x and box.periodic_y:
        boxsize = [box.Lx, box.Ly]
    elif box.periodic_x or box.periodic_y:
        raise NotImplementedError("mixed periodicity needs the brute-force path")
    tree = cKDTree(pts, boxsize=boxsize)
    rows = []
    hmax = float(h.max())
    # candidates within the largest radius, then the per-node predicate
    sel = np.asarray(rows_of, dtype=np.int64)
    assert np.all(np.diff(sel) > 0), "rows in increasing order"
    cand = tree.query_ball_point(pts[sel], r=2.0 * hmax * (1.0 + 1e-9), return_sorted=True)
    for k, i in enumerate(sel):
        c = np.asarray(cand[k], dtype=np.int64)
        c = c[c != i]
        dx = min_image(x[c] - x[i], box.Lx, box.periodic_x)
        dy = min_image(y[c] - y[i], box.Ly, box.periodic_y)
        rows.append(np.sort(c[in_stencil(dx, dy, h[i])]))
    counts = np.zeros(n, dtype=np.int64)
    counts[sel] = [r.size for r in rows]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(counts)
    col = np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, np.int64)
    return row_ptr, col


def neighbours_rows(x, y, h, box, nodes) -> tuple:
    """The stencils of the listed nodes only, by testing every j (brute force
    per row), as a CSR over all N nodes whose other rows are empty: for
    sampled checks of node sets too large for the full search."""
    n = x.size
    nodes = sorted(set(int(i) for i in nodes))
    rows = {}
    for i in nodes:
        dx = min_image(x - x[i], box.Lx, box.periodic_x)
        dy = min_image(y - y[i], box.Ly, box.periodic_y)
        sel = in_stencil(dx, dy, h[i])
        sel[i] = False
        rows[i] = np.nonzero(sel)[0]
    counts = np.zeros(n, dtype=np.int64)
    for i, r in rows.items():
        counts[i] = r.size
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(counts)
    col = (np.concatenate([rows[i] for i in nodes]).astype(np.int64) if nodes
           else np.zeros(0, np.int64))
    return row_ptr, col


# ---------------------------------------------------------------------------
# Sections "LABFM" and "New ABFs": basis functions, moment matrix, weights
# ---------------------------------------------------------------------------

def wendland_c2(q: np.ndarray) -> np.ndarray:
    """Wendland C2 radial function of q = |r|/h with support q < 2."""
    t = np.clip(1.0 - 0.5 * q, 0.0, None)
    return np.where(q < 2.0, t ** 4 * (1.0 + 2.0 * q), 0.0)


def hermite_phys(a: int, z: np.ndarray) -> np.ndarray:
    """Physicists' Hermite polynomial H_a(z): H_0 = 1, H_1 = 2z,
    H_{k+1} = 2z H_k - 2k H_{k-1}."""
    h0 = np.ones_like(z)
    if a == 0:
        return h0
    h1 = 2.0 * z
    for k in range(1, a):
        h0, h1 = h1, 2.0 * z * h1 - 2.0 * k * h0
    return h1


def taylor_monomials(xs: np.ndarray, ys: np.ndarray, m: int) -> np.ndarray:
    """Scaled monomial vector X~_ji = X_ji . H_i: entry (a, b) is
    (x/h)^a (y/h)^b / (a! b!) for the already scaled xs = x/h, ys = y/h.
    Shape (..., n)."""
    cols = []
    for a, b in monomial_exponents(m):
        cols.append(xs ** a * ys ** b / (math.factorial(a) * math.factorial(b)))
    return np.stack(cols, axis=-1)


def hermite_abfs(xs: np.ndarray, ys: np.ndarray, m: int) -> np.ndarray:
    """Hermite ABFs: W^q = psi(|r|/h) H_a(x/(h sqrt2)) H_b(y/(h sqrt2)) / sqrt(2^(a+b)).
    Shape (..., n)."""
    psi = wendland_c2(np.sqrt(xs * xs + ys * ys))
    r2 = math.sqrt(2.0)
    cols = []
    for a, b in monomial_exponents(m):
        cols.append(psi * hermite_phys(a, xs / r2) * hermite_phys(b, ys / r2)
                    / math.sqrt(2.0 ** (a + b)))
    return np.stack(cols, axis=-1)


def filter_power(m: int) -> int:
    """Order of the hyperviscous filter operator: m if even, else m - 1."""
    return m if m % 2 == 0 else m - 1


def target_vectors(m: int, h: float) -> np.ndarray:
    """C~^d = C^d . H for d in (x, y, L, xx, xy, hyp); shape (n, 6).

    C^x, C^y, C^L as printed; xx and xy select one second derivative; hyp is
    nabla^m' = sum_p binom(m'/2, p) d^m'/dx^(2p) dy^(m'-2p)."""
    ex = monomial_exponents(m)
    idx = {ab: q for q, ab in enumerate(ex)}
    C = np.zeros((len(ex), 6))
    C[idx[(1, 0)], OP_X] = 1.0
    C[idx[(0, 1)], OP_Y] = 1.0
    if m >= 2:
        C[idx[(2, 0)], OP_L] = 1.0
        C[idx[(0, 2)], OP_L] = 1.0
        C[idx[(2, 0)], OP_XX] = 1.0
        C[idx[(1, 1)], OP_XY] = 1.0
    mp = filter_power(m)
    if mp >= 2:
        half = mp // 2
        for p in range(half + 1):
            C[idx[(2 * p, mp - 2 * p)], OP_HYP] = float(math.comb(half, p))
    scale = np.array([h ** (-(a + b)) for a, b in ex])
    return C * scale[:, None]


def moment_matrix(Xt: np.ndarray, W: np.ndarray) -> np.ndarray:
    """M_i = sum_j X~_ji (outer) W_ji: rows are monomials, columns basis
    functions. Xt, W have shape (K, n)."""
    return Xt.T @ W


def node_weights(dx: np.ndarray, dy: np.ndarray, h: float, s: float, m: int) -> dict:
    """One node's weights w^d_ji for the six operators, its filter coefficient
    and a status code, from the offsets r_ji = (dx, dy) of its K neighbours."""
    n = n_moments(m)
    K = dx.size
    xs, ys = dx / h, dy / h
    Xt = taylor_monomials(xs, ys, m)
    W = hermite_abfs(xs, ys, m)
    M = moment_matrix(Xt, W)
    C = target_vectors(m, h)
    status = STATUS_OK
    if K < n:
        status = STATUS_FEW_NEIGHBOURS
    try:
        Psi = np.linalg.solve(M, C)
    except np.linalg.LinAlgError:
        Psi = np.full((n, 6), np.nan)
        status = STATUS_SINGULAR
    w = (W @ Psi).T  # (6, K): w^d_ji = W_ji . Psi^d_i
    kappa, fstat = filter_coefficient(dx, dy, s, w[OP_HYP])
    if status == STATUS_OK and fstat != STATUS_OK:
        status = fstat
    return {"w": w, "kappa": kappa, "status": status, "M": M, "C": C, "Psi": Psi}


def filter_coefficient(dx, dy, s: float, w_hyp: np.ndarray, k: float = None) -> tuple:
    """F_0 = sum_j [1 - cos(k x_ji) cos(k y_ji)] w^hyp_ji and kappa = 2/(3 F_0),
    so that the filter leaves 1/3 of that mode, with k two-thirds of the
    Nyquist wavenumber pi/s, i.e. k = 2 pi / (3 s) (the default).

    The paper's printed phase 3 pi x / (2 s) is 1.5 times the Nyquist
    wavenumber (the wavelength 4s/3, two-thirds of the Nyquist wavelength 2s,
    which is what the sentence after the kappa equation names); on a
    near-lattice it aliases to a low wavenumber, F_0 gets small or changes
    sign at some nodes and the filter then amplifies instead of damping. The
    next paragraph names "two-thirds the Nyquist wavenumber", which is the
    reading taken here. ``k`` overrides the wavenumber (the tests use it to
    show what the printed phase does)."""
    a = 2.0 * math.pi / (3.0 * s) if k is None else float(k)
    phi = 1.0 - np.cos(a * dx) * np.cos(a * dy)
    F0 = float(np.sum(phi * w_hyp))
    if not np.isfinite(F0) or F0 == 0.0:
        return 0.0, STATUS_BAD_FILTER
    return 2.0 / (3.0 * F0), STATUS_OK


def stencil_offsets(x, y, box, row_ptr, col, i) -> tuple:
    """r_ji = r_j - r_i (nearest periodic image) for the neighbours of i."""
    c = col[row_ptr[i]:row_ptr[i + 1]]
    dx = min_image(x[c] - x[i], box.Lx, box.periodic_x)
    dy = min_image(y[c] - y[i], box.Ly, box.periodic_y)
    return dx, dy


def weights(x, y, h, s, m, row_ptr, col, box, nodes=None) -> dict:
    """Weights for every node (or the listed ``nodes``).

    Returns w (6, nnz) laid out like ``col`` (entries of unlisted nodes are
    NaN), kappa (N,), rowsum (6, N) = sum_j w^d_ji, status (N,)."""
    N = x.size
    nnz = int(row_ptr[-1])
    m = np.broadcast_to(np.asarray(m), (N,))
    w = np.full((6, nnz), np.nan)
    kappa = np.full(N, np.nan)
    rowsum = np.full((6, N), np.nan)
    status = np.full(N, -1, dtype=np.int8)
    it = range(N) if nodes is None else nodes
    for i in it:
        dx, dy = stencil_offsets(x, y, box, row_ptr, col, i)
        r = node_weights(dx, dy, float(h[i]), float(s[i]), int(m[i]))
        w[:, row_ptr[i]:row_ptr[i + 1]] = r["w"]
        kappa[i] = r["kappa"]
        rowsum[:, i] = r["w"].sum(axis=1)
        status[i] = r["status"]
    return {"w": w, "kappa": kappa, "rowsum": rowsum, "status": status}


def weights_batched(x, y, h, s, m: int, row_ptr, col, box, chunk: int = 4096,
                    start: int = 0, stop: int = None) -> dict:
    """Same steps as ``weights`` for a uniform order m, run over a stack of
    nodes at once. Rows are padded to the longest row of the stack and padded
    entries are masked out of every sum. Only nodes start..stop-1 are built
    (all by default); the entries of the others are left unset."""
    N = x.size
    stop = N if stop is None else stop
    nnz = int(row_ptr[-1])
    n = n_moments(m)
    K = np.diff(row_ptr)
    w = np.empty((6, nnz))
    kappa = np.empty(N)
    rowsum = np.empty((6, N))
    status = np.zeros(N, dtype=np.int8)
    for lo in range(start, stop, chunk):
        hi = min(stop, lo + chunk)
        Kmax = int(K[lo:hi].max()) if hi > lo else 0
        B = hi - lo
        idx = np.arange(Kmax)[None, :]
        valid = idx < K[lo:hi, None]
        e = np.where(valid, row_ptr[lo:hi, None] + idx, 0)
        cj = col[e]
        ii = np.arange(lo, hi)[:, None]
        dx = min_image(x[cj] - x[ii], box.Lx, box.periodic_x)
        dy = min_image(y[cj] - y[ii], box.Ly, box.periodic_y)
        hh = h[lo:hi, None]
        Xt = taylor_monomials(dx / hh, dy / hh, m) * valid[..., None]
        Wb = hermite_abfs(dx / hh, dy / hh, m) * valid[..., None]
        M = np.einsum("bkp,bkq->bpq", Xt, Wb)
        C = np.stack([target_vectors(m, float(h[i])) for i in range(lo, hi)])
        try:
            Psi = np.linalg.solve(M, C)
        except np.linalg.LinAlgError:
            Psi = np.empty((B, n, 6))
            for b in range(B):
                try:
                    Psi[b] = np.linalg.solve(M[b], C[b])
                except np.linalg.LinAlgError:
                    Psi[b] = np.nan
                    status[lo + b] = STATUS_SINGULAR
        wb = np.einsum("bkq,bqd->bdk", Wb, Psi) * valid[:, None, :]
        a = 2.0 * math.pi / (3.0 * s[lo:hi, None])
        phi = (1.0 - np.cos(a * dx) * np.cos(a * dy)) * valid
        F0 = np.sum(phi * wb[:, OP_HYP, :], axis=1)
        bad = ~np.isfinite(F0) | (F0 == 0.0)
        kappa[lo:hi] = np.where(bad, 0.0, 2.0 / (3.0 * np.where(bad, 1.0, F0)))
        status[lo:hi] = np.where((status[lo:hi] == 0) & bad, STATUS_BAD_FILTER, status[lo:hi])
        status[lo:hi] = np.where((status[lo:hi] == 0) & (K[lo:hi] < n),
                                 STATUS_FEW_NEIGHBOURS, status[lo:hi])
        rowsum[:, lo:hi] = wb.sum(axis=2).T
        for b in range(B):
            k = K[lo + b]
            w[:, row_ptr[lo + b]:row_ptr[lo + b] + k] = wb[b, :, :k]
    return {"w": w, "kappa": kappa, "rowsum": rowsum, "status": status}


# ---------------------------------------------------------------------------
# Section "Stencil optimisation"
# ---------------------------------------------------------------------------

STENCIL_H0_OVER_S = 2.8   # initial h_i = 2.8 s_i
STENCIL_SHRINK = 0.99     # h_i <- 0.99 h_i while both tests pass
STENCIL_GAIN_MAX = 1.01   # largest accepted amplitude response
STENCIL_N_K = 16          # wavenumbers k_Ny/16 ... k_Ny of the amplitude test


def laplacian_residual(r: dict, h: float, m: int) -> float:
    """alpha_L = || M Psi^L - C^L ||_2 of the node's unscaled system (the
    scaled system M~ Psi = C~ is the unscaled one with row p multiplied by
    h^-(a+b); C^L is 1 at x^2 and y^2)."""
    deg = np.array([a + b for a, b in monomial_exponents(m)], dtype=float)
    res = r["M"] @ r["Psi"][:, OP_L] - r["C"][:, OP_L]
    return float(np.linalg.norm(res * h ** deg))


def amplitude_responses(dx, dy, w: np.ndarray, s: float, n_k: int = STENCIL_N_K) -> tuple:
    """A^x = L^x(sin k x)/k, A^y = L^y(sin k y)/k and
    A^L = L^L(1/2 - cos(k x) cos(k y)/2)/k^2 at k = q k_Ny/n_k, q = 1..n_k,
    k_Ny = pi/s (the fields vanish at the node itself)."""
    k = (math.pi / s) * np.arange(1, n_k + 1) / n_k
    ax = np.sin(np.outer(k, dx)) @ w[OP_X] / k
    ay = np.sin(np.outer(k, dy)) @ w[OP_Y] / k
    al = (0.5 - 0.5 * np.cos(np.outer(k, dx)) * np.cos(np.outer(k, dy))) @ w[OP_L] / k ** 2
    return ax, ay, al


STENCIL_RES_COEF = 1e4    # residual bound coefficient (the paper prints 1e-4 for its solver)


def optimise_stencil_node(dx0, dy0, h0: float, s: float, m: int,
                          res_coef: float = STENCIL_RES_COEF,
                          shrink: float = STENCIL_SHRINK, gain_max: float = STENCIL_GAIN_MAX,
                          max_iter: int = 200) -> tuple:
    """The paper's loop for one node, on the offsets of its h0 stencil (the
    neighbours beyond 2h have psi = 0 and drop out): build the system at h,
    stop if the Laplacian residual exceeds res_coef eps n^4/(h m) or any
    amplitude response exceeds gain_max, else keep h and shrink it. Returns
    the last accepted h (h0 if none), the number k of shrinks that led to it
    (h = h0 shrink^k, formed by repeated multiplication), and the test values
    at the scale that stopped the loop."""
    n = n_moments(m)
    eps = np.finfo(float).eps
    h, k, best, kbest = h0, 0, h0, 0
    while True:
        r = node_weights(dx0, dy0, h, s, m)
        alpha = laplacian_residual(r, h, m) if np.all(np.isfinite(r["Psi"])) else math.inf
        alpha0 = res_coef * eps * n ** 4 / (h * m)
        amax = math.nan
        ok = alpha <= alpha0
        if ok:
            ax, ay, al = amplitude_responses(dx0, dy0, r["w"], s)
            amax = float(max(ax.max(), ay.max(), al.max()))
            ok = amax <= gain_max
        if not ok or k > max_iter:
            return best, kbest, {"alpha": alpha, "alpha0": alpha0, "amax": amax}
        best, kbest = h, k
        h = h * shrink
        k += 1


def optimise_stencils(x, y, s, m, box, h0=None, nodes=None, **kw) -> tuple:
    """optimise_stencil_node for every node (or the listed ones) on the
    stencils of radius 2 h0 (h0 = 2.8 s by default). Returns h (N,), with h0
    at unlisted nodes, and the accepted-shrink counts (-1 at unlisted
    nodes)."""
    N = x.size
    m = np.broadcast_to(np.asarray(m), (N,))
    h0 = STENCIL_H0_OVER_S * np.asarray(s) if h0 is None else np.asarray(h0)
    listed = range(N) if nodes is None else nodes
    rp, col = (neighbours(x, y, h0, box) if nodes is None
               else neighbours_rows(x, y, h0, box, list(listed)))
    h = np.array(h0, dtype=float, copy=True)
    iters = np.full(N, -1, dtype=np.int64)
    for i in listed:
        dx, dy = stencil_offsets(x, y, box, rp, col, i)
        h[i], iters[i], _ = optimise_stencil_node(dx, dy, float(h0[i]), float(s[i]), int(m[i]),
                                                  **kw)
    return h, iters


# ---------------------------------------------------------------------------
# Equation general_do: the discrete operator
# ---------------------------------------------------------------------------

def apply_op(row_ptr, col, w_d: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """L^d_i(phi) = sum_j (phi_j - phi_i) w^d_ji, summed in ascending j."""
    N = row_ptr.size - 1
    K = np.diff(row_ptr)
    rows = np.repeat(np.arange(N), K)
    terms = (phi[col] - phi[rows]) * w_d
    # bincount adds the terms one after another in storage order, i.e. each
    # row in ascending j
    if np.iscomplexobj(terms):
        return (np.bincount(rows, weights=terms.real, minlength=N)
                + 1j * np.bincount(rows, weights=terms.imag, minlength=N))
    return np.bincount(rows, weights=terms, minlength=N)


# ---------------------------------------------------------------------------
# Section "Implementation for isothermal flows": right-hand side, RK, filter
# ---------------------------------------------------------------------------

# RK3(2)4[2R+]C of Kennedy, Carpenter & Lewis (2000), in 2R form: the Butcher
# matrix has a_{i,j} = b_j for j < i-1, so only a_{i+1,i} and b_i are needed.
RK_A_SUB = (Fraction(11847461282814, 36547543011857),
            Fraction(3943225443063, 7078155732230),
            Fraction(-346793006927, 4029903576067))
RK_B = (Fraction(1017324711453, 9774461848756),
        Fraction(8237718856693, 13685301971492),
        Fraction(57731312506979, 19404895981398),
        Fraction(-101169746363290, 37734290219643))


def butcher_tableau() -> tuple:
    """Full (A, b, c) of the 2R scheme as exact fractions."""
    s = 4
    A = [[Fraction(0)] * s for _ in range(s)]
    for i in range(1, s):
        for j in range(i - 1):
            A[i][j] = RK_B[j]
        A[i][i - 1] = RK_A_SUB[i - 1]
    c = [sum(row) for row in A]
    return A, list(RK_B), c


def ns_rhs(lnrho, u, v, W: dict, prm) -> tuple:
    """Right-hand side of the isothermal Navier-Stokes equations in
    (ln rho, u, v) with the full viscous stress (equation icns).

    W holds row_ptr, col and the operator weights w (6, nnz)."""
    rp, col, w = W["row_ptr"], W["col"], W["w"]

    def L(d, f):
        return apply_op(rp, col, w[d], f)

    lx, ly = L(OP_X, lnrho), L(OP_Y, lnrho)
    ux, uy, uL, uxx, uxy = (L(OP_X, u), L(OP_Y, u), L(OP_L, u), L(OP_XX, u), L(OP_XY, u))
    vx, vy, vL, vxx, vxy = (L(OP_X, v), L(OP_Y, v), L(OP_L, v), L(OP_XX, v), L(OP_XY, v))
    uyy = uL - uxx
    vyy = vL - vxx
    rho = np.exp(lnrho)
    nu = prm.mu / rho
    r_l = -(u * lx + v * ly) - (ux + vy)
    r_u = (-(u * ux + v * uy) - prm.c2 * lx
           + nu * (4.0 / 3.0 * uxx + uyy + 1.0 / 3.0 * vxy) + prm.gx)
    r_v = (-(u * vx + v * vy) - prm.c2 * ly
           + nu * (4.0 / 3.0 * vyy + vxx + 1.0 / 3.0 * uxy) + prm.gy)
    return r_l, r_u, r_v


def filter_fields(fields: tuple, W: dict) -> tuple:
    """phi~_i = phi_i + kappa_i L^hyp_i(phi) for each evolved field."""
    rp, col, w, kappa = W["row_ptr"], W["col"], W["w"], W["kappa"]
    return tuple(f + kappa * apply_op(rp, col, w[OP_HYP], f) for f in fields)


def time_step(s, lnrho, u, v, prm, conv_coef: float = 1.0, visc_coef: float = 0.4) -> float:
    """Equation dt: min over nodes of min(1.0 s/(|u|+c), 0.4 s^2 rho / mu)
    (the two coefficients can be given; those are the paper's)."""
    c = math.sqrt(prm.c2)
    speed = np.sqrt(u * u + v * v)
    conv = conv_coef * s / (speed + c)
    visc = visc_coef * s * s * np.exp(lnrho) / prm.mu
    return float(np.min(np.minimum(conv, visc)))


def rk_integrate(q: tuple, rhs, dt: float, n_steps: int, after_step=None) -> tuple:
    """n_steps of the four-stage low-storage scheme: two registers, q (the
    solution) and Y (the stage value). At stage i: F = rhs(Y); Y = q + dt
    a_{i+1,i} F (stages 1-3, using q before its update); q = q + dt b_i F.
    ``after_step`` (the filter) maps the new q after every complete step."""
    a = [float(v) for v in RK_A_SUB]
    b = [float(v) for v in RK_B]
    q = tuple(np.array(f, dtype=np.result_type(f, float), copy=True) for f in q)
    for _ in range(n_steps):
        Y = q
        for i in range(4):
            F = rhs(*Y)
            if i < 3:
                Y = tuple(qk + (dt * a[i]) * fk for qk, fk in zip(q, F))
            q = tuple(qk + (dt * b[i]) * fk for qk, fk in zip(q, F))
        if after_step is not None:
            q = after_step(q)
    return q


def rk_run(lnrho, u, v, W: dict, prm, dt: float, n_steps: int, filt: bool = True) -> tuple:
    """Evolve (ln rho, u, v) by n_steps RK steps with the filter after each."""
    rhs = lambda l_, u_, v_: ns_rhs(l_, u_, v_, W, prm)  # noqa: E731
    post = (lambda q: filter_fields(q, W)) if filt else None
    return rk_integrate((lnrho, u, v), rhs, dt, n_steps, post)


def ns_rhs_at(lnrho, u, v, x, y, h, s, m, row_ptr, col, box, prm, nodes) -> np.ndarray:
    """Right-hand side of eq. icns at the listed nodes only, each from its own
    weights (the derivatives at a node need only that node's stencil).
    Returns (3, len(nodes))."""
    m = np.broadcast_to(np.asarray(m), (x.size,))
    out = np.empty((3, len(nodes)))
    for k, i in enumerate(nodes):
        dx, dy = stencil_offsets(x, y, box, row_ptr, col, i)
        w = node_weights(dx, dy, float(h[i]), float(s[i]), int(m[i]))["w"]
        c = col[row_ptr[i]:row_ptr[i + 1]]
        dl, du, dv = lnrho[c] - lnrho[i], u[c] - u[i], v[c] - v[i]
        lx, ly = np.sum(dl * w[OP_X]), np.sum(dl * w[OP_Y])
        ux, uy, uL, uxx, uxy = (np.sum(du * w[d]) for d in (OP_X, OP_Y, OP_L, OP_XX, OP_XY))
        vx, vy, vL, vxx, vxy = (np.sum(dv * w[d]) for d in (OP_X, OP_Y, OP_L, OP_XX, OP_XY))
        nu = prm.mu / math.exp(lnrho[i])
        out[0, k] = -(u[i] * lx + v[i] * ly) - (ux + vy)
        out[1, k] = (-(u[i] * ux + v[i] * uy) - prm.c2 * lx
                     + nu * (4.0 / 3.0 * uxx + (uL - uxx) + 1.0 / 3.0 * vxy) + prm.gx)
        out[2, k] = (-(u[i] * vx + v[i] * vy) - prm.c2 * ly
                     + nu * (4.0 / 3.0 * (vL - vxx) + vxx + 1.0 / 3.0 * uxy) + prm.gy)
    return out


# ---------------------------------------------------------------------------
# Adjoint (reverse mode) of the filtered RK time loop
# ---------------------------------------------------------------------------

def operator_matrices(W: dict) -> list:
    """A_d = [w^d_ij] - diag(sum_j w^d_ij): L^d(phi) = A_d phi, as scipy CSR."""
    from scipy import sparse

    rp, col, w = W["row_ptr"], W["col"], W["w"]
    N = rp.size - 1
    mats = []
    for d in range(6):
        Wd = sparse.csr_matrix((w[d], col, rp), shape=(N, N))
        S = np.asarray(Wd.sum(axis=1)).ravel()
        mats.append((Wd - sparse.diags(S)).tocsr())
    return mats


def ns_rhs_vjp(lnrho, u, v, W: dict, prm, rbar: tuple, mats=None) -> tuple:
    """Vector-Jacobian product of ns_rhs: given adjoints (Rl, Ru, Rv) of the
    right-hand side, the adjoints of (ln rho, u, v). Derived by hand from the
    expressions of ns_rhs; operator adjoints are the transposes A_d^T."""
    if mats is None:
        mats = operator_matrices(W)
    A = mats
    Rl, Ru, Rv = rbar
    lx, ly = A[OP_X] @ lnrho, A[OP_Y] @ lnrho
    ux, uy, uL, uxx, uxy = (A[d] @ u for d in (OP_X, OP_Y, OP_L, OP_XX, OP_XY))
    vx, vy, vL, vxx, vxy = (A[d] @ v for d in (OP_X, OP_Y, OP_L, OP_XX, OP_XY))
    uyy = uL - uxx
    vyy = vL - vxx
    nu = prm.mu / np.exp(lnrho)
    visc_u = 4.0 / 3.0 * uxx + uyy + 1.0 / 3.0 * vxy
    visc_v = 4.0 / 3.0 * vyy + vxx + 1.0 / 3.0 * uxy
    # adjoints of the derivative fields
    b_lx = -u * Rl - prm.c2 * Ru
    b_ly = -v * Rl - prm.c2 * Rv
    b_ux = -Rl - u * Ru
    b_uy = -v * Ru
    b_uxx = nu * Ru * (4.0 / 3.0)
    b_uyy = nu * Ru
    b_vxy = nu * Ru / 3.0
    b_vx = -u * Rv
    b_vy = -Rl - v * Rv
    b_vyy = nu * Rv * (4.0 / 3.0)
    b_vxx = nu * Rv
    b_uxy = nu * Rv / 3.0
    # uyy = uL - uxx, vyy = vL - vxx
    b_uL = b_uyy
    b_uxx = b_uxx - b_uyy
    b_vL = b_vyy
    b_vxx = b_vxx - b_vyy
    T = lambda d, g: A[d].T @ g  # noqa: E731
    lbar = T(OP_X, b_lx) + T(OP_Y, b_ly) - nu * (Ru * visc_u + Rv * visc_v)
    ubar = (T(OP_X, b_ux) + T(OP_Y, b_uy) + T(OP_L, b_uL) + T(OP_XX, b_uxx) + T(OP_XY, b_uxy)
            - Rl * lx - Ru * ux - Rv * vx)
    vbar = (T(OP_X, b_vx) + T(OP_Y, b_vy) + T(OP_L, b_vL) + T(OP_XX, b_vxx) + T(OP_XY, b_vxy)
            - Rl * ly - Ru * uy - Rv * vy)
    return lbar, ubar, vbar


def rk_adjoint(lnrho, u, v, W: dict, prm, dt: float, n_steps: int, qbar: tuple,
               filt: bool = True) -> tuple:
    """Adjoint of rk_run: given the adjoint of the state after n_steps, the
    adjoint of the initial state. Written on the full Butcher tableau
    Y_i = q + dt sum_{j<i} a_ij F_j, q' = q + dt sum_i b_i F_i, q+ = filter(q'):
        qbar' = (I + diag(kappa) A_hyp)^T qbar+,
        Fbar_i = dt (b_i qbar' + sum_{k>i} a_ki Ybar_k),  Ybar_i = J_R(Y_i)^T Fbar_i,
        qbar = qbar' + sum_i Ybar_i,
    with every forward state stored."""
    mats = operator_matrices(W)
    A, b, _ = butcher_tableau()
    Af = [[float(a) for a in row] for row in A]
    bf = [float(x) for x in b]
    kappa = W["kappa"]
    rhs = lambda l_, u_, v_: ns_rhs(l_, u_, v_, W, prm)  # noqa: E731
    states = [tuple(np.array(f, dtype=float) for f in (lnrho, u, v))]
    for _ in range(n_steps):
        states.append(rk_run(*states[-1], W, prm, dt, 1, filt=filt))
    qb = tuple(np.array(f, dtype=float) for f in qbar)
    for k in range(n_steps - 1, -1, -1):
        q = states[k]
        Y, F = [], []
        for i in range(4):
            Yi = tuple(q[f] + dt * sum(Af[i][j] * F[j][f] for j in range(i)) for f in range(3))
            Y.append(Yi)
            F.append(rhs(*Yi))
        if filt:
            qb = tuple(g + mats[OP_HYP].T @ (kappa * g) for g in qb)
        Ybar = [None] * 4
        for i in range(3, -1, -1):
            Fb = tuple(dt * (bf[i] * qb[f] + sum(Af[k2][i] * Ybar[k2][f] for k2 in range(i + 1, 4)))
                       for f in range(3))
            Ybar[i] = ns_rhs_vjp(*Y[i], W, prm, Fb, mats)
        qb = tuple(qb[f] + sum(Ybar[i][f] for i in range(4)) for f in range(3))
    return qb
