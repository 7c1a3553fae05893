"""Parity of the boundary scheme on the GPU (labfm_boundary_weights and the
wall equation of the stage kernels) with the FP64 CPU oracle, and the
Poiseuille start-up against its analytic solution.

Gates: boundary weights within 1e-12 relative l2 per row (the strip rows come
from a 4 x 4 solve and fixed differences; the other rows keep the build's
cond-based bound), right-hand sides and RK states within 1e-12 relative
(measured: 1e-14 to 2.4e-13), the float32 copies the rounded float64
weights."""
import math

import numpy as np
import pytest

from oracle import boundaries_oracle as B
from oracle import labfm_oracle as O
from paper_2102_02019_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_02019_amd import labfm

    labfm.lib()
    return torch.device("cuda:0")


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_channel(nodes, strips, dev, f32=False):
    from paper_2102_02019_amd import labfm

    x, y, h, s = (T(a, dev) for a in (nodes.x, nodes.y, nodes.h, nodes.s))
    rp, col = labfm.build_neighbours(x, y, h, nodes.box)
    ops = labfm.build_weights(x, y, h, s, T(nodes.m, dev), nodes.box, rp, col, f32=f32)
    labfm.boundary_weights(x, y, h, s, nodes.box, ops, T(strips.column, dev),
                           T(strips.normal, dev))
    torch.cuda.synchronize()
    return ops


@pytest.fixture(scope="module")
def ch20(dev):
    nodes, strips = inputs.channel(20)
    return nodes, strips, gpu_channel(nodes, strips, dev, f32=True), B.channel_weights(nodes, strips)


def _cond2d(nodes, W, i):
    dx, dy = O.stencil_offsets(nodes.x, nodes.y, nodes.box, W["row_ptr"], W["col"], i)
    r = O.node_weights(dx, dy, nodes.h[i], nodes.s[i], int(nodes.m[i]))
    return np.linalg.cond(r["M"])


def _check_channel_weights(nodes, strips, ops, W):
    rp = W["row_ptr"]
    assert np.array_equal(ops.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(ops.col.cpu().numpy(), W["col"])
    w = ops.w.cpu().numpy()
    kappa = ops.kappa.cpu().numpy()
    worst = {}
    for i in range(nodes.n):
        a, b = rp[i], rp[i + 1]
        lvl = strips.level[i]
        tol2d = max(1e-12, 100 * _cond2d(nodes, W, i) * 2.2e-16) if lvl != 0 else TOL
        for d in range(6):
            boundary = lvl == 0 or (lvl in (1, 2) and d in (O.OP_X, O.OP_Y))
            tol = TOL if boundary else tol2d
            e = rel(w[d, a:b], W["w"][d, a:b])
            key = "strip rows" if boundary else "2D rows / their gate"
            worst[key] = max(worst.get(key, 0.0), e if boundary else e / tol)
            assert e <= tol, (i, lvl, d)
        # kappa comes from the filter weights: the 1D solve at wall nodes, the
        # two-dimensional one elsewhere
        assert abs(kappa[i] - W["kappa"][i]) <= max(1e-9, tol2d) * abs(W["kappa"][i]), i
    print(f"gate channel weights: {worst}")
    assert np.array_equal(ops.status.cpu().numpy(), W["status"])
    assert np.array_equal(ops.wall_normal.cpu().numpy(), W["wall_normal"])


def test_channel_weights_match_oracle(ch20):
    nodes, strips, ops, W = ch20
    _check_channel_weights(nodes, strips, ops, W)
    # the float32 copies and first moments follow the replaced weights
    w = ops.w.cpu().numpy()
    assert np.array_equal(ops.w32.cpu().numpy(), w.astype(np.float32))
    mom = ops.mom32.cpu().numpy()
    assert np.all(mom[:, strips.column[:, 0]] == 0.0)


def test_channel_weights_ragged(dev):
    """13 columns (a ragged last tile), another seed and bulk order 8."""
    nodes, strips = inputs.channel(13, m=8, seed=21)
    _check_channel_weights(nodes, strips, gpu_channel(nodes, strips, dev),
                           B.channel_weights(nodes, strips))


def test_channel_without_columns_is_unchanged(dev):
    """count = 0: the weights stay those of the build; wall_normal is zero."""
    from paper_2102_02019_amd import labfm

    nodes, _ = inputs.channel(12)
    x, y, h, s = (T(a, dev) for a in (nodes.x, nodes.y, nodes.h, nodes.s))
    rp, col = labfm.build_neighbours(x, y, h, nodes.box)
    ops = labfm.build_weights(x, y, h, s, T(nodes.m, dev), nodes.box, rp, col)
    w0 = ops.w.clone()
    labfm.boundary_weights(x, y, h, s, nodes.box, ops,
                           torch.zeros((0, 5), dtype=torch.int32, device=dev),
                           torch.zeros((0, 2), dtype=torch.float64, device=dev))
    assert torch.equal(ops.w, w0)
    assert torch.count_nonzero(ops.wall_normal).item() == 0


@pytest.mark.parametrize("bad", ["range", "twice", "normal"])
def test_bad_columns_are_rejected(dev, bad):
    from paper_2102_02019_amd import labfm

    nodes, strips = inputs.channel(12)
    x, y, h, s = (T(a, dev) for a in (nodes.x, nodes.y, nodes.h, nodes.s))
    rp, col = labfm.build_neighbours(x, y, h, nodes.box)
    ops = labfm.build_weights(x, y, h, s, T(nodes.m, dev), nodes.box, rp, col)
    column, normal = strips.column.copy(), strips.normal.copy()
    if bad == "range":
        column[3, 2] = nodes.n
    elif bad == "twice":
        column[4, 1] = column[5, 1]
    else:
        normal[2] *= 1.5
    with pytest.raises(labfm.LabfmError) as e:
        labfm.boundary_weights(x, y, h, s, nodes.box, ops, T(column, dev), T(normal, dev))
    assert e.value.code == labfm.ERR_ARG


def _smooth_state(nodes, amp=1.0):
    """Fields with u = v = 0 on both walls and ln rho varying everywhere."""
    x, y = nodes.x, nodes.y
    tp = 2.0 * math.pi
    lnrho = 0.01 * np.cos(tp * x) * (1.0 + y + y * y)
    u = amp * np.sin(tp * x) * y * (1.0 - y)
    v = amp * (np.cos(tp * x) * y * y * (1.0 - y) ** 2 + 0.3 * y * (1.0 - y))
    return lnrho, u, v


def test_channel_rhs_matches_oracle(dev, ch20):
    from paper_2102_02019_amd import labfm

    nodes, strips, ops, W = ch20
    flow = inputs.FlowParams(c2=400.0, mu=0.1, gx=0.8, gy=-0.5)
    l, u, v = _smooth_state(nodes)
    got = labfm.ns_rhs(T(np.concatenate([l, u, v]), dev), ops, flow).cpu().numpy().reshape(3, -1)
    ref = B.channel_rhs(l, u, v, W, flow)
    wall = strips.column[:, 0]
    assert np.all(got[1:, wall] == 0.0)
    print(f"gate channel rhs: {[rel(got[k], ref[k]) for k in range(3)]} "
          f"wall {rel(got[0, wall], ref[0][wall])}")
    for k in range(3):
        assert rel(got[k], ref[k]) <= TOL, k
    assert rel(got[0, wall], ref[0][wall]) <= TOL


def _compare_state(got, ref):
    g = got.reshape(3, -1)
    return [rel(np.exp(g[0]), np.exp(ref[0])), rel(g[1], ref[1]), rel(g[2], ref[2])]


@pytest.mark.parametrize("graph", [False, True])
def test_channel_rk_matches_oracle(dev, ch20, graph):
    """40 filtered steps from a disturbed state, body force along the walls."""
    from paper_2102_02019_amd import labfm

    nodes, strips, ops, W = ch20
    P = inputs.POISEUILLE
    flow = P.flow()
    l, u, v = _smooth_state(nodes, amp=0.2)
    dt = O.time_step(nodes.s, l, u, v, flow)
    q = T(np.concatenate([l, u, v]), dev)
    labfm.rk_step(q, ops, flow, dt, 40, use_graph=graph, check_finite=True)
    ref = B.channel_run(l, u, v, W, flow, dt, 40)
    got = q.cpu().numpy()
    errs = _compare_state(got, ref)
    print(f"gate channel rk(graph={graph}): {errs}")
    assert max(errs) <= TOL, errs
    wall = strips.column[:, 0]
    assert np.all(got.reshape(3, -1)[1:, wall] == 0.0)


def test_channel_float32_weights(dev, ch20):
    """The float32 precisions run the wall scheme too: 40 steps of the
    Poiseuille start-up stay within 1e-6 of float64."""
    from paper_2102_02019_amd import labfm

    nodes, strips, ops, W = ch20
    P = inputs.POISEUILLE
    flow = P.flow()
    dt, _ = B.poiseuille_steps(nodes, P, flow, 1.0)
    z = np.zeros(3 * nodes.n)
    ref = T(z, dev)
    labfm.rk_step(ref, ops, flow, dt, 40)
    for prec in (labfm.F32W, labfm.F32_COMP):
        q = T(z, dev)
        labfm.rk_step(q, ops, flow, dt, 40, prec=prec)
        d = (q - ref).abs().max().item()
        assert d <= 1e-6 * ref.abs().max().item(), (prec, d)


def test_adjoint_rejects_walls(dev, ch20):
    from paper_2102_02019_amd import labfm

    import ctypes

    nodes, strips, ops, W = ch20
    q = T(np.zeros(3 * nodes.n), dev)
    out = torch.empty_like(q)
    c = ops._c()
    tr = labfm._Transpose(None, None, None, None)
    prm = labfm._RKParams(400.0, 0.1, 0.8, 0.0, 1e-3, 1, 0)
    code = labfm.lib().labfm_rk_adjoint(labfm._ptr(q), labfm._ptr(q), labfm._ptr(out),
                                        ctypes.byref(c), ctypes.byref(tr), ctypes.byref(prm),
                                        2, 1, None, 0, labfm._stream())
    assert code == labfm.ERR_UNSUPPORTED
    assert "wall" in labfm.lib().labfm_last_error().decode()


# ---------------------------------------------------------------------------
# Poiseuille start-up (section "Poiseuille flow")
# ---------------------------------------------------------------------------

def _gpu_poiseuille(dev, nx, t_star):
    from paper_2102_02019_amd import labfm

    P = inputs.POISEUILLE
    flow = P.flow()
    nodes, strips = inputs.channel(nx)
    ops = gpu_channel(nodes, strips, dev)
    assert np.all(ops.status.cpu().numpy() == 0)
    dt, n = B.poiseuille_steps(nodes, P, flow, t_star)
    q = T(np.zeros(3 * nodes.n), dev)
    labfm.rk_step(q, ops, flow, dt, n, use_graph=True, check_finite=True)
    g = q.cpu().numpy().reshape(3, -1)
    ua = B.poiseuille_startup(nodes.y, P.time(t_star), P.H, P.mu / P.rho0, P.gx)
    return nodes, g, B.velocity_error(g[1], g[2], ua)


def test_poiseuille_startup_matches_oracle(dev):
    """The whole start-up to t* = 1 at s = H/20 (400 steps) against the
    oracle's run, state by state."""
    P = inputs.POISEUILLE
    flow = P.flow()
    nodes, g, err = _gpu_poiseuille(dev, 20, 1.0)
    strips = inputs.channel(20)[1]
    W = B.channel_weights(nodes, strips)
    dt, n = B.poiseuille_steps(nodes, P, flow, 1.0)
    z = np.zeros(nodes.n)
    ref = B.channel_run(z, z, z, W, flow, dt, n)
    # v is rounding noise (|v| ~ 1e-7 against |u| ~ 0.6): the velocity is
    # compared as a vector
    e_rho = rel(np.exp(g[0]), np.exp(ref[0]))
    e_vel = rel(np.concatenate([g[1], g[2]]), np.concatenate([ref[1], ref[2]]))
    print(f"gate poiseuille start-up: rho {e_rho} velocity {e_vel}")
    assert max(e_rho, e_vel) <= 1e-12, (e_rho, e_vel)
    ua = B.poiseuille_startup(nodes.y, P.time(1.0), P.H, P.mu / P.rho0, P.gx)
    assert err == pytest.approx(B.velocity_error(ref[1], ref[2], ua), rel=1e-6)


def test_poiseuille_convergence(dev):
    """Velocity error at t* = 1 for s = H/20, H/40, H/80: about fourth order
    (the paper reports ~4)."""
    errs = [_gpu_poiseuille(dev, nx, 1.0)[2] for nx in (20, 40, 80)]
    rates = [math.log(errs[k] / errs[k + 1]) / math.log(2.0) for k in range(2)]
    print("poiseuille t*=1 errors", errs, "rates", rates)
    assert errs[-1] < 1e-5
    assert min(rates) > 3.5, (errs, rates)


def test_poiseuille_steady_state(dev):
    """At t* = 20 the flow is steady (the parabola); the error falls with s
    (the paper reports fifth order)."""
    errs = [_gpu_poiseuille(dev, nx, 20.0)[2] for nx in (20, 40)]
    rate = math.log(errs[0] / errs[1]) / math.log(2.0)
    print("poiseuille t*=20 errors", errs, "rate", rate)
    assert errs[1] < errs[0] / 8.0, errs


def test_channel_full_size_sampled(dev):
    """The benchmark's channel (n_x = 1024, 1,049,600 nodes, m = 6 in the bulk)
    built on the GPU in the benchmark's configuration: sampled strip columns
    (all five levels) and bulk nodes against the oracle's per-row stencils,
    weights, kappa, status and right-hand side."""
    from paper_2102_02019_amd import labfm

    nodes, strips = inputs.channel(1024)
    ops = gpu_channel(nodes, strips, dev)
    cols = [0, 311, 777, 1023, 1024, 1500, 2047]
    rng = np.random.default_rng(17)
    bulk = rng.choice(np.nonzero(strips.level < 0)[0], 24, replace=False)
    rows = sorted(set(int(i) for i in strips.column[cols].ravel()) | set(int(i) for i in bulk))
    rp, col = O.neighbours_rows(nodes.x, nodes.y, nodes.h, nodes.box, rows)
    W2 = O.weights(nodes.x, nodes.y, nodes.h, nodes.s, nodes.m, rp, col, nodes.box, nodes=rows)
    W = B.boundary_weights(nodes, strips, rp, col, W2, columns=cols)
    rp_g = ops.row_ptr.cpu().numpy()
    kappa = ops.kappa.cpu().numpy()
    status = ops.status.cpu().numpy()
    wn = ops.wall_normal.cpu().numpy()
    for i in rows:
        a, b = rp[i], rp[i + 1]
        ga, gb = int(rp_g[i]), int(rp_g[i + 1])
        assert np.array_equal(ops.col[ga:gb].cpu().numpy(), col[a:b]), i
        w = ops.w[:, ga:gb].cpu().numpy()
        lvl = strips.level[i]
        tol2d = max(1e-12, 100 * _cond2d(nodes, W, i) * 2.2e-16) if lvl != 0 else TOL
        for d in range(6):
            boundary = lvl == 0 or (lvl in (1, 2) and d in (O.OP_X, O.OP_Y))
            assert rel(w[d], W["w"][d, a:b]) <= (TOL if boundary else tol2d), (i, lvl, d)
        assert abs(kappa[i] - W["kappa"][i]) <= max(1e-9, tol2d) * abs(W["kappa"][i]), i
        assert status[i] == W["status"][i], i
        assert np.array_equal(wn[i], W["wall_normal"][i]), i
    flow = inputs.FlowParams(c2=400.0, mu=0.1, gx=0.8, gy=-0.5)
    l, u, v = _smooth_state(nodes)
    got = labfm.ns_rhs(T(np.concatenate([l, u, v]), dev), ops, flow).cpu().numpy().reshape(3, -1)
    ref = B.channel_rhs(l, u, v, W, flow)
    errs = [np.max(np.abs(got[k][rows] - ref[k][rows])) / (np.max(np.abs(ref[k][rows])) + 1e-300)
            for k in range(3)]
    print(f"gate channel 1.05M sampled rhs: {errs}")
    for k in range(3):
        assert errs[k] <= 1e-12, k


def test_cylinder_matches_oracle(dev):
    """A curved no-slip wall (the paper's cylinder geometry): normals in every
    direction, strip rows along arcs, a body force with g.n != 0 on the wall.
    All weights, the right-hand side and 10 filtered steps against the
    oracle."""
    from paper_2102_02019_amd import labfm

    nodes, strips = inputs.cylinder(64)
    ops = gpu_channel(nodes, strips, dev)
    W = B.channel_weights(nodes, strips)
    _check_channel_weights(nodes, strips, ops, W)
    tp = 2.0 * math.pi
    r = np.hypot(nodes.x - 0.5, nodes.y - 0.5)
    wall = strips.column[:, 0]
    l = 0.01 * np.cos(tp * nodes.x) * np.sin(tp * nodes.y)
    u = 0.5 * (r - 0.2) * np.sin(tp * nodes.y)
    v = 0.5 * (r - 0.2) * np.cos(tp * nodes.x)
    u[wall] = 0.0
    v[wall] = 0.0
    flow = inputs.FlowParams(c2=400.0, mu=0.05, gx=0.3, gy=0.1)
    got = labfm.ns_rhs(T(np.concatenate([l, u, v]), dev), ops, flow).cpu().numpy().reshape(3, -1)
    ref = B.channel_rhs(l, u, v, W, flow)
    print(f"gate cylinder rhs: {[rel(got[k], ref[k]) for k in range(3)]}")
    for k in range(3):
        assert rel(got[k], ref[k]) <= TOL, k
    assert rel(got[0, wall], ref[0][wall]) <= TOL
    dt = O.time_step(nodes.s, l, u, v, flow)
    q = T(np.concatenate([l, u, v]), dev)
    labfm.rk_step(q, ops, flow, dt, 10, check_finite=True)
    refq = B.channel_run(l, u, v, W, flow, dt, 10)
    errs = _compare_state(q.cpu().numpy(), refq)
    print(f"gate cylinder rk: {errs}")
    assert max(errs) <= TOL, errs
