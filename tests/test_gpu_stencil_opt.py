"""Stencil optimisation on the GPU (section "Stencil optimisation") against
the oracle's per-node loop, and the optimised stencils in use."""
import numpy as np
import pytest
import torch

from oracle import labfm_oracle as O
from paper_2102_02019_amd import inputs

pytestmark = pytest.mark.gpu


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_02019_amd import labfm

    labfm.lib()
    return torch.device("cuda:0")


def _gpu_opt(nodes, dev, **kw):
    from paper_2102_02019_amd import labfm

    x, y, s = T(nodes.x, dev), T(nodes.y, dev), T(nodes.s, dev)
    h0 = T(O.STENCIL_H0_OVER_S * nodes.s, dev)
    h, k = labfm.optimise_stencils(x, y, s, T(nodes.m, dev), nodes.box, h0=h0, **kw)
    return h.cpu().numpy(), k.cpu().numpy()


def _disputed_step_margins(nodes, i, k_lo):
    """The oracle's test values at the scale where the GPU and the oracle
    decided differently, h* = h0 0.99^(k_lo + 1): the Laplacian residual
    over its bound, and the largest amplitude response."""
    h0 = O.STENCIL_H0_OVER_S * nodes.s
    rp, col = O.neighbours_rows(nodes.x, nodes.y, h0, nodes.box, [i])
    dx, dy = O.stencil_offsets(nodes.x, nodes.y, nodes.box, rp, col, i)
    hh = h0[i]
    for _ in range(k_lo + 1):
        hh = hh * O.STENCIL_SHRINK
    m = int(nodes.m[i])
    r = O.node_weights(dx, dy, hh, float(nodes.s[i]), m)
    alpha = O.laplacian_residual(r, hh, m)
    alpha0 = O.STENCIL_RES_COEF * np.finfo(float).eps * O.n_moments(m) ** 4 / (hh * m)
    ax, ay, al = O.amplitude_responses(dx, dy, r["w"], float(nodes.s[i]))
    return alpha / alpha0, float(max(ax.max(), ay.max(), al.max()))


def _check_against_oracle(nodes, h, k, sample):
    """Same number of shrinks as the oracle at (nearly) every sampled node:
    at most one step apart, and only where the step in dispute is marginal
    for the oracle itself: its Laplacian residual within a factor 10 of the
    bound (the residual is a rounding-level quantity, which two float64
    solvers reproduce only to within such a factor), or the residual test
    passed and the largest amplitude response within 1e-6 of 1.01 (the
    responses of two correct solves differ by about cond(M) eps). The scales
    are h0 0.99^k formed by repeated multiplication."""
    ho, ko = O.optimise_stencils(nodes.x, nodes.y, nodes.s, nodes.m, nodes.box,
                                 h0=O.STENCIL_H0_OVER_S * nodes.s, nodes=sample)
    d = np.abs(k[sample] - ko[sample])
    assert d.max() <= 1, (sample, k[sample], ko[sample])
    assert np.mean(d > 0) <= 0.05, np.mean(d > 0)
    for i in np.asarray(sample)[d > 0]:
        ratio, amax = _disputed_step_margins(nodes, int(i), int(min(k[i], ko[i])))
        print(f"disputed node {i}: gpu {k[i]} oracle {ko[i]} shrinks; at the disputed step "
              f"residual/bound {ratio:.3g}, largest response {amax:.12f}")
        marginal_residual = 0.1 <= ratio <= 10.0
        marginal_gain = ratio <= 1.0 and abs(amax - O.STENCIL_GAIN_MAX) <= 1e-6
        assert marginal_residual or marginal_gain, (i, ratio, amax)
    for i in sample:
        hh = O.STENCIL_H0_OVER_S * nodes.s[i]
        for _ in range(int(k[i])):
            hh = hh * 0.99
        assert h[i] == hh


def test_stencil_optimisation_matches_oracle(dev):
    """40 x 40 jittered nodes, m = 6, from h0 = 2.8 s."""
    nodes = inputs.jittered_lattice(40, L=1.0, seed=3, m=6, h_over_s=O.STENCIL_H0_OVER_S)
    h, k = _gpu_opt(nodes, dev)
    assert np.all(k > 0)
    _check_against_oracle(nodes, h, k, list(range(0, nodes.n, 37)))
    ratio = h / nodes.s
    assert 1.35 < ratio.mean() < 1.95


def test_stencil_optimisation_mixed_orders(dev):
    """Graded node set with orders 4, 6 and 10 in one launch."""
    nodes = inputs.graded_holes(20000, seed=3)
    h, k = _gpu_opt(nodes, dev)
    sample = []
    for m in (4, 6, 10):
        idx = np.nonzero(nodes.m == m)[0]
        sample += list(idx[:: max(1, idx.size // 6)][:6])
    _check_against_oracle(nodes, h, k, sample)


def test_optimised_stencils_in_use(dev):
    """65,536 nodes, m = 6: the optimised stencils hold fewer neighbours than
    the uniform h/s = 2.2 ones, every node's system is regular, and the
    operators stay accurate on a smooth field (smaller stencils trade some
    low-wavenumber accuracy for their modal response)."""
    from paper_2102_02019_amd import labfm

    nodes = inputs.TG256_M6.nodes()
    h, k = _gpu_opt(nodes, dev)
    x, y, s, m = (T(a, dev) for a in (nodes.x, nodes.y, nodes.s, nodes.m))
    rp0, _ = labfm.build_neighbours(x, y, T(nodes.h, dev), nodes.box)  # uniform 2.2 s
    rp1, col1 = labfm.build_neighbours(x, y, T(h, dev), nodes.box)
    K0 = rp0[-1].item() / nodes.n
    K1 = rp1[-1].item() / nodes.n
    assert K1 < 0.8 * K0, (K0, K1)
    ops = labfm.build_weights(x, y, T(h, dev), s, m, nodes.box, rp1, col1)
    assert int((ops.status != 0).sum().item()) == 0
    f = np.sin(nodes.x) * np.cos(2 * nodes.y)
    d = labfm.apply_operators(ops, T(f, dev), 0x07).cpu().numpy()
    ex = [np.cos(nodes.x) * np.cos(2 * nodes.y), -2 * np.sin(nodes.x) * np.sin(2 * nodes.y), -5 * f]
    for j in range(3):
        assert np.linalg.norm(d[j] - ex[j]) / np.linalg.norm(ex[j]) < 1e-6, j
