"""Pins of the oracle's stencil search (the stencil definition of the paper's
LABFM section: all j with |r_ji| <= 2 h_i) against a pure-Python pair loop."""
import math

import numpy as np

from oracle import labfm_oracle as O
from paper_2102_02019_amd import inputs


def _python_pairs(x, y, h, box):
    """Every pair tested with Python floats (IEEE double, each operation
    rounded on its own), nearest periodic image taken explicitly."""
    n = len(x)
    out = []
    for i in range(n):
        row = []
        for j in range(n):
            if j == i:
                continue
            dx = float(x[j]) - float(x[i])
            dy = float(y[j]) - float(y[i])
            if box.periodic_x:
                if dx > 0.5 * box.Lx:
                    dx -= box.Lx
                elif dx < -0.5 * box.Lx:
                    dx += box.Lx
            if box.periodic_y:
                if dy > 0.5 * box.Ly:
                    dy -= box.Ly
                elif dy < -0.5 * box.Ly:
                    dy += box.Ly
            r = 2.0 * float(h[i])
            if dx * dx + dy * dy <= r * r:
                row.append(j)
        out.append(row)
    return out


def _csr_rows(rp, col):
    return [list(col[rp[i]:rp[i + 1]]) for i in range(rp.size - 1)]


def test_bruteforce_matches_python_pairs_random_cloud():
    x, y, box = inputs.random_cloud(300, L=1.0, seed=3)
    h = np.random.default_rng(4).uniform(0.02, 0.08, 300)
    rp, col = O.neighbours_bruteforce(x, y, h, box)
    assert _csr_rows(rp, col) == _python_pairs(x, y, h, box)


def test_bruteforce_matches_python_pairs_nonperiodic():
    x, y, box = inputs.random_cloud(250, L=1.0, seed=5, periodic=False)
    h = np.full(250, 0.06)
    rp, col = O.neighbours_bruteforce(x, y, h, box)
    assert _csr_rows(rp, col) == _python_pairs(x, y, h, box)


def test_tree_path_matches_bruteforce():
    nodes = inputs.jittered_lattice(72, seed=7, m=6)  # 5184 nodes > 4096
    rp1, col1 = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
    # force the pairwise path on the same arrays
    rp2, col2 = O.neighbours_bruteforce(nodes.x, nodes.y, nodes.h, nodes.box)
    assert np.array_equal(rp1, rp2) and np.array_equal(col1, col2)


def test_row_ranges_match_bruteforce():
    """Rows computed a range at a time (as when a large node set is split over
    processes) are the brute-force rows, and the other rows stay empty."""
    nodes = inputs.jittered_lattice(40, seed=9, m=8)
    rp2, col2 = O.neighbours_bruteforce(nodes.x, nodes.y, nodes.h, nodes.box)
    for a, b in ((0, 1), (100, 517), (1590, nodes.n)):
        rp, col = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box, nodes=range(a, b))
        assert np.all(np.diff(rp)[:a] == 0) and np.all(np.diff(rp)[b:] == 0)
        for i in range(a, b):
            assert np.array_equal(col[rp[i]:rp[i + 1]], col2[rp2[i]:rp2[i + 1]]), i


def test_periodic_wrap_and_tie_included():
    # four points: a corner pair that only touch through both periodic edges,
    # and a pair at exactly 2h (0.5 = 2 * 0.25, all exactly representable)
    x = np.array([0.01, 0.99, 0.25, 0.75])
    y = np.array([0.01, 0.99, 0.5, 0.5])
    h = np.array([0.02, 0.02, 0.25, 0.25])
    box = inputs.Box(1.0, 1.0, True, True)
    rp, col = O.neighbours_bruteforce(x, y, h, box)
    rows = _csr_rows(rp, col)
    assert rows[0] == [1] and rows[1] == [0]
    assert rows[2] == [3] and rows[3] == [2]
    # without periodicity the corner pair is far apart
    rp, col = O.neighbours_bruteforce(x, y, h, inputs.Box(1.0, 1.0, False, False))
    assert _csr_rows(rp, col)[0] == []


def test_lattice_population():
    """On the +/-0.3 s jittered lattice the stencil sizes are those the
    workloads were chosen for (~4 pi (h/s)^2 in the paper's estimate)."""
    for m, lo, hi in ((4, 26, 33), (6, 57, 64), (8, 86, 94)):
        nodes = inputs.jittered_lattice(48, seed=11, m=m)
        rp, _ = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
        k = np.diff(rp).mean()
        assert lo < k < hi


def test_rows_of_listed_nodes_match_full_search():
    """The per-row search used for sampled checks of large node sets gives
    the same rows as the full search; unlisted rows are empty."""
    x, y, box = inputs.random_cloud(3000, L=1.0, seed=7)
    h = np.full(x.size, 0.02) * (1.0 + 0.5 * np.sin(7 * x))
    rp, col = O.neighbours(x, y, h, box)
    sample = [0, 17, 1500, 2999]
    rp2, col2 = O.neighbours_rows(x, y, h, box, sample)
    for i in range(x.size):
        got = col2[rp2[i]:rp2[i + 1]]
        if i in sample:
            assert np.array_equal(got, col[rp[i]:rp[i + 1]])
        else:
            assert got.size == 0


# ---------------------------------------------------------------------------
# Morton binning
# ---------------------------------------------------------------------------

def _z_less(p, q):
    """Z-order comparison without interleaving (the dimension whose
    coordinates differ in the highest bit decides; at equal bit levels y is
    the more significant, as it sits above x in the interleaved key)."""
    def less_msb(a, b):
        return a < b and a < (a ^ b)

    j, best = 1, 0
    for d in (1, 0):
        v = p[d] ^ q[d]
        if less_msb(best, v):
            j, best = d, v
    return (p[j] > q[j]) - (p[j] < q[j])


def test_morton_permutation_against_a_z_order_comparator():
    import functools

    from paper_2102_02019_amd import inputs as I

    rng = np.random.default_rng(3)
    for trial in range(4):
        n = 300
        x = rng.uniform(0.0, 1.0, n)
        y = rng.uniform(0.0, 0.7, n)
        box = I.Box(1.0, 0.7, True, True)
        cell = [0.013, 0.05, 0.1, 0.33][trial]
        perm = O.morton_permutation(x, y, box, cell)
        ncx, ncy = math.ceil(1.0 / cell), math.ceil(0.7 / cell)
        cells = [(min(int(math.floor(x[i] / cell)), ncx - 1), min(int(math.floor(y[i] / cell)), ncy - 1))
                 for i in range(n)]
        ref = sorted(range(n), key=functools.cmp_to_key(
            lambda a, b: _z_less(cells[a], cells[b]) or (a > b) - (a < b)))
        assert list(perm) == ref


def test_morton_permutation_of_the_lattice_is_the_generators_order():
    """The jittered lattice leaves its generator in the Z-order of its lattice
    cells; re-binning the (unjittered) cell centres reproduces that order."""
    from paper_2102_02019_amd import inputs as I

    nodes = I.jittered_lattice(32, L=1.0, jitter=0.0, seed=1, m=4, morton=False)
    perm = O.morton_permutation(nodes.x, nodes.y, nodes.box, 1.0 / 32)
    ordered = I.jittered_lattice(32, L=1.0, jitter=0.0, seed=1, m=4, morton=True)
    assert np.array_equal(nodes.x[perm], ordered.x) and np.array_equal(nodes.y[perm], ordered.y)
