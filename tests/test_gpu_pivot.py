"""The weight build's LU on given systems (labfm_solve_systems: the
rows-in-registers kernel's pivot search, elimination and back substitution
run on caller-supplied [M~ | C~] in place of the systems it assembles).

Partial pivoting takes the largest |entry| of the column (section "The Local
Anisotropic Basis Function Method": each node's system is solved by LU with
partial pivoting). The candidates here differ only in their lowest mantissa
bits, fewer than 128 units in the last place apart, so a comparison of
truncated magnitudes would call them equal: the kernel must still take the
larger one, and the lowest row only when the magnitudes are equal. The
solutions are checked against numpy.linalg.solve, and on dense systems the
pivot sequence against LAPACK's (scipy.linalg.lu_factor)."""
import numpy as np
import pytest
import scipy.linalg
import torch

pytestmark = pytest.mark.gpu

ORDERS = list(range(1, 11))


def moments(m):
    return (m * m + 3 * m) // 2


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_02019_amd import labfm

    labfm.lib()
    return torch.device("cuda:0")


def _ulps_apart(x, k):
    """|x| moved up by k units in the last place, with x's sign."""
    b = np.array([abs(x)], dtype=np.float64).view(np.uint64) + np.uint64(k)
    return float(np.copysign(b.view(np.float64)[0], x))


def block_system(n, rng, first_rows=None):
    """[A | C] whose columns pair up (2b, 2b+1) on two rows each (a lone
    last column when n is odd); every other entry of those columns is an
    exact zero, so column 2b's candidates are exactly its two given
    entries. Returns the system and the expected pivot row of each column:
    the larger magnitude, the lower row on a tie."""
    rows = rng.permutation(n)
    if first_rows is not None:  # the rows of block 0 chosen by the caller
        rest = [r for r in rows if r not in first_rows]
        rows = np.array(list(first_rows) + rest)
    A = np.zeros((n, n))
    piv = np.empty(n, dtype=np.int64)
    kinds = []
    for b in range(n // 2):
        r1, r2 = int(rows[2 * b]), int(rows[2 * b + 1])
        x = rng.uniform(0.5, 2.0) * rng.choice([-1.0, 1.0])
        kind = ("near", "tie", "far")[b % 3]
        if kind == "near":
            y = _ulps_apart(x, int(rng.integers(1, 100))) * rng.choice([-1.0, 1.0])
        elif kind == "tie":
            y = -x if rng.random() < 0.5 else x
        else:
            y = rng.uniform(0.5, 2.0) * rng.choice([-1.0, 1.0])
        if rng.random() < 0.5:
            x, y = y, x
        A[r1, 2 * b], A[r2, 2 * b] = x, y
        if abs(x) > abs(y):
            p, o = r1, r2
        elif abs(y) > abs(x):
            p, o = r2, r1
        else:
            p, o = min(r1, r2), max(r1, r2)
        # second column: the other row keeps a large entry after elimination
        while True:
            bp, bo = rng.uniform(-1.0, 1.0, 2)
            if abs(bo - A[o, 2 * b] / A[p, 2 * b] * bp) > 0.5:
                break
        A[p, 2 * b + 1], A[o, 2 * b + 1] = bp, bo
        piv[2 * b], piv[2 * b + 1] = p, o
        kinds.append(kind)
    if n % 2:
        r = int(rows[n - 1])
        A[r, n - 1] = rng.uniform(0.5, 2.0)
        piv[n - 1] = r
    C = rng.standard_normal((n, 6))
    return np.hstack([A, C]), piv, kinds


def _solve(m, systems, dev):
    from paper_2102_02019_amd import labfm

    psi, piv, st = labfm.solve_systems(m, torch.from_numpy(np.ascontiguousarray(systems)).to(dev))
    torch.cuda.synchronize()
    return psi.cpu().numpy(), piv.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("m", ORDERS)
def test_pivots_of_near_ties_and_ties(dev, m):
    """Near ties (1-99 ulps), exact ties and separated pairs in every block:
    each column's pivot is the row the rule names; Psi matches numpy."""
    n = moments(m)
    rng = np.random.default_rng(100 + m)
    systems, expect = [], []
    for _ in range(24):
        S, piv, _ = block_system(n, rng)
        systems.append(S)
        expect.append(piv)
    psi, piv, st = _solve(m, np.stack(systems), dev)
    assert (st == 0).all()
    np.testing.assert_array_equal(piv, np.stack(expect))
    for k, S in enumerate(systems):
        ref = np.linalg.solve(S[:, :n], S[:, n:])
        err = np.abs(psi[k] - ref).max() / np.abs(ref).max()
        assert err <= 1e-14, (m, k, err)


def test_order10_first_pivot_against_row_64(dev):
    """Order 10 (65 rows, one beyond the wavefront): the first column's pivot
    is chosen among lanes 0..63 and the extra row 64; row 64 wins only when
    strictly larger, a near tie or a tie with a lower row goes by the rule."""
    m, n = 10, 65
    rng = np.random.default_rng(7)
    systems, expect = [], []
    for low in (0, 17, 63):
        for _ in range(6):
            S, piv, _ = block_system(n, rng, first_rows=(low, 64))
            systems.append(S)
            expect.append(piv)
    assert any(e[0] == 64 for e in expect) and any(e[0] != 64 for e in expect)
    psi, piv, st = _solve(m, np.stack(systems), dev)
    assert (st == 0).all()
    np.testing.assert_array_equal(piv, np.stack(expect))
    for k, S in enumerate(systems):
        ref = np.linalg.solve(S[:, :n], S[:, n:])
        assert np.abs(psi[k] - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("m", [2, 5, 8, 9, 10])
def test_dense_systems_match_lapack(dev, m):
    """Dense random systems: the pivot sequence equals LAPACK's (rows as
    given), Psi matches numpy.linalg.solve within the LU's forward error
    bound, and the residual is at rounding level."""
    n = moments(m)
    rng = np.random.default_rng(200 + m)
    systems = rng.standard_normal((16, n, n + 6))
    psi, piv, st = _solve(m, systems, dev)
    assert (st == 0).all()
    eps = np.finfo(np.float64).eps
    for k in range(len(systems)):
        A, C = systems[k][:, :n], systems[k][:, n:]
        _, ipiv = scipy.linalg.lu_factor(A)
        order = np.arange(n)
        for c in range(n):
            order[[c, ipiv[c]]] = order[[ipiv[c], c]]
        np.testing.assert_array_equal(piv[k], order, err_msg=f"m={m} system {k}")
        ref = np.linalg.solve(A, C)
        cond = np.linalg.cond(A)
        fwd = np.abs(psi[k] - ref).max() / np.abs(ref).max()
        assert fwd <= 10 * n * cond * eps, (m, k, fwd, cond)
        res = np.abs(A @ psi[k] - C).max() / (np.abs(A).max() * np.abs(psi[k]).max())
        assert res <= 10 * n * eps, (m, k, res)


def test_singular_systems_are_flagged(dev):
    """A zero column makes its system singular (status set, nothing
    written); the other systems of the call are solved as usual."""
    m, n = 6, moments(6)
    rng = np.random.default_rng(3)
    systems = rng.standard_normal((3, n, n + 6))
    systems[1][:, 4] = 0.0
    psi, piv, st = _solve(m, systems, dev)
    assert list(st) == [0, 1, 0]
    assert (piv[1] == -1).all() and (psi[1] == 0.0).all()
    for k in (0, 2):
        ref = np.linalg.solve(systems[k][:, :n], systems[k][:, n:])
        assert np.abs(psi[k] - ref).max() <= 1e-10 * np.abs(ref).max()
