"""Pins of the oracle's basis functions against the paper's printed lists and
against library routines (CPU only)."""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite as nphermite
from scipy import special

from oracle import labfm_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "monomial_order.txt")


def _golden():
    entries, ns = [], {}
    for line in open(GOLDEN):
        line = line.strip()
        if line.startswith("# n "):
            _, _, m, n = line.split()
            ns[int(m)] = int(n)
        elif line and not line.startswith("#"):
            q, a, b, div = map(int, line.split())
            entries.append((q, a, b, div))
    return entries, ns


def test_monomial_order_matches_printed_vector():
    entries, _ = _golden()
    ex = O.monomial_exponents(4)
    for q, a, b, div in entries:
        assert ex[q] == (a, b)
        assert math.factorial(a) * math.factorial(b) == div
    # the vector ends with y^m / m!
    for m in (2, 4, 6, 8, 10):
        assert O.monomial_exponents(m)[-1] == (0, m)


def test_vector_length_formula():
    _, ns = _golden()
    for m, n in ns.items():
        assert O.n_moments(m) == n == len(O.monomial_exponents(m))


def test_taylor_monomials_values():
    rng = np.random.default_rng(0)
    xs, ys = rng.uniform(-2, 2, 7), rng.uniform(-2, 2, 7)
    X = O.taylor_monomials(xs, ys, 6)
    for q, (a, b) in enumerate(O.monomial_exponents(6)):
        ref = np.array([float(x) ** a * float(y) ** b for x, y in zip(xs, ys)])
        ref /= special.factorial(a) * special.factorial(b)
        np.testing.assert_allclose(X[:, q], ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("a", range(0, 11))
def test_hermite_matches_library(a):
    z = np.linspace(-2.5, 2.5, 41)
    c = np.zeros(a + 1)
    c[a] = 1.0
    ref_np = nphermite.hermval(z, c)
    ref_sp = special.eval_hermite(a, z)
    got = O.hermite_phys(a, z)
    scale = np.max(np.abs(ref_np)) + 1.0
    assert np.max(np.abs(got - ref_np)) <= 1e-13 * scale
    assert np.max(np.abs(got - ref_sp)) <= 1e-13 * scale


def test_hermite_abf_orthogonality_weight():
    """Hermite ABFs with psi = 1 reduce to products of physicists' Hermite
    polynomials, orthogonal under exp(-z^2) (Gauss-Hermite quadrature)."""
    z, wq = nphermite.hermgauss(30)
    for a in range(6):
        for b in range(6):
            s = np.sum(wq * O.hermite_phys(a, z) * O.hermite_phys(b, z))
            exact = math.sqrt(math.pi) * 2 ** a * math.factorial(a) if a == b else 0.0
            assert abs(s - exact) <= 1e-9 * max(1.0, exact)


def test_wendland_is_the_c2_compact_quintic():
    """psi is the unique degree-5 polynomial on [0,2) with a fourfold root at
    q=2 (C2 and compact), psi(0)=1 and psi'(0)=0 (smooth at the origin)."""
    q = np.linspace(0.0, 1.999, 400)
    coef = np.polynomial.polynomial.polyfit(q, O.wendland_c2(q), 7)
    # exact degree 5: higher coefficients vanish
    assert np.all(np.abs(coef[6:]) < 1e-9)
    p = np.polynomial.Polynomial(coef[:6])
    for k in range(4):
        assert abs(p.deriv(k)(2.0) if k else p(2.0)) < 1e-8
    assert abs(p(0.0) - 1.0) < 1e-12
    assert abs(p.deriv(1)(0.0)) < 1e-9
    # compact support and positivity inside it
    assert np.all(O.wendland_c2(np.array([2.0, 2.5, 10.0])) == 0.0)
    assert np.all(O.wendland_c2(q) > 0.0)


def test_hermite_abf_equals_probabilists_product():
    """W^q = psi He_a(x/h) He_b(y/h): the sqrt(2) scaling of the paper's
    physicists' form is the probabilists' Hermite polynomial."""
    rng = np.random.default_rng(1)
    xs, ys = rng.uniform(-1.5, 1.5, 50), rng.uniform(-1.5, 1.5, 50)
    W = O.hermite_abfs(xs, ys, 10)
    psi = O.wendland_c2(np.hypot(xs, ys))
    for q, (a, b) in enumerate(O.monomial_exponents(10)):
        ref = psi * special.eval_hermitenorm(a, xs) * special.eval_hermitenorm(b, ys)
        np.testing.assert_allclose(W[:, q], ref, rtol=1e-11, atol=1e-11)


def test_target_vectors():
    h = 0.37
    C = O.target_vectors(6, h)
    ex = O.monomial_exponents(6)
    idx = {ab: q for q, ab in enumerate(ex)}
    # x, y, L as printed (before scaling), scaled by h^-(a+b)
    assert C[idx[(1, 0)], O.OP_X] == pytest.approx(1 / h)
    assert C[idx[(0, 1)], O.OP_Y] == pytest.approx(1 / h)
    assert C[idx[(2, 0)], O.OP_L] == pytest.approx(h ** -2)
    assert C[idx[(0, 2)], O.OP_L] == pytest.approx(h ** -2)
    assert np.count_nonzero(C[:, O.OP_L]) == 2
    # nabla^6 = d6x + 3 d4x d2y + 3 d2x d4y + d6y
    hyp = {ab: C[q, O.OP_HYP] * h ** 6 for ab, q in idx.items() if C[q, O.OP_HYP] != 0}
    assert hyp == pytest.approx({(6, 0): 1, (4, 2): 3, (2, 4): 3, (0, 6): 1})
    # odd m uses nabla^(m-1)
    C5 = O.target_vectors(5, 1.0)
    idx5 = {ab: q for q, ab in enumerate(O.monomial_exponents(5))}
    assert C5[idx5[(4, 0)], O.OP_HYP] == 1 and C5[idx5[(2, 2)], O.OP_HYP] == 2
