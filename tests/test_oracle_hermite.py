"""Pins of the oracle's 1D Hermite matrix H (Sec. 3.1; interpolant of Eq. 3).

H maps the scaled derivatives [L0..Lm, R0..Rm] at xi = -1/2, +1/2 to the
monomial coefficients b_0..b_{2m+1} of the interpolating polynomial about the
cell centre. The pins do not reuse the oracle's construction:
  * an exact-rational brute-force solve of the interpolation system,
  * the textbook cubic Hermite basis (m = 1),
  * reproduction of random polynomials, with derivatives taken by numpy's
    polynomial routines, and failure one degree above 2m+1.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import Polynomial

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hermite_matrices.txt")


@pytest.mark.parametrize("m", [1, 2, 3])
def test_H_matches_exact_rational_solve_bitwise(oracle_mod, m):
    H = oracle_mod.hermite_matrix(m)
    E = np.array([[float(v) for v in row] for row in oracle_mod.exact_hermite_matrix(m)])
    assert np.array_equal(H, E)


def test_H_m4_within_rounding(oracle_mod):
    # m = 4 has entries with more significant bits; long-double elimination
    # leaves a few units of rounding there (m = 4 is outside the library's range)
    H = oracle_mod.hermite_matrix(4)
    E = np.array([[float(v) for v in row] for row in oracle_mod.exact_hermite_matrix(4)])
    assert np.abs(H - E).max() <= 1e-15 * np.abs(E).max()


def test_H_m1_equals_textbook_cubic_hermite(oracle_mod):
    # Cubic Hermite basis on t in [0, 1]: value/slope at t = 0 and t = 1.
    h00 = Polynomial([1, 0, -3, 2])
    h10 = Polynomial([0, 1, -2, 1])
    h01 = Polynomial([0, 0, 3, -2])
    h11 = Polynomial([0, 0, -1, 1])
    t_of_xi = Polynomial([0.5, 1.0])  # t = xi + 1/2, and d/dt = d/dxi
    cols = [h(t_of_xi).coef for h in (h00, h10, h01, h11)]
    expect = np.zeros((4, 4))
    for c, coef in enumerate(cols):
        expect[: len(coef), c] = coef
    assert np.array_equal(oracle_mod.hermite_matrix(1), expect)


def _taylor_at(poly: Polynomial, x: float, m: int):
    return [poly.deriv(k)(x) / math.factorial(k) if k else poly(x) for k in range(m + 1)]


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_H_reproduces_polynomials_of_degree_2m_plus_1(oracle_mod, m):
    rng = np.random.default_rng(100 + m)
    H = oracle_mod.hermite_matrix(m)
    P = 2 * m + 2
    for _ in range(20):
        b = rng.standard_normal(P)
        p = Polynomial(b)
        data = np.array(_taylor_at(p, -0.5, m) + _taylor_at(p, 0.5, m))
        assert np.allclose(H @ data, b, rtol=0, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("m", [1, 2, 3])
def test_H_fails_one_degree_higher(oracle_mod, m):
    # the interpolant is unique among degree <= 2m+1; xi^(2m+2) is not reproduced
    H = oracle_mod.hermite_matrix(m)
    P = 2 * m + 2
    p = Polynomial([0] * P + [1.0])
    data = np.array(_taylor_at(p, -0.5, m) + _taylor_at(p, 0.5, m))
    b = H @ data
    assert np.abs(b).max() > 1e-3
    # and the interpolant differs from xi^(2m+2) inside the cell
    xs = np.linspace(-0.4, 0.4, 9)
    assert np.abs(Polynomial(b)(xs) - p(xs)).max() > 1e-4


@pytest.mark.parametrize("m", [1, 2, 3])
def test_H_matches_golden_fixture(oracle_mod, m):
    """tests/golden/hermite_matrices.txt is written by
    tests/golden/make_golden.py from the exact-rational oracle routine."""
    rows = {}
    with open(GOLDEN) as fh:
        cur = None
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("m="):
                cur = int(line[2:])
                rows[cur] = []
            else:
                rows[cur].append([Fraction(v) for v in line.split()])
    G = np.array([[float(v) for v in r] for r in rows[m]])
    assert np.array_equal(oracle_mod.hermite_matrix(m), G)
