"""Pins of the oracle's per-cell steps: interpolation (Sec. 3.1, Alg. 1-2,
Eq. 3) and evolution (Sec. 3.2, Alg. 3-4, and the multi-stage variant).

Independent references used here:
  * numpy's polynomial derivative/evaluation routines (corner data of a known
    tensor polynomial) - the interpolant of a polynomial of per-axis degree
    <= 2m+1 is that polynomial;
  * d'Alembert plane waves f(k.xi - lam*sigma), exact solutions of the wave
    equation for any polynomial f, expanded by the multinomial theorem;
  * harmonic polynomials (Lap = 0), which must stay fixed or drift linearly;
  * scipy's matrix exponential of the system operator, with the Laplacian
    taken by numpy's polyder, for the exact solution operator on random data;
  * for RK4: the algebraic identity with the 4-term Taylor series at one
    substep, and convergence to the exact operator as substeps grow.
"""
import math

import numpy as np
import pytest
import scipy.linalg
from numpy.polynomial import polynomial as npoly


def _corner_data(b: np.ndarray, m: int) -> np.ndarray:
    """uloc[a3][a2][a1] of the tensor polynomial sum b[j3,j2,j1] xi3^j3 xi2^j2 xi1^j1
    with a = side*(m+1) + d, side 0 at xi = -1/2. numpy's polyval3d(x, y, z, c)
    uses c[i, j, k] x^i y^j z^k, so x = xi3, y = xi2, z = xi1."""
    M, P = m + 1, 2 * m + 2
    uloc = np.zeros((P, P, P))
    for d3 in range(M):
        for d2 in range(M):
            for d1 in range(M):
                c = b
                c = npoly.polyder(c, m=d3, axis=0) if d3 else c
                c = npoly.polyder(c, m=d2, axis=1) if d2 else c
                c = npoly.polyder(c, m=d1, axis=2) if d1 else c
                scale = 1.0 / (math.factorial(d1) * math.factorial(d2) * math.factorial(d3))
                for s3 in range(2):
                    for s2 in range(2):
                        for s1 in range(2):
                            x3, x2, x1 = s3 - 0.5, s2 - 0.5, s1 - 0.5
                            uloc[s3 * M + d3, s2 * M + d2, s1 * M + d1] = scale * npoly.polyval3d(x3, x2, x1, c)
    return uloc


@pytest.mark.parametrize("m", [1, 2, 3])
def test_interpolation_reproduces_tensor_polynomials(oracle_mod, m):
    P = 2 * m + 2
    rng = np.random.default_rng(7 + m)
    for _ in range(3):
        b = rng.standard_normal((P, P, P))
        R = oracle_mod.interpolate_cell(m, _corner_data(b, m))
        # rounding of the corner data is amplified by up to ||H||_inf^3
        # (about 3.8e5 for m = 3); a wrong sign or index gives O(1) errors
        tol = 1e-12 if m < 3 else 2e-11
        assert np.abs(R - b).max() <= tol * np.abs(b).max()


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_interpolation_is_sharp(oracle_mod, m, axis):
    # one degree too many along one axis is not reproduced
    P = 2 * m + 2
    shape = [P, P, P]
    shape[axis] = P + 1
    b = np.zeros(shape)
    idx = [0, 0, 0]
    idx[axis] = P
    b[tuple(idx)] = 1.0
    R = oracle_mod.interpolate_cell(m, _corner_data(b, m))
    trunc = b[:P, :P, :P]
    assert np.abs(R - trunc).max() > 1e-3


def _linear_form_power(kvec, p, P):
    """Coefficient tensor [j3, j2, j1] of (k1 xi1 + k2 xi2 + k3 xi3)^p by the
    multinomial theorem."""
    T = np.zeros((P, P, P))
    k1, k2, k3 = kvec
    for a in range(p + 1):
        for bb in range(p + 1 - a):
            c = p - a - bb
            if a < P and bb < P and c < P:
                T[c, bb, a] += math.factorial(p) / (math.factorial(a) * math.factorial(bb) * math.factorial(c)) \
                    * k1 ** a * k2 ** bb * k3 ** c
    return T


def _plane_wave(kvec, f_coef, P):
    """Coefficient tensor of f(k.xi) for a 1D polynomial f."""
    T = np.zeros((P, P, P))
    for p, fp in enumerate(f_coef):
        if fp != 0:
            T += fp * _linear_form_power(kvec, p, P)
    return T


@pytest.mark.parametrize("m", [1, 2, 3])
def test_taylor_evolution_exact_on_plane_waves(oracle_mod, m):
    """u = f(k.xi - lam sigma) + g(k'.xi + lam sigma) with |k| = |k'| = 1 solves
    u_sigma = lam vt, vt_sigma = lam Lap u, vt = -f'(..) + g'(..)."""
    P = 2 * m + 2
    lam = 0.25
    rng = np.random.default_rng(30 + m)
    for _ in range(4):
        k = rng.standard_normal(3)
        k /= np.linalg.norm(k)
        k2 = rng.standard_normal(3)
        k2 /= np.linalg.norm(k2)
        f = npoly.Polynomial(rng.standard_normal(P))
        g = npoly.Polynomial(rng.standard_normal(P))
        Ru = _plane_wave(k, f.coef, P) + _plane_wave(k2, g.coef, P)
        Rv = _plane_wave(k, -f.deriv().coef, P) + _plane_wave(k2, g.deriv().coef, P)
        fs = f(npoly.Polynomial([-lam, 1.0]))   # f(s - lam)
        gs = g(npoly.Polynomial([lam, 1.0]))    # g(s + lam)
        Eu = _plane_wave(k, fs.coef, P) + _plane_wave(k2, gs.coef, P)
        Ev = _plane_wave(k, -fs.deriv().coef, P) + _plane_wave(k2, gs.deriv().coef, P)
        Wu, Wv = oracle_mod.evolve_taylor(m, oracle_mod.exact_q(m), lam, Ru, Rv)
        scale = max(np.abs(Eu).max(), np.abs(Ev).max())
        assert np.abs(Wu - Eu).max() <= 1e-12 * scale
        assert np.abs(Wv - Ev).max() <= 1e-12 * scale


@pytest.mark.parametrize("m", [2, 3])
def test_taylor_evolution_on_harmonic_polynomials(oracle_mod, m):
    """Re((xi1 + i xi2)^(2m+1)) * xi3 is harmonic: as u it stays fixed and as
    vt it makes u grow by lam * sigma * (that polynomial)."""
    P = 2 * m + 2
    p = 2 * m + 1
    T = np.zeros((P, P, P))
    for a in range(p + 1):
        # Re of C(p,a) xi1^a (i xi2)^(p-a): i^(p-a) real when p-a even
        e = p - a
        if e % 2 == 0:
            T[1, e, a] = math.comb(p, a) * (-1) ** (e // 2)
    lam = 0.25
    Wu, Wv = oracle_mod.evolve_taylor(m, oracle_mod.exact_q(m), lam, T, np.zeros_like(T))
    assert np.array_equal(Wu, T) and np.abs(Wv).max() == 0.0
    Wu, Wv = oracle_mod.evolve_taylor(m, oracle_mod.exact_q(m), lam, np.zeros_like(T), T)
    assert np.allclose(Wu, lam * T, rtol=0, atol=1e-13 * np.abs(T).max())
    assert np.allclose(Wv, T, rtol=0, atol=1e-13 * np.abs(T).max())


def _system_matrix(m, lam):
    """L = lam * [[0, I], [Lap, 0]] on the 2 P^3 coefficient space, with Lap
    built from numpy's polyder (coefficients ordered [j3, j2, j1])."""
    P = 2 * m + 2
    n = P ** 3
    Lap = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        E = e.reshape(P, P, P)
        out = np.zeros((P, P, P))
        for axis in range(3):
            d = npoly.polyder(E, m=2, axis=axis)
            pad = [(0, 0)] * 3
            pad[axis] = (0, 2)
            out += np.pad(d, pad)
        Lap[:, col] = out.ravel()
    L = np.zeros((2 * n, 2 * n))
    L[:n, n:] = lam * np.eye(n)
    L[n:, :n] = lam * Lap
    return L


@pytest.mark.parametrize("m", [1, 2, 3])
def test_taylor_exact_q_equals_matrix_exponential(oracle_mod, m):
    P = 2 * m + 2
    lam = 0.25
    L = _system_matrix(m, lam)
    E = scipy.linalg.expm(L)
    rng = np.random.default_rng(50 + m)
    Ru = rng.standard_normal((P, P, P))
    Rv = rng.standard_normal((P, P, P))
    ref = E @ np.concatenate([Ru.ravel(), Rv.ravel()])
    Wu, Wv = oracle_mod.evolve_taylor(m, oracle_mod.exact_q(m), lam, Ru, Rv)
    got = np.concatenate([Wu.ravel(), Wv.ravel()])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("m", [1, 2, 3])
def test_system_operator_nilpotency_index(oracle_mod, m):
    """Lap^(3m+1) = 0 and Lap^(3m) != 0 on degree <= 2m+1 per axis, hence
    L^(6m+2) = 0 and L^(6m+1) != 0: q = 6m+1 Taylor stages are exact and more
    stages change nothing beyond rounding."""
    P = 2 * m + 2
    rng = np.random.default_rng(60 + m)
    W = rng.standard_normal((P, P, P))
    for _ in range(3 * m):
        W = oracle_mod.laplacian(m, W)
    assert np.abs(W).max() > 1.0
    W = oracle_mod.laplacian(m, W)
    assert np.abs(W).max() == 0.0
    Ru, Rv = rng.standard_normal((P, P, P)), rng.standard_normal((P, P, P))
    a = oracle_mod.evolve_taylor(m, 6 * m + 1, 0.25, Ru, Rv)
    b = oracle_mod.evolve_taylor(m, 6 * m + 3, 0.25, Ru, Rv)   # the paper's d(2m+1) stages
    s = np.abs(a[0]).max()
    assert np.abs(a[0] - b[0]).max() <= 1e-13 * s and np.abs(a[1] - b[1]).max() <= 1e-13 * s
    # at lam = 1 the last stage is visible above rounding
    a = oracle_mod.evolve_taylor(m, 6 * m + 1, 1.0, Ru, Rv)
    c = oracle_mod.evolve_taylor(m, 6 * m, 1.0, Ru, Rv)
    s = np.abs(a[0]).max()
    # L^(6m+1) (Ru, Rv) = lam^(6m+1) (Lap^(3m) Rv, 0): the last stage reaches u only
    assert np.abs(a[0] - c[0]).max() > 1e-12 * s


@pytest.mark.parametrize("m", [1, 2, 3])
def test_rk4_one_substep_is_four_term_taylor(oracle_mod, m):
    # classical RK4 applied to a linear autonomous ODE is its degree-4 Taylor polynomial
    P = 2 * m + 2
    rng = np.random.default_rng(70 + m)
    Ru, Rv = rng.standard_normal((P, P, P)), rng.standard_normal((P, P, P))
    a = oracle_mod.evolve_rk4(m, 1, 0.25, Ru, Rv)
    b = oracle_mod.evolve_taylor(m, 4, 0.25, Ru, Rv)
    s = max(np.abs(b[0]).max(), np.abs(b[1]).max())
    assert np.abs(a[0] - b[0]).max() <= 1e-13 * s and np.abs(a[1] - b[1]).max() <= 1e-13 * s


@pytest.mark.parametrize("m", [1, 3])
def test_rk4_converges_to_exact_operator_at_fourth_order(oracle_mod, m):
    P = 2 * m + 2
    lam = 0.25
    rng = np.random.default_rng(80 + m)
    Ru, Rv = rng.standard_normal((P, P, P)), rng.standard_normal((P, P, P))
    ex = oracle_mod.evolve_taylor(m, 6 * m + 1, lam, Ru, Rv)
    errs = []
    for S in (2, 4, 8):
        a = oracle_mod.evolve_rk4(m, S, lam, Ru, Rv)
        errs.append(max(np.abs(a[0] - ex[0]).max(), np.abs(a[1] - ex[1]).max()))
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 3.5 < r1 < 4.8 and 3.5 < r2 < 4.8, (errs, r1, r2)
