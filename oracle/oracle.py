"""Python side of the CPU oracle (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's ``cpu_baseline`` leg may
import this module. It loads ``liboracle.so`` built from ``hermite_oracle.c``
with gcc, and adds an exact-rational construction of the 1D Hermite matrix.

Citations refer to Vargas, Chan, Hagstrom, Warburton, "GPU Acceleration of
Hermite Methods for the Simulation of Wave Propagation" (arXiv:1609.09841).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hermite_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_LD_PATH = os.path.join(_HERE, "liboracle_ld.so")
_lib = None
_lib_ld = None

__all__ = [
    "build_oracle", "load", "exact_hermite_matrix", "hermite_matrix",
    "interpolate_cell", "laplacian", "evolve_taylor", "evolve_rk4",
    "gather_cell", "half_step", "run", "point", "point_box", "exact_q",
    "gauss_taylor", "ricker_taylor", "evolve_taylor_forced", "run_forced",
    "advection_q", "evolve_advection", "run_advection",
    "adjoint_half_step", "source_term", "run_series", "adjoint_series",
]


def build_oracle(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, no fast-math), and its
    long-double twin used only to measure the FP64 rounding floor."""
    for path, extra in ((_LIB_PATH, []), (_LIB_LD_PATH, ["-DORACLE_REAL=long double"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                   "-ffp-contract=off", *extra, "-o", tmp, _SRC, "-lm"]
            subprocess.check_call(cmd)
            os.replace(tmp, path)
    return _LIB_PATH


def load(ld: bool = False):
    """The FP64 oracle library, or (ld=True) its long-double twin."""
    global _lib, _lib_ld
    if (_lib_ld if ld else _lib) is not None:
        return _lib_ld if ld else _lib
    path = _LIB_LD_PATH if ld else _LIB_PATH
    if not os.path.exists(path):
        build_oracle(force=True)
    lib = ctypes.CDLL(path)
    real = ctypes.c_longdouble if ld else ctypes.c_double
    dp = ctypes.POINTER(real)
    i, d = ctypes.c_int, real
    lib.oracle_hermite_matrix.argtypes = [i, dp]
    lib.oracle_hermite_matrix.restype = i
    lib.oracle_interpolate_cell.argtypes = [i, dp, dp, dp]
    lib.oracle_interpolate_cell.restype = None
    lib.oracle_laplacian.argtypes = [i, dp, dp]
    lib.oracle_laplacian.restype = None
    lib.oracle_evolve_taylor.argtypes = [i, i, d, dp, dp]
    lib.oracle_evolve_taylor.restype = None
    lib.oracle_evolve_rk4.argtypes = [i, i, d, dp, dp]
    lib.oracle_evolve_rk4.restype = None
    lib.oracle_gather_cell.argtypes = [i, i, dp, i, i, i, dp]
    lib.oracle_gather_cell.restype = None
    lib.oracle_half_step.argtypes = [i, i, dp, d, i, i, dp, dp, i]
    lib.oracle_half_step.restype = None
    lib.oracle_run.argtypes = [i, i, d, d, i, i, i, dp, dp]
    lib.oracle_run.restype = i
    lib.oracle_point.argtypes = [i, i, d, d, i, i, i, dp, dp, i, i, i, dp]
    lib.oracle_point.restype = i
    lib.oracle_point_box.argtypes = [i, i, d, d, i, i, i, dp, dp, dp]
    lib.oracle_point_box.restype = i
    lib.oracle_gauss_taylor.argtypes = [d, d, d, i, dp]
    lib.oracle_gauss_taylor.restype = i
    lib.oracle_ricker_taylor.argtypes = [d, d, d, d, i, dp]
    lib.oracle_ricker_taylor.restype = i
    lib.oracle_evolve_taylor_forced.argtypes = [i, i, d, dp, dp, dp, dp]
    lib.oracle_evolve_taylor_forced.restype = None
    lib.oracle_run_forced.argtypes = [i, i, d, d, i, i, dp, dp, dp, d, d, d, d]
    lib.oracle_run_forced.restype = i
    lib.oracle_evolve_advection.argtypes = [i, i, d, dp]
    lib.oracle_evolve_advection.restype = None
    lib.oracle_half_step_advection.argtypes = [i, i, dp, d, i, dp, dp, i]
    lib.oracle_half_step_advection.restype = None
    lib.oracle_run_advection.argtypes = [i, i, d, d, i, i, dp]
    lib.oracle_run_advection.restype = i
    lib.oracle_evolve_taylor_T.argtypes = [i, i, d, dp, dp]
    lib.oracle_evolve_taylor_T.restype = None
    lib.oracle_interpolate_cell_T.argtypes = [i, dp, dp, dp]
    lib.oracle_interpolate_cell_T.restype = None
    lib.oracle_adjoint_half_step.argtypes = [i, i, dp, d, i, dp, dp, i]
    lib.oracle_adjoint_half_step.restype = None
    lib.oracle_source_term.argtypes = [i, i, d, d, i, i, d, dp, d, d, d, d, dp]
    lib.oracle_source_term.restype = i
    if ld:
        _lib_ld = lib
    else:
        _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.longdouble and np.longdouble != np.float64:
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble))
    assert a.dtype == np.float64
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def exact_q(m: int) -> int:
    """Stage count at which the Taylor series of the wave system is exact on
    the cell space: each axis absorbs at most m second derivatives of a
    degree-(2m+1) polynomial, so Lap^(3m+1) = 0 and L^(6m+2) = 0."""
    return 6 * m + 1


def exact_hermite_matrix(m: int) -> list[list[Fraction]]:
    """Brute-force exact solve of the 1D two-point Hermite interpolation system.

    Unknowns: monomial coefficients b_0..b_{2m+1} of p(xi) about the cell
    centre. Equations: the k-th Taylor coefficient of p at xi = -1/2 and at
    xi = +1/2 equals the given scaled derivative (Sec. 2, Eq. 2-3). Solved by
    Gauss-Jordan elimination over the rationals; returns H with b = H @ data,
    data ordered [L0..Lm, R0..Rm].
    """
    M, P = m + 1, 2 * m + 2
    half = Fraction(1, 2)
    rows = []
    for side in (0, 1):
        x = -half if side == 0 else half
        for k in range(M):
            row = []
            for j in range(P):
                if j < k:
                    row.append(Fraction(0))
                else:
                    # k-th Taylor coefficient of xi^j at x: C(j,k) x^(j-k)
                    c = Fraction(1)
                    for t in range(1, k + 1):
                        c = c * (j - k + t) / t
                    row.append(c * x ** (j - k))
            rows.append(row)
    aug = [rows[r] + [Fraction(int(r == c)) for c in range(P)] for r in range(P)]
    for col in range(P):
        piv = next(r for r in range(col, P) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        d = aug[col][col]
        aug[col] = [v / d for v in aug[col]]
        for r in range(P):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[col])]
    return [[aug[j][P + r] for r in range(P)] for j in range(P)]


def hermite_matrix(m: int) -> np.ndarray:
    """The C oracle's H (long-double Gauss-Jordan rounded to FP64)."""
    P = 2 * m + 2
    H = np.zeros((P, P))
    rc = load().oracle_hermite_matrix(m, _ptr(H))
    if rc != 0:
        raise ValueError(f"oracle_hermite_matrix({m}) failed: {rc}")
    return H


def interpolate_cell(m: int, uloc: np.ndarray, H: np.ndarray | None = None) -> np.ndarray:
    """Alg. 2 on one cell: uloc[a3][a2][a1] -> monomial coefficients R[j3][j2][j1]."""
    P = 2 * m + 2
    H = hermite_matrix(m) if H is None else np.ascontiguousarray(H, dtype=np.float64)
    uloc = np.ascontiguousarray(uloc, dtype=np.float64).reshape(P, P, P)
    R = np.zeros((P, P, P))
    load().oracle_interpolate_cell(m, _ptr(H), _ptr(uloc), _ptr(R))
    return R


def laplacian(m: int, W: np.ndarray) -> np.ndarray:
    P = 2 * m + 2
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(P, P, P)
    out = np.zeros((P, P, P))
    load().oracle_laplacian(m, _ptr(W), _ptr(out))
    return out


def evolve_taylor(m: int, q: int, lam: float, Ru: np.ndarray, Rv: np.ndarray):
    P = 2 * m + 2
    a = np.array(Ru, dtype=np.float64).reshape(P, P, P).copy()
    b = np.array(Rv, dtype=np.float64).reshape(P, P, P).copy()
    load().oracle_evolve_taylor(m, q, lam, _ptr(a), _ptr(b))
    return a, b


def evolve_rk4(m: int, S: int, lam: float, Ru: np.ndarray, Rv: np.ndarray):
    P = 2 * m + 2
    a = np.array(Ru, dtype=np.float64).reshape(P, P, P).copy()
    b = np.array(Rv, dtype=np.float64).reshape(P, P, P).copy()
    load().oracle_evolve_rk4(m, S, lam, _ptr(a), _ptr(b))
    return a, b


def gather_cell(n: int, m: int, g: np.ndarray, i: int, j: int, k: int) -> np.ndarray:
    P = 2 * m + 2
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros((P, P, P))
    load().oracle_gather_cell(n, m, _ptr(g), i, j, k, _ptr(out))
    return out


def half_step(n: int, m: int, lam: float, src: np.ndarray, to_dual: bool,
              evolution: str = "taylor", param: int | None = None) -> np.ndarray:
    """One half step on internal variables (u, (h/c) u_t), arrays [2][M^3][n^3]."""
    evo, param = _evo(m, evolution, param)
    H = hermite_matrix(m)
    src = np.ascontiguousarray(src, dtype=np.float64)
    dst = np.zeros_like(src)
    load().oracle_half_step(n, m, _ptr(H), lam, evo, param, _ptr(src), _ptr(dst), int(bool(to_dual)))
    return dst


def _evo(m, evolution, param):
    if evolution == "taylor":
        return 0, exact_q(m) if param is None else int(param)
    if evolution == "rk4":
        return 1, 1 if param is None else int(param)
    raise ValueError(evolution)


def run(n: int, m: int, cfl: float, c: float, u: np.ndarray, ut: np.ndarray, nsteps: int,
        evolution: str = "taylor", param: int | None = None, ld: bool = False):
    """Advance primal-grid scaled derivatives (u, u_t), each [M^3][n^3] (any
    shape with that many elements, layout [d3][d2][d1][k][j][i]), by nsteps
    full steps. Returns new (u, ut) float64 arrays of the same shape.
    ld=True runs the long-double twin (rounding-floor measurements only)."""
    evo, param = _evo(m, evolution, param)
    shape = np.shape(u)
    dt = np.longdouble if ld else np.float64
    a = np.array(u, dtype=np.float64).astype(dt).ravel().copy()
    b = np.array(ut, dtype=np.float64).astype(dt).ravel().copy()
    M3 = (m + 1) ** 3
    assert a.size == M3 * n ** 3 and b.size == a.size
    rc = load(ld).oracle_run(n, m, float(cfl), float(c), evo, param, int(nsteps), _ptr(a), _ptr(b))
    if rc != 0:
        raise ValueError(f"oracle_run failed: {rc}")
    return a.astype(np.float64).reshape(shape), b.astype(np.float64).reshape(shape)


def point(n: int, m: int, cfl: float, c: float, u: np.ndarray, ut: np.ndarray, nsteps: int,
          i: int, j: int, k: int, evolution: str = "taylor", param: int | None = None):
    """Values (u then u_t, 2*M^3 scaled derivatives) at primal node (i,j,k)
    after nsteps full steps, from its dependency cone only."""
    evo, param = _evo(m, evolution, param)
    a = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
    b = np.ascontiguousarray(np.asarray(ut, dtype=np.float64).ravel())
    out = np.zeros(2 * (m + 1) ** 3)
    rc = load().oracle_point(n, m, float(cfl), float(c), evo, param, int(nsteps),
                             _ptr(a), _ptr(b), i, j, k, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_point failed: {rc}")
    return out


def point_box(n: int, m: int, cfl: float, c: float, ubox: np.ndarray, utbox: np.ndarray, nsteps: int,
              evolution: str = "taylor", param: int | None = None, ld: bool = False):
    """Values (u then u_t) at the centre primal node of a (2*nsteps+1)^3 box of
    primal nodes, laid out [M^3][w][w][w], after nsteps full steps (grid of n
    cells per side, so h = 1/n). ld=True runs the long-double twin (rounding
    floor measurements only)."""
    evo, param = _evo(m, evolution, param)
    dt = np.longdouble if ld else np.float64
    a = np.ascontiguousarray(np.asarray(ubox, dtype=np.float64).astype(dt).ravel())
    b = np.ascontiguousarray(np.asarray(utbox, dtype=np.float64).astype(dt).ravel())
    w = 2 * nsteps + 1
    assert a.size == (m + 1) ** 3 * w ** 3 and b.size == a.size
    out = np.zeros(2 * (m + 1) ** 3, dtype=dt)
    rc = load(ld).oracle_point_box(n, m, float(cfl), float(c), evo, param, int(nsteps),
                                   _ptr(a), _ptr(b), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_point_box failed: {rc}")
    return out.astype(np.float64)


# --- point source (forced wave equation) -----------------------------------

def gauss_taylor(d: float, sigma: float, h: float, K: int) -> np.ndarray:
    """Scaled Taylor coefficients h^a/a! g1^(a), a < K, of the unit-mass 1D
    Gaussian factor at nearest-image offset d from the source (sigma <= 0:
    the uniform factor 1)."""
    out = np.zeros(K)
    rc = load().oracle_gauss_taylor(float(d), float(sigma), float(h), int(K), _ptr(out))
    if rc != 0:
        raise ValueError(rc)
    return out


def ricker_taylor(ta: float, tau: float, f0: float, t0: float, K: int) -> np.ndarray:
    """Time Taylor coefficients tau^k/k! w^(k)(ta), k < K, of the Ricker
    wavelet (1 - 2 beta s^2) exp(-beta s^2), s = t - t0, beta = (pi f0)^2."""
    out = np.zeros(K)
    rc = load().oracle_ricker_taylor(float(ta), float(tau), float(f0), float(t0), int(K), _ptr(out))
    if rc != 0:
        raise ValueError(rc)
    return out


def evolve_taylor_forced(m: int, q: int, lam: float, Ru, Rv, G, wk):
    """Forced Taylor evolution of one cell (forward series recursion)."""
    P = 2 * m + 2
    a = np.array(Ru, dtype=np.float64).reshape(P, P, P).copy()
    b = np.array(Rv, dtype=np.float64).reshape(P, P, P).copy()
    g = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(P, P, P))
    w = np.ascontiguousarray(np.asarray(wk, dtype=np.float64))
    assert w.size >= q
    load().oracle_evolve_taylor_forced(m, q, lam, _ptr(a), _ptr(b), _ptr(g), _ptr(w))
    return a, b


def run_forced(n: int, m: int, cfl: float, c: float, u, ut, nsteps: int, source: dict, q: int | None = None,
               ld: bool = False):
    """As run() with Taylor evolution and the point source
    source = {"x": (x, y, z), "sigma": s, "freq": f0, "t0": t0, "amplitude": a}.
    ld=True runs the long-double twin (rounding-floor measurements only)."""
    q = exact_q(m) if q is None else int(q)
    shape = np.shape(u)
    dt = np.longdouble if ld else np.float64
    a = np.array(u, dtype=np.float64).astype(dt).ravel().copy()
    b = np.array(ut, dtype=np.float64).astype(dt).ravel().copy()
    sx = np.ascontiguousarray(np.asarray(source["x"], dtype=np.float64).astype(dt))
    rc = load(ld).oracle_run_forced(n, m, float(cfl), float(c), q, int(nsteps), _ptr(a), _ptr(b), _ptr(sx),
                                    float(source["sigma"]), float(source["freq"]), float(source["t0"]),
                                    float(source["amplitude"]))
    if rc != 0:
        raise ValueError(f"oracle_run_forced failed: {rc}")
    return a.astype(np.float64).reshape(shape), b.astype(np.float64).reshape(shape)


# --- advection (the paper's Eq. 1) -------------------------------------------

def advection_q(m: int) -> int:
    """Stage count 3(2m+1) of Sec. 3.2: exact for the advection equation."""
    return 3 * (2 * m + 1)


def evolve_advection(m: int, q: int, lam: float, R: np.ndarray) -> np.ndarray:
    """Alg. 4 for u_sigma = lam (sum_x d/dxi_x) u on one cell's coefficients R[j3][j2][j1]."""
    P = 2 * m + 2
    a = np.array(R, dtype=np.float64).reshape(P, P, P).copy()
    load().oracle_evolve_advection(m, int(q), float(lam), _ptr(a))
    return a


def run_advection(n: int, m: int, cfl: float, c: float, u, nsteps: int, q: int | None = None,
                  ld: bool = False) -> np.ndarray:
    """nsteps full steps of u_t = c (u_x1 + u_x2 + u_x3) from primal-grid data u
    ((m+1)^3 n^3 scaled derivatives, layout [d3][d2][d1][k][j][i]).
    ld=True runs the long-double twin (rounding-floor measurements only)."""
    q = advection_q(m) if q is None else int(q)
    shape = np.shape(u)
    dt = np.longdouble if ld else np.float64
    a = np.array(u, dtype=np.float64).astype(dt).ravel().copy()
    assert a.size == (m + 1) ** 3 * n ** 3
    rc = load(ld).oracle_run_advection(n, m, float(cfl), float(c), q, int(nsteps), _ptr(a))
    if rc != 0:
        raise ValueError(f"oracle_run_advection failed: {rc}")
    return a.astype(np.float64).reshape(shape)


# --- adjoint (gradients of receiver traces) ----------------------------------

def adjoint_half_step(n: int, m: int, lam: float, lam_dst: np.ndarray, to_dual: bool, q: int | None = None):
    """Transpose of half_step (Taylor, q stages) on internal variables
    [2][M^3][n^3]: the adjoint of the source grid from that of the
    destination grid."""
    q = exact_q(m) if q is None else int(q)
    H = hermite_matrix(m)
    a = np.ascontiguousarray(lam_dst, dtype=np.float64)
    out = np.zeros_like(a)
    load().oracle_adjoint_half_step(n, m, _ptr(H), float(lam), q, _ptr(a), _ptr(out), int(bool(to_dual)))
    return out


def source_term(n: int, m: int, cfl: float, c: float, to_dual: bool, ta: float, source: dict,
                q: int | None = None) -> np.ndarray:
    """The point source's contribution to one half step starting at ta
    (internal variables [2][M^3][n^3] on the destination grid)."""
    q = exact_q(m) if q is None else int(q)
    M3 = (m + 1) ** 3
    out = np.zeros(2 * M3 * n ** 3)
    sx = np.ascontiguousarray(np.asarray(source["x"], dtype=np.float64))
    rc = load().oracle_source_term(n, m, float(cfl), float(c), q, int(bool(to_dual)), float(ta), _ptr(sx),
                                   float(source["sigma"]), float(source["freq"]), float(source["t0"]),
                                   float(source["amplitude"]), _ptr(out))
    if rc != 0:
        raise ValueError(rc)
    return out


def run_series(n: int, m: int, cfl: float, c: float, u0, ut0, nsteps: int, source: dict | None, amps,
               receivers, q: int | None = None):
    """Forward run whose source term in half step s (two per full step) is
    multiplied by amps[s]; returns the traces [nsteps][R] of u at the primal
    receiver nodes (i, j, k) after each full step, and the final (u, ut)."""
    q = exact_q(m) if q is None else int(q)
    M3 = (m + 1) ** 3
    nn = n ** 3
    h = 1.0 / n
    dt = cfl * h / c
    lam = c * 0.5 * dt / h
    a = np.concatenate([np.asarray(u0, dtype=np.float64).ravel(), (h / c) * np.asarray(ut0, dtype=np.float64).ravel()])
    rec = [(k * n + j) * n + i for (i, j, k) in receivers]
    traces = np.zeros((nsteps, len(rec)))
    for s in range(nsteps):
        b = half_step(n, m, lam, a, True, "taylor", q)
        if source is not None:
            b += amps[2 * s] * source_term(n, m, cfl, c, True, s * dt, source, q)
        a = half_step(n, m, lam, b, False, "taylor", q)
        if source is not None:
            a += amps[2 * s + 1] * source_term(n, m, cfl, c, False, s * dt + 0.5 * dt, source, q)
        traces[s] = a[rec]
    return traces, a[:M3 * nn].copy(), (c / h) * a[M3 * nn:]


def adjoint_series(n: int, m: int, cfl: float, c: float, nsteps: int, source: dict | None, receivers, residual,
                   q: int | None = None):
    """Gradients of sum_{s, r} residual[s][r] traces[s][r] (traces of
    run_series) with respect to u0, ut0 (flat [M^3 n^3]) and amps (2 nsteps):
    the adjoint recursion run backwards with adjoint_half_step."""
    q = exact_q(m) if q is None else int(q)
    M3 = (m + 1) ** 3
    nn = n ** 3
    h = 1.0 / n
    dt = cfl * h / c
    lam = c * 0.5 * dt / h
    rec = [(k * n + j) * n + i for (i, j, k) in receivers]
    residual = np.asarray(residual, dtype=np.float64)
    g = np.zeros(2 * M3 * nn)
    gamps = np.zeros(2 * nsteps)
    for s in range(nsteps - 1, -1, -1):
        for r, node in enumerate(rec):
            g[node] += residual[s, r]
        if source is not None:
            gamps[2 * s + 1] = g @ source_term(n, m, cfl, c, False, s * dt + 0.5 * dt, source, q)
        mu = adjoint_half_step(n, m, lam, g, False, q)
        if source is not None:
            gamps[2 * s] = mu @ source_term(n, m, cfl, c, True, s * dt, source, q)
        g = adjoint_half_step(n, m, lam, mu, True, q)
    return g[:M3 * nn].copy(), (h / c) * g[M3 * nn:], gamps
