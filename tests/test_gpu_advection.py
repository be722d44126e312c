"""GPU parity of the advection half step (the paper's Eq. 1) against the CPU
oracle's Eq. 5 / Alg. 4 recursion, through the C ABI.

The library composes interpolation, the exact Taylor series (a translation)
and truncation into one separable operator per axis; the oracle follows the
paper's steps. Tolerance: relative L2 <= 1e-12, or at m = 3 within the
measured FP64 rounding floor of the oracle (oracle vs its long-double twin):
within 3x that floor, and at least as close to the long-double result as the
FP64 oracle (within 50%).
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1609_09841_amd import binding as B
from paper_1609_09841_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-12


def rel(a, b):
    return I.rel_l2(np.asarray(a), np.asarray(b))


def gpu_advect(n, m, u0, steps, cfl=0.5, c=1.0, **kw):
    print(f"[gpu_advect] n={n} m={m} steps={steps} cfl={cfl} c={c} {kw}", flush=True)
    with B.Solver(n, m, cfl, c, equation="advection", **kw) as s:
        s.set_initial(u0, None)
        s.step(steps)
        u, ut, t = s.gather()
    assert ut is None
    return u, t


def _check(n, m, u0, steps, cfl=0.5, c=1.0, q=None, **kw):
    gu, t = gpu_advect(n, m, u0, steps, cfl, c, **({"q": q} if q else {}), **kw)
    ou = O.run_advection(n, m, cfl, c, u0, steps, q)
    e = rel(gu, ou)
    assert math.isclose(t, steps * cfl / n / c, rel_tol=1e-15)
    if e <= TOL:
        print(f"  gpu-oracle {e:.2e}", flush=True)
        return e
    lu = O.run_advection(n, m, cfl, c, u0, steps, q, ld=True)
    f = rel(ou, lu)
    print(f"  gpu-oracle {e:.2e}; oracle-ld {f:.2e}; gpu-ld {rel(gu, lu):.2e}", flush=True)
    assert e <= max(TOL, 3 * f) and rel(gu, lu) <= max(TOL, 1.5 * f), (e, f)
    return e


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "two"])
@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("n", [2, 3, 5, 8, 13])
def test_random_data_small_grids(n, m, fused):
    M = m + 1
    u0 = np.random.default_rng(100 * n + m).standard_normal((M, M, M, n, n, n))
    _check(n, m, u0, 2, fused=fused)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_two_kernel_organisation_matches_fused(m):
    """Interpolation to the coefficients in memory, then the translation
    kernel, against the fused kernel (independent code paths)."""
    n = 11
    u0, _ = I.fourier_initial(n, m, nmodes=3, kmax=2)
    a, _ = gpu_advect(n, m, u0.numpy(), 5, fused=True)
    b, _ = gpu_advect(n, m, u0.numpy(), 5, fused=False)
    assert rel(b, a) <= (1e-13 if m < 3 else 1e-11)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_smooth_data_several_steps(m):
    n = 16
    u0, _ = I.fourier_initial(n, m, nmodes=4, kmax=3)
    _check(n, m, u0.numpy(), 8)


@pytest.mark.parametrize("m", [1, 3])
def test_stage_counts_and_speed(m):
    n = 7
    M = m + 1
    u0 = np.random.default_rng(7 + m).standard_normal((M, M, M, n, n, n))
    _check(n, m, u0, 2, q=3 * (2 * m + 1) + 4)
    _check(n, m, u0, 2, cfl=0.9, c=2.3)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_cfl_one_is_a_shift_by_one_node(m):
    n = 6
    M = m + 1
    u0 = np.random.default_rng(70 + m).standard_normal((M, M, M, n, n, n))
    gu, _ = gpu_advect(n, m, u0, 2, cfl=1.0)
    ref = np.roll(u0, (-2, -2, -2), axis=(3, 4, 5))
    assert np.abs(gu - ref).max() <= {1: 1e-13, 2: 1e-11, 3: 1e-8}[m] * np.abs(u0).max()


def _window(u, i, j, k, w):
    """(M, M, M, w, w, w) periodic window of u whose centre is node (i, j, k)."""
    n = u.shape[-1]
    r = w // 2
    ix = [(i - r + a) % n for a in range(w)]
    jx = [(j - r + a) % n for a in range(w)]
    kx = [(k - r + a) % n for a in range(w)]
    return np.ascontiguousarray(u[..., kx, :, :][..., :, jx, :][..., :, :, ix])


def test_full_size_sampled_150_cube_m3():
    """The paper's advection grid (150^3 cells), m = 3, seeded Fourier data,
    4 steps. Sampled nodes against the oracle: a half step in the cell
    variables depends on lam = cfl/2 only, so the oracle run on the periodic
    (2s+1)^3 window around a node gives that node's value after s steps (the
    window's wrapped edges stay outside the node's dependency cone). Also the
    node values against the exact translated modes."""
    n, m, steps, cfl = 150, 3, 4, 0.5
    w = 2 * steps + 1
    modes = I.fourier_modes(nmodes=8, kmax=8)
    u0d, _ = I.fourier_exact(n, m, modes, t=0.0, device="cuda")
    print(f"[gpu_advect] n={n} m={m} steps={steps} full size, device data", flush=True)
    with B.Solver(n, m, cfl, 1.0, equation="advection") as s:
        s.set_initial(u0d)
        s.step(steps)
        gu, _, t = s.gather()
    u0 = u0d.cpu().numpy()
    del u0d
    rng = np.random.default_rng(150)
    worst = 0.0
    for (i, j, k) in [(0, 0, 0), (n - 1, n - 1, n - 1)] + [tuple(rng.integers(0, n, 3)) for _ in range(10)]:
        box = _window(u0, i, j, k, w)
        ob = O.run_advection(w, m, cfl, 1.0, box, steps)[..., steps, steps, steps]
        lb = O.run_advection(w, m, cfl, 1.0, box, steps, ld=True)[..., steps, steps, steps]
        g = gu[..., k, j, i]
        e, f = rel(g, ob), rel(ob, lb)
        worst = max(worst, e)
        assert e <= max(TOL, 3 * f) and rel(g, lb) <= max(TOL, 1.5 * f), ((i, j, k), e, f)
    print(f"  sampled nodes: worst gpu-oracle {worst:.2e}", flush=True)
    shifted = [(kv, A, phi + 2 * math.pi * t * sum(kv)) for (kv, A, phi) in modes]
    ue, _ = I.fourier_exact(n, m, shifted, t=0.0, device="cuda")
    err = I.rel_l2(torch.as_tensor(gu[0, 0, 0], device="cuda"), ue[0, 0, 0])
    print(f"  node values vs exact translation after {steps} steps: {err:.2e}", flush=True)
    assert err < 1e-6


def test_advection_option_errors():
    o = B.hermite_default_options()
    o.equation = B.HERMITE_EQ_ADVECTION
    for field, value in (("precision", B.HERMITE_PREC_FP32), ("evolution", B.HERMITE_EVOLVE_RK4), ("q", 6)):
        oo = B.hermite_options.from_buffer_copy(o)
        setattr(oo, field, value)
        rc, h = B.hermite_create(8, 2, 0.5, 1.0, oo)
        assert rc == B.HERMITE_EUNSUPPORTED and h is None, field
    with B.Solver(6, 2, equation="advection") as s:
        with pytest.raises(B.HermiteError) as e:
            s.set_source({"x": (0.5, 0.5, 0.5), "sigma": 0.1, "freq": 1.0, "t0": 0.0, "amplitude": 1.0})
        assert e.value.code == B.HERMITE_EUNSUPPORTED
