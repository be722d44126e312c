"""Seeded synthetic initial data for the Hermite wave solver.

This module holds no part of the method: it only evaluates closed-form
solutions of u_tt = c^2 Lap u on the periodic unit cube and their scaled
derivatives h^{|d|}/d! D^d (the nodal unknowns of the paper's Eq. 2), so that
both the HIP path and the CPU oracle are fed, and judged, with the same data.

Arrays are float64 tensors of shape (M, M, M, n, n, n) = [d3][d2][d1][k][j][i]
with M = m + 1 and i (x1) fastest, the nodal layout of the paper's Sec. 3.1.
Node (i, j, k) sits at (i, j, k) * h on the primal grid, h = 1/n, and at
(i + 1/2, j + 1/2, k + 1/2) * h on the dual grid.
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = [
    "fourier_modes", "fourier_initial", "fourier_exact", "standing_mode",
    "plane_waves_1d", "rel_l2", "batch_shots",
]


def fourier_modes(seed: int = 1609, nmodes: int = 8, kmax: int = 8):
    """Seeded list of (k, A, phi): integer wave vectors with components in
    [1, kmax] times a random sign, amplitudes ~ N(0, 1), phases ~ U(0, 2 pi).
    Draw order per mode: k magnitudes, k signs, A, phi."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(nmodes):
        k = rng.integers(1, kmax + 1, 3) * rng.choice([-1, 1], 3)
        A = float(rng.standard_normal())
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
        modes.append((tuple(int(v) for v in k), A, phi))
    return modes


def _coords(n: int, staggered: bool, device, dtype):
    shift = 0.5 if staggered else 0.0
    x = (torch.arange(n, device=device, dtype=dtype) + shift) / n
    return x


def fourier_exact(n: int, m: int, modes, t: float = 0.0, c: float = 1.0,
                  staggered: bool = False, device="cpu"):
    """Scaled derivatives of u = sum A cos(2 pi k.x + phi) cos(2 pi |k| c t)
    and of u_t at time t, both shaped (M, M, M, n, n, n)."""
    dt = torch.float64
    M = m + 1
    h = 1.0 / n
    x = _coords(n, staggered, device, dt)
    u = torch.zeros((M, M, M, n, n, n), device=device, dtype=dt)
    ut = torch.zeros_like(u)
    for (k, A, phi) in modes:
        kx, ky, kz = k
        theta = (2 * math.pi * kz * x).view(n, 1, 1) + (2 * math.pi * ky * x).view(1, n, 1) \
            + (2 * math.pi * kx * x).view(1, 1, n) + phi
        cth, sth = torch.cos(theta), torch.sin(theta)
        # cos(theta + r pi/2) for r = 0..3
        rot = [cth, -sth, -cth, sth]
        omega = 2 * math.pi * math.sqrt(kx * kx + ky * ky + kz * kz) * c
        tu, tv = math.cos(omega * t), -omega * math.sin(omega * t)
        for d3 in range(M):
            for d2 in range(M):
                for d1 in range(M):
                    s = A * ((2 * math.pi * kx * h) ** d1 / math.factorial(d1)) \
                        * ((2 * math.pi * ky * h) ** d2 / math.factorial(d2)) \
                        * ((2 * math.pi * kz * h) ** d3 / math.factorial(d3))
                    base = rot[(d1 + d2 + d3) % 4]
                    if tu != 0.0:
                        u[d3, d2, d1].add_(base, alpha=s * tu)
                    if tv != 0.0:
                        ut[d3, d2, d1].add_(base, alpha=s * tv)
        del theta, cth, sth, rot
    return u, ut


def fourier_initial(n: int, m: int, seed: int = 1609, nmodes: int = 8, kmax: int = 8,
                    device="cpu"):
    """Initial data of the seeded Fourier-mode workload: u0 = sum of modes,
    u_t = 0."""
    return fourier_exact(n, m, fourier_modes(seed, nmodes, kmax), 0.0, 1.0, False, device)


def standing_mode(n: int, m: int, t: float = 0.0, c: float = 1.0, k=(1, 1, 1),
                  staggered: bool = False, device="cpu"):
    """u = sin(2 pi k1 x1) sin(2 pi k2 x2) sin(2 pi k3 x3) cos(2 pi |k| c t)
    and u_t, as scaled derivatives."""
    dt = torch.float64
    M = m + 1
    h = 1.0 / n
    x = _coords(n, staggered, device, dt)
    omega = 2 * math.pi * math.sqrt(sum(kk * kk for kk in k)) * c
    tu, tv = math.cos(omega * t), -omega * math.sin(omega * t)
    axes = []
    for kk in k:
        a = 2 * math.pi * kk
        # d-th scaled derivative of sin(a x): (a h)^d / d! sin(a x + d pi/2)
        axes.append([((a * h) ** d / math.factorial(d)) * torch.sin(a * x + d * math.pi / 2)
                     for d in range(M)])
    u = torch.empty((M, M, M, n, n, n), device=device, dtype=dt)
    for d3 in range(M):
        for d2 in range(M):
            for d1 in range(M):
                u[d3, d2, d1] = axes[2][d3].view(n, 1, 1) * axes[1][d2].view(1, n, 1) \
                    * axes[0][d1].view(1, 1, n)
    return u * tu, u * tv


def plane_waves_1d(n: int, m: int, kx: int = 1, t: float = 0.0, c: float = 1.0, phi: float = 0.3,
                   device="cpu"):
    """u = cos(2 pi kx x1 + phi) cos(2 pi |kx| c t): data that depends on x1
    only (every derivative in x2 or x3 vanishes)."""
    return fourier_exact(n, m, [((kx, 0, 0), 1.0, phi)], t, c, False, device)


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 over all entries."""
    x = torch.as_tensor(x, dtype=torch.float64)
    ref = torch.as_tensor(ref, dtype=torch.float64).to(x.device)
    den = torch.linalg.vector_norm(ref).item()
    num = torch.linalg.vector_norm(x - ref).item()
    return num / den if den > 0 else num


def batch_shots(seed: int = 1609, count: int = 64, sizes=(32, 48, 64, 96), orders=(1, 2, 3), c: float = 1.0):
    """Seeded shot list of the batched point-source workload: per shot, in
    this draw order, cells per side from `sizes`, order m from `orders`, and
    the source point uniform in [0, 1)^3. Each source is a Gaussian of width
    sigma = 2h with a Ricker wavelet of about 8 cells per dominant wavelength
    (f0 = c / (8h)) peaking at t0 = 1.2 / f0, unit amplitude; zero initial
    data. Shot dicts: {"n", "m", "source": {"x", "sigma", "freq", "t0",
    "amplitude"}}."""
    rng = np.random.default_rng(seed)
    shots = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        m = int(rng.choice(orders))
        x = tuple(float(v) for v in rng.uniform(0.0, 1.0, 3))
        f0 = c * n / 8.0
        shots.append({"n": n, "m": m, "source": {"x": x, "sigma": 2.0 / n, "freq": f0, "t0": 1.2 / f0,
                                                  "amplitude": 1.0}})
    return shots
