"""GPU: mixed-precision contractions (FP32, split BF16x3) of the m = 3 fused
half step, against the plain FP64 path and the CPU oracle.

The low-precision part is the remainder after the FP64 corner mean, so its
rounding is relative to sum |K'| |x| of the class operator, which at m = 3 is
large for the high-order derivatives (monomial-basis cancellation). Bounds
below are per field, rel L2 over all DOFs and over the node values (d = 0)
separately; the project's 1e-6 target for the mixed path is measured and
reported by the benchmark, not asserted here.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_09841_amd import binding as B
from paper_1609_09841_amd import inputs as I

pytestmark = pytest.mark.gpu

# rel L2 bounds (all DOFs, node values d = 0) per precision
BOUNDS = {"fp32": (1e-3, 1e-6), "bf16x3": (1e-1, 1e-4)}
RANDOM_BOUNDS = {"fp32": 1e-5, "bf16x3": 1e-3}


def run(n, u0, ut0, steps, precision, **kw):
    print(f"[mixed] n={n} steps={steps} precision={precision} {kw}", flush=True)
    with B.Solver(n, 3, precision=precision, **kw) as s:
        s.set_initial(u0, ut0)
        s.step(steps)
        u, ut, _ = s.gather()
    return u, ut


def rel(a, b):
    return I.rel_l2(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("evolution", ["taylor", "rk4"])
def test_smooth_data_against_fp64_and_oracle(precision, evolution):
    n, steps = 16, 4
    u0, ut0 = I.fourier_exact(n, 3, I.fourier_modes(kmax=1), t=0.05)
    u0, ut0 = u0.numpy(), ut0.numpy()
    gu, gv = run(n, u0, ut0, steps, "fp64", evolution=evolution)
    mu, mv = run(n, u0, ut0, steps, precision, evolution=evolution)
    ou, ov = O.run(n, 3, 0.5, 1.0, u0, ut0, steps, evolution)
    all_b, node_b = BOUNDS[precision]
    for name, (m_, g_, o_) in {"u": (mu, gu, ou), "u_t": (mv, gv, ov)}.items():
        e_all, e_node, e_or = rel(m_, g_), rel(m_[0, 0, 0], g_[0, 0, 0]), rel(m_, o_)
        print(f"  {precision} {evolution} {name}: vs fp64 all {e_all:.2e} nodes {e_node:.2e}; vs oracle {e_or:.2e}",
              flush=True)
        assert e_all <= all_b and e_node <= node_b and e_or <= all_b


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n", [2, 5, 7, 17])
def test_random_data_ragged_grids(precision, n):
    """Random data, no cancellation to amplify rounding: every class, lane and
    tail position of the kernel must agree with FP64 to the low precision."""
    rng = np.random.default_rng(7 * n)
    u0 = rng.standard_normal((4, 4, 4, n, n, n))
    ut0 = rng.standard_normal((4, 4, 4, n, n, n)) * n
    gu, gv = run(n, u0, ut0, 1, "fp64")
    mu, mv = run(n, u0, ut0, 1, precision)
    eu, ev = rel(mu, gu), rel(mv, gv)
    print(f"  {precision} n={n}: u {eu:.2e} u_t {ev:.2e}", flush=True)
    assert eu <= RANDOM_BOUNDS[precision] and ev <= RANDOM_BOUNDS[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_constant_data_exact(precision):
    """A constant u: only the corner mean of d = 0 is non-zero, which is FP64,
    and the low-precision remainder is exactly zero."""
    n = 6
    z = np.zeros((4, 4, 4, n, n, n))
    c = z.copy()
    c[0, 0, 0] = 1.375
    u, ut = run(n, c, z, 3, precision)
    assert np.array_equal(u, c) and np.all(ut == 0)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_poisoned_destination_fully_written(precision):
    n = 9
    u0, ut0 = I.fourier_exact(n, 3, I.fourier_modes(kmax=1), t=0.05)
    a, b = run(n, u0.numpy(), ut0.numpy(), 2, precision, poison=True)
    c, d = run(n, u0.numpy(), ut0.numpy(), 2, precision)
    assert np.isfinite(a).all() and np.isfinite(b).all()
    assert np.array_equal(a, c) and np.array_equal(b, d)
