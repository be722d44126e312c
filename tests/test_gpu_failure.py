"""Failure detection forced from the host (no kernel faults, no hangs):
non-finite state after instability or bad input, out-of-memory on absurd
sizes, and the poisoned-destination check staying clean."""
import numpy as np
import pytest

from paper_1609_09841_amd import binding as B
from paper_1609_09841_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_finite_after_normal_steps_and_with_poisoned_destinations():
    n, m = 8, 2
    u0, ut0 = I.fourier_initial(n, m, nmodes=2, kmax=2)
    for poison in (False, True):
        with B.Solver(n, m, poison=poison) as s:
            s.set_initial(u0.numpy(), ut0.numpy())
            s.step(3)
            assert s.finite()


def test_nan_in_initial_data_is_detected():
    n, m = 6, 1
    u0, ut0 = I.fourier_initial(n, m, nmodes=2, kmax=2)
    u0 = u0.numpy().copy()
    u0[1, 0, 1, 2, 3, 4] = np.nan
    with B.Solver(n, m) as s:
        s.set_initial(u0, ut0.numpy())
        assert not s.finite()
        s.step(2)
        assert not s.finite()


def test_instability_beyond_the_stable_cfl_range_is_detected():
    """cfl = 1 is allowed by the half-step condition of Sec. 2 but unstable in
    3D (amplification ~1.3 per half step): rounding grows until it overflows."""
    n, m = 16, 1
    u0, ut0 = I.standing_mode(n, m)
    print("[instability] n=16 m=1 cfl=1.0 3000 steps", flush=True)
    with B.Solver(n, m, 1.0, 1.0) as s:
        s.set_initial(u0.numpy(), ut0.numpy())
        s.step(3000)
        assert not s.finite()
    with B.Solver(n, m, 0.5, 1.0) as s:
        s.set_initial(u0.numpy(), ut0.numpy())
        s.step(3000)
        assert s.finite()


def test_absurd_size_reports_out_of_memory():
    """1290^3 cells at m = 3 need about 4.4 TB of grids."""
    rc, h = B.hermite_create(1290, 3, 0.5, 1.0)
    assert rc == B.HERMITE_ENOMEM and h is None
    assert "hipMalloc" in B.hermite_last_error(None)
