"""The stability statement of the C header, on the oracle: the half-step
condition of Sec. 2 (cfl <= 1) is necessary but not sufficient in 3D;
Taylor evolution is stable at cfl 0.5 (the workloads') and 0.75, and grows
at cfl 1.0."""
import numpy as np
import pytest

from paper_1609_09841_amd import inputs as I


def _growth(O, cfl, steps, n=8, m=1):
    rng = np.random.default_rng(3)
    M = m + 1
    u0 = rng.standard_normal((M, M, M, n, n, n))
    ut0 = rng.standard_normal((M, M, M, n, n, n))
    u, ut = O.run(n, m, cfl, 1.0, u0, ut0, steps)
    return np.sqrt(np.sum(u ** 2)) / np.sqrt(np.sum(u0 ** 2))


@pytest.mark.parametrize("cfl", [0.5, 0.75])
def test_taylor_stable_below_the_documented_limit(oracle_mod, cfl):
    assert _growth(oracle_mod, cfl, 60) < 2.0


def test_taylor_grows_at_cfl_one(oracle_mod):
    assert _growth(oracle_mod, 1.0, 60) > 1e3
