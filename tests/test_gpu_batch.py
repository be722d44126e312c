"""GPU tests of batches of independent shots (hermite_batch_*), through the
C ABI.

A batched launch runs the same per-cell arithmetic as the single-grid fused
kernels (same operators, same kernel bodies), so every shot of a batch must
equal, bit for bit, a single-grid context run of that shot; and each shot is
checked against the CPU oracle (unforced or forced) with the single-grid
tolerance (relative L2 <= 1e-12, or within the measured FP64 floor at m = 3).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1609_09841_amd import binding as B
from paper_1609_09841_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-12


def rel(a, b):
    return I.rel_l2(np.asarray(a), np.asarray(b))


def _source(n, rng):
    f0 = n / 8.0
    return {"x": tuple(rng.uniform(0, 1, 3)), "sigma": 2.0 / n, "freq": f0, "t0": 1.2 / f0, "amplitude": 1.0}


def _shots(seed, count, ns, ms, with_source):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(ns))
        m = int(rng.choice(ms))
        out.append({"n": n, "m": m, "source": _source(n, rng) if with_source else None})
    return out


def _initial(sh, seed):
    rng = np.random.default_rng(seed)
    M, n = sh["m"] + 1, sh["n"]
    return rng.standard_normal((M, M, M, n, n, n)), rng.standard_normal((M, M, M, n, n, n))


def _single(sh, u0, ut0, steps, cfl=0.5, c=1.0, **kw):
    with B.Solver(sh["n"], sh["m"], cfl, c, **kw) as s:
        s.set_initial(u0, ut0)
        if sh.get("source") is not None:
            s.set_source(sh["source"])
        s.step(steps)
        return s.gather()


def _oracle_check(sh, u0, ut0, steps, gu, gv, cfl=0.5, c=1.0):
    n, m = sh["n"], sh["m"]
    if sh.get("source") is not None:
        ou, ov = O.run_forced(n, m, cfl, c, u0, ut0, steps, sh["source"])
        lo = lambda: O.run_forced(n, m, cfl, c, u0, ut0, steps, sh["source"], ld=True)
    else:
        ou, ov = O.run(n, m, cfl, c, u0, ut0, steps)
        lo = lambda: O.run(n, m, cfl, c, u0, ut0, steps, ld=True)
    eu, ev = rel(gu, ou), rel(gv, ov)
    if eu <= TOL and ev <= TOL:
        return
    lu, lv = lo()
    fu, fv = rel(ou, lu), rel(ov, lv)
    print(f"  shot n={n} m={m}: gpu-oracle {eu:.2e} {ev:.2e}, floor {fu:.2e} {fv:.2e}", flush=True)
    assert eu <= max(TOL, 3 * fu) and ev <= max(TOL, 3 * fv), (eu, ev, fu, fv)


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "direct"])
def test_uneven_batch_equals_single_runs_and_oracle(graph):
    shots = [{"n": 5, "m": 1}, {"n": 8, "m": 3}, {"n": 7, "m": 2}, {"n": 12, "m": 1},
             {"n": 6, "m": 3}, {"n": 9, "m": 2}, {"n": 3, "m": 3}]
    steps = 3
    print(f"[batch] {shots} graph={graph}", flush=True)
    data = [_initial(sh, 10 + i) for i, sh in enumerate(shots)]
    with B.Batch(shots, graph=graph) as b:
        for i, (u0, ut0) in enumerate(data):
            b.set_initial(i, u0, ut0)
        b.step(steps)
        res = [b.gather(i) for i in range(len(shots))]
        for m in (1, 2, 3):
            ch, ms = b.tuning(m)
            assert 0 <= ch < (3 if m < 3 else 4) and ms > 0
    for sh, (u0, ut0), (gu, gv, t) in zip(shots, data, res):
        su, sv, st = _single(sh, u0, ut0, steps)
        assert np.array_equal(gu, su) and np.array_equal(gv, sv), sh
        assert t == st and math.isclose(t, steps * 0.5 / sh["n"], rel_tol=1e-15)
        _oracle_check(sh, u0, ut0, steps, gu, gv)


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "direct"])
def test_forced_shots_from_zero_data(graph):
    """The batched-shot workload's shape scaled down: zero data, a width-2h
    Gaussian source with a Ricker wavelet of about 8 cells per wavelength."""
    shots = _shots(4, 9, (8, 10, 12), (1, 2, 3), True)
    steps = 6
    print(f"[batch forced] {shots}", flush=True)
    with B.Batch(shots, graph=graph) as b:
        b.step(steps)
        res = [b.gather(i) for i in range(len(shots))]
    for sh, (gu, gv, t) in zip(shots, res):
        M, n = sh["m"] + 1, sh["n"]
        z = np.zeros((M, M, M, n, n, n))
        su, sv, _ = _single(sh, z, z, steps)
        assert np.array_equal(gu, su) and np.array_equal(gv, sv), sh
        assert np.abs(gu).max() > 0
        _oracle_check(sh, z, z, steps, gu, gv)


def test_autotune_and_graph_do_not_change_results():
    shots = _shots(7, 6, (6, 9, 16, 17), (1, 2, 3), True)
    data = [_initial(sh, 30 + i) for i, sh in enumerate(shots)]
    outs = []
    for graph, tune in ((True, True), (False, False), (True, False)):
        with B.Batch(shots, graph=graph, autotune=tune) as b:
            for i, (u0, ut0) in enumerate(data):
                b.set_initial(i, u0, ut0)
            b.step(2)
            b.step(0)
            b.step(1)
            outs.append([b.gather(i) for i in range(len(shots))])
    for other in outs[1:]:
        for a, c in zip(outs[0], other):
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])


def test_set_initial_restarts_one_shot_only():
    shots = [{"n": 8, "m": 2, "source": _source(8, np.random.default_rng(1))},
             {"n": 6, "m": 3, "source": _source(6, np.random.default_rng(2))},
             {"n": 7, "m": 1}]
    data = [_initial(sh, 50 + i) for i, sh in enumerate(shots)]
    with B.Batch(shots) as b:
        for i, (u0, ut0) in enumerate(data):
            b.set_initial(i, u0, ut0)
        b.step(3)
        b.set_initial(0, *data[0])   # shot 0 back to t = 0
        b.step(2)
        res = [b.gather(i) for i in range(len(shots))]
    ref = [_single(sh, *d, s) for sh, d, s in zip(shots, data, (2, 5, 5))]
    for (gu, gv, t), (su, sv, st) in zip(res, ref):
        assert np.array_equal(gu, su) and np.array_equal(gv, sv) and t == st


def test_zero_batch_stays_zero_and_null_initial_zeroes():
    shots = [{"n": 9, "m": 3}, {"n": 5, "m": 1}]
    with B.Batch(shots) as b:
        b.step(2)
        for i in range(2):
            u, ut, _ = b.gather(i)
            assert not u.any() and not ut.any()
        b.set_initial(1, *_initial(shots[1], 3))
        b.step(1)
        assert np.abs(b.gather(1)[0]).max() > 0
        b.set_initial(1)
        u, ut, t = b.gather(1)
        assert not u.any() and not ut.any() and t == 0.0


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_precision_batch_equals_single_runs(precision):
    shots = [{"n": 8, "m": 3}, {"n": 11, "m": 3, "source": _source(11, np.random.default_rng(5))},
             {"n": 7, "m": 2}]
    data = [_initial(sh, 70 + i) for i, sh in enumerate(shots)]
    with B.Batch(shots, precision=precision) as b:
        for i, (u0, ut0) in enumerate(data):
            b.set_initial(i, u0, ut0)
        b.step(2)
        res = [b.gather(i) for i in range(len(shots))]
    for sh, (u0, ut0), (gu, gv, _) in zip(shots, data, res):
        kw = {"precision": precision} if sh["m"] == 3 else {}
        su, sv, _ = _single(sh, u0, ut0, 2, **kw)
        assert np.array_equal(gu, su) and np.array_equal(gv, sv), sh


def test_rk4_and_other_cfl_batch():
    shots = [{"n": 6, "m": 1}, {"n": 8, "m": 3}, {"n": 5, "m": 2}]
    data = [_initial(sh, 90 + i) for i, sh in enumerate(shots)]
    with B.Batch(shots, cfl=0.3, c=1.7, evolution="rk4", rk_substeps=2) as b:
        for i, (u0, ut0) in enumerate(data):
            b.set_initial(i, u0, ut0)
        b.step(2)
        res = [b.gather(i) for i in range(len(shots))]
    for sh, (u0, ut0), (gu, gv, t) in zip(shots, data, res):
        su, sv, st = _single(sh, u0, ut0, 2, cfl=0.3, c=1.7, evolution="rk4", rk_substeps=2)
        assert np.array_equal(gu, su) and np.array_equal(gv, sv) and t == st


def test_batch_argument_errors():
    with B.Batch([{"n": 4, "m": 1}, {"n": 5, "m": 3}]) as b:
        lib = B.load()
        assert lib.hermite_batch_set_initial(b._b, 2, None, None) == B.HERMITE_EINVAL
        assert lib.hermite_batch_gather(b._b, -1, None, None, None) == B.HERMITE_EINVAL
        assert lib.hermite_batch_step(b._b, -1) == B.HERMITE_EINVAL
        with pytest.raises(B.HermiteError):
            b.tuning(2)   # no shot of order 2
        u = np.zeros(8 * 64)
        assert lib.hermite_batch_set_initial(b._b, 0, B._dptr(u), None) == B.HERMITE_EINVAL


def test_full_size_shots_equal_single_runs_bitwise():
    """Shots at the batched workload's sizes (n up to 96, every order, with
    sources): each equals its single-grid run bit for bit after a few steps
    (the per-cell arithmetic is shared, so at full size too)."""
    rng = np.random.default_rng(11)
    shots = [{"n": 96, "m": 3, "source": _source(96, rng)}, {"n": 64, "m": 2, "source": _source(64, rng)},
             {"n": 48, "m": 1, "source": _source(48, rng)}, {"n": 32, "m": 3, "source": None},
             {"n": 96, "m": 1, "source": None}]
    steps = 5
    print(f"[batch full size] {[(s['n'], s['m']) for s in shots]}", flush=True)
    data = [I.fourier_initial(sh["n"], sh["m"], nmodes=4, kmax=4) for sh in shots]
    with B.Batch(shots) as b:
        for i, (u0, ut0) in enumerate(data):
            b.set_initial(i, u0.numpy(), ut0.numpy())
        b.step(steps)
        res = [b.gather(i) for i in range(len(shots))]
    for sh, (u0, ut0), (gu, gv, _) in zip(shots, data, res):
        su, sv, _ = _single(sh, u0.numpy(), ut0.numpy(), steps)
        assert np.array_equal(gu, su) and np.array_equal(gv, sv), (sh["n"], sh["m"])


def test_graph_replays_interleaved_with_eager_work():
    """Each replay of the captured step, with eager work of the library
    (gathers: copies and scaling kernels) and synchronisations between
    replays, equals the same steps launched directly."""
    shots = _shots(13, 5, (7, 10, 16), (1, 2, 3), True)
    data = [_initial(sh, 200 + i) for i, sh in enumerate(shots)]
    with B.Batch(shots, graph=True) as g, B.Batch(shots, graph=False) as d:
        for i, (u0, ut0) in enumerate(data):
            g.set_initial(i, u0, ut0)
            d.set_initial(i, u0, ut0)
        for step in range(4):
            g.step(1)
            d.step(1)
            for i in range(len(shots)):
                a, b = g.gather(i), d.gather(i)
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (step, i)
            g.sync()
