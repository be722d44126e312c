"""GPU tests of receivers and the adjoint sweep (transposed half steps),
through the C ABI, and of the autograd Function built on them.

References: the GPU forward itself through <F x, y> = <x, F^T y> (the
definition of the transpose), the CPU oracle's adjoint recursion
(oracle.adjoint_series, pinned against central differences of the oracle's
forward), and central differences of the quadratic misfit evaluated with
the GPU forward (exact up to rounding for a quadratic).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1609_09841_amd import binding as B
from paper_1609_09841_amd import inputs as I
from paper_1609_09841_amd.autograd import receiver_traces

pytestmark = pytest.mark.gpu


def rel(a, b):
    return I.rel_l2(np.asarray(a), np.asarray(b))


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _src(n, t0=0.1, amp=30.0):
    f0 = n / 8.0
    return {"x": (0.41, 0.52, 0.37), "sigma": 2.0 / n, "freq": f0, "t0": t0, "amplitude": amp}


@pytest.mark.parametrize("evolution", ["taylor", "rk4"])
@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("n", [5, 8])
def test_transpose_dot_product_identity(n, m, evolution):
    steps = 3
    M = m + 1
    rng = np.random.default_rng(10 * n + m)
    x = [rng.standard_normal((M, M, M, n, n, n)) for _ in range(2)]
    y = [rng.standard_normal((M, M, M, n, n, n)) for _ in range(2)]
    print(f"[adjoint dot] n={n} m={m} {evolution}", flush=True)
    with B.Solver(n, m, 0.5, 1.3, evolution=evolution) as s:
        s.set_initial(*x)
        s.step(steps)
        fu, fut, _ = s.gather()
        gu = torch.empty((M, M, M, n, n, n), dtype=torch.float64, device="cuda")
        gut = torch.empty_like(gu)
        s.adjoint_init(_t(y[0]), _t(y[1]))
        s.adjoint_step(steps)
        s.adjoint_gather(gu, gut)
        s.sync()
    lhs = np.sum(fu * y[0]) + np.sum(fut * y[1])
    rhs = np.sum(x[0] * gu.cpu().numpy()) + np.sum(x[1] * gut.cpu().numpy())
    scale = np.sqrt(np.sum(fu ** 2) + np.sum(fut ** 2)) * np.sqrt(np.sum(y[0] ** 2) + np.sum(y[1] ** 2))
    err = abs(lhs - rhs) / scale
    print(f"  <Fx,y> {lhs:.6e} <x,F^T y> {rhs:.6e} rel {err:.2e}", flush=True)
    assert err <= {1: 1e-13, 2: 1e-13, 3: 1e-11}[m]


def test_step_record_traces_equal_gathered_values():
    n, m = 7, 2
    u0, ut0 = I.fourier_initial(n, m, nmodes=3, kmax=2)
    rec = [(0, 0, 0), (3, 5, 6), (6, 1, 2), (3, 5, 6)]
    with B.Solver(n, m) as s:
        s.set_receivers(rec)
        s.set_initial(u0.numpy(), ut0.numpy())
        tr = torch.empty((4, len(rec)), dtype=torch.float64, device="cuda")
        s.step_record(4, tr)
        u, _, _ = s.gather()
    ou, _ = O.run(n, m, 0.5, 1.0, u0.numpy(), ut0.numpy(), 4)
    got = tr.cpu().numpy()[-1]
    assert np.array_equal(got, np.array([u[0, 0, 0, k, j, i] for (i, j, k) in rec]))
    assert rel(got, [ou[0, 0, 0, k, j, i] for (i, j, k) in rec]) <= 1e-12


@pytest.mark.parametrize("m", [1, 2, 3])
def test_gradients_match_oracle_adjoint(m):
    n, steps, cfl, c = 6, 3, 0.5, 1.3
    M = m + 1
    rng = np.random.default_rng(m)
    u0 = rng.standard_normal((M, M, M, n, n, n))
    ut0 = rng.standard_normal((M, M, M, n, n, n))
    amps = rng.uniform(0.5, 1.5, 2 * steps)
    src = _src(n)
    rec = [(0, 0, 4), (3, 1, 4), (5, 4, 4), (2, 2, 1)]
    res = rng.standard_normal((steps, len(rec)))
    print(f"[adjoint vs oracle] n={n} m={m}", flush=True)
    with B.Solver(n, m, cfl, c) as s:
        s.set_receivers(rec)
        s.set_source(src)
        s.set_initial(u0, ut0)
        a = _t(amps)
        s.set_source_series(a)
        tr = torch.empty((steps, len(rec)), dtype=torch.float64, device="cuda")
        s.step_record(steps, tr)
        gu = torch.empty((M, M, M, n, n, n), dtype=torch.float64, device="cuda")
        gut = torch.empty_like(gu)
        ga = torch.empty(2 * steps, dtype=torch.float64, device="cuda")
        s.adjoint_init()
        s.adjoint_step(steps, _t(res), ga)
        s.adjoint_gather(gu, gut)
        s.sync()
    otr, _, _ = O.run_series(n, m, cfl, c, u0, ut0, steps, src, amps, rec)
    ogu, ogut, oga = O.adjoint_series(n, m, cfl, c, steps, src, rec, res)
    tol = 1e-12 if m < 3 else 1e-10
    e = (rel(tr.cpu(), otr), rel(gu.cpu().numpy().ravel(), ogu), rel(gut.cpu().numpy().ravel(), ogut),
         rel(ga.cpu(), oga))
    print(f"  traces {e[0]:.2e} gu {e[1]:.2e} gut {e[2]:.2e} gamps {e[3]:.2e}", flush=True)
    assert max(e) <= tol, e


def test_autograd_gradient_matches_central_differences():
    """torch.autograd through the library: J = 1/2 |traces - obs|^2, gradient
    against central differences of J evaluated with the GPU forward."""
    n, m, steps = 12, 2, 6
    M = m + 1
    rng = np.random.default_rng(7)
    u0 = _t(rng.standard_normal((M, M, M, n, n, n)))
    ut0 = _t(rng.standard_normal((M, M, M, n, n, n)))
    amps = _t(rng.uniform(0.5, 1.5, 2 * steps))
    rec = [(i, (3 * i) % n, 9) for i in range(8)]
    obs = _t(rng.standard_normal((steps, len(rec))))
    with B.Solver(n, m) as s:
        s.set_receivers(rec)
        s.set_source(_src(n, t0=0.05))

        def J(a, b, c):
            return 0.5 * ((receiver_traces(s, a, b, c, steps) - obs) ** 2).sum()

        x = [u0.clone().requires_grad_(), ut0.clone().requires_grad_(), amps.clone().requires_grad_()]
        val = J(*x)
        grads = torch.autograd.grad(val, x)
        for which in range(3):
            d = [torch.zeros_like(v) for v in x]
            d[which] = _t(rng.standard_normal(tuple(x[which].shape)))
            eps = 1e-3
            with torch.no_grad():
                jp = J(*[v + eps * dv for v, dv in zip(x, d)]).item()
                jm = J(*[v - eps * dv for v, dv in zip(x, d)]).item()
            fd = (jp - jm) / (2 * eps)
            ad = sum((g * dv).sum().item() for g, dv in zip(grads, d))
            print(f"  direction {which}: fd {fd:.10e} adjoint {ad:.10e}", flush=True)
            assert fd == pytest.approx(ad, rel=1e-7)


def test_adjoint_errors():
    with B.Solver(5, 1) as s:
        with pytest.raises(B.HermiteError) as e:
            s.adjoint_init()
        assert e.value.code == B.HERMITE_ESTATE
        with pytest.raises(B.HermiteError) as e:
            s.set_receivers([(0, 0, 5)])
        assert e.value.code == B.HERMITE_EINVAL
        with pytest.raises(B.HermiteError) as e:
            s.set_source_series(_t(np.ones(4)))
        assert e.value.code == B.HERMITE_ESTATE
        s.set_source(_src(5))
        s.set_source_series(_t(np.ones(4)))
        z = np.zeros((2, 2, 2, 5, 5, 5))
        s.set_initial(z, z)
        s.step(2)
        with pytest.raises(B.HermiteError) as e:
            s.step(1)   # the series covers 4 half steps
        assert e.value.code == B.HERMITE_EINVAL
        s.adjoint_init()
        with pytest.raises(B.HermiteError) as e:
            s.adjoint_step(3)   # only 2 steps to reverse
        assert e.value.code == B.HERMITE_EINVAL
    with B.Solver(5, 1, equation="advection") as s:
        s.set_initial(np.zeros((2, 2, 2, 5, 5, 5)))
        with pytest.raises(B.HermiteError) as e:
            s.adjoint_init()
        assert e.value.code == B.HERMITE_EUNSUPPORTED


def test_differentiation_workload_small_copy():
    """The differentiation workload's shape on a 16^3, m = 2 copy: Ricker
    source at the cube centre, receivers on the node plane z = 0.75, misfit
    against traces from perturbed initial data. Checks: the dot-product
    identity of the whole sweep, and central differences of J for u0, u_t0
    and the source series."""
    n, m, steps = 16, 2, 10
    M = m + 1
    rng = np.random.default_rng(1609)
    src = {"x": (0.5, 0.5, 0.5), "sigma": 2.0 / n, "freq": n / 8.0, "t0": 0.05, "amplitude": 20.0}
    kz = int(round(0.75 * n))
    rec = [(int(i), int(j), kz) for i, j in zip(rng.integers(0, n, 32), rng.integers(0, n, 32))]
    u0 = _t(rng.standard_normal((M, M, M, n, n, n)))
    ut0 = _t(rng.standard_normal((M, M, M, n, n, n)))
    du = _t(rng.standard_normal((M, M, M, n, n, n)))
    amps = _t(np.ones(2 * steps))
    print(f"[differentiation copy] n={n} m={m} receivers on k={kz}", flush=True)
    with B.Solver(n, m) as s:
        s.set_receivers(rec)
        s.set_source(src)
        with torch.no_grad():
            obs = receiver_traces(s, u0 + 0.1 * du, ut0, amps, steps)

        def J(a, b, c):
            return 0.5 * ((receiver_traces(s, a, b, c, steps) - obs) ** 2).sum()

        x = [u0.clone().requires_grad_(), ut0.clone().requires_grad_(), amps.clone().requires_grad_()]
        grads = torch.autograd.grad(J(*x), x)
        for which in range(3):
            d = [torch.zeros_like(v) for v in x]
            d[which] = _t(rng.standard_normal(tuple(x[which].shape)))
            eps = 1e-3
            with torch.no_grad():
                fd = (J(*[v + eps * dv for v, dv in zip(x, d)]).item()
                      - J(*[v - eps * dv for v, dv in zip(x, d)]).item()) / (2 * eps)
            ad = sum((g * dv).sum().item() for g, dv in zip(grads, d))
            print(f"  direction {which}: fd {fd:.10e} adjoint {ad:.10e}", flush=True)
            assert fd == pytest.approx(ad, rel=1e-7)
        # dot-product identity of the sweep: <F x, y> = <x, F^T y>
        y = [rng.standard_normal((M, M, M, n, n, n)) for _ in range(2)]
        xs = [rng.standard_normal((M, M, M, n, n, n)) for _ in range(2)]
    with B.Solver(n, m) as s:
        s.set_initial(*xs)
        s.step(steps)
        fu, fut, _ = s.gather()
        gu = torch.empty((M, M, M, n, n, n), dtype=torch.float64, device="cuda")
        gut = torch.empty_like(gu)
        s.adjoint_init(_t(y[0]), _t(y[1]))
        s.adjoint_step(steps)
        s.adjoint_gather(gu, gut)
        s.sync()
    lhs = np.sum(fu * y[0]) + np.sum(fut * y[1])
    rhs = np.sum(xs[0] * gu.cpu().numpy()) + np.sum(xs[1] * gut.cpu().numpy())
    scale = np.sqrt(np.sum(fu ** 2) + np.sum(fut ** 2)) * np.sqrt(np.sum(y[0] ** 2) + np.sum(y[1] ** 2))
    assert abs(lhs - rhs) / scale <= 1e-13


@pytest.mark.parametrize("kernel", ["mfma", "valu"])
def test_m3_adjoint_on_contexts_of_other_forward_kernels(kernel):
    """A context whose forward half step is not the default kernel has no
    work queue until the adjoint needs one: its transposed half steps equal
    those of a default context bit for bit (odd n, so the last row pair of
    some XCDs has no upper row)."""
    n, steps, M = 21, 3, 4
    rng = np.random.default_rng(2100)
    x = [rng.standard_normal((M, M, M, n, n, n)) for _ in range(2)]
    y = [rng.standard_normal((M, M, M, n, n, n)) for _ in range(2)]
    print(f"[adjoint queue] n={n} kernel={kernel}", flush=True)
    out = {}
    for kern in ("auto", kernel):
        with B.Solver(n, 3, 0.5, 1.0, kernel=kern) as s:
            s.set_initial(*x)
            s.step(steps)
            gu = torch.empty((M, M, M, n, n, n), dtype=torch.float64, device="cuda")
            gut = torch.empty_like(gu)
            s.adjoint_init(_t(y[0]), _t(y[1]))
            s.adjoint_step(steps)
            s.adjoint_gather(gu, gut)
            s.sync()
            out[kern] = (gu.cpu().numpy(), gut.cpu().numpy())
    assert np.array_equal(out["auto"][0], out[kernel][0]) and np.array_equal(out["auto"][1], out[kernel][1])
