"""GPU tests of z-slabs of a sharded periodic grid (hermite_slab_*), through
the C ABI.

A slab runs the same per-cell arithmetic as the cube's fused matrix-core
kernel (same operator, same batch of 16 cells per MFMA), only over its own
cell planes with the neighbour planes held as halos. So slabs that exchange
their boundary planes every half step (here on one device, by plane copies
on one stream, the stand-in for peer copies between GPUs) must reproduce
the single-grid run bit for bit, and with it the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1609_09841_amd import binding as B
from paper_1609_09841_amd import inputs as I

pytestmark = pytest.mark.gpu


def _cube(n, u0, ut0, steps, **kw):
    with B.Solver(n, 3, **kw) as s:
        s.set_initial(u0, ut0)
        s.step(steps)
        u, ut, _ = s.gather()
    return u, ut


def _run_slabs(n, splits, u0, ut0, steps, **kw):
    """Slabs of the given plane counts (bottom to top) on one torch stream;
    halos exchanged before every half step. Returns the gathered grid."""
    stream = torch.cuda.Stream()
    z = np.cumsum([0] + list(splits))
    slabs = [B.Slab(n, nz, stream=stream, **kw) for nz in splits]
    try:
        for g, sl in enumerate(slabs):
            sl.set_initial(u0[:, :, :, z[g]:z[g + 1]], ut0[:, :, :, z[g]:z[g + 1]])
        G = len(slabs)
        nxt = B.HERMITE_SLAB_PRIMAL_HALO
        for _ in range(2 * steps):
            for g, sl in enumerate(slabs):
                if nxt == B.HERMITE_SLAB_PRIMAL_HALO:
                    sl.copy_plane_from(B.HERMITE_SLAB_PRIMAL_HALO, slabs[(g + 1) % G], B.HERMITE_SLAB_PRIMAL_FIRST)
                else:
                    sl.copy_plane_from(B.HERMITE_SLAB_DUAL_HALO, slabs[(g - 1) % G], B.HERMITE_SLAB_DUAL_LAST)
            for sl in slabs:
                nxt = sl.half_step()
        parts = [sl.gather() for sl in slabs]
        t = parts[0][2]
        assert all(p[2] == t for p in parts)
        return np.concatenate([p[0] for p in parts], axis=3), np.concatenate([p[1] for p in parts], axis=3), t
    finally:
        for sl in slabs:
            sl.close()


@pytest.mark.parametrize("n", [5, 12, 20])
def test_one_slab_holding_the_grid_equals_the_cube(n):
    """nz = n, halos copied from the slab's own boundary planes (the
    periodic wrap)."""
    rng = np.random.default_rng(n)
    u0 = rng.standard_normal((4, 4, 4, n, n, n))
    ut0 = rng.standard_normal((4, 4, 4, n, n, n))
    print(f"[slab self] n={n}", flush=True)
    su, sut, t = _run_slabs(n, [n], u0, ut0, 3)
    cu, cut = _cube(n, u0, ut0, 3)
    assert np.array_equal(su, cu) and np.array_equal(sut, cut)
    assert t == pytest.approx(3 * 0.5 / n, rel=1e-15)


@pytest.mark.parametrize("splits", [(4, 4, 4), (5, 4, 3), (1, 7, 2, 2), (12,)])
def test_exchanging_slabs_equal_the_cube_and_the_oracle(splits):
    n = 12
    rng = np.random.default_rng(sum(splits) * 7 + len(splits))
    u0 = rng.standard_normal((4, 4, 4, n, n, n))
    ut0 = rng.standard_normal((4, 4, 4, n, n, n))
    print(f"[slab exchange] n={n} splits={splits}", flush=True)
    su, sut, _ = _run_slabs(n, splits, u0, ut0, 2)
    cu, cut = _cube(n, u0, ut0, 2)
    assert np.array_equal(su, cu) and np.array_equal(sut, cut)
    ou, out_ = O.run(n, 3, 0.5, 1.0, u0, ut0, 2)
    eu, ev = I.rel_l2(su, ou), I.rel_l2(sut, out_)
    if eu > 1e-12 or ev > 1e-12:
        lu, lv = O.run(n, 3, 0.5, 1.0, u0, ut0, 2, ld=True)
        fu, fv = I.rel_l2(ou, lu), I.rel_l2(out_, lv)
        print(f"  slab-oracle {eu:.2e} {ev:.2e}, floor {fu:.2e} {fv:.2e}", flush=True)
        assert eu <= max(1e-12, 3 * fu) and ev <= max(1e-12, 3 * fv)


def test_rk4_slabs_equal_the_cube():
    n = 9
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal((4, 4, 4, n, n, n))
    ut0 = rng.standard_normal((4, 4, 4, n, n, n))
    su, sut, _ = _run_slabs(n, (3, 6), u0, ut0, 2, evolution="rk4", rk_substeps=2, cfl=0.3, c=1.7)
    cu, cut = _cube(n, u0, ut0, 2, evolution="rk4", rk_substeps=2, cfl=0.3, c=1.7)
    assert np.array_equal(su, cu) and np.array_equal(sut, cut)


def test_one_devices_share_of_the_128_cube():
    """The 128^3 workload cut into 8 slabs of 128 x 128 x 16 cells (one
    device's share of an 8-way split): the slabs reproduce the cube."""
    n, steps = 128, 2
    u0, ut0 = I.fourier_initial(n, 3)
    u0, ut0 = u0.numpy(), ut0.numpy()
    print("[slab 128^3 / 8]", flush=True)
    su, sut, _ = _run_slabs(n, [16] * 8, u0, ut0, steps)
    cu, cut = _cube(n, u0, ut0, steps)
    assert np.array_equal(su, cu) and np.array_equal(sut, cut)


def test_slab_state_and_argument_errors():
    n = 6
    with B.Slab(n, 3) as sl:
        with pytest.raises(B.HermiteError) as e:
            sl.half_step()
        assert e.value.code == B.HERMITE_ESTATE
        with pytest.raises(B.HermiteError) as e:
            sl.plane(7)
        assert e.value.code == B.HERMITE_EINVAL
        z = np.zeros((4, 4, 4, 3, n, n))
        sl.set_initial(z, z)
        assert sl.half_step() == B.HERMITE_SLAB_DUAL_HALO
        with pytest.raises(B.HermiteError) as e:
            sl.gather()   # odd number of half steps
        assert e.value.code == B.HERMITE_ESTATE
        assert sl.half_step() == B.HERMITE_SLAB_PRIMAL_HALO
        u, ut, t = sl.gather()
        assert not u.any() and not ut.any() and t == pytest.approx(0.5 / n)
        p0, pitch = sl.plane(B.HERMITE_SLAB_PRIMAL_FIRST)
        p1, _ = sl.plane(B.HERMITE_SLAB_PRIMAL_HALO)
        assert p1 - p0 == 3 * n * n * 8 and pitch >= 4 * n * n * 8
        with B.Slab(n + 1, 3) as other:
            with pytest.raises(B.HermiteError) as e:
                sl.copy_plane_from(B.HERMITE_SLAB_PRIMAL_HALO, other, B.HERMITE_SLAB_PRIMAL_FIRST)
            assert e.value.code == B.HERMITE_EINVAL


def _run_slabs_split(n, splits, u0, ut0, steps, comm_stream=False):
    """As _run_slabs, each half step in two parts: the interior cells, then
    (after the halo copies) the boundary plane. With comm_stream the copies
    run on a second stream, overlapping the interior parts, ordered by
    events."""
    stream = torch.cuda.Stream()
    comm = torch.cuda.Stream() if comm_stream else None
    z = np.cumsum([0] + list(splits))
    slabs = [B.Slab(n, nz, stream=stream) for nz in splits]
    try:
        for g, sl in enumerate(slabs):
            sl.set_initial(u0[:, :, :, z[g]:z[g + 1]], ut0[:, :, :, z[g]:z[g + 1]])
        G = len(slabs)
        for _ in range(2 * steps):
            ready = torch.cuda.Event()
            ready.record(stream)              # the planes to copy are final
            halos = [sl.half_step_part(B.HERMITE_SLAB_INTERIOR) for sl in slabs]
            cs = comm if comm_stream else stream
            if comm_stream:
                comm.wait_event(ready)
            for g, sl in enumerate(slabs):
                if halos[g] == B.HERMITE_SLAB_PRIMAL_HALO:
                    sl.copy_plane_from(halos[g], slabs[(g + 1) % G], B.HERMITE_SLAB_PRIMAL_FIRST, stream=cs)
                else:
                    sl.copy_plane_from(halos[g], slabs[(g - 1) % G], B.HERMITE_SLAB_DUAL_LAST, stream=cs)
            if comm_stream:
                done = torch.cuda.Event()
                done.record(comm)
                stream.wait_event(done)
            for sl in slabs:
                sl.half_step_part(B.HERMITE_SLAB_BOUNDARY)
        parts = [sl.gather() for sl in slabs]
        return np.concatenate([p[0] for p in parts], axis=3), np.concatenate([p[1] for p in parts], axis=3)
    finally:
        for sl in slabs:
            sl.close()


@pytest.mark.parametrize("comm_stream", [False, True], ids=["one_stream", "copies_overlapping"])
@pytest.mark.parametrize("splits", [(4, 4, 4), (1, 5, 6), (12,)])
def test_split_half_steps_equal_the_cube(splits, comm_stream):
    n = 12
    rng = np.random.default_rng(40 + len(splits))
    u0 = rng.standard_normal((4, 4, 4, n, n, n))
    ut0 = rng.standard_normal((4, 4, 4, n, n, n))
    print(f"[slab split] splits={splits} comm_stream={comm_stream}", flush=True)
    su, sut = _run_slabs_split(n, splits, u0, ut0, 2, comm_stream)
    cu, cut = _cube(n, u0, ut0, 2)
    assert np.array_equal(su, cu) and np.array_equal(sut, cut)


def test_split_part_order_errors():
    n = 6
    with B.Slab(n, 3) as sl:
        z = np.zeros((4, 4, 4, 3, n, n))
        sl.set_initial(z, z)
        with pytest.raises(B.HermiteError) as e:
            sl.half_step_part(B.HERMITE_SLAB_BOUNDARY)
        assert e.value.code == B.HERMITE_ESTATE
        assert sl.half_step_part(B.HERMITE_SLAB_INTERIOR) == B.HERMITE_SLAB_PRIMAL_HALO
        for part in (B.HERMITE_SLAB_INTERIOR, B.HERMITE_SLAB_ALL):
            with pytest.raises(B.HermiteError) as e:
                sl.half_step_part(part)
            assert e.value.code == B.HERMITE_ESTATE
        with pytest.raises(B.HermiteError) as e:
            sl.gather()
        assert e.value.code == B.HERMITE_ESTATE
        assert sl.half_step_part(B.HERMITE_SLAB_BOUNDARY) == B.HERMITE_SLAB_DUAL_HALO
        assert sl.half_step_part(B.HERMITE_SLAB_INTERIOR) == B.HERMITE_SLAB_DUAL_HALO
        assert sl.half_step_part(B.HERMITE_SLAB_BOUNDARY) == B.HERMITE_SLAB_PRIMAL_HALO
        with pytest.raises(B.HermiteError) as e:
            sl.half_step_part(0)
        assert e.value.code == B.HERMITE_EINVAL
        sl.gather()
