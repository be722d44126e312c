"""ctypes binding of libhermite.so (the C ABI in include/hermite.h).

Argument marshalling only: every step of the half step runs in the library's
HIP kernels. Loading fails loudly when the library is missing; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhermite.so")

HERMITE_OK = 0
HERMITE_EINVAL = -1
HERMITE_ENOMEM = -2
HERMITE_EDEVICE = -3
HERMITE_ESTATE = -4
HERMITE_EUNSUPPORTED = -5

HERMITE_PREC_FP64 = 0
HERMITE_PREC_FP32 = 1
HERMITE_PREC_BF16X3 = 2
HERMITE_EVOLVE_TAYLOR = 0
HERMITE_EVOLVE_RK4 = 1
HERMITE_KERNEL_AUTO = 0
HERMITE_KERNEL_MFMA = 1
HERMITE_KERNEL_VALU = 2
HERMITE_KERNEL_MFMA4 = 3
HERMITE_EQ_WAVE = 0
HERMITE_EQ_ADVECTION = 1
HERMITE_SLAB_PRIMAL_FIRST = 0
HERMITE_SLAB_PRIMAL_HALO = 1
HERMITE_SLAB_DUAL_LAST = 2
HERMITE_SLAB_DUAL_HALO = 3
HERMITE_SLAB_INTERIOR = 1
HERMITE_SLAB_BOUNDARY = 2
HERMITE_SLAB_ALL = 3
EQUATIONS = {"wave": HERMITE_EQ_WAVE, "advection": HERMITE_EQ_ADVECTION}
KERNELS = {"auto": HERMITE_KERNEL_AUTO, "mfma": HERMITE_KERNEL_MFMA, "valu": HERMITE_KERNEL_VALU,
           "mfma4": HERMITE_KERNEL_MFMA4}

PRECISIONS = {"fp64": HERMITE_PREC_FP64, "fp32": HERMITE_PREC_FP32, "bf16x3": HERMITE_PREC_BF16X3}
EVOLUTIONS = {"taylor": HERMITE_EVOLVE_TAYLOR, "rk4": HERMITE_EVOLVE_RK4}

# every symbol include/hermite.h declares
EXPORTS = (
    "hermite_default_options", "hermite_create", "hermite_set_initial", "hermite_set_initial_device",
    "hermite_step", "hermite_gather", "hermite_gather_device", "hermite_sync", "hermite_get_time",
    "hermite_destroy", "hermite_last_error", "hermite_set_source",
    "hermite_batch_default_options", "hermite_batch_create", "hermite_batch_set_initial", "hermite_batch_step",
    "hermite_batch_gather", "hermite_batch_sync", "hermite_batch_tuning", "hermite_batch_destroy",
    "hermite_batch_last_error", "hermite_set_receivers", "hermite_set_source_series", "hermite_step_record",
    "hermite_adjoint_init", "hermite_adjoint_step", "hermite_adjoint_gather", "hermite_state_finite",
    "hermite_slab_create", "hermite_slab_set_initial", "hermite_slab_plane", "hermite_slab_half_step",
    "hermite_slab_half_step_part",
    "hermite_slab_gather", "hermite_slab_copy_plane", "hermite_slab_sync", "hermite_slab_destroy",
    "hermite_slab_last_error",
)


class hermite_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("evolution", ctypes.c_int),
        ("rk_substeps", ctypes.c_int),
        ("q", ctypes.c_int),
        ("fused", ctypes.c_int),
        ("poison", ctypes.c_int),
        ("kernel", ctypes.c_int),
        ("equation", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class hermite_source(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_double * 3),
        ("sigma", ctypes.c_double),
        ("freq", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("amplitude", ctypes.c_double),
    ]


class hermite_shot(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int),
        ("m", ctypes.c_int),
        ("has_source", ctypes.c_int),
        ("source", hermite_source),
    ]


class hermite_batch_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("evolution", ctypes.c_int),
        ("rk_substeps", ctypes.c_int),
        ("q", ctypes.c_int),
        ("graph", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class HermiteError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hermite error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libhermite.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1609_09841_amd.build.build() "
                          "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    opt_p = ctypes.POINTER(hermite_options)
    lib.hermite_default_options.argtypes = [opt_p]
    lib.hermite_default_options.restype = None
    lib.hermite_create.argtypes = [ip, ip, ctypes.c_double, ctypes.c_double, opt_p, ctypes.POINTER(vp)]
    lib.hermite_create.restype = ip
    lib.hermite_set_initial.argtypes = [vp, dp, dp]
    lib.hermite_set_initial.restype = ip
    lib.hermite_set_initial_device.argtypes = [vp, vp, vp]
    lib.hermite_set_initial_device.restype = ip
    lib.hermite_step.argtypes = [vp, ip]
    lib.hermite_step.restype = ip
    lib.hermite_gather.argtypes = [vp, dp, dp, dp]
    lib.hermite_gather.restype = ip
    lib.hermite_gather_device.argtypes = [vp, vp, vp]
    lib.hermite_gather_device.restype = ip
    lib.hermite_sync.argtypes = [vp]
    lib.hermite_sync.restype = ip
    lib.hermite_get_time.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong), dp]
    lib.hermite_get_time.restype = ip
    lib.hermite_destroy.argtypes = [vp]
    lib.hermite_destroy.restype = None
    lib.hermite_set_source.argtypes = [vp, ctypes.POINTER(hermite_source)]
    lib.hermite_set_source.restype = ip
    lib.hermite_last_error.argtypes = [vp]
    lib.hermite_last_error.restype = ctypes.c_char_p
    lib.hermite_state_finite.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.hermite_state_finite.restype = ip
    lib.hermite_set_receivers.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.hermite_set_receivers.restype = ip
    lib.hermite_set_source_series.argtypes = [vp, vp, ctypes.c_longlong]
    lib.hermite_set_source_series.restype = ip
    lib.hermite_step_record.argtypes = [vp, ip, vp]
    lib.hermite_step_record.restype = ip
    lib.hermite_adjoint_init.argtypes = [vp, vp, vp]
    lib.hermite_adjoint_init.restype = ip
    lib.hermite_adjoint_step.argtypes = [vp, ip, vp, vp]
    lib.hermite_adjoint_step.restype = ip
    lib.hermite_adjoint_gather.argtypes = [vp, vp, vp]
    lib.hermite_adjoint_gather.restype = ip
    bopt_p = ctypes.POINTER(hermite_batch_options)
    lib.hermite_batch_default_options.argtypes = [bopt_p]
    lib.hermite_batch_default_options.restype = None
    lib.hermite_batch_create.argtypes = [ip, ctypes.POINTER(hermite_shot), ctypes.c_double, ctypes.c_double, bopt_p,
                                         ctypes.POINTER(vp)]
    lib.hermite_batch_create.restype = ip
    lib.hermite_batch_set_initial.argtypes = [vp, ip, dp, dp]
    lib.hermite_batch_set_initial.restype = ip
    lib.hermite_batch_step.argtypes = [vp, ip]
    lib.hermite_batch_step.restype = ip
    lib.hermite_batch_gather.argtypes = [vp, ip, dp, dp, dp]
    lib.hermite_batch_gather.restype = ip
    lib.hermite_batch_sync.argtypes = [vp]
    lib.hermite_batch_sync.restype = ip
    lib.hermite_batch_tuning.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int), dp]
    lib.hermite_batch_tuning.restype = ip
    lib.hermite_batch_destroy.argtypes = [vp]
    lib.hermite_batch_destroy.restype = None
    lib.hermite_batch_last_error.argtypes = [vp]
    lib.hermite_batch_last_error.restype = ctypes.c_char_p
    lib.hermite_slab_create.argtypes = [ip, ip, ip, ctypes.c_double, ctypes.c_double, opt_p, ctypes.POINTER(vp)]
    lib.hermite_slab_create.restype = ip
    lib.hermite_slab_set_initial.argtypes = [vp, dp, dp]
    lib.hermite_slab_set_initial.restype = ip
    lib.hermite_slab_plane.argtypes = [vp, ip, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
    lib.hermite_slab_plane.restype = ip
    lib.hermite_slab_half_step.argtypes = [vp, ctypes.POINTER(ip)]
    lib.hermite_slab_half_step.restype = ip
    lib.hermite_slab_half_step_part.argtypes = [vp, ip, ctypes.POINTER(ip)]
    lib.hermite_slab_half_step_part.restype = ip
    lib.hermite_slab_gather.argtypes = [vp, dp, dp, ctypes.POINTER(ctypes.c_double)]
    lib.hermite_slab_gather.restype = ip
    lib.hermite_slab_copy_plane.argtypes = [vp, ip, vp, ip, vp]
    lib.hermite_slab_copy_plane.restype = ip
    lib.hermite_slab_sync.argtypes = [vp]
    lib.hermite_slab_sync.restype = ip
    lib.hermite_slab_destroy.argtypes = [vp]
    lib.hermite_slab_destroy.restype = None
    lib.hermite_slab_last_error.argtypes = [vp]
    lib.hermite_slab_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, ctx=None):
    if rc != HERMITE_OK:
        msg = load().hermite_last_error(ctx).decode(errors="replace")
        raise HermiteError(rc, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --- functions with the C names (thin wrappers returning status codes) -----

def hermite_default_options() -> hermite_options:
    o = hermite_options()
    load().hermite_default_options(ctypes.byref(o))
    return o


def hermite_create(n_cells: int, m: int, cfl: float, c: float, opt: hermite_options | None = None):
    """Returns (status, ctx handle or None)."""
    h = ctypes.c_void_p()
    rc = load().hermite_create(int(n_cells), int(m), float(cfl), float(c),
                               ctypes.byref(opt) if opt is not None else None, ctypes.byref(h))
    return rc, (h if rc == HERMITE_OK else None)


def hermite_set_source(ctx, src: hermite_source | None) -> int:
    return load().hermite_set_source(ctx, ctypes.byref(src) if src is not None else None)


def make_source(x, sigma: float, freq: float, t0: float, amplitude: float) -> hermite_source:
    s = hermite_source()
    for i in range(3):
        s.x[i] = float(x[i])
    s.sigma, s.freq, s.t0, s.amplitude = float(sigma), float(freq), float(t0), float(amplitude)
    return s


def hermite_last_error(ctx=None) -> str:
    return load().hermite_last_error(ctx).decode(errors="replace")


# --- a small owning wrapper ------------------------------------------------

class Solver:
    """One hermite_ctx. Host arrays are numpy float64 of shape
    (M, M, M, n, n, n) or flat; device arrays are torch CUDA float64 tensors."""

    def __init__(self, n: int, m: int, cfl: float = 0.5, c: float = 1.0, *, precision: str = "fp64",
                 evolution: str = "taylor", q: int = 0, rk_substeps: int = 1, fused: bool = True,
                 poison: bool = False, kernel: str = "auto", equation: str = "wave", stream=None):
        lib = load()
        o = hermite_default_options()
        o.precision = PRECISIONS[precision]
        o.evolution = EVOLUTIONS[evolution]
        o.q = int(q)
        o.rk_substeps = int(rk_substeps)
        o.fused = int(bool(fused))
        o.poison = int(bool(poison))
        o.kernel = KERNELS[kernel]
        o.equation = EQUATIONS[equation]
        self.nf = 1 if equation == "advection" else 2
        if stream is not None:
            o.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        self.n, self.m = int(n), int(m)
        self.M3 = (self.m + 1) ** 3
        self.size = self.M3 * self.n ** 3
        self._stream = stream
        rc, h = hermite_create(n, m, cfl, c, o)
        _check(rc, None)
        self._ctx = h
        self._lib = lib

    @property
    def handle(self):
        return self._ctx

    def set_initial(self, u, ut=None):
        """ut is ignored (may be None) for advection."""
        if hasattr(u, "is_cuda") and u.is_cuda:
            assert str(u.dtype) == "torch.float64" and u.is_contiguous() and u.numel() == self.size
            vp = ctypes.c_void_p(ut.data_ptr()) if (ut is not None and self.nf == 2) else None
            if self.nf == 2:
                assert ut.dtype == u.dtype and ut.is_contiguous() and ut.numel() == self.size
            _check(self._lib.hermite_set_initial_device(self._ctx, ctypes.c_void_p(u.data_ptr()), vp), self._ctx)
            return
        a = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).ravel()
        assert a.size == self.size
        if self.nf == 1:
            _check(self._lib.hermite_set_initial(self._ctx, _dptr(a), None), self._ctx)
            return
        b = np.ascontiguousarray(np.asarray(ut, dtype=np.float64)).ravel()
        assert b.size == self.size
        _check(self._lib.hermite_set_initial(self._ctx, _dptr(a), _dptr(b)), self._ctx)

    def set_source(self, source: dict | None):
        """Point source {"x", "sigma", "freq", "t0", "amplitude"}; None removes it."""
        src = None if source is None else make_source(source["x"], source["sigma"], source["freq"],
                                                     source["t0"], source["amplitude"])
        _check(hermite_set_source(self._ctx, src), self._ctx)

    def step(self, nsteps: int = 1):
        _check(self._lib.hermite_step(self._ctx, int(nsteps)), self._ctx)

    # --- receivers and the adjoint sweep (device arrays are torch tensors) ---

    def set_receivers(self, ijk):
        """Primal receiver nodes [(i, j, k), ...]; [] removes them."""
        arr = (ctypes.c_int * (3 * len(ijk)))(*[int(v) for p in ijk for v in p])
        _check(self._lib.hermite_set_receivers(self._ctx, len(ijk), arr), self._ctx)
        self.nrec = len(ijk)

    def set_source_series(self, amps):
        """Scale the source of half step h by amps[h] (CUDA float64 tensor kept
        alive by this object); None removes the scaling."""
        if amps is None:
            _check(self._lib.hermite_set_source_series(self._ctx, None, 0), self._ctx)
            self._amps = None
            return
        assert amps.is_cuda and str(amps.dtype) == "torch.float64" and amps.is_contiguous()
        self._amps = amps
        _check(self._lib.hermite_set_source_series(self._ctx, ctypes.c_void_p(amps.data_ptr()), amps.numel()),
               self._ctx)

    def step_record(self, nsteps: int, traces):
        assert traces.is_cuda and traces.is_contiguous() and traces.numel() == nsteps * self.nrec
        _check(self._lib.hermite_step_record(self._ctx, int(nsteps), ctypes.c_void_p(traces.data_ptr())), self._ctx)

    def adjoint_init(self, lam_u=None, lam_ut=None):
        a = ctypes.c_void_p(lam_u.data_ptr()) if lam_u is not None else None
        b = ctypes.c_void_p(lam_ut.data_ptr()) if lam_ut is not None else None
        _check(self._lib.hermite_adjoint_init(self._ctx, a, b), self._ctx)

    def adjoint_step(self, nsteps: int, res=None, grad_amps=None):
        a = ctypes.c_void_p(res.data_ptr()) if res is not None else None
        b = ctypes.c_void_p(grad_amps.data_ptr()) if grad_amps is not None else None
        _check(self._lib.hermite_adjoint_step(self._ctx, int(nsteps), a, b), self._ctx)

    def adjoint_gather(self, gu=None, gut=None):
        a = ctypes.c_void_p(gu.data_ptr()) if gu is not None else None
        b = ctypes.c_void_p(gut.data_ptr()) if gut is not None else None
        _check(self._lib.hermite_adjoint_gather(self._ctx, a, b), self._ctx)

    def sync(self):
        _check(self._lib.hermite_sync(self._ctx), self._ctx)

    def finite(self) -> bool:
        """True if every DOF of the (adjoint) state is finite."""
        f = ctypes.c_int()
        _check(self._lib.hermite_state_finite(self._ctx, ctypes.byref(f)), self._ctx)
        return bool(f.value)

    def gather(self):
        """(u, ut, t) as numpy arrays shaped (M, M, M, n, n, n); ut is None
        for advection."""
        M, n = self.m + 1, self.n
        u = np.empty((M, M, M, n, n, n))
        ut = np.empty_like(u) if self.nf == 2 else None
        t = ctypes.c_double()
        _check(self._lib.hermite_gather(self._ctx, _dptr(u), _dptr(ut) if ut is not None else None,
                                        ctypes.byref(t)), self._ctx)
        return u, ut, t.value

    def gather_device(self, u, ut=None):
        assert u.is_cuda and u.numel() == self.size
        vp = None
        if ut is not None and self.nf == 2:
            assert ut.is_cuda and ut.numel() == self.size
            vp = ctypes.c_void_p(ut.data_ptr())
        _check(self._lib.hermite_gather_device(self._ctx, ctypes.c_void_p(u.data_ptr()), vp), self._ctx)

    def time(self):
        t, s, dt = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
        _check(self._lib.hermite_get_time(self._ctx, ctypes.byref(t), ctypes.byref(s), ctypes.byref(dt)), self._ctx)
        return t.value, s.value, dt.value

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            self._lib.hermite_destroy(self._ctx)
            self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- batches of independent shots -------------------------------------------

def hermite_batch_default_options() -> hermite_batch_options:
    o = hermite_batch_options()
    load().hermite_batch_default_options(ctypes.byref(o))
    return o


def make_shots(shots) -> ctypes.Array:
    """shots: list of {"n": cells per side, "m": order, "source": dict or None}."""
    arr = (hermite_shot * len(shots))()
    for i, sh in enumerate(shots):
        arr[i].n_cells = int(sh["n"])
        arr[i].m = int(sh["m"])
        src = sh.get("source")
        arr[i].has_source = int(src is not None)
        if src is not None:
            arr[i].source = make_source(src["x"], src["sigma"], src["freq"], src["t0"], src["amplitude"])
    return arr


def hermite_batch_create(shots, cfl: float, c: float, opt: hermite_batch_options | None = None):
    """Returns (status, batch handle or None)."""
    arr = make_shots(shots)
    h = ctypes.c_void_p()
    rc = load().hermite_batch_create(len(shots), arr, float(cfl), float(c),
                                     ctypes.byref(opt) if opt is not None else None, ctypes.byref(h))
    return rc, (h if rc == HERMITE_OK else None)


def hermite_batch_last_error(b=None) -> str:
    return load().hermite_batch_last_error(b).decode(errors="replace")


def _bcheck(rc: int, b=None):
    if rc != HERMITE_OK:
        raise HermiteError(rc, hermite_batch_last_error(b))


class Batch:
    """One hermite_batch: independent shots of uneven sizes and orders stepped
    together. Host arrays are numpy float64 of shape (M, M, M, n, n, n)."""

    def __init__(self, shots, cfl: float = 0.5, c: float = 1.0, *, precision: str = "fp64",
                 evolution: str = "taylor", q: int = 0, rk_substeps: int = 1, graph: bool = True,
                 autotune: bool = True, stream=None):
        lib = load()
        o = hermite_batch_default_options()
        o.precision = PRECISIONS[precision]
        o.evolution = EVOLUTIONS[evolution]
        o.q = int(q)
        o.rk_substeps = int(rk_substeps)
        o.graph = int(bool(graph))
        o.autotune = int(bool(autotune))
        if stream is not None:
            o.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        self.shots = [dict(sh) for sh in shots]
        self._stream = stream
        rc, h = hermite_batch_create(self.shots, cfl, c, o)
        _bcheck(rc, None)
        self._b = h
        self._lib = lib

    def __len__(self):
        return len(self.shots)

    def set_initial(self, shot: int, u=None, ut=None):
        if u is None and ut is None:
            _bcheck(self._lib.hermite_batch_set_initial(self._b, int(shot), None, None), self._b)
            return
        sh = self.shots[shot]
        size = (sh["m"] + 1) ** 3 * sh["n"] ** 3
        a = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).ravel()
        b = np.ascontiguousarray(np.asarray(ut, dtype=np.float64)).ravel()
        assert a.size == size and b.size == size
        _bcheck(self._lib.hermite_batch_set_initial(self._b, int(shot), _dptr(a), _dptr(b)), self._b)

    def step(self, nsteps: int = 1):
        _bcheck(self._lib.hermite_batch_step(self._b, int(nsteps)), self._b)

    def sync(self):
        _bcheck(self._lib.hermite_batch_sync(self._b), self._b)

    def gather(self, shot: int):
        sh = self.shots[shot]
        M, n = sh["m"] + 1, sh["n"]
        u = np.empty((M, M, M, n, n, n))
        ut = np.empty_like(u)
        t = ctypes.c_double()
        _bcheck(self._lib.hermite_batch_gather(self._b, int(shot), _dptr(u), _dptr(ut), ctypes.byref(t)), self._b)
        return u, ut, t.value

    def tuning(self, m: int):
        ch, ms = ctypes.c_int(), ctypes.c_double()
        _bcheck(self._lib.hermite_batch_tuning(self._b, int(m), ctypes.byref(ch), ctypes.byref(ms)), self._b)
        return ch.value, ms.value

    def close(self):
        if getattr(self, "_b", None) is not None:
            self._lib.hermite_batch_destroy(self._b)
            self._b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- z-slabs of a sharded grid ---------------------------------------------

def hermite_slab_last_error(sl=None) -> str:
    return load().hermite_slab_last_error(sl).decode(errors="replace")


def _scheck(rc: int, sl=None):
    if rc != HERMITE_OK:
        raise HermiteError(rc, hermite_slab_last_error(sl))


class Slab:
    """One hermite_slab: the node planes z0 .. z0+nz-1 of a periodic n x n x N
    grid (m = 3, fused FP64 on the matrix cores). Host arrays are numpy
    float64 of shape (M, M, M, nz, n, n). The caller fills the halo plane a
    half step reads (plane(which) gives its device address and row stride)."""

    def __init__(self, n: int, nz: int, m: int = 3, cfl: float = 0.5, c: float = 1.0, *,
                 evolution: str = "taylor", q: int = 0, rk_substeps: int = 1, stream=None):
        lib = load()
        o = hermite_default_options()
        o.evolution = EVOLUTIONS[evolution]
        o.q = int(q)
        o.rk_substeps = int(rk_substeps)
        if stream is not None:
            o.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        h = ctypes.c_void_p()
        _scheck(lib.hermite_slab_create(int(n), int(nz), int(m), float(cfl), float(c), ctypes.byref(o),
                                        ctypes.byref(h)), None)
        self._s, self._lib = h, lib
        self.n, self.nz, self.m = int(n), int(nz), int(m)
        self.rows = 2 * (m + 1) ** 3
        self._stream = stream

    def set_initial(self, u, ut):
        size = (self.m + 1) ** 3 * self.nz * self.n ** 2
        a = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).ravel()
        b = np.ascontiguousarray(np.asarray(ut, dtype=np.float64)).ravel()
        assert a.size == size and b.size == size
        _scheck(self._lib.hermite_slab_set_initial(self._s, _dptr(a), _dptr(b)), self._s)

    def plane(self, which: int):
        """(device address, row stride in bytes) of a HERMITE_SLAB_* plane:
        2 (m+1)^3 rows of n^2 doubles."""
        p, pitch = ctypes.c_void_p(), ctypes.c_size_t()
        _scheck(self._lib.hermite_slab_plane(self._s, int(which), ctypes.byref(p), ctypes.byref(pitch)), self._s)
        return p.value, pitch.value

    def half_step(self) -> int:
        """Enqueue one half step; returns the HERMITE_SLAB_*_HALO plane the next one reads."""
        nxt = ctypes.c_int()
        _scheck(self._lib.hermite_slab_half_step(self._s, ctypes.byref(nxt)), self._s)
        return nxt.value

    def gather(self):
        M = self.m + 1
        u = np.empty((M, M, M, self.nz, self.n, self.n))
        ut = np.empty_like(u)
        t = ctypes.c_double()
        _scheck(self._lib.hermite_slab_gather(self._s, _dptr(u), _dptr(ut), ctypes.byref(t)), self._s)
        return u, ut, t.value

    def half_step_part(self, part: int) -> int:
        """hermite_slab_half_step_part: HERMITE_SLAB_INTERIOR, _BOUNDARY or _ALL;
        returns the halo plane that the next part or half step reads."""
        nxt = ctypes.c_int()
        _scheck(self._lib.hermite_slab_half_step_part(self._s, int(part), ctypes.byref(nxt)), self._s)
        return nxt.value

    def copy_plane_from(self, which: int, src: "Slab", src_which: int, stream=None):
        """Fill plane `which` of this slab from plane `src_which` of `src`
        (hermite_slab_copy_plane), on `stream` (a torch stream or handle;
        None: this slab's stream)."""
        st = None if stream is None else ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        _scheck(self._lib.hermite_slab_copy_plane(self._s, int(which), src._s, int(src_which), st), self._s)

    def sync(self):
        _scheck(self._lib.hermite_slab_sync(self._s), self._s)

    def close(self):
        if getattr(self, "_s", None) is not None:
            self._lib.hermite_slab_destroy(self._s)
            self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

