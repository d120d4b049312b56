"""Thin ctypes binding of the C ABI in include/lc.h.

Every entry point of the library has a function of the same name here that
only marshals arguments; all arithmetic runs in the HIP kernels of liblc.so.
PyTorch provides device memory and the stream.  If the shared library is
missing this module raises on import: there is no fallback path.

The convenience class :class:`Solver` owns the torch buffers of one grid.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblc.so")

LC_OK, LC_EINVAL, LC_ENOMEM, LC_EDEVICE, LC_ENONFINITE, LC_ESTATE, LC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LC_D2Q9, LC_D3Q19 = 0, 1
LC_FP64, LC_FP32_DEV, LC_MIXED, LC_FP32_SR = 0, 1, 2, 3
LC_VARIANT_AUTO, LC_VARIANT_STAGED, LC_VARIANT_SPLIT, LC_VARIANT_FUSED = 0, 1, 2, 3
LC_COLL_BGK, LC_COLL_MRT = 0, 1
LC_STENCIL_COMPACT, LC_STENCIL_ISOTROPIC = 0, 1
LC_OBS_MASS, LC_OBS_MOM, LC_OBS_UMAX, LC_OBS_S, LC_OBS_ALL = 1, 2, 4, 8, 15
LC_FIELD_F, LC_FIELD_Q, LC_FIELD_RHO, LC_FIELD_U, LC_FIELD_FORCE, LC_FIELD_S = range(6)

LATTICES = {"D2Q9": LC_D2Q9, "D3Q19": LC_D3Q19}
PRECISIONS = {"fp64": LC_FP64, "fp32dev": LC_FP32_DEV, "mixed": LC_MIXED, "fp32sr": LC_FP32_SR}


class lc_grid(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class lc_params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("A0", "gamma", "K", "Gamma", "xi", "eta", "tau")]


class lc_buffers(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p * 2), ("Q", ctypes.c_void_p * 2), ("scratch", ctypes.c_void_p)]


class lc_observables(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("mom", ctypes.c_double * 3), ("umax", ctypes.c_double),
                ("ssum", ctypes.c_double), ("ssum_half", ctypes.c_double), ("step", ctypes.c_int64),
                ("nonfinite", ctypes.c_int32), ("half_axis", ctypes.c_int32)]


class LCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lc error %d: %s" % (code, msg))
        self.code = code


def _load():
    # torch ships its own HIP runtime under the same soname as ROCm's; the
    # first one loaded serves the whole process.  Loading torch first makes
    # the library share torch's runtime (and so its devices and streams)
    # whichever module the caller imported first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library %s is missing: build it with "
                          "`python -m paper_1907_13415_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sigs = {
        "lc_last_error": ([], ctypes.c_char_p),
        "lc_lattice_info": ([ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_double)], ctypes.c_int32),
        "lc_buffer_bytes": ([P(lc_grid), P(ctypes.c_size_t), P(ctypes.c_size_t), P(ctypes.c_size_t)], ctypes.c_int32),
        "lc_init": ([P(lc_grid), P(lc_params), P(lc_buffers), ctypes.c_void_p, P(ctypes.c_void_p)], ctypes.c_int32),
        "lc_set_params": ([ctypes.c_void_p, P(lc_params)], ctypes.c_int32),
        "lc_set_variant": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
        "lc_set_chunk": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
        "lc_set_stencil": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
        "lc_load_state": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int32),
        "lc_step": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int32),
        "lc_observe": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32, P(lc_observables)], ctypes.c_int32),
        "lc_export": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p], ctypes.c_int32),
        "lc_sync": ([ctypes.c_void_p], ctypes.c_int32),
        "lc_vjp_step": ([ctypes.c_void_p] * 6, ctypes.c_int32),
        "lc_vjp_history_bytes": ([P(lc_grid), ctypes.c_int32], ctypes.c_size_t),
        "lc_set_collision": ([ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32], ctypes.c_int32),
        "lc_vjp_backward_bytes": ([P(lc_grid), ctypes.c_int32], ctypes.c_size_t),
        "lc_vjp_backward": ([ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_void_p), P(ctypes.c_void_p),
                             P(ctypes.c_int32)] + [ctypes.c_void_p] * 4, ctypes.c_int32),
        "lc_vjp_segment": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 4,
                           ctypes.c_int32),
        "lc_set_timing": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
        "lc_get_timing": ([ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int64)], ctypes.c_int32),
        "lc_step_count": ([ctypes.c_void_p], ctypes.c_int64),
        "lc_free": ([ctypes.c_void_p], ctypes.c_int32),
        "lc_batch_layout": ([ctypes.c_int32, P(lc_grid), P(ctypes.c_size_t), P(ctypes.c_size_t),
                             P(ctypes.c_size_t), P(ctypes.c_size_t), P(ctypes.c_size_t)], ctypes.c_int32),
        "lc_batch_init": ([ctypes.c_int32, P(lc_grid), P(lc_params), P(lc_buffers), ctypes.c_void_p,
                           P(ctypes.c_void_p)], ctypes.c_int32),
        "lc_batch_load_state": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int32),
        "lc_batch_step": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int32),
        "lc_batch_set_tile": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
        "lc_batch_set_tiles": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32], ctypes.c_int32),
        "lc_batch_set_collision": ([ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32],
                                   ctypes.c_int32),
        "lc_batch_set_stencil": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
        "lc_batch_autotune": ([ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_double)],
                              ctypes.c_int32),
        "lc_batch_observe": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32, P(lc_observables)], ctypes.c_int32),
        "lc_batch_export": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p], ctypes.c_int32),
        "lc_batch_free": ([ctypes.c_void_p], ctypes.c_int32),
        "lc_step_static": ([P(lc_grid), P(lc_params), P(ctypes.c_void_p), P(ctypes.c_void_p), ctypes.c_int32,
                            ctypes.c_int64, ctypes.c_void_p], ctypes.c_int32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def _check(rc):
    if rc != LC_OK:
        raise LCError(rc, _lib.lc_last_error().decode())
    return rc


# ---------------------------------------------------------------- raw calls
def lc_last_error():
    return _lib.lc_last_error().decode()


def lc_lattice_info(lattice):
    q = ctypes.c_int32()
    c = (ctypes.c_int32 * 57)()
    w = (ctypes.c_double * 19)()
    _check(_lib.lc_lattice_info(lattice, ctypes.byref(q), c, w))
    n = q.value
    return np.array(c[: 3 * n], dtype=np.int64).reshape(n, 3), np.array(w[:n])


def make_grid(lattice, precision, nx, ny, nz=1):
    return lc_grid(lattice, precision, nx, ny, nz)


def make_params(A0, gamma, K, Gamma, xi, tau, eta=None):
    if eta is None:
        eta = (tau - 0.5) / 3.0
    return lc_params(A0, gamma, K, Gamma, xi, eta, tau)


def lc_buffer_bytes(grid):
    fb, qb, sb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.lc_buffer_bytes(ctypes.byref(grid), ctypes.byref(fb), ctypes.byref(qb), ctypes.byref(sb)))
    return fb.value, qb.value, sb.value


def lc_init(grid, params, bufs, stream):
    ctx = ctypes.c_void_p()
    _check(_lib.lc_init(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(bufs),
                        ctypes.c_void_p(stream), ctypes.byref(ctx)))
    return ctx


def lc_set_params(ctx, params):
    _check(_lib.lc_set_params(ctx, ctypes.byref(params)))


def lc_set_variant(ctx, variant):
    _check(_lib.lc_set_variant(ctx, variant))


def lc_set_chunk(ctx, planes):
    _check(_lib.lc_set_chunk(ctx, int(planes)))


def lc_set_stencil(ctx, stencil):
    _check(_lib.lc_set_stencil(ctx, int(stencil)))


def lc_load_state(ctx, f_ptr, q_ptr):
    _check(_lib.lc_load_state(ctx, ctypes.c_void_p(f_ptr), ctypes.c_void_p(q_ptr)))


def lc_step(ctx, n):
    _check(_lib.lc_step(ctx, int(n)))


def lc_observe(ctx, mask=LC_OBS_ALL, half_axis=0, allow_nonfinite=False):
    o = lc_observables()
    rc = _lib.lc_observe(ctx, mask, half_axis, ctypes.byref(o))
    if not (allow_nonfinite and rc == LC_ENONFINITE):
        _check(rc)
    return dict(mass=o.mass, mom=np.array(o.mom[:]), umax=o.umax, ssum=o.ssum, ssum_half=o.ssum_half,
                step=o.step, nonfinite=o.nonfinite, status=rc)


def lc_export(ctx, field, dst_ptr):
    _check(_lib.lc_export(ctx, field, ctypes.c_void_p(dst_ptr)))


def lc_vjp_step(ctx, f_ptr, q_ptr, adj_f_ptr, adj_q_ptr, dparams_ptr):
    _check(_lib.lc_vjp_step(ctx, ctypes.c_void_p(f_ptr), ctypes.c_void_p(q_ptr), ctypes.c_void_p(adj_f_ptr),
                            ctypes.c_void_p(adj_q_ptr), ctypes.c_void_p(dparams_ptr)))


def lc_vjp_history_bytes(grid, n):
    return _lib.lc_vjp_history_bytes(ctypes.byref(grid), int(n))


def lc_vjp_segment(ctx, f_ck_ptr, q_ck_ptr, n, hist_ptr, adj_f_ptr, adj_q_ptr, dparams_ptr):
    _check(_lib.lc_vjp_segment(ctx, ctypes.c_void_p(f_ck_ptr), ctypes.c_void_p(q_ck_ptr), int(n),
                               ctypes.c_void_p(hist_ptr), ctypes.c_void_p(adj_f_ptr), ctypes.c_void_p(adj_q_ptr),
                               ctypes.c_void_p(dparams_ptr)))


def lc_set_collision(ctx, kind, rates=()):
    n = len(rates)
    arr = (ctypes.c_double * max(n, 1))(*[float(r) for r in rates])
    _check(_lib.lc_set_collision(ctx, int(kind), arr if n else None, n))


def lc_vjp_backward_bytes(grid, n):
    return _lib.lc_vjp_backward_bytes(ctypes.byref(grid), int(n))


def lc_vjp_backward(ctx, f_ck_ptrs, q_ck_ptrs, ns, hist_ptr, adj_f_ptr, adj_q_ptr, dparams_ptr):
    """f_ck_ptrs, q_ck_ptrs, ns: sequences (forward order) of checkpoint
    device pointers and segment lengths."""
    k = len(ns)
    fa = (ctypes.c_void_p * k)(*f_ck_ptrs)
    qa = (ctypes.c_void_p * k)(*q_ck_ptrs)
    na = (ctypes.c_int32 * k)(*[int(n) for n in ns])
    _check(_lib.lc_vjp_backward(ctx, k, fa, qa, na, ctypes.c_void_p(hist_ptr), ctypes.c_void_p(adj_f_ptr),
                                ctypes.c_void_p(adj_q_ptr), ctypes.c_void_p(dparams_ptr)))


def lc_set_timing(ctx, enable):
    _check(_lib.lc_set_timing(ctx, 1 if enable else 0))


def lc_get_timing(ctx):
    ms = (ctypes.c_double * 2)()
    n = (ctypes.c_int64 * 2)()
    _check(_lib.lc_get_timing(ctx, ms, n))
    return list(ms), list(n)


def lc_sync(ctx):
    _check(_lib.lc_sync(ctx))


def lc_step_count(ctx):
    return _lib.lc_step_count(ctx)


def lc_free(ctx):
    _check(_lib.lc_free(ctx))


LC_STATIC_SCRATCH_BYTES = 64 << 20


def lc_step_static(grid, params, f_ptrs, q_ptrs, parity, n, stream):
    """f_ptrs, q_ptrs: the two device pointers of each buffer pair."""
    fa = (ctypes.c_void_p * 2)(*f_ptrs)
    qa = (ctypes.c_void_p * 2)(*q_ptrs)
    _check(_lib.lc_step_static(ctypes.byref(grid), ctypes.byref(params), fa, qa, int(parity), int(n),
                               ctypes.c_void_p(stream)))


# ------------------------------------------------------------ convenience
def _torch():
    import torch
    return torch


class Solver:
    """One grid: torch-owned buffers plus a library context.

    lattice: "D2Q9" | "D3Q19"; precision: "fp64", "fp32dev" (f as float
    deviations from the rest weights, Q in float, float arithmetic),
    "fp32sr" (the same storage; bulk molecular field summed in double and
    the Q update rounded stochastically) or "mixed" (f as float deviations,
    Q and its right-hand side in double);
    shape: (nz, ny, nx); params: (A0, gamma, K, Gamma, xi, tau).
    """

    def __init__(self, lattice, precision, shape, params, device="cuda", stream=None, variant=LC_VARIANT_AUTO):
        torch = _torch()
        self.torch = torch
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.grid = make_grid(LATTICES[lattice], PRECISIONS[precision], nx, ny, nz)
        self.params = make_params(*params)
        fb, qb, sb = lc_buffer_bytes(self.grid)
        self.q = fb // (self.N * (8 if precision == "fp64" else 4))
        self.device = torch.device(device)
        # raw byte buffers: torch's allocator returns 512-byte aligned blocks
        self._f = [torch.empty(fb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self._Q = [torch.empty(qb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self._scratch = torch.empty(max(sb, 256), dtype=torch.uint8, device=self.device)
        self.bufs = lc_buffers((ctypes.c_void_p * 2)(self._f[0].data_ptr(), self._f[1].data_ptr()),
                               (ctypes.c_void_p * 2)(self._Q[0].data_ptr(), self._Q[1].data_ptr()),
                               self._scratch.data_ptr())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # the library works on self.stream: keep torch from reusing these
        # blocks before that stream's work on them is done
        for t in self._f + self._Q + [self._scratch]:
            t.record_stream(self.stream)
        self.ctx = lc_init(self.grid, self.params, self.bufs, self.stream.cuda_stream)
        if variant != LC_VARIANT_AUTO:
            lc_set_variant(self.ctx, variant)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                _lib.lc_free(ctx)
            except Exception:
                pass
            self.ctx = None

    def set_variant(self, v):
        lc_set_variant(self.ctx, v)

    def set_collision(self, kind, rates=()):
        lc_set_collision(self.ctx, kind, rates)

    def set_chunk(self, planes):
        lc_set_chunk(self.ctx, planes)

    def set_stencil(self, stencil):
        lc_set_stencil(self.ctx, stencil)

    def set_params(self, params):
        self.params = make_params(*params)
        lc_set_params(self.ctx, self.params)

    def load(self, q5, f=None):
        """q5: (5, nz, ny, nx) array; f: (q, nz, ny, nx) logical populations
        or None for the fluid at rest."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            qd = torch.as_tensor(np.ascontiguousarray(q5, dtype=np.float64)).to(self.device)
            fd = None if f is None else torch.as_tensor(np.ascontiguousarray(f, dtype=np.float64)).to(self.device)
            lc_load_state(self.ctx, None if fd is None else fd.data_ptr(), qd.data_ptr())
            self.stream.synchronize()

    def step(self, n):
        lc_step(self.ctx, n)

    def observe(self, mask=LC_OBS_ALL, half_axis=0, allow_nonfinite=False):
        return lc_observe(self.ctx, mask, half_axis, allow_nonfinite)

    def export(self, field):
        torch = self.torch
        ncomp = {LC_FIELD_F: self.q, LC_FIELD_Q: 5, LC_FIELD_RHO: 1, LC_FIELD_U: 3,
                 LC_FIELD_FORCE: 3, LC_FIELD_S: 1}[field]
        with torch.cuda.stream(self.stream):
            out = torch.zeros((ncomp,) + self.shape, dtype=torch.float64, device=self.device)
            lc_export(self.ctx, field, out.data_ptr())
            self.stream.synchronize()
        return out.cpu().numpy()

    def sync(self):
        lc_sync(self.ctx)


# ---------------------------------------------------------------- batched form
def lc_batch_layout(grids):
    n = len(grids)
    ga = (lc_grid * n)(*grids)
    fb, qb, sb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    fo = (ctypes.c_size_t * n)()
    qo = (ctypes.c_size_t * n)()
    _check(_lib.lc_batch_layout(n, ga, ctypes.byref(fb), ctypes.byref(qb), ctypes.byref(sb), fo, qo))
    return fb.value, qb.value, sb.value, list(fo), list(qo)


def lc_batch_init(grids, params, arena, stream):
    n = len(grids)
    ga = (lc_grid * n)(*grids)
    pa = (lc_params * n)(*params)
    b = ctypes.c_void_p()
    _check(_lib.lc_batch_init(n, ga, pa, ctypes.byref(arena), ctypes.c_void_p(stream), ctypes.byref(b)))
    return b


def lc_batch_load_state(b, k, f_ptr, q_ptr):
    _check(_lib.lc_batch_load_state(b, k, ctypes.c_void_p(f_ptr), ctypes.c_void_p(q_ptr)))


def lc_batch_step(b, n):
    _check(_lib.lc_batch_step(b, int(n)))


def lc_batch_set_tile(b, v):
    _check(_lib.lc_batch_set_tile(b, int(v)))


def lc_batch_set_tiles(b, v_lb, v_q):
    _check(_lib.lc_batch_set_tiles(b, int(v_lb), int(v_q)))


def lc_batch_set_stencil(b, stencil):
    _check(_lib.lc_batch_set_stencil(b, int(stencil)))


def lc_batch_set_collision(b, kind, rates=()):
    n = len(rates)
    arr = (ctypes.c_double * max(n, 1))(*[float(r) for r in rates])
    _check(_lib.lc_batch_set_collision(b, int(kind), arr if n else None, n))


def lc_batch_autotune(b, trial_steps):
    ch = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(_lib.lc_batch_autotune(b, int(trial_steps), ctypes.byref(ch), ctypes.byref(ms)))
    return ch.value, ms.value


def lc_batch_observe(b, n, mask=LC_OBS_ALL, half_axis=0):
    out = (lc_observables * n)()
    _check(_lib.lc_batch_observe(b, mask, half_axis, out))
    return [dict(mass=o.mass, mom=np.array(o.mom[:]), umax=o.umax, ssum=o.ssum, ssum_half=o.ssum_half,
                 step=o.step, nonfinite=o.nonfinite) for o in out]


def lc_batch_export(b, k, field, dst_ptr):
    _check(_lib.lc_batch_export(b, k, field, ctypes.c_void_p(dst_ptr)))


def lc_batch_free(b):
    _check(_lib.lc_batch_free(b))


class BatchSolver:
    """Many independent D2Q9 grids advanced together.

    shapes: list of (ny, nx); params: list of (A0, gamma, K, Gamma, xi, tau);
    precision: "fp64", "fp32dev", "fp32sr" or "mixed".
    """

    def __init__(self, precision, shapes, params, device="cuda", stream=None):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.shapes = [(1, ny, nx) for (ny, nx) in shapes]
        self.n = len(shapes)
        self.grids = [make_grid(LC_D2Q9, PRECISIONS[precision], nx, ny, 1) for (ny, nx) in shapes]
        self.params = [make_params(*p) for p in params]
        fb, qb, sb, self.f_off, self.q_off = lc_batch_layout(self.grids)
        self._f = [torch.empty(fb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self._Q = [torch.empty(qb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self._scratch = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.arena = lc_buffers((ctypes.c_void_p * 2)(self._f[0].data_ptr(), self._f[1].data_ptr()),
                                (ctypes.c_void_p * 2)(self._Q[0].data_ptr(), self._Q[1].data_ptr()),
                                self._scratch.data_ptr())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        for t in self._f + self._Q + [self._scratch]:
            t.record_stream(self.stream)
        self.b = lc_batch_init(self.grids, self.params, self.arena, self.stream.cuda_stream)

    def __del__(self):
        b = getattr(self, "b", None)
        if b:
            try:
                _lib.lc_batch_free(b)
            except Exception:
                pass
            self.b = None

    def load(self, k, q5, f=None):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            qd = torch.as_tensor(np.ascontiguousarray(q5, dtype=np.float64)).to(self.device)
            fd = None if f is None else torch.as_tensor(np.ascontiguousarray(f, dtype=np.float64)).to(self.device)
            lc_batch_load_state(self.b, k, None if fd is None else fd.data_ptr(), qd.data_ptr())
            self.stream.synchronize()

    def step(self, n):
        lc_batch_step(self.b, n)

    def set_tile(self, v):
        lc_batch_set_tile(self.b, v)

    def set_tiles(self, v_lb, v_q):
        lc_batch_set_tiles(self.b, v_lb, v_q)

    def set_collision(self, kind, rates=()):
        lc_batch_set_collision(self.b, kind, rates)

    def set_stencil(self, stencil):
        lc_batch_set_stencil(self.b, stencil)

    def autotune(self, trial_steps=20):
        return lc_batch_autotune(self.b, trial_steps)

    def observe(self, mask=LC_OBS_ALL, half_axis=0):
        return lc_batch_observe(self.b, self.n, mask, half_axis)

    def export(self, k, field):
        torch = self.torch
        ncomp = {LC_FIELD_F: 9, LC_FIELD_Q: 5, LC_FIELD_RHO: 1, LC_FIELD_U: 3, LC_FIELD_FORCE: 3, LC_FIELD_S: 1}[field]
        with torch.cuda.stream(self.stream):
            out = torch.zeros((ncomp,) + self.shapes[k], dtype=torch.float64, device=self.device)
            lc_batch_export(self.b, k, field, out.data_ptr())
            self.stream.synchronize()
        return out.cpu().numpy()
