"""TEST INFRASTRUCTURE ONLY: the double-precision CPU oracle.

A plain, slow reference of one time step of the hybrid lattice-Boltzmann /
finite-difference scheme of Coelho, Araujo and Telo da Gama (arXiv:1907.13415),
written in C (``lc_oracle.c``) and loaded here through ctypes.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the GPU library never does, and the two share no code.

Array conventions (numpy, float64, C order):
  f  : (q, nz, ny, nx)  populations in the oracle's velocity order;
  q5 : (5, nz, ny, nx)  order tensor (xx, xy, xz, yy, yz), Qzz = -Qxx - Qyy;
  params: (A0, gamma, K, Gamma, xi, tau).

Stencils: ``stencil="compact"`` (the default) takes the central differences
and compact Laplacian of Sec. 1.2.2; ``stencil="isotropic"`` takes every
derivative of the step from the lattice's own velocity set and weights (the
option Sec. 2.2 closes on for reducing spurious currents).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lc_oracle.c")
_LIB = os.path.join(_HERE, "liblc_oracle.so")
_OPC_SRC = os.path.join(_HERE, "opcount.cpp")
_OPC_BIN = os.path.join(_HERE, "opcount")

D2Q9 = 0
D3Q19 = 1

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source file into a shared library at `out` (gcc,
    -O2, no floating-point contraction)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle (see compile_source) if its library is missing or
    older than the source; with force, also the operation counter."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    if force:
        build_opcount(force=True)
    return _LIB


def build_opcount(force: bool = False) -> str:
    """Compile opcount.cpp (the oracle's source counted operation by
    operation, see that file) with g++ if the program is missing or older
    than either source."""
    stale = not os.path.exists(_OPC_BIN) or any(
        os.path.getmtime(_OPC_BIN) < os.path.getmtime(s) for s in (_SRC, _OPC_SRC))
    if force or stale:
        tmp = _OPC_BIN + ".tmp%d" % os.getpid()
        subprocess.run(["g++", "-O1", "-fpermissive", "-fopenmp", "-w", "-o", tmp, _OPC_SRC, "-lm"], check=True)
        os.replace(tmp, _OPC_BIN)
    return _OPC_BIN


def opcount(lat: int, n: int, mrt: bool = False, stencil: str = "compact") -> dict:
    """Floating-point operations of one oracle step on an n x n (D2Q9) or
    n^3 (D3Q19) grid: counts of additions (and subtractions),
    multiplications, divisions, square roots and comparisons, and the
    operations per site."""
    import json
    if stencil not in STENCILS:
        raise ValueError("stencil must be one of %s" % sorted(STENCILS))
    exe = build_opcount()
    r = subprocess.run([exe, str(int(lat)), str(int(n)), str(int(bool(mrt))), str(STENCILS[stencil])],
                       check=True, stdout=subprocess.PIPE, text=True)
    return json.loads(r.stdout)


def _load():
    """Load the oracle library: the one built from lc_oracle.c, or, when the
    environment names one in LC_ORACLE_LIBRARY, that library (the tests that
    plant mistakes in a copy of the source run the pins against it)."""
    global _lib
    if _lib is None:
        path = os.environ.get("LC_ORACLE_LIBRARY") or build()
        lib = ctypes.CDLL(path)
        lib.lco_lattice.argtypes = [ctypes.c_int, _ip, _dp]
        lib.lco_lattice.restype = ctypes.c_int
        lib.lco_run.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp, ctypes.c_long]
        lib.lco_run.restype = ctypes.c_int
        lib.lco_run_coll.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp, _dp, ctypes.c_long]
        lib.lco_run_coll.restype = ctypes.c_int
        lib.lco_mrt_basis.argtypes = [ctypes.c_int, _dp]
        lib.lco_mrt_basis.restype = ctypes.c_int
        lib.lco_fields.argtypes = [ctypes.c_int] * 4 + [_dp] * 12
        lib.lco_fields.restype = ctypes.c_int
        lib.lco_rate.argtypes = [ctypes.c_int] * 3 + [_dp] * 6
        lib.lco_rate.restype = ctypes.c_int
        lib.lco_stress.argtypes = [ctypes.c_int] * 3 + [_dp] * 5
        lib.lco_stress.restype = ctypes.c_int
        lib.lco_feq.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        lib.lco_feq.restype = None
        lib.lco_source.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        lib.lco_source.restype = None
        lib.lco_observe.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp, ctypes.c_int, _dp]
        lib.lco_observe.restype = ctypes.c_int
        lib.lco_set_threads.argtypes = [ctypes.c_int]
        lib.lco_set_threads.restype = None
        lib.lco_threads.argtypes = []
        lib.lco_threads.restype = ctypes.c_int
        lib.lco_set_stencil.argtypes = [ctypes.c_int]
        lib.lco_set_stencil.restype = ctypes.c_int
        lib.lco_stencil.argtypes = []
        lib.lco_stencil.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _params(p):
    a = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
    assert a.shape == (6,), "params = (A0, gamma, K, Gamma, xi, tau)"
    return a


def threads() -> int:
    """Host threads the oracle's whole-grid loops use."""
    return int(_load().lco_threads())


def set_threads(n: int) -> None:
    """Set the host threads of the oracle's whole-grid loops (n >= 1)."""
    _load().lco_set_threads(int(n))


STENCILS = {"compact": 0, "isotropic": 1}


@contextlib.contextmanager
def _stencil(name):
    """Select the difference stencil for the duration of one call."""
    if name not in STENCILS:
        raise ValueError("stencil must be one of %s" % sorted(STENCILS))
    lib = _load()
    old = lib.lco_stencil()
    if lib.lco_set_stencil(STENCILS[name]) != 0:
        raise ValueError("lco_set_stencil failed")
    try:
        yield lib
    finally:
        lib.lco_set_stencil(old)


def lattice(lat: int):
    """Velocity table c (q, 3) and weights w (q,) of the oracle."""
    c = np.zeros(19 * 3, dtype=np.int32)
    w = np.zeros(19, dtype=np.float64)
    q = _load().lco_lattice(lat, c.ctypes.data_as(_ip), w.ctypes.data_as(_dp))
    if q < 0:
        raise ValueError("unknown lattice")
    return c[: 3 * q].reshape(q, 3).astype(np.int64), w[:q].copy()


def _dims(q5):
    assert q5.ndim == 4 and q5.shape[0] == 5
    nz, ny, nx = q5.shape[1:]
    return nx, ny, nz


def run(lat, f, q5, params, nsteps, rates=None, stencil="compact"):
    """Advance (f, q5) by nsteps; returns new arrays.  With rates (q values,
    one per moment of the MRT basis, see mrt_basis) the collision is MRT,
    else BGK; `stencil` as in the module notes."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    q5 = np.array(q5, dtype=np.float64, order="C", copy=True)
    nx, ny, nz = _dims(q5)
    p = _params(params)
    r = None
    if rates is not None:
        r = np.ascontiguousarray(np.asarray(rates, dtype=np.float64))
        assert r.shape == (f.shape[0],), "one rate per moment"
    with _stencil(stencil) as lib:
        if r is None:
            rc = lib.lco_run(lat, nx, ny, nz, _ptr(p), _ptr(f), _ptr(q5), int(nsteps))
        else:
            rc = lib.lco_run_coll(lat, nx, ny, nz, _ptr(p), _ptr(r), _ptr(f), _ptr(q5), int(nsteps))
    if rc != 0:
        raise ValueError("lco_run failed: %d" % rc)
    return f, q5


def mrt_basis(lat):
    """The MRT moment matrix M (q, q): row k = moment k at each velocity.
    D2Q9: rho, e, eps, jx, qx, jy, qy, pxx, pxy; D3Q19: rho, e, eps, jx, qx,
    jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz."""
    q = 9 if lat == D2Q9 else 19
    M = np.zeros((q, q))
    assert _load().lco_mrt_basis(lat, _ptr(M)) == q
    return M


# moment groups of the MRT bases: conserved, shear (relaxed at 1/tau) and the
# other (non-hydrodynamic) groups in the order the library takes their rates
MRT_GROUPS = {
    D2Q9: dict(conserved=[0, 3, 5], shear=[7, 8], ghosts=[[1], [2], [4, 6]]),
    D3Q19: dict(conserved=[0, 3, 5, 7], shear=[9, 11, 13, 14, 15],
                ghosts=[[1], [2], [4, 6, 8], [10, 12], [16, 17, 18]]),
}


def mrt_rates(lat, tau, ghost_rates):
    """Per-moment rate vector: conserved and shear moments at 1/tau, each
    non-hydrodynamic group at its rate (D2Q9: s_e, s_eps, s_q; D3Q19: s_e,
    s_eps, s_q, s_pi, s_m)."""
    g = MRT_GROUPS[lat]
    q = 9 if lat == D2Q9 else 19
    r = np.full(q, 1.0 / tau)
    assert len(ghost_rates) == len(g["ghosts"])
    for ks, v in zip(g["ghosts"], ghost_rates):
        r[ks] = v
    return r


def fields(lat, f, q5, params, stencil="compact"):
    """Intermediates of one step at state (f, q5)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    q5 = np.ascontiguousarray(q5, dtype=np.float64)
    nx, ny, nz = _dims(q5)
    sh = (nz, ny, nx)
    out = dict(rho=np.zeros(sh), u=np.zeros((3,) + sh), F=np.zeros((3,) + sh),
               H=np.zeros((3, 3) + sh), tau=np.zeros((3, 3) + sh), G=np.zeros((3, 3) + sh),
               R=np.zeros((5,) + sh), Rp=np.zeros((5,) + sh), S=np.zeros((3, 3) + sh))
    p = _params(params)
    with _stencil(stencil) as lib:
        rc = lib.lco_fields(lat, nx, ny, nz, _ptr(p), _ptr(f), _ptr(q5),
                            *[_ptr(out[k]) for k in ("rho", "u", "F", "H", "tau", "G", "R", "Rp", "S")])
    if rc != 0:
        raise ValueError("lco_fields failed: %d" % rc)
    return out


def rate(q5, u, params):
    """Beris-Edwards rate R (5 comps), co-rotational S and H (3x3) for given u."""
    q5 = np.ascontiguousarray(q5, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    nx, ny, nz = _dims(q5)
    sh = (nz, ny, nx)
    R = np.zeros((5,) + sh)
    S = np.zeros((3, 3) + sh)
    H = np.zeros((3, 3) + sh)
    p = _params(params)
    rc = _load().lco_rate(nx, ny, nz, _ptr(p), _ptr(q5), _ptr(u), _ptr(R), _ptr(S), _ptr(H))
    if rc != 0:
        raise ValueError("lco_rate failed")
    return R, S, H


def stress(q5, params):
    """Stress tau (3x3), body force F (3) and molecular field H (3x3)."""
    q5 = np.ascontiguousarray(q5, dtype=np.float64)
    nx, ny, nz = _dims(q5)
    sh = (nz, ny, nx)
    tau = np.zeros((3, 3) + sh)
    F = np.zeros((3,) + sh)
    H = np.zeros((3, 3) + sh)
    p = _params(params)
    rc = _load().lco_stress(nx, ny, nz, _ptr(p), _ptr(q5), _ptr(tau), _ptr(F), _ptr(H))
    if rc != 0:
        raise ValueError("lco_stress failed")
    return tau, F, H


def feq(lat, rho, u):
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    q = 9 if lat == D2Q9 else 19
    out = np.zeros(q)
    _load().lco_feq(lat, float(rho), _ptr(u), _ptr(out))
    return out


def source(lat, tau, u, F):
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    F = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(3))
    q = 9 if lat == D2Q9 else 19
    out = np.zeros(q)
    _load().lco_source(lat, float(tau), _ptr(u), _ptr(F), _ptr(out))
    return out


def observe(lat, f, q5, params, half_axis=0, stencil="compact"):
    """mass, lattice momentum (3), max |u|, sum S, half-domain sum S."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    q5 = np.ascontiguousarray(q5, dtype=np.float64)
    nx, ny, nz = _dims(q5)
    out = np.zeros(7)
    p = _params(params)
    with _stencil(stencil) as lib:
        rc = lib.lco_observe(lat, nx, ny, nz, _ptr(p), _ptr(f), _ptr(q5), int(half_axis), _ptr(out))
    if rc != 0:
        raise ValueError("lco_observe failed")
    return dict(mass=out[0], mom=out[1:4].copy(), umax=out[4], ssum=out[5], ssum_half=out[6])


def rest_populations(lat, shape, rho=1.0, rel=None):
    """f_i = w_i rho (1 + rel_i) with the oracle's own weights."""
    _, w = lattice(lat)
    f = np.empty((len(w),) + tuple(shape))
    for i, wi in enumerate(w):
        f[i] = wi * rho
    if rel is not None:
        f *= 1.0 + rel
    return f
