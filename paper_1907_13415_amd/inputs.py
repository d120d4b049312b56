"""Seeded synthetic inputs for the hybrid LB / finite-difference step.

This module only builds initial states and parameter sets; it holds none of
the time-stepping arithmetic.  Both the GPU library's tests and the CPU oracle
consume the same arrays from here.

Array conventions (float64, C order):
  q5  : (5, nz, ny, nx), components (xx, xy, xz, yy, yz) of the order tensor;
  rel : (q, nz, ny, nx) optional relative perturbation of the populations,
        f_i = w_i * rho0 * (1 + rel_i), applied by each side with its own
        lattice weights.

The uniaxial form Q = S (n n - I/3) is the definition of the order tensor in
Sec. 1.1 of the paper.  Geometries follow the paper's flat interface (Sec. 2.1:
nematic slab in the middle, isotropic outside) and circular domain (Sec. 2.2),
with the seeded sizes, angles and noise of the workload definitions below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# (A0, gamma, K, Gamma, xi, tau)
WORKLOAD_PARAMS = (1.0, 2.7, 0.04, 0.3, 0.7, 1.0)
# Parameter set of Sec. 2 (resolved interface, correlation length 2).
PAPER_PARAMS = (0.1, 2.7, 0.04, 0.34, 0.7, 1.5)


def eta_of(tau: float) -> float:
    """Dynamic viscosity matching tau at rho0 = 1 (c_s^2 (tau - 1/2))."""
    return (tau - 0.5) / 3.0


def with_gamma(params, gamma):
    p = list(params)
    p[1] = float(gamma)
    return tuple(p)


def uniaxial_q5(S, n):
    """Five stored components of S (n n - I/3); S (...), n (3, ...)."""
    S = np.asarray(S, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    out = np.empty((5,) + S.shape)
    out[0] = S * (n[0] * n[0] - 1.0 / 3.0)
    out[1] = S * (n[0] * n[1])
    out[2] = S * (n[0] * n[2])
    out[3] = S * (n[1] * n[1] - 1.0 / 3.0)
    out[4] = S * (n[1] * n[2])
    return out


def tanh_edge(d, width=4.0, s_n=1.0 / 3.0):
    """(S_n/2)(1 - tanh(d/width)): S_n inside (d < 0), 0 outside."""
    return 0.5 * s_n * (1.0 - np.tanh(np.asarray(d, dtype=np.float64) / width))


@dataclass
class Workload:
    name: str
    lattice: str            # "D2Q9" | "D3Q19"
    shape: tuple            # (nz, ny, nx)
    q5: np.ndarray
    params: tuple
    steps: int
    half_axis: int = 0
    rel: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def flat_slab_2d(nx, ny, theta, half_width=None, width=4.0, s_n=1.0 / 3.0):
    """Nematic slab centred at x = nx/2 (half width nx/4 by default) with an
    in-plane director at angle theta; isotropic outside."""
    hw = nx / 4.0 if half_width is None else half_width
    x = np.arange(nx, dtype=np.float64)
    S1 = tanh_edge(np.abs(x - nx / 2.0) - hw, width, s_n)
    S = np.broadcast_to(S1[None, None, :], (1, ny, nx))
    n = np.zeros((3, 1, ny, nx))
    n[0] = math.cos(theta)
    n[1] = math.sin(theta)
    return uniaxial_q5(S, n)


def paper_flat(nx, ny, half_width=None):
    """Sec. 2.1 setup: nematic slab in the middle of a periodic box, director
    vertical (along y), isotropic elsewhere, tanh edges of width 2 lambda = 4
    at S_n = 1/3."""
    return flat_slab_2d(nx, ny, math.pi / 2, half_width=half_width)


def paper_circle(n=100, radius=25.0, angle_deg=0.0, width=4.0, s_n=1.0 / 3.0):
    """Sec. 2.2 setup: a nematic disc of the given radius centred in an n x n
    periodic box, uniform director n = (sin a, cos a, 0) (a = 0: vertical),
    tanh edge of width 2 lambda = 4."""
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    r = np.hypot(x - n / 2.0, y - n / 2.0)
    S = tanh_edge(r - radius, width, s_n)[None]
    a = math.radians(angle_deg)
    nvec = np.zeros((3, 1, n, n))
    nvec[0] = math.sin(a)
    nvec[1] = math.cos(a)
    return uniaxial_q5(S, nvec)


def config0():
    """128 x 16 D2Q9 flat interface, director angle theta ~ U[0, pi)."""
    rng = np.random.default_rng(0)
    theta = math.pi * rng.random()
    q5 = flat_slab_2d(128, 16, theta, half_width=32.0)
    return Workload("flat128x16_d2q9_fp64", "D2Q9", (1, 16, 128), q5, WORKLOAD_PARAMS, 2000,
                    half_axis=0, extra=dict(theta=theta))


def droplet_2d(n, radius, rng, width=4.0, noise=0.05, s_n=1.0 / 3.0):
    """Circular nematic domain centred at (n/2, n/2), radial director plus a
    uniform per-site angle perturbation in [-noise, noise] (row-major draw)."""
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    dx, dy = x - n / 2.0, y - n / 2.0
    r = np.hypot(dx, dy)
    phi = np.arctan2(dy, dx)  # atan2(0, 0) = 0
    phi = phi + rng.uniform(-noise, noise, size=(n, n))
    S = tanh_edge(r - radius, width, s_n)[None]
    nvec = np.zeros((3, 1, n, n))
    nvec[0, 0] = np.cos(phi)
    nvec[1, 0] = np.sin(phi)
    return uniaxial_q5(S, nvec)


def config1(dgamma=0.0, n=256):
    """256^2 D2Q9 droplet of radius 40, radial + noise director."""
    rng = np.random.default_rng(1)
    q5 = droplet_2d(n, 40.0 * n / 256.0, rng)
    return Workload("droplet%d_d2q9" % n, "D2Q9", (1, n, n), q5,
                    with_gamma(WORKLOAD_PARAMS, 2.7 + dgamma), 20000, half_axis=0,
                    extra=dict(dgamma=dgamma))


def slab_3d(n, rng, noise=1e-4, width=4.0, s_n=1.0 / 3.0, dtype=np.float64):
    """n^3 planar nematic slab for n/4 <= z < 3n/4, random uniform director,
    Gaussian noise of standard deviation `noise` on each stored component."""
    g = rng.standard_normal(3)
    nvec = g / np.linalg.norm(g)
    z = np.arange(n, dtype=np.float64)
    S1 = tanh_edge(np.abs(z - n / 2.0) - n / 4.0, width, s_n)
    base = np.empty(5)
    nn = np.outer(nvec, nvec)
    base[:] = [nn[0, 0] - 1 / 3.0, nn[0, 1], nn[0, 2], nn[1, 1] - 1 / 3.0, nn[1, 2]]
    q5 = np.empty((5, n, n, n), dtype=dtype)
    for c in range(5):
        q5[c] = (S1[:, None, None] * base[c]).astype(dtype)
    for c in range(5):  # component-major, then z, y, x
        q5[c] += rng.normal(0.0, noise, size=(n, n, n)).astype(dtype)
    return q5, nvec


def config2(n=256):
    """256^3 D3Q19 planar slab, random director, 1e-4 noise."""
    rng = np.random.default_rng(2)
    q5, nvec = slab_3d(n, rng)
    return Workload("slab%d3_d3q19" % n, "D3Q19", (n, n, n), q5, WORKLOAD_PARAMS, 500,
                    half_axis=2, extra=dict(director=nvec))


BATCH_SIZES = (64, 96, 128, 192, 256, 384, 512)


def config3(ngrids=64):
    """Temperature sweep: per grid a square size from BATCH_SIZES and
    gamma ~ U[2.62, 2.78] (drawn as pairs), then the director angles."""
    rng = np.random.default_rng(3)
    sizes, gammas = [], []
    for _ in range(ngrids):
        sizes.append(int(rng.choice(BATCH_SIZES)))
        gammas.append(float(rng.uniform(2.62, 2.78)))
    thetas = [math.pi * float(rng.random()) for _ in range(ngrids)]
    grids = []
    for L, g, th in zip(sizes, gammas, thetas):
        q5 = flat_slab_2d(L, L, th)
        grids.append(Workload("flat%d_sweep" % L, "D2Q9", (1, L, L), q5,
                              with_gamma(WORKLOAD_PARAMS, g), 5000, half_axis=0,
                              extra=dict(theta=th)))
    return grids


def config4(n=256):
    """Adjoint workload: the droplet at dgamma = 0.005, the target disc of
    radius 36, and 16 seeded (component, y, x) probe entries."""
    w = config1(0.005, n)
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    r = np.hypot(x - n / 2.0, y - n / 2.0)
    s_target = tanh_edge(r - 36.0 * n / 256.0)[None]
    rng = np.random.default_rng(4)
    probes = []
    while len(probes) < 16:
        c = int(rng.choice([0, 1, 3]))
        ang = rng.uniform(0, 2 * math.pi)
        rad = rng.uniform(36.0, 44.0) * n / 256.0
        px = int(round(n / 2.0 + rad * math.cos(ang))) % n
        py = int(round(n / 2.0 + rad * math.sin(ang))) % n
        probes.append((c, 0, py, px))
    w.name = "adjoint_droplet%d" % n
    w.steps = 2000
    w.extra.update(s_target=s_target, probes=probes)
    return w


def random_q5(shape, rng, amp=0.2):
    """Random symmetric traceless tensors with entries of size ~amp."""
    nz, ny, nx = shape
    A = rng.normal(0.0, amp, size=(3, 3, nz, ny, nx))
    A = 0.5 * (A + A.transpose(1, 0, 2, 3, 4))
    tr = (A[0, 0] + A[1, 1] + A[2, 2]) / 3.0
    for a in range(3):
        A[a, a] -= tr
    return np.stack([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2]])


def random_rel(q, shape, rng, amp=1e-3):
    """Relative population perturbations of size ~amp."""
    return rng.normal(0.0, amp, size=(q,) + tuple(shape))
