"""Pins of the oracle's multiple-relaxation-time (MRT) collision.

The paper ran an MRT operator but gives neither its moment matrix nor its
rates (Sec. 1.2.1 defers them to another paper).  The oracle uses the
standard orthogonal bases (Lallemand and Luo for D2Q9, d'Humieres et al. for
D3Q19) and collides in moment space, transforming back with the inverse of
an orthogonal basis, M^T diag(1/|m_k|^2).  What fixes it independently of its
own code:
  - the D2Q9 matrix equals the published one; both bases are orthogonal and
    carry density, momentum and the traceless stress as rows;
  - with every rate equal to 1/tau it is the BGK step (already pinned);
  - any rates keep a uniform equilibrium unchanged and conserve mass and
    momentum, also over hundreds of steps, where a systematic leak would
    accumulate;
  - the shear rate alone sets the viscosity: a shear wave decays at
    nu = (tau - 1/2)/3 whatever the other rates are;
  - the other rates act only on non-equilibrium parts, so they change a
    trajectory away from equilibrium, and the static flat interface at
    coexistence stays static.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1907_13415_amd import inputs

D2, D3 = oracle.D2Q9, oracle.D3Q19
PAPER = inputs.PAPER_PARAMS

# D2Q9 moment matrix of Lallemand and Luo (2000), velocities in the order
# rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-) (the oracle's order).
LL_D2Q9 = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)


def test_d2q9_basis_is_the_published_matrix():
    np.testing.assert_array_equal(oracle.mrt_basis(D2), LL_D2Q9)


@pytest.mark.parametrize("lat", [D2, D3])
def test_basis_orthogonal_with_hydrodynamic_rows(lat):
    M = oracle.mrt_basis(lat)
    c, _ = oracle.lattice(lat)
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert abs(np.linalg.det(M)) > 1.0
    g = oracle.MRT_GROUPS[lat]
    cons = g["conserved"]
    np.testing.assert_array_equal(M[cons[0]], np.ones(len(c)))
    for a, k in enumerate(cons[1:]):
        np.testing.assert_array_equal(M[k], c[:, a])
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    c2 = cx * cx + cy * cy + cz * cz
    if lat == D2:
        shear = [cx * cx - cy * cy, cx * cy]
    else:
        shear = [3 * cx * cx - c2, cy * cy - cz * cz, cx * cy, cy * cz, cx * cz]
    for k, row in zip(g["shear"], shear):
        np.testing.assert_array_equal(M[k], row)
    # every row is in exactly one group
    allk = sorted(cons + g["shear"] + [k for grp in g["ghosts"] for k in grp])
    assert allk == list(range(len(c)))


def _random_state(lat, shape, seed):
    rng = np.random.default_rng(seed)
    _, w = oracle.lattice(lat)
    q5 = inputs.random_q5(shape, rng, amp=0.1)
    f = oracle.rest_populations(lat, shape, rel=inputs.random_rel(len(w), shape, rng, amp=3e-3))
    return f, q5


GHOSTS = {D2: (1.19, 1.4, 1.1), D3: (1.19, 1.4, 1.2, 1.4, 1.98)}


@pytest.mark.parametrize("lat,shape", [(D2, (1, 9, 11)), (D3, (5, 6, 7))])
def test_equal_rates_is_bgk(lat, shape):
    f, q5 = _random_state(lat, shape, 21)
    p = (1.0, 2.7, 0.04, 0.3, 0.7, 1.3)
    q = f.shape[0]
    fa, qa = oracle.run(lat, f, q5, p, 20)
    fb, qb = oracle.run(lat, f, q5, p, 20, rates=np.full(q, 1 / p[5]))
    assert np.abs(fb - fa).max() < 1e-15 and np.abs(qb - qa).max() < 1e-15
    # the moment-group helper maps the same thing
    np.testing.assert_array_equal(oracle.mrt_rates(lat, p[5], [1 / p[5]] * len(GHOSTS[lat])), np.full(q, 1 / p[5]))


@pytest.mark.parametrize("lat", [D2, D3])
def test_uniform_equilibrium_is_invariant(lat):
    shape = (1, 4, 5) if lat == D2 else (3, 4, 5)
    u = [0.03, -0.02, 0.01 if lat == D3 else 0.0]
    feq = oracle.feq(lat, 1.02, u)
    f = np.broadcast_to(feq[(slice(None),) + (None,) * 3], (len(feq),) + shape).copy()
    q5 = np.zeros((5,) + shape)
    r = oracle.mrt_rates(lat, 0.9, GHOSTS[lat])
    f1, _ = oracle.run(lat, f, q5, (1.0, 2.7, 0.04, 0.3, 0.7, 0.9), 3, rates=r)
    assert np.abs(f1 - f).max() < 1e-15  # a few ulps of the populations


@pytest.mark.parametrize("lat,shape", [(D2, (1, 10, 12)), (D3, (5, 6, 7))])
def test_conservation_with_any_rates(lat, shape):
    f, q5 = _random_state(lat, shape, 22)
    c, _ = oracle.lattice(lat)
    p = (1.0, 2.7, 0.04, 0.3, 0.7, 1.5)
    f1, _ = oracle.run(lat, f, q5, p, 20, rates=oracle.mrt_rates(lat, p[5], GHOSTS[lat]))
    assert abs(f1.sum() - f.sum()) / f.sum() < 1e-14
    j0 = np.tensordot(c.T, f, axes=1).reshape(3, -1).sum(axis=1)
    j1 = np.tensordot(c.T, f1, axes=1).reshape(3, -1).sum(axis=1)
    np.testing.assert_allclose(j1, j0, rtol=0, atol=1e-14 * f.size)


@pytest.mark.parametrize("lat,axis", [(D2, 1), (D3, 2)])
def test_shear_wave_viscosity_set_by_shear_rate(lat, axis):
    n = 64
    shape = [1, 1, 1]
    shape[2 - axis] = n
    shape = tuple(shape)
    c, _ = oracle.lattice(lat)
    k = 2 * math.pi / n
    coord = np.indices(shape)[2 - axis]
    ux = 1e-4 * np.sin(k * coord)
    f = np.zeros((len(c),) + shape)
    for idx in np.ndindex(shape):
        f[(slice(None),) + idx] = oracle.feq(lat, 1.0, [ux[idx], 0, 0])
    q5 = np.zeros((5,) + shape)
    tau = 0.8
    p = (1.0, 2.7, 0.04, 0.3, 0.0, tau)
    nu = (tau - 0.5) / 3
    for ghosts in (GHOSTS[lat], tuple(1.7 for _ in GHOSTS[lat])):
        r = oracle.mrt_rates(lat, tau, ghosts)
        fa, qa = oracle.run(lat, f, q5, p, 200, rates=r)
        fb, _ = oracle.run(lat, fa, qa, p, 1000, rates=r)
        amp = []
        for ff in (fa, fb):
            jx = np.tensordot(c[:, 0], ff, axes=1)
            amp.append((jx * np.sin(k * coord)).sum() * 2 / jx.size)
        rate = -math.log(amp[1] / amp[0]) / 1000
        assert abs(rate / (nu * k * k) - 1) < 5e-3, (ghosts, rate, nu * k * k)


@pytest.mark.parametrize("lat,shape", [(D2, (1, 9, 11)), (D3, (5, 6, 7))])
def test_other_rates_act_away_from_equilibrium(lat, shape):
    f, q5 = _random_state(lat, shape, 23)
    p = (1.0, 2.7, 0.04, 0.3, 0.7, 1.3)
    fa, _ = oracle.run(lat, f, q5, p, 5)
    fb, _ = oracle.run(lat, f, q5, p, 5, rates=oracle.mrt_rates(lat, p[5], GHOSTS[lat]))
    assert np.abs(fb - fa).max() > 1e-6


@pytest.mark.slow
def test_static_flat_interface_with_mrt():
    """Paper parameters at gamma = 2.7: with other rates the relaxed slab is
    still static (the rates do not enter the order-tensor equilibrium)."""
    nx, ny = 128, 2
    q5 = inputs.flat_slab_2d(nx, ny, math.pi / 2)
    f = oracle.rest_populations(D2, (1, ny, nx))
    r = oracle.mrt_rates(D2, PAPER[5], GHOSTS[D2])
    f, q5 = oracle.run(D2, f, q5, PAPER, 6000, rates=r)
    o0 = oracle.observe(D2, f, q5, PAPER)
    f2, q2 = oracle.run(D2, f, q5, PAPER, 1000, rates=r)
    o1 = oracle.observe(D2, f2, q2, PAPER)
    assert o1["umax"] < 1e-9
    assert abs((o1["ssum_half"] - o0["ssum_half"]) / (2 / 3)) < 1e-7


@pytest.mark.parametrize("lat,shape,steps", [(D3, (16, 16, 16), 400), (D2, (1, 48, 48), 1000)])
def test_momentum_conserved_over_a_long_run(lat, shape, steps):
    """The collision conserves mass and momentum (Sec. 1.2.1) at every site
    and step, so on a periodic grid the lattice momentum may change only by
    round-off that does not accumulate: over hundreds of steps of the slab
    recipe (a nearly static state, whose rounding repeats from step to step)
    it must stay within 1e-12 in total.  A back-transform whose entries are
    rounded independently (a generic numerical inverse of M) leaks a fixed
    fraction of the density into the momentum at every site and step, and
    fails this by orders of magnitude."""
    c, _ = oracle.lattice(lat)
    if lat == D3:
        w = inputs.config2(shape[0])
        q5, p = w.q5, w.params
    else:
        q5 = inputs.flat_slab_2d(shape[2], shape[1], 0.4, half_width=shape[2] / 4)
        p = inputs.WORKLOAD_PARAMS
    f = oracle.rest_populations(lat, shape)
    j0 = np.tensordot(c.T.astype(float), f, axes=1).reshape(3, -1).sum(axis=1)
    f1, _ = oracle.run(lat, f, q5, p, steps, rates=oracle.mrt_rates(lat, p[5], GHOSTS[lat]))
    j1 = np.tensordot(c.T.astype(float), f1, axes=1).reshape(3, -1).sum(axis=1)
    assert np.abs(j1 - j0).max() < 1e-12, j1 - j0
