"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Double precision must agree with the oracle to 1e-12 in the normwise metric
of gpu_util.rel_err (field scales: f 1/36, Q 1/3, rho 1, u c_s); the FP32
deviation form must keep S within 1e-5 of the double-precision oracle.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1907_13415_amd import inputs
from gpu_util import SCALES, rel_err, require_gpu

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
VARIANTS = None  # filled lazily: variants the library provides


def _lc():
    require_gpu()
    from paper_1907_13415_amd import lc
    return lc


def _variants(lc):
    out = []
    for v in (lc.LC_VARIANT_STAGED, lc.LC_VARIANT_SPLIT, lc.LC_VARIANT_FUSED):
        out.append(v)
    return out


def _solver(lc, lat, prec, shape, params, variant):
    s = lc.Solver("D2Q9" if lat == 0 else "D3Q19", prec, shape, params)
    try:
        s.set_variant(variant)
    except lc.LCError as e:
        if e.code == lc.LC_EUNSUPPORTED:
            pytest.skip("variant %d not provided for this grid" % variant)
        raise
    return s


def _announce(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare_state(lc, s, f_ref, q_ref, tol, what):
    f = s.export(lc.LC_FIELD_F)
    q = s.export(lc.LC_FIELD_Q)
    ef = rel_err(f, f_ref, SCALES["f"])
    eq = rel_err(q, q_ref, SCALES["q"])
    _announce("%s: err f %.3e  Q %.3e" % (what, ef, eq))
    assert ef < tol and eq < tol, (what, ef, eq)


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_parity_flat_interface_128x16_fp64(variant):
    """Flat-interface workload (128 x 16 D2Q9, seeded director angle) after
    1000 and 2000 steps."""
    lc = _lc()
    w = inputs.config0()
    _announce("parity flat 128x16 variant %d" % variant)
    s = _solver(lc, 0, "fp64", w.shape, w.params, variant)
    s.load(w.q5)
    f_ref = oracle.rest_populations(oracle.D2Q9, w.shape)
    q_ref = w.q5
    for target in (1000, 2000):
        f_ref, q_ref = oracle.run(oracle.D2Q9, f_ref, q_ref, w.params, 1000)
        s.step(1000)
        _compare_state(lc, s, f_ref, q_ref, TOL64, "flat step %d" % target)


_SLAB_REF = {}


def _slab_reference(n, steps):
    """Oracle run of the D3Q19 slab recipe at n^3 (cached per size and step)."""
    key = (n, steps)
    if key not in _SLAB_REF:
        w = inputs.config2(n)
        _SLAB_REF[key] = oracle.run(oracle.D3Q19, oracle.rest_populations(oracle.D3Q19, w.shape), w.q5, w.params,
                                    steps)
    return _SLAB_REF[key]


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_parity_slab_32cubed_d3q19_1000_steps(variant):
    """The slab recipe on a 32^3 D3Q19 grid in double precision for 1000
    steps (several z-chunks and tiles, periodic wrap in every direction)."""
    lc = _lc()
    w = inputs.config2(32)
    _announce("parity slab 32^3 d3q19 1000 steps variant %d" % variant)
    s = _solver(lc, 1, "fp64", w.shape, w.params, variant)
    s.set_chunk(8)  # four z-chunks, so chunk boundaries are crossed
    s.load(w.q5)
    s.step(1000)
    f_ref, q_ref = _slab_reference(32, 1000)
    _compare_state(lc, s, f_ref, q_ref, TOL64, "slab 32^3 step 1000")


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("lat,shape", [(0, (1, 23, 37)), (0, (1, 70, 130)), (1, (9, 11, 13)), (1, (17, 6, 67))])
def test_parity_random_state_ragged(variant, lat, shape):
    """Random Q and perturbed populations on ragged grids spanning several
    tiles: exercises every term, halo and wrap-around."""
    lc = _lc()
    _announce("parity random lat %d shape %s variant %d" % (lat, shape, variant))
    rng = np.random.default_rng(100 + lat)
    q = 9 if lat == 0 else 19
    q5 = inputs.random_q5(shape, rng, amp=0.12)
    rel = inputs.random_rel(q, shape, rng, amp=2e-3)
    p = (1.0, 2.72, 0.05, 0.3, 0.7, 1.3)
    f0 = oracle.rest_populations(lat, shape, rel=rel)
    c_gpu, w_gpu = lc.lc_lattice_info(lat)
    c_or, _ = oracle.lattice(lat)
    assert np.array_equal(c_gpu, c_or)
    f_gpu = w_gpu.reshape((q, 1, 1, 1)) * (1.0 + rel)
    s = _solver(lc, lat, "fp64", shape, p, variant)
    s.load(q5, f_gpu)
    f_ref, q_ref = oracle.run(lat, f0, q5, p, 12)
    s.step(12)
    _compare_state(lc, s, f_ref, q_ref, TOL64, "random")
    fl = oracle.fields(lat, f_ref, q_ref, p)
    for field, key, sc in ((lc.LC_FIELD_RHO, "rho", 1.0), (lc.LC_FIELD_U, "u", SCALES["u"]),
                           (lc.LC_FIELD_FORCE, "F", SCALES["F"])):
        got = s.export(field)
        want = fl[key] if key != "rho" else fl[key][None]
        e = rel_err(got, want, sc)
        assert e < TOL64, (key, e)


def test_observables_match_oracle():
    lc = _lc()
    rng = np.random.default_rng(7)
    shape = (1, 40, 48)
    q5 = inputs.random_q5(shape, rng, amp=0.1)
    rel = inputs.random_rel(9, shape, rng, amp=1e-3)
    p = (1.0, 2.7, 0.04, 0.3, 0.7, 1.0)
    _, w = lc.lc_lattice_info(0)
    s = lc.Solver("D2Q9", "fp64", shape, p)
    s.load(q5, w.reshape(9, 1, 1, 1) * (1 + rel))
    s.step(5)
    f_ref, q_ref = oracle.run(0, oracle.rest_populations(0, shape, rel=rel), q5, p, 5)
    for ax in (0, 1):
        o = s.observe(half_axis=ax)
        r = oracle.observe(0, f_ref, q_ref, p, half_axis=ax)
        assert abs(o["mass"] - r["mass"]) < 1e-12 * r["mass"]
        np.testing.assert_allclose(o["mom"], r["mom"], rtol=0, atol=1e-13)
        assert abs(o["umax"] - r["umax"]) < 1e-12 * SCALES["u"]
        assert abs(o["ssum"] - r["ssum"]) < 1e-12 * r["ssum"]
        assert abs(o["ssum_half"] - r["ssum_half"]) < 1e-12 * r["ssum"]
        assert o["step"] == 5 and o["nonfinite"] == 0


def test_observables_3d_half_axis_z_match_oracle():
    lc = _lc()
    rng = np.random.default_rng(8)
    shape = (12, 10, 14)
    q5 = inputs.random_q5(shape, rng, amp=0.1)
    rel = inputs.random_rel(19, shape, rng, amp=1e-3)
    p = (1.0, 2.7, 0.04, 0.3, 0.7, 1.0)
    _, w = lc.lc_lattice_info(1)
    s = lc.Solver("D3Q19", "fp64", shape, p)
    s.load(q5, w.reshape(19, 1, 1, 1) * (1 + rel))
    s.step(4)
    f_ref, q_ref = oracle.run(1, oracle.rest_populations(1, shape, rel=rel), q5, p, 4)
    for ax in (0, 1, 2):
        o = s.observe(half_axis=ax)
        r = oracle.observe(1, f_ref, q_ref, p, half_axis=ax)
        assert abs(o["mass"] - r["mass"]) < 1e-12 * r["mass"]
        np.testing.assert_allclose(o["mom"], r["mom"], rtol=0, atol=1e-13)
        assert abs(o["umax"] - r["umax"]) < 1e-12 * SCALES["u"]
        assert abs(o["ssum"] - r["ssum"]) < 1e-12 * r["ssum"]
        assert abs(o["ssum_half"] - r["ssum_half"]) < 1e-12 * r["ssum"]


def test_set_params_between_steps_equals_a_restart():
    """Changing the parameters between steps (a temperature quench) gives the
    same state, bit for bit, as exporting, loading into a fresh context with
    the new parameters and stepping there."""
    lc = _lc()
    w = inputs.config0()
    p2 = inputs.with_gamma(w.params, 2.705)
    a = lc.Solver("D2Q9", "fp64", w.shape, w.params)
    a.load(w.q5)
    a.step(30)
    f_mid, q_mid = a.export(lc.LC_FIELD_F), a.export(lc.LC_FIELD_Q)
    a.set_params(p2)
    a.step(30)
    b = lc.Solver("D2Q9", "fp64", w.shape, p2)
    b.load(q_mid, f_mid)
    b.step(30)
    assert np.array_equal(a.export(lc.LC_FIELD_Q), b.export(lc.LC_FIELD_Q))
    assert np.array_equal(a.export(lc.LC_FIELD_F), b.export(lc.LC_FIELD_F))


def test_nonfinite_state_is_reported():
    lc = _lc()
    shape = (1, 16, 16)
    q5 = np.zeros((5,) + shape)
    q5[0, 0, 3, 4] = np.nan
    s = lc.Solver("D2Q9", "fp64", shape, inputs.WORKLOAD_PARAMS)
    s.load(q5)
    o = s.observe(allow_nonfinite=True)
    assert o["nonfinite"] == 1 and o["status"] == lc.LC_ENONFINITE
    with pytest.raises(lc.LCError) as e:
        s.observe()
    assert e.value.code == lc.LC_ENONFINITE


def test_mass_conserved_on_gpu():
    lc = _lc()
    w = inputs.config1(0.005, n=128)
    s = lc.Solver("D2Q9", "fp64", w.shape, w.params)
    s.load(w.q5)
    m0 = s.observe()["mass"]
    s.step(500)
    o = s.observe()
    assert abs(o["mass"] - m0) < 1e-12 * m0
    assert np.abs(o["mom"]).max() < 1e-12


# (the staged variant, 1, has no mixed-precision form)
@pytest.mark.parametrize("prec,variant", [("fp32dev", 1), ("fp32dev", 2), ("fp32dev", 3), ("fp32sr", 2),
                                          ("fp32sr", 3), ("mixed", 2), ("mixed", 3)])
def test_float_populations_conserve_mass(prec, variant):
    """The float deviation forms on the 256^2 droplet for 5000 steps: total
    mass within float rounding of its start (summed per site it may drift by
    ~1e-10 per site and step at random; the density part of the equilibrium
    formed as rho - 1 from the rounded rho drifted it by 7e-2)."""
    lc = _lc()
    w = inputs.config1(0.0)
    s = _solver(lc, 0, prec, w.shape, w.params, variant)
    s.load(w.q5)
    m0 = s.observe()["mass"]
    s.step(5000)
    o = s.observe()
    _announce("%s variant %d: mass drift over 5000 steps %.2e (of %.0f)" % (prec, variant, o["mass"] - m0, m0))
    assert abs(o["mass"] - m0) < 1e-4


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_fp32dev_within_tolerance_on_S(variant):
    """FP32 deviation storage against the double-precision oracle:
    |S32 - S64| <= 1e-5 everywhere on the flat-interface workload."""
    lc = _lc()
    w = inputs.config0()
    _announce("fp32dev flat 128x16 variant %d" % variant)
    s = _solver(lc, 0, "fp32dev", w.shape, w.params, variant)
    s.load(w.q5)
    f_ref, q_ref = oracle.run(0, oracle.rest_populations(0, w.shape), w.q5, w.params, 1000)
    s.step(1000)
    S_gpu = s.export(lc.LC_FIELD_S)[0]
    S_ref = np.sqrt(1.5 * (q_ref[0] ** 2 + q_ref[3] ** 2 + (q_ref[0] + q_ref[3]) ** 2
                           + 2 * (q_ref[1] ** 2 + q_ref[2] ** 2 + q_ref[4] ** 2)))
    err = np.abs(S_gpu - S_ref).max()
    _announce("fp32dev max |dS| = %.3e" % err)
    assert err < 1e-5


def test_fp32dev_slab_256cubed_500_steps_within_tolerance_on_S():
    """The 256^3 D3Q19 slab over its 500 steps in the FP32 deviation form
    against double precision on the GPU (which matches the oracle to
    1e-12): |S32 - S64| <= 1e-5 at every site."""
    import torch
    lc = _lc()
    w = inputs.config2(256)
    _announce("fp32dev vs fp64, 256^3 slab, 500 steps")
    S = []
    for prec in ("fp64", "fp32dev"):
        s = lc.Solver("D3Q19", prec, w.shape, w.params)
        s.load(w.q5)
        s.step(500)
        S.append(_export_dev(lc, s, lc.LC_FIELD_S, 1))
        del s
        torch.cuda.empty_cache()
    err = float((S[1] - S[0]).abs().max().item())
    _announce("  max |S32 - S64| = %.3e" % err)
    assert err < 1e-5


def _export_dev(lc, s, field, ncomp):
    import torch
    out = torch.empty((ncomp,) + s.shape, dtype=torch.float64, device=s.device)
    with torch.cuda.stream(s.stream):
        lc.lc_export(s.ctx, field, out.data_ptr())
    s.stream.synchronize()
    return out


def _patch(t, z, y, x, r):
    """(C, 2r+1, 2r+1, 2r+1) periodic patch of a device tensor around (z, y, x)."""
    import torch
    nz, ny, nx = t.shape[1:]
    iz = torch.tensor([(z + d) % nz for d in range(-r, r + 1)], device=t.device)
    iy = torch.tensor([(y + d) % ny for d in range(-r, r + 1)], device=t.device)
    ix = torch.tensor([(x + d) % nx for d in range(-r, r + 1)], device=t.device)
    return t[:, iz][:, :, iy][:, :, :, ix].cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("fp32dev", 2e-6), ("fp32sr", 2e-6), ("fp64", 1e-12)])
def test_full_size_slab_256cubed_sampled_sites(prec, tol):
    """The 256^3 D3Q19 slab workload in the launch configuration the
    benchmark times: one GPU step from a developed state is compared, at
    sampled sites (tile corners, chunk boundaries, periodic edges and random
    sites), with the oracle run on a periodic patch of radius 6 around each
    site (the step depends on Q within 4 sites and f within 2)."""
    lc = _lc()
    _announce("full-size 256^3 %s" % prec)
    w = inputs.config2(256)
    s = lc.Solver("D3Q19", prec, w.shape, w.params)
    s.load(w.q5)
    s.step(3)
    f0 = _export_dev(lc, s, lc.LC_FIELD_F, 19)
    q0 = _export_dev(lc, s, lc.LC_FIELD_Q, 5)
    s.step(1)
    f1 = _export_dev(lc, s, lc.LC_FIELD_F, 19)
    q1 = _export_dev(lc, s, lc.LC_FIELD_Q, 5)
    rng = np.random.default_rng(42)
    sites = [(0, 0, 0), (255, 255, 255), (31, 7, 31), (32, 8, 32), (127, 128, 64), (191, 3, 250), (64, 64, 0),
             (96, 255, 33)]
    sites += [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(40)]
    r = 6
    worst_f = worst_q = 0.0
    for (z, y, x) in sites:
        fp = _patch(f0, z, y, x, r)
        qp = _patch(q0, z, y, x, r)
        fr, qr = oracle.run(oracle.D3Q19, fp, qp, w.params, 1)
        got_f = f1[:, z, y, x].cpu().numpy()
        got_q = q1[:, z, y, x].cpu().numpy()
        worst_f = max(worst_f, np.abs(got_f - fr[:, r, r, r]).max() / (1 / 3))
        worst_q = max(worst_q, np.abs(got_q - qr[:, r, r, r]).max() / (1 / 3))
    _announce("256^3 %s sampled: err f %.3e Q %.3e" % (prec, worst_f, worst_q))
    assert worst_f < tol and worst_q < tol


@pytest.mark.parametrize("prec", ["fp64"])
def test_full_size_droplet_256sq_fp64(prec):
    """The 256^2 droplet workload (delta gamma = 0.005) on the full grid
    for 200 steps, in the launch configuration of the library default."""
    lc = _lc()
    w = inputs.config1(0.005)
    s = lc.Solver("D2Q9", prec, w.shape, w.params)
    s.load(w.q5)
    s.step(200)
    f_ref, q_ref = oracle.run(0, oracle.rest_populations(0, w.shape), w.q5, w.params, 200)
    _compare_state(lc, s, f_ref, q_ref, TOL64, "droplet 256^2 step 200")


@pytest.mark.parametrize("lat,shape", [(0, (1, 40, 56)), (1, (12, 10, 14))])
def test_resume_from_export_is_bitexact(lat, shape):
    """Checkpoint/resume: n steps equal n/2 steps, lc_export of (f, Q), a
    fresh context, lc_load_state and n/2 more steps, bit for bit (FP64)."""
    lc = _lc()
    rng = np.random.default_rng(50 + lat)
    q5 = inputs.random_q5(shape, rng, amp=0.1)
    p = (1.0, 2.72, 0.05, 0.3, 0.7, 1.3)
    name = "D2Q9" if lat == 0 else "D3Q19"
    a = lc.Solver(name, "fp64", shape, p)
    a.load(q5)
    a.step(40)
    b = lc.Solver(name, "fp64", shape, p)
    b.load(q5)
    b.step(20)
    f_mid, q_mid = b.export(lc.LC_FIELD_F), b.export(lc.LC_FIELD_Q)
    c = lc.Solver(name, "fp64", shape, p)
    c.load(q_mid, f_mid)
    c.step(20)
    assert np.array_equal(a.export(lc.LC_FIELD_F), c.export(lc.LC_FIELD_F))
    assert np.array_equal(a.export(lc.LC_FIELD_Q), c.export(lc.LC_FIELD_Q))
    assert c.observe()["step"] == 20


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_shift_equivariance_on_gpu_bitexact(variant):
    """A one-site periodic shift of the initial state shifts the result bit
    for bit (per-site arithmetic does not depend on the tile position)."""
    lc = _lc()
    shape = (20, 24, 40)
    rng = np.random.default_rng(60)
    q5 = inputs.random_q5(shape, rng, amp=0.1)
    out = []
    for sh in (0, 1):
        s = _solver(lc, 1, "fp64", shape, (1.0, 2.72, 0.05, 0.3, 0.7, 1.3), variant)
        s.load(np.roll(q5, sh, axis=3))
        s.step(6)
        out.append(s.export(lc.LC_FIELD_Q))
    assert np.array_equal(np.roll(out[0], 1, axis=3), out[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32dev", "mixed", "fp32sr"])
def test_z_chunk_does_not_change_the_result(prec):
    """The z-chunk of the two sweeps only decides which block marches which
    planes (and where the boundary planes are recomputed): the state after a
    few steps is bit-identical for any chunk, on a grid whose depth no chunk
    divides evenly (with stochastic rounding too: its uniform numbers depend
    on the site index and the step only)."""
    lc = _lc()
    shape = (23, 9, 70)
    rng = np.random.default_rng(61)
    q5 = inputs.random_q5(shape, rng, amp=0.12)
    _, w = lc.lc_lattice_info(1)
    f = w.reshape((19, 1, 1, 1)) * (1.0 + inputs.random_rel(19, shape, rng, amp=2e-3))
    p = (1.0, 2.72, 0.05, 0.3, 0.7, 1.3)
    out = {}
    for zc in (0, 1, 5, 23, 64, 2 ** 31 - 1):
        _announce("z-chunk %d (%s)" % (zc, prec))
        s = lc.Solver("D3Q19", prec, shape, p)
        s.set_chunk(zc)
        s.load(q5, f)
        s.step(6)
        out[zc] = (s.export(lc.LC_FIELD_F), s.export(lc.LC_FIELD_Q))
    for zc in (1, 5, 23, 64, 2 ** 31 - 1):
        assert np.array_equal(out[zc][0], out[0][0]) and np.array_equal(out[zc][1], out[0][1]), zc
