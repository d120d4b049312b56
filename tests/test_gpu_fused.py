"""The single-pass step (LC_VARIANT_FUSED) against the two-sweep step.

Both variants evaluate every site with the same per-site arithmetic in the
same order (stress, body force, moments, collision; predictor and
corrector of Sec. 1.2.2), so from the same storage state they must give the
same bits, in every precision, on ragged grids whose edges cut tiles, with
z-chunks that cut the march, and on grids smaller than the tile.  Parity of
the fused variant with the oracle is tested in test_gpu_parity.py and
test_gpu_edges.py."""
import sys

import numpy as np
import pytest

from paper_1907_13415_amd import inputs
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

PARAMS = (1.0, 2.72, 0.05, 0.3, 0.7, 1.3)


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _pair(lc, lat, prec, shape, rng, chunk=0, mrt=None):
    q = 9 if lat == 0 else 19
    q5 = inputs.random_q5(shape, rng, amp=0.12)
    rel = inputs.random_rel(q, shape, rng, amp=2e-3)
    _, w = lc.lc_lattice_info(lat)
    f = w.reshape((q, 1, 1, 1)) * (1.0 + rel)
    out = []
    for variant in (lc.LC_VARIANT_SPLIT, lc.LC_VARIANT_FUSED):
        s = lc.Solver("D2Q9" if lat == 0 else "D3Q19", prec, shape, PARAMS)
        s.set_variant(variant)
        if chunk:
            s.set_chunk(chunk)
        if mrt is not None:
            s.set_collision(lc.LC_COLL_MRT, mrt)
        s.load(q5, f)
        out.append(s)
    return out


def _same(lc, a, b, n):
    import torch
    torch.cuda.synchronize()
    p = n & 1
    return torch.equal(a._f[p], b._f[p]) and torch.equal(a._Q[p], b._Q[p])


@pytest.mark.parametrize("prec", ["fp64", "fp32dev", "mixed", "fp32sr"])
# two-dimensional shapes: the library's single pass takes 16x8 tiles with
# 1024 threads on grids of at most 256 such tiles (23x37, 70x130), 32x8
# tiles with 1024 threads on at most 256 of those (130x250), with 512
# threads on at most 1024 (300x301), else with 256 threads (270x1030)
@pytest.mark.parametrize("lat,shape,chunk", [(0, (1, 23, 37), 0), (0, (1, 70, 130), 0), (0, (1, 130, 250), 0),
                                             (0, (1, 300, 301), 0), (0, (1, 270, 1030), 0), (1, (9, 11, 13), 0),
                                             (1, (17, 6, 67), 5), (1, (40, 20, 36), 0), (1, (13, 18, 35), 3),
                                             (1, (7, 9, 40), 1)])
def test_fused_equals_split_bitwise(prec, lat, shape, chunk):
    require_gpu()
    from paper_1907_13415_amd import lc
    _say("fused vs split: lat %d %s %s chunk %d" % (lat, prec, shape, chunk))
    rng = np.random.default_rng(500 + lat)
    a, b = _pair(lc, lat, prec, shape, rng, chunk)
    for n in (1, 6):
        a.step(n)
        b.step(n)
    assert _same(lc, a, b, 7), (lat, prec, shape)


@pytest.mark.parametrize("lat,shape,rates", [(0, (1, 33, 45), (1.64, 1.54, 1.9)),
                                             (0, (1, 130, 250), (1.64, 1.54, 1.9)),
                                             (1, (11, 9, 35), (1.19, 1.4, 1.2, 1.4, 1.98))])
def test_fused_equals_split_with_mrt(lat, shape, rates):
    require_gpu()
    from paper_1907_13415_amd import lc
    _say("fused vs split MRT: lat %d %s" % (lat, shape))
    rng = np.random.default_rng(520 + lat)
    for prec in ("fp64", "fp32dev"):
        a, b = _pair(lc, lat, prec, shape, rng, 0, rates)
        a.step(5)
        b.step(5)
        assert _same(lc, a, b, 5), (lat, prec)


def test_fused_full_size_slab_equals_split():
    """The 256^3 slab recipe in FP32 over 20 steps in the launch shape the
    benchmark times: the two variants agree bit for bit."""
    require_gpu()
    import torch
    from paper_1907_13415_amd import lc
    w = inputs.config2(256)
    _say("fused vs split: 256^3 fp32dev slab, 20 steps")
    res = []
    for variant in (lc.LC_VARIANT_SPLIT, lc.LC_VARIANT_FUSED):
        s = lc.Solver("D3Q19", "fp32dev", w.shape, w.params)
        s.set_variant(variant)
        s.load(w.q5)
        s.step(20)
        torch.cuda.synchronize()
        res.append((s._f[0].clone(), s._Q[0].clone()))
        del s
        torch.cuda.empty_cache()
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("prec", ["fp64", "fp32dev", "fp32sr", "mixed"])
@pytest.mark.parametrize("n", [64, 256, 384, 385])
def test_auto_variant_on_small_2d_grids(prec, n):
    """AUTO runs the single pass on D2Q9 grids of at most 384^2 sites and
    the two sweeps above: either way its state equals the explicit two-sweep
    variant bit for bit (64^2 and 256^2 in the two shapes with 1024 threads
    per tile, 384^2 with 512, 385^2 just above)."""
    require_gpu()
    from paper_1907_13415_amd import lc
    rng = np.random.default_rng(900 + n)
    shape = (1, n, n)
    q5 = inputs.random_q5(shape, rng, amp=0.12)
    rel = inputs.random_rel(9, shape, rng, amp=2e-3)
    _, w = lc.lc_lattice_info(0)
    f = w.reshape((9, 1, 1, 1)) * (1.0 + rel)
    runs = []
    for variant in (lc.LC_VARIANT_AUTO, lc.LC_VARIANT_SPLIT):
        s = lc.Solver("D2Q9", prec, shape, PARAMS)
        s.set_variant(variant)
        s.load(q5, f)
        s.step(9)
        runs.append(s)
    _say("auto vs split, D2Q9 %s %dx%d" % (prec, n, n))
    assert _same(lc, runs[0], runs[1], 9)
