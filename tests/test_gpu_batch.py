"""GPU tests of the batched form: many grids of different sizes and gamma in
one launch per sweep, replayed from a HIP graph.

Every grid of a batch must reproduce the single-grid path exactly (the
per-site arithmetic does not depend on tile shape or on which block runs a
tile), across graph replays with eager work in between, and match the CPU
oracle to the double-precision tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1907_13415_amd import inputs
from gpu_util import SCALES, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _lc():
    require_gpu()
    from paper_1907_13415_amd import lc
    return lc


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


SHAPES = [(23, 37), (64, 64), (40, 96), (16, 16), (70, 130)]


def _batch_inputs(seed):
    rng = np.random.default_rng(seed)
    q5s, params = [], []
    for k, (ny, nx) in enumerate(SHAPES):
        q5s.append(inputs.random_q5((1, ny, nx), rng, amp=0.12))
        params.append(inputs.with_gamma((1.0, 2.7, 0.05, 0.3, 0.7, 1.3), 2.66 + 0.03 * k))
    return q5s, params


@pytest.mark.parametrize("prec", ["fp32dev", "fp64", "fp32sr", "mixed"])
def test_batch_equals_single_grid_across_graph_replays(prec):
    """With stochastic rounding too: a graph replay draws the uniform
    numbers of the steps it advances, as the single grid does."""
    lc = _lc()
    _say("batch vs single %s" % prec)
    q5s, params = _batch_inputs(1)
    b = lc.BatchSolver(prec, SHAPES, params)
    singles = []
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
        s = lc.Solver("D2Q9", prec, (1,) + SHAPES[k], params[k])
        s.load(q5)
        singles.append(s)
    done = 0
    for chunk in (64, 64, 11, 64):  # graph replay, replay, eager tail, replay from odd parity
        b.step(chunk)
        for s in singles:
            s.step(chunk)
        done += chunk
        # eager work and synchronisation between replays
        obs = b.observe()
        for k, s in enumerate(singles):
            fb, qb = b.export(k, lc.LC_FIELD_F), b.export(k, lc.LC_FIELD_Q)
            fs, qs = s.export(lc.LC_FIELD_F), s.export(lc.LC_FIELD_Q)
            assert np.array_equal(fb, fs) and np.array_equal(qb, qs), (k, done)
            o = s.observe()
            assert obs[k]["mass"] == o["mass"] and obs[k]["ssum_half"] == o["ssum_half"]
            assert obs[k]["step"] == done


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6])
def test_batch_every_tile_shape_matches_oracle_fp64(tile):
    """Each tile shape (32x8, 64x4, 16x16, 32x16, 64x8, 64x16, 128x8) agrees
    with the double-precision oracle."""
    lc = _lc()
    q5s, params = _batch_inputs(2)
    b = lc.BatchSolver("fp64", SHAPES, params)
    b.set_tile(tile)
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
    b.step(70)
    for k, q5 in enumerate(q5s):
        f_ref, q_ref = oracle.run(0, oracle.rest_populations(0, (1,) + SHAPES[k]), q5, params[k], 70)
        ef = rel_err(b.export(k, lc.LC_FIELD_F), f_ref, SCALES["f"])
        eq = rel_err(b.export(k, lc.LC_FIELD_Q), q_ref, SCALES["q"])
        assert ef < 1e-12 and eq < 1e-12, (tile, k, ef, eq)


def test_batch_autotune_keeps_results():
    lc = _lc()
    q5s, params = _batch_inputs(2)
    ref = lc.BatchSolver("fp32dev", SHAPES, params)
    for k, q5 in enumerate(q5s):
        ref.load(k, q5)
    b = lc.BatchSolver("fp32dev", SHAPES, params)
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
    chosen, ms = b.autotune(5)
    _say("autotune chose tiles %d, %d (%.3f ms/step)" % (chosen % 7, chosen // 7, ms))
    assert 0 <= chosen < 49 and ms > 0
    ref.set_tiles(chosen % 7, chosen // 7)
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
        ref.load(k, q5)
    b.step(70)
    ref.step(70)
    for k in range(len(SHAPES)):
        assert np.array_equal(ref.export(k, lc.LC_FIELD_Q), b.export(k, lc.LC_FIELD_Q))


def test_batch_fp64_matches_oracle():
    lc = _lc()
    q5s, params = _batch_inputs(3)
    b = lc.BatchSolver("fp64", SHAPES, params)
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
    b.step(70)
    for k, q5 in enumerate(q5s):
        f_ref, q_ref = oracle.run(0, oracle.rest_populations(0, (1,) + SHAPES[k]), q5, params[k], 70)
        ef = rel_err(b.export(k, lc.LC_FIELD_F), f_ref, SCALES["f"])
        eq = rel_err(b.export(k, lc.LC_FIELD_Q), q_ref, SCALES["q"])
        assert ef < 1e-12 and eq < 1e-12, (k, ef, eq)


def test_temperature_sweep_workload_full_size():
    """The 64-grid sweep (sizes 64..512, gamma in [2.62, 2.78]) at full size:
    sampled grids equal the single-grid path after 70 steps (graph path)."""
    lc = _lc()
    ws = inputs.config3()
    shapes = [w.shape[1:] for w in ws]
    b = lc.BatchSolver("fp32dev", shapes, [w.params for w in ws])
    for k, w in enumerate(ws):
        b.load(k, w.q5)
    b.step(70)
    sizes = [s[0] for s in shapes]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), len(ws) // 2})
    for k in picks:
        s = lc.Solver("D2Q9", "fp32dev", ws[k].shape, ws[k].params)
        s.load(ws[k].q5)
        s.step(70)
        assert np.array_equal(b.export(k, lc.LC_FIELD_Q), s.export(lc.LC_FIELD_Q)), k
        assert np.array_equal(b.export(k, lc.LC_FIELD_F), s.export(lc.LC_FIELD_F)), k
    obs = b.observe()
    assert all(o["nonfinite"] == 0 for o in obs)


def test_sweep_front_speeds_fp32_against_fp64():
    """The reported quantity of the sweep, the front speed of each grid
    between steps 1000 and 5000, in the float forms (FP32 deviation, FP32
    with stochastic rounding) against double precision: grids whose front
    moves (neither melted nor filled) agree to a small fraction of their
    speed."""
    lc = _lc()
    ws = inputs.config3()
    shapes = [w.shape[1:] for w in ws]
    half = {}
    for prec in ("fp64", "fp32dev", "fp32sr"):
        b = lc.BatchSolver(prec, shapes, [w.params for w in ws])
        for k, w in enumerate(ws):
            b.load(k, w.q5)
        b.step(1000)
        o0 = b.observe(half_axis=0)
        b.step(4000)
        o1 = b.observe(half_axis=0)
        half[prec] = [(a["ssum_half"], c["ssum_half"], c["ssum"]) for a, c in zip(o0, o1)]
        del b
    for prec in ("fp32dev", "fp32sr"):
        worst, n = 0.0, 0
        for w, h64, h32 in zip(ws, half["fp64"], half[prec]):
            L, g = w.shape[2], w.params[1]
            if g < 8.0 / 3.0:
                continue
            sn = 0.25 + 0.75 * (1.0 - 8.0 / (3.0 * g)) ** 0.5
            if h64[2] < 1e-6 * L * L or h64[2] > 0.99 * sn * L * L:
                continue  # melted or filled
            v64 = (h64[1] - h64[0]) / (sn * L) / 4000
            v32 = (h32[1] - h32[0]) / (sn * L) / 4000
            if abs(v64) < 1e-7:
                continue
            worst = max(worst, abs(v32 - v64) / abs(v64))
            n += 1
        print("sweep front speeds, %d moving grids: worst %s relative error %.2e" % (n, prec, worst), flush=True)
        assert n >= 10 and worst < 1e-3  # measured 1.3e-5 (FP32 deviation), 4.3e-6 (stochastic rounding) over 24 moving grids


@pytest.mark.parametrize("prec,iso", [("fp32dev", False), ("fp32sr", False), ("mixed", False), ("fp32dev", True),
                                      ("fp64", True)])
def test_batch_tile_shapes_agree_bitwise(prec, iso):
    """Every site runs the same code wherever it falls in a tile, so every
    tile shape of either sweep gives identical results (seven pairings that
    use each shape once in each sweep), with the isotropic stencils too."""
    lc = _lc()
    q5s, params = _batch_inputs(4)
    res = []
    for v in range(7):
        b = lc.BatchSolver(prec, SHAPES, params)
        b.set_tiles(v, (3 * v + 1) % 7)
        if iso:
            b.set_stencil(lc.LC_STENCIL_ISOTROPIC)
        for k, q5 in enumerate(q5s):
            b.load(k, q5)
        b.step(70)
        res.append([(b.export(k, lc.LC_FIELD_Q), b.export(k, lc.LC_FIELD_F)) for k in range(len(SHAPES))])
    for v in range(1, 7):
        for k in range(len(SHAPES)):
            assert np.array_equal(res[0][k][0], res[v][k][0]), (v, k)
            assert np.array_equal(res[0][k][1], res[v][k][1]), (v, k)


@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_batch_mrt_equals_single_grid(prec):
    """The multiple-relaxation-time collision in the batched form: every
    grid, with its own tau among the group rates, equals the same grid
    stepped alone with that collision, across graph replays and an eager
    tail; bad rates are refused and BGK restores the default operator."""
    lc = _lc()
    _say("batch MRT vs single %s" % prec)
    q5s, params = _batch_inputs(7)
    params = [p[:5] + (1.0 + 0.1 * k,) for k, p in enumerate(params)]  # a tau per grid
    rates = (1.64, 1.54, 1.9)
    b = lc.BatchSolver(prec, SHAPES, params)
    b.set_collision(lc.LC_COLL_MRT, rates)
    for bad in ((1.64, 1.54), (1.64, 2.0, 1.9), (0.0, 1.54, 1.9)):
        with pytest.raises(lc.LCError) as e:
            b.set_collision(lc.LC_COLL_MRT, bad)
        assert e.value.code == lc.LC_EINVAL
    with pytest.raises(lc.LCError):
        b.set_collision(7)
    b.set_collision(lc.LC_COLL_MRT, rates)  # the refused calls left nothing half set
    singles = []
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
        s = lc.Solver("D2Q9", prec, (1,) + SHAPES[k], params[k])
        s.set_collision(lc.LC_COLL_MRT, rates)
        s.load(q5)
        singles.append(s)
    for chunk in (64, 11, 64):
        b.step(chunk)
        for s in singles:
            s.step(chunk)
        for k, s in enumerate(singles):
            assert np.array_equal(b.export(k, lc.LC_FIELD_F), s.export(lc.LC_FIELD_F)), (k, chunk)
            assert np.array_equal(b.export(k, lc.LC_FIELD_Q), s.export(lc.LC_FIELD_Q)), (k, chunk)
    # back to BGK: equals a batch that never left it
    b.set_collision(lc.LC_COLL_BGK)
    ref = lc.BatchSolver(prec, SHAPES, params)
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
        ref.load(k, q5)
    b.step(70)
    ref.step(70)
    for k in range(len(SHAPES)):
        assert np.array_equal(b.export(k, lc.LC_FIELD_Q), ref.export(k, lc.LC_FIELD_Q)), k


@pytest.mark.parametrize("prec,coll", [("fp64", "bgk"), ("fp32dev", "bgk"), ("fp64", "mrt")])
def test_batch_isotropic_stencils_equal_single_grid(prec, coll):
    """The isotropic stencils in the batched form: every grid equals the same
    grid stepped alone with them (states and the force export, which
    differentiates the stress with the same stencils), across graph replays
    and an eager tail; the float forms without them are refused."""
    lc = _lc()
    _say("batch isotropic vs single %s %s" % (prec, coll))
    q5s, params = _batch_inputs(8)
    rates = (1.64, 1.54, 1.9)
    b = lc.BatchSolver(prec, SHAPES, params)
    b.set_stencil(lc.LC_STENCIL_ISOTROPIC)
    if coll == "mrt":
        b.set_collision(lc.LC_COLL_MRT, rates)
    singles = []
    for k, q5 in enumerate(q5s):
        b.load(k, q5)
        s = lc.Solver("D2Q9", prec, (1,) + SHAPES[k], params[k])
        s.set_stencil(lc.LC_STENCIL_ISOTROPIC)
        if coll == "mrt":
            s.set_collision(lc.LC_COLL_MRT, rates)
        s.load(q5)
        singles.append(s)
    for chunk in (64, 11):
        b.step(chunk)
        for s in singles:
            s.step(chunk)
        for k, s in enumerate(singles):
            for field in (lc.LC_FIELD_F, lc.LC_FIELD_Q, lc.LC_FIELD_FORCE):
                assert np.array_equal(b.export(k, field), s.export(field)), (k, chunk, field)
    for other in ("fp32sr", "mixed"):
        ob = lc.BatchSolver(other, SHAPES[:1], params[:1])
        with pytest.raises(lc.LCError) as e:
            ob.set_stencil(lc.LC_STENCIL_ISOTROPIC)
        assert e.value.code == lc.LC_EUNSUPPORTED
