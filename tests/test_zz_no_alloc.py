"""lc_step_static, the step for callers that cannot allocate device memory,
against lc_step on a context over the same initial storage buffers: the two
run the same sweeps, so the results must agree bit for bit.  Three calls in
a row on one GPU, each on a smaller input than the one before, so the
library's fixed scratch array is reused with stale contents from a larger
grid."""
import numpy as np
import pytest

from gpu_util import require_gpu
from paper_1907_13415_amd import inputs


PARAMS = (1.0, 2.7, 0.04, 0.3, 0.7, 1.2)

# (lattice, precision, (nz, ny, nx), steps), in decreasing size
CASES = [("D3Q19", "fp32dev", (40, 36, 70), 5),
         ("D3Q19", "mixed", (21, 18, 33), 4),
         ("D2Q9", "fp64", (1, 34, 50), 3)]


def _state(lc, lattice, shape, rng):
    _, w = lc.lc_lattice_info(lc.LATTICES[lattice])
    q5 = inputs.random_q5(shape, rng, amp=0.15)
    rel = inputs.random_rel(len(w), shape, rng, amp=2e-3)
    f = np.stack([wi * (1.0 + rel[i]) for i, wi in enumerate(w)])
    return f, q5


@pytest.mark.gpu
def test_static_step_equals_context_step_on_shrinking_grids():
    require_gpu()
    import torch
    from paper_1907_13415_amd import lc
    rng = np.random.default_rng(60)
    for lattice, precision, shape, n in CASES:
        print("static step: %s %s %s, %d steps" % (lattice, precision, shape, n), flush=True)
        s = lc.Solver(lattice, precision, shape, PARAMS, device="cuda:0")
        f, q5 = _state(lc, lattice, shape, rng)
        s.load(q5, f)
        # the storage form after the load is in buffer 0 of each pair
        f_init = s._f[0].clone()
        fc = [s._f[0].clone(), torch.full_like(s._f[1], 255)]
        qc = [s._Q[0].clone(), torch.full_like(s._Q[1], 255)]
        torch.cuda.synchronize()
        s.step(n)
        lc.lc_step_static(s.grid, s.params, [t.data_ptr() for t in fc], [t.data_ptr() for t in qc], 0, n,
                          s.stream.cuda_stream)
        torch.cuda.synchronize()
        out = n & 1
        assert lc.lc_step_count(s.ctx) == n
        assert torch.equal(s._f[out], fc[out]), (lattice, precision, shape)
        assert torch.equal(s._Q[out], qc[out]), (lattice, precision, shape)
        # and the result is a real step: it differs from the initial state
        assert not torch.equal(fc[out], f_init)
