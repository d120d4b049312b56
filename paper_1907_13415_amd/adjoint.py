"""Gradients through many steps of the hybrid scheme: a torch.autograd.Function
over the library's forward step (lc_step) and reverse step (lc_vjp_step),
with checkpoint-and-recompute.

Forward: the state is saved every `every` steps (logical f and Q in double,
on the device).  Backward (lc_vjp_backward): segments are processed last to
first; each is replayed from its checkpoint with every intermediate state
kept, then the reverse steps walk it back, and the replay of the next
segment overlaps that walk on a second stream.  Memory: one checkpoint per
segment plus the histories of two segments.  All arithmetic runs in the HIP
kernels; this module only owns buffers and passes pointers.

Two-dimensional (D2Q9) grids in double precision.
"""
from __future__ import annotations

import torch

from . import lc


class LCSolve(torch.autograd.Function):
    """q_final = LCSolve.apply(q0, gamma, K, Gamma, cfg)

    q0: (5, 1, ny, nx) float64 CUDA tensor, the initial order tensor (the
        fluid starts at rest, f = w_i);
    gamma, K, Gamma: float64 scalar tensors;
    cfg: dict(A0=, xi=, tau=, steps=, every=100).
    Returns the order tensor after cfg["steps"] steps.
    """

    @staticmethod
    def forward(ctx, q0, gamma, K, Gamma, cfg):
        for name, t in (("q0", q0), ("gamma", gamma), ("K", K), ("Gamma", Gamma)):
            if not torch.is_tensor(t) or t.dtype != torch.float64:
                raise TypeError("%s must be a float64 tensor" % name)
        steps = int(cfg["steps"])
        every = int(cfg.get("every", 100))
        if steps < 0 or every < 1:
            raise ValueError("steps must be >= 0 and every >= 1 (got %d, %d)" % (steps, every))
        params = (cfg["A0"], float(gamma), float(K), float(Gamma), cfg["xi"], cfg["tau"])
        shape = tuple(q0.shape[1:])
        s = lc.Solver("D2Q9", "fp64", shape, params, device=q0.device)
        s.stream.wait_stream(torch.cuda.current_stream(q0.device))  # q0 may still be in flight
        with torch.cuda.stream(s.stream):
            q0c = q0.detach().contiguous()
            lc.lc_load_state(s.ctx, None, q0c.data_ptr())
            checkpoints = []
            done = 0
            while done < steps:
                f_ck = torch.empty((9,) + shape, dtype=torch.float64, device=q0.device)
                q_ck = torch.empty((5,) + shape, dtype=torch.float64, device=q0.device)
                lc.lc_export(s.ctx, lc.LC_FIELD_F, f_ck.data_ptr())
                lc.lc_export(s.ctx, lc.LC_FIELD_Q, q_ck.data_ptr())
                n = min(every, steps - done)
                checkpoints.append((f_ck, q_ck, n))
                s.step(n)
                done += n
            q_final = torch.empty((5,) + shape, dtype=torch.float64, device=q0.device)
            lc.lc_export(s.ctx, lc.LC_FIELD_Q, q_final.data_ptr())
        s.stream.synchronize()
        ctx.solver = s
        ctx.checkpoints = checkpoints
        ctx.shape = shape
        return q_final

    @staticmethod
    def backward(ctx, grad_q):
        s = ctx.solver
        shape = ctx.shape
        dev = grad_q.device
        if not ctx.checkpoints:  # zero steps: q_final is q0
            zero = torch.zeros((), dtype=torch.float64, device=dev)
            return grad_q.detach().to(torch.float64).clone(), zero, zero.clone(), zero.clone(), None
        s.stream.wait_stream(torch.cuda.current_stream(dev))  # grad_q may still be in flight
        with torch.cuda.stream(s.stream):
            adj_q = grad_q.detach().to(torch.float64).contiguous().clone()
            adj_f = torch.zeros((9,) + shape, dtype=torch.float64, device=dev)
            dparams = torch.zeros(3, dtype=torch.float64, device=dev)
            every = max(n for _, _, n in ctx.checkpoints)
            hist = torch.empty(lc.lc_vjp_backward_bytes(s.grid, every), dtype=torch.uint8, device=dev)
            # segments are replayed on a second stream of the library while
            # the previous one is walked back
            lc.lc_vjp_backward(s.ctx, [f.data_ptr() for f, _, _ in ctx.checkpoints],
                               [q.data_ptr() for _, q, _ in ctx.checkpoints], [n for _, _, n in ctx.checkpoints],
                               hist.data_ptr(), adj_f.data_ptr(), adj_q.data_ptr(), dparams.data_ptr())
        s.stream.synchronize()
        return adj_q, dparams[0], dparams[1], dparams[2], None


def solve(q0, gamma, K, Gamma, **cfg):
    """Functional form of LCSolve.apply."""
    return LCSolve.apply(q0, gamma, K, Gamma, cfg)


def order_parameter(q5):
    """S = sqrt(1.5 Q:Q) of a (5, ...) tensor of stored components."""
    xx, xy, xz, yy, yz = q5
    qq = xx * xx + yy * yy + (xx + yy) * (xx + yy) + 2 * (xy * xy + xz * xz + yz * yz)
    return torch.sqrt(1.5 * qq)
