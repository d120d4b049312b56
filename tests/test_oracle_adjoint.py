"""Pins of the differentiable CPU twin (oracle/torch_step.py) used to check
the GPU reverse step: its forward step equals the C oracle's, and its
autograd gradients equal central finite differences of itself."""
import numpy as np
import pytest
import torch

import oracle
from oracle import torch_step
from paper_1907_13415_amd import inputs


def _random_state(shape, seed):
    rng = np.random.default_rng(seed)
    q5 = inputs.random_q5(shape, rng, amp=0.12)
    f = oracle.rest_populations(oracle.D2Q9, shape, rel=inputs.random_rel(9, shape, rng, amp=2e-3))
    return f, q5


@pytest.mark.parametrize("steps", [1, 4])
def test_torch_twin_matches_c_oracle(steps):
    p = (0.9, 2.72, 0.06, 0.31, 0.7, 1.3)
    f, q5 = _random_state((1, 9, 11), 20)
    fr, qr = oracle.run(oracle.D2Q9, f, q5, p, steps)
    ft = torch.tensor(f[:, 0])
    qt = torch.tensor(q5[:, 0])
    for _ in range(steps):
        ft, qt = torch_step.step(ft, qt, *p)
    np.testing.assert_allclose(ft.numpy(), fr[:, 0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(qt.numpy(), qr[:, 0], rtol=0, atol=1e-14)


def test_torch_twin_gradients_match_finite_differences():
    p = [0.9, 2.72, 0.06, 0.31, 0.7, 1.3]
    f, q5 = _random_state((1, 7, 8), 21)
    rng = np.random.default_rng(22)
    wf = torch.tensor(rng.normal(size=(9, 7, 8)))
    wq = torch.tensor(rng.normal(size=(5, 7, 8)))

    def loss(ft, qt, g, K, G):
        for _ in range(3):
            ft, qt = torch_step.step(ft, qt, p[0], g, K, G, p[4], p[5])
        return (wf * ft).sum() + (wq * qt).sum()

    qt = torch.tensor(q5[:, 0], requires_grad=True)
    ft = torch.tensor(f[:, 0], requires_grad=True)
    g = torch.tensor(p[1], dtype=torch.float64, requires_grad=True)
    K = torch.tensor(p[2], dtype=torch.float64, requires_grad=True)
    G = torch.tensor(p[3], dtype=torch.float64, requires_grad=True)
    loss(ft, qt, g, K, G).backward()
    h = 1e-6
    with torch.no_grad():
        for idx in [(0, 3, 4), (1, 0, 7), (3, 6, 2), (4, 2, 2)]:
            qp = qt.detach().clone(); qp[idx] += h
            qm = qt.detach().clone(); qm[idx] -= h
            fd = (loss(ft.detach(), qp, g, K, G) - loss(ft.detach(), qm, g, K, G)) / (2 * h)
            assert abs(fd.item() - qt.grad[idx].item()) < 1e-6 * max(1.0, abs(fd.item()))
        for name, t in (("gamma", g), ("K", K), ("Gamma", G)):
            tp = t.detach() + h
            tm = t.detach() - h
            args_p = dict(g=g.detach(), K=K.detach(), G=G.detach())
            args_m = dict(args_p)
            key = {"gamma": "g", "K": "K", "Gamma": "G"}[name]
            args_p[key] = tp
            args_m[key] = tm
            fd = (loss(ft.detach(), qt.detach(), **args_p) - loss(ft.detach(), qt.detach(), **args_m)) / (2 * h)
            assert abs(fd.item() - t.grad.item()) < 1e-6 * max(1.0, abs(fd.item())), name
