"""TEST INFRASTRUCTURE ONLY: a differentiable CPU twin of one D2Q9 step.

The same time step as the C oracle (molecular field Eq. 4, stress Eq. 6 and
its divergence, force-corrected velocity Eq. 9, Heun predictor-corrector of
Sec. 1.2.2, BGK collision with forcing, periodic streaming), written again
with whole-grid torch operations in double precision so that torch's
autograd supplies exact vector-Jacobian products and parameter gradients.
It is pinned to the C oracle (tests/test_oracle_adjoint.py) and used to
check the GPU reverse step.  Only tests may import it.

Arrays: f (9, ny, nx), q5 (5, ny, nx); shifts are periodic.
"""
from __future__ import annotations

import torch

# D2Q9 velocities and weights, the order used throughout (rest, axes, diagonals)
C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4


def shift(a, dx, dy):
    """a(x - dx, y - dy): the field moved by (+dx, +dy) on the periodic grid."""
    return torch.roll(a, shifts=(dy, dx), dims=(-2, -1))


def ddx(a):
    """Central difference along x: [a(x+1) - a(x-1)] / 2."""
    return (torch.roll(a, -1, dims=-1) - torch.roll(a, 1, dims=-1)) / 2


def ddy(a):
    return (torch.roll(a, -1, dims=-2) - torch.roll(a, 1, dims=-2)) / 2


def lap(a):
    return (torch.roll(a, -1, -1) + torch.roll(a, 1, -1) + torch.roll(a, -1, -2) + torch.roll(a, 1, -2) - 4 * a)


def full(q5):
    xx, xy, xz, yy, yz = q5
    return torch.stack([torch.stack([xx, xy, xz]), torch.stack([xy, yy, yz]), torch.stack([xz, yz, -xx - yy])])


def five(T):
    return torch.stack([T[0, 0], T[0, 1], T[0, 2], T[1, 1], T[1, 2]])


def molecular_field(q5, A0, gamma, K):
    """Eq. (4): H = -A0(1-g/3)Q - A0 g (Tr Q^2 I/3 - Q Q) - A0 g Q Tr Q^2 + K lap Q."""
    Q = full(q5)
    I = torch.eye(3, dtype=Q.dtype).reshape(3, 3, 1, 1)
    tr2 = (Q * Q).sum(dim=(0, 1))
    QQ = torch.einsum("ag...,bg...->ab...", Q, Q)
    L = full(lap(q5))
    return (-A0 * (1 - gamma / 3) * Q - A0 * gamma * (tr2 * I / 3 - QQ) - A0 * gamma * Q * tr2 + K * L)


def grad(q5):
    """d_g Q for g = x, y (z derivatives vanish in two dimensions)."""
    return [full(ddx(q5)), full(ddy(q5)), torch.zeros_like(full(q5))]


def stress(q5, H, xi, K):
    """Eq. (6) without the hydrostatic part."""
    Q = full(q5)
    I = torch.eye(3, dtype=Q.dtype).reshape(3, 3, 1, 1)
    Qp = Q + I / 3
    qh = (Q * H).sum(dim=(0, 1))
    dQ = grad(q5)
    E = torch.stack([torch.stack([(dQ[a] * dQ[b]).sum(dim=(0, 1)) for b in range(3)]) for a in range(3)])
    HQp = torch.einsum("ag...,gb...->ab...", H, Qp)
    QpH = torch.einsum("ag...,gb...->ab...", Qp, H)
    QH = torch.einsum("ag...,gb...->ab...", Q, H)
    HQ = torch.einsum("ag...,gb...->ab...", H, Q)
    return 2 * xi * Qp * qh - xi * HQp - xi * QpH - K * E + QH - HQ


def rate(q5, u, G, A0, gamma, K, Gamma, xi):
    """Eq. (1)-(2): R = Gamma H + S - (u . grad) Q on the stored components;
    u = (ux, uy), G[a][b] = d_b u_a (3x3 with zero z row and column)."""
    Q = full(q5)
    I = torch.eye(3, dtype=Q.dtype).reshape(3, 3, 1, 1)
    Qp = Q + I / 3
    H = molecular_field(q5, A0, gamma, K)
    D = (G + G.transpose(0, 1)) / 2
    Wv = (G - G.transpose(0, 1)) / 2
    qg = torch.einsum("ge...,eg...->...", Q, G)
    S = (torch.einsum("ag...,bg...->ab...", xi * D + Wv, Qp) + torch.einsum("ag...,gb...->ab...", Qp, xi * D - Wv)
         - 2 * xi * Qp * qg)
    adv = u[0] * ddx(q5) + u[1] * ddy(q5)
    return Gamma * five(H) + five(S) - adv


def step(f, q5, A0, gamma, K, Gamma, xi, tau):
    """One step; returns (f', q5')."""
    H = molecular_field(q5, A0, gamma, K)
    tau_s = stress(q5, H, xi, K)
    Fx = ddx(tau_s[0, 0]) + ddy(tau_s[0, 1])
    Fy = ddx(tau_s[1, 0]) + ddy(tau_s[1, 1])
    rho = f.sum(dim=0)
    jx = sum(C[i][0] * f[i] for i in range(9))
    jy = sum(C[i][1] * f[i] for i in range(9))
    ux = (jx + Fx / 2) / rho
    uy = (jy + Fy / 2) / rho
    z = torch.zeros_like(ux)
    G = torch.stack([torch.stack([ddx(ux), ddy(ux), z]), torch.stack([ddx(uy), ddy(uy), z]), torch.stack([z, z, z])])
    u = (ux, uy)
    R = rate(q5, u, G, A0, gamma, K, Gamma, xi)
    qp = q5 + R
    Rp = rate(qp, u, G, A0, gamma, K, Gamma, xi)
    q_new = q5 + (R + Rp) / 2
    uu = ux * ux + uy * uy
    out = []
    for i, (cx, cy) in enumerate(C):
        cu = cx * ux + cy * uy
        feq = W[i] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
        src = W[i] * (1 - 1 / (2 * tau)) * (3 * (cx * Fx + cy * Fy) * (1 + 3 * cu) - 3 * (ux * Fx + uy * Fy))
        post = f[i] - (f[i] - feq) / tau + src
        out.append(shift(post, cx, cy))
    return torch.stack(out), q_new
