"""Pins of the reference gradient (autograd of the plain torch grid
formulation with frozen timesteps): central finite differences of the same
frozen-timestep map, and the forward/reverse dot-product identity. CPU only."""
import numpy as np
import torch

from oracle import torch_ref
from paper_2202_12309_amd import inputs


def _state(N=8, blk=8, seed=9):
    n, nrb = (blk,) * 3, (N // blk,) * 3
    lv = inputs.uniform_leaves(nrb)
    U = inputs.smooth_density(lv, n, nrb, seed=5, amp=3e-2)
    U = U + 0.05 * inputs.turbulent_box(lv, n, nrb, seed=seed) - 0.05 * inputs.uniform_state(lv, n)
    return torch.tensor(torch_ref.blocks_to_global(U, lv, n, nrb))


def _loss(G, dts, tgt):
    GN, _ = torch_ref.run(G, len(dts), dts=dts)
    return 0.5 * ((GN[0] - tgt) ** 2).sum() / G[0].numel()


def test_reference_gradient_matches_finite_differences():
    G0 = _state()
    _, dts = torch_ref.run(G0, 4)
    tgt = G0[0] * 1.01
    G = G0.clone().requires_grad_(True)
    _loss(G, dts, tgt).backward()
    g = G.grad
    rng = np.random.default_rng(0)
    good = 0
    for trial in range(4):
        v = torch.tensor(rng.normal(size=G0.shape)) * torch.tensor([1, .3, .3, .3, 1.])[:, None, None, None]
        dirder = float((g * v).sum())
        fd = []
        for h in (1e-6, 5e-7):
            fd.append(float((_loss(G0 + h * v, dts, tgt) - _loss(G0 - h * v, dts, tgt)) / (2 * h)))
        if abs(fd[1] - dirder) <= max(1e-7 * abs(dirder), 2 * abs(fd[0] - fd[1])):
            good += 1
    assert good >= 3


def test_forward_reverse_dot_product():
    G0 = _state()
    _, dts = torch_ref.run(G0, 3)

    def F(G):
        return torch_ref.run(G, 3, dts=dts)[0]
    rng = np.random.default_rng(1)
    v = torch.tensor(rng.normal(size=G0.shape))
    w = torch.tensor(rng.normal(size=G0.shape))
    _, jv = torch.func.jvp(F, (G0,), (v,))
    _, vjp = torch.func.vjp(F, G0)
    jtw = vjp(w)[0]
    lhs, rhs = float((jv * w).sum()), float((v * jtw).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
