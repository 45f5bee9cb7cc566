"""Seeded operands of many two-site problems drawn directly in device memory
(the uneven batch is tens of GB, too large to draw on the host).

The recipe is that of `heff_problem`: complex Gaussian blocks, Hermitian per
channel, L/R scaled by 1/sqrt(D), W by 1/sqrt(d w_in w_out), theta of unit
norm.  Complex tensors are planar torch tensors [2, ...] in float64; the W
blocks are small and drawn on the host (numpy complex).
"""
import numpy as np


def _herm_planar(x):
    """(X + X^H)/2 over the last two axes of a planar [2, ..., n, n] tensor."""
    import torch
    re = 0.5 * (x[0] + x[0].transpose(-1, -2))
    im = 0.5 * (x[1] - x[1].transpose(-1, -2))
    return torch.stack([re, im]).contiguous()


def batch_operands(seed, shapes, device="cuda"):
    """One dict per shape (Dl, d1, d2, Dr, wl, wc, wr) with planar device
    tensors L [2][wl][Dl][Dl], R [2][wr][Dr][Dr], theta [2][Dl][d1][d2][Dr]
    and host complex W1 [wl][wc][d1][d1], W2 [wc][wr][d2][d2]."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    out = []
    for (Dl, d1, d2, Dr, wl, wc, wr) in shapes:
        def dev(*shape):
            return torch.randn(2, *shape, dtype=torch.float64, device=device, generator=gen)

        def wblock(win, wout, d):
            x = rng.standard_normal((win, wout, d, d)) + 1j * rng.standard_normal((win, wout, d, d))
            x = 0.5 * (x + np.conj(np.swapaxes(x, -1, -2)))
            return x / np.sqrt(d * win * wout)

        L = _herm_planar(dev(wl, Dl, Dl)) / np.sqrt(Dl)
        R = _herm_planar(dev(wr, Dr, Dr)) / np.sqrt(Dr)
        th = dev(Dl, d1, d2, Dr)
        th /= torch.linalg.vector_norm(th)
        out.append(dict(L=L, R=R, theta=th, W1=wblock(wl, wc, d1), W2=wblock(wc, wr, d2)))
    return out
