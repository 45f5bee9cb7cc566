"""Seeded random operands for a single effective-Hamiltonian problem.

Environments L[w] (D_l x D_l), R[w] (D_r x D_r) and MPO blocks W[w, w'] (d x d)
are complex Gaussian and Hermitised per channel ((X + X^H)/2), scaled so that
the resulting operator has norm of order one; theta is complex Gaussian.
Arrays are complex128 numpy arrays in the index order used everywhere in this
project:  L[w, a, a'], W[w, w', s, s'], R[w, b, b'], theta[a, s, t, b].
"""
import numpy as np


def _cgauss(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _herm(x):
    return 0.5 * (x + np.conj(np.swapaxes(x, -1, -2)))


def heff_problem(seed, Dl, d1, d2, Dr, wl, wc, wr, two_site=True, w_density=1.0):
    """Operands of one two-site (or, with two_site=False, one-site) problem.

    w_density < 1 zeroes whole (w, w') blocks of W at random, which gives the
    block-sparse channel structure of a vibronic MPO.
    """
    rng = np.random.default_rng(seed)
    L = _herm(_cgauss(rng, (wl, Dl, Dl))) / np.sqrt(Dl)
    R = _herm(_cgauss(rng, (wr, Dr, Dr))) / np.sqrt(Dr)

    def wblock(win, wout, d):
        W = _herm(_cgauss(rng, (win, wout, d, d))) / np.sqrt(d * win * wout)
        if w_density < 1.0:
            mask = rng.random((win, wout)) < w_density
            mask[0, 0] = True
            W = W * mask[:, :, None, None]
        return W

    if two_site:
        W1 = wblock(wl, wc, d1)
        W2 = wblock(wc, wr, d2)
        theta = _cgauss(rng, (Dl, d1, d2, Dr))
        theta /= np.linalg.norm(theta)
        return dict(L=L, W1=W1, W2=W2, R=R, theta=theta)
    W = wblock(wl, wr, d1)
    theta = _cgauss(rng, (Dl, d1, Dr))
    theta /= np.linalg.norm(theta)
    return dict(L=L, W=W, R=R, theta=theta)


def heff_batch_shapes(seed, n=256, Dlo=16, Dhi=256, dlo=4, dhi=30, wlo=4, whi=24, scale=1.0):
    """Uneven two-site problem shapes (D_l, d1, d2, D_r, w_l, w_c, w_r), each
    drawn uniformly from the given integer ranges; `scale` shrinks the bond
    dimensions (for oracle-sized versions of the same draw)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        Dl, Dr = rng.integers(Dlo, Dhi + 1, 2)
        d1, d2 = rng.integers(dlo, dhi + 1, 2)
        wl, wc, wr = rng.integers(wlo, whi + 1, 3)
        Dl = max(1, int(round(Dl * scale)))
        Dr = max(1, int(round(Dr * scale)))
        out.append(tuple(int(x) for x in (Dl, d1, d2, Dr, wl, wc, wr)))
    return out
