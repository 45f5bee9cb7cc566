"""Observables of an MPS (Sections 2.1.1 and 3.1).

All values are raw expectation values <psi|O|psi> (no division by the norm):
after truncation ||psi||^2 = 1 - (sum of discarded weights).
"""
import numpy as np

from .hamiltonian import local_matrix, site_dims
from .tdvp import env_boundary, env_left


def overlap(bra, ket):
    """<bra|ket> by the zipper contraction (eqs. overlap 1 / overlap 2)."""
    E = np.ones((1, 1), dtype=complex)
    for a, b in zip(bra, ket):
        X = np.einsum("bB,BsA->bsA", E, b, optimize=True)
        E = np.einsum("bsa,bsA->aA", a.conj(), X, optimize=True)
    return complex(E[0, 0])


def expectation(mps, W):
    L = env_boundary()
    for a, w in zip(mps, W):
        L = env_left(L, a, w)
    return complex(L[0, 0, 0])


def single_site_mpo(model, site, key):
    """A w = 1 MPO: the local operator `key` on `site`, identity elsewhere."""
    out = []
    for s, d in enumerate(site_dims(model)):
        m = local_matrix(model, s, key) if s == site else np.eye(d, dtype=complex)
        out.append(m[None, None, :, :])
    return out


def populations(model, mps):
    """P_i = <psi| |i><i| x 1 |psi> for every electronic state i."""
    el = list(model["order"]).index(-1)
    return np.array([expectation(mps, single_site_mpo(model, el, ("proj", i))).real
                     for i in range(model["n_el"])])


def norm2(mps):
    return overlap(mps, mps).real


def energy(mps, W):
    return expectation(mps, W).real
