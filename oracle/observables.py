"""Observables of an MPS (Sections 2.1.1 and 3.1).

All values are raw expectation values <psi|O|psi> (no division by the norm):
after truncation ||psi||^2 = 1 - (sum of discarded weights).
"""
import numpy as np

from . import HBAR
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
    """P_i = <psi| |i><i| x 1 |psi> for every electronic state i (with one
    site per state: <psi| n_i |psi>)."""
    from .hamiltonian import el_site_of, per_state
    if per_state(model):
        return np.array([expectation(mps, single_site_mpo(model, el_site_of(model, i), "occ")).real
                         for i in range(model["n_el"])])
    el = list(model["order"]).index(-1)
    return np.array([expectation(mps, single_site_mpo(model, el, ("proj", i))).real
                     for i in range(model["n_el"])])


def norm2(mps):
    return overlap(mps, mps).real


def energy(mps, W):
    return expectation(mps, W).real


def absorption_spectrum(C, dt_fs, E, tau_fs):
    """sigma(E) = (1 / (pi hbar)) Re int_0^T C(t) exp(i E t / hbar) exp(-t / tau) dt
    from C(t_k) = <psi(0)|psi(t_k)> at t_k = k dt (k = 0 .. N-1, T = (N-1) dt),
    by the trapezoid rule.  The paper shows spectra obtained from C(t) with a
    damping time tau (Section 3.1, pyrazine spectra with tau = 30 and 50 fs)
    without printing the transform; this is the standard one-sided form,
    which assumes C(-t) = conj(C(t)).  E in eV, result in 1/eV."""
    C = np.asarray(C, dtype=complex)
    E = np.asarray(E, dtype=float)
    assert len(C) >= 2, "the trapezoid rule needs two samples"
    t = dt_fs * np.arange(len(C))
    w = np.full(len(C), dt_fs)
    w[0] *= 0.5
    w[-1] *= 0.5
    out = np.zeros(len(E))
    for m, e in enumerate(E):
        out[m] = np.sum(w * C * np.exp(1j * e * t / HBAR - t / tau_fs)).real
    return out / (np.pi * HBAR)
