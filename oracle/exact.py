"""Exact references: propagation in the full product space (eqs. propagator,
time evolution) and closed forms used to pin the oracle."""
import numpy as np
import scipy.sparse.linalg as spla

from . import HBAR
from .hamiltonian import dense_hamiltonian, el_site_of, per_state, site_dims


def product_vector(model):
    dims = site_dims(model)
    v = np.zeros(int(np.prod(dims)), dtype=complex)
    idx = 0
    for d, k in zip(dims, model["occ"]):
        idx = idx * d + int(k)
    v[idx] = 1.0
    return v


def evolve(model, psi0, times):
    """psi(t) = exp(-i H t / hbar) psi0 at every t in `times` (fs)."""
    H = dense_hamiltonian(model)
    out = []
    for t in times:
        out.append(spla.expm_multiply(-1j * (t / HBAR) * H, psi0))
    return out


def el_populations(model, psi):
    dims = site_dims(model)
    p = np.abs(psi.reshape(dims)) ** 2
    if per_state(model):  # P_i = <n_i>: weight with site of state i occupied
        out = []
        for i in range(model["n_el"]):
            e = el_site_of(model, i)
            out.append(np.take(p, 1, axis=e).sum())
        return np.array(out)
    el = list(model["order"]).index(-1)
    axes = tuple(a for a in range(len(dims)) if a != el)
    return p.sum(axis=axes)


def displaced_autocorrelation(t, E, omegas, kappas):
    """C(t) = <psi(0)|psi(t)> for one electronic state of energy E with
    harmonic modes w_I (n_I + 1/2) + kappa_I q_I, starting from the vacuum:
    C = exp(-iEt/hbar) prod_I exp(-i w t/2hbar + i S w t/hbar - S (1 - e^{-i w t/hbar})),
    S_I = kappa_I^2 / (2 w_I^2) (untruncated oscillators)."""
    t = np.asarray(t, dtype=float)
    out = np.exp(-1j * E * t / HBAR)
    for w, k in zip(omegas, kappas):
        S = k * k / (2.0 * w * w)
        x = w * t / HBAR
        out = out * np.exp(-0.5j * x + 1j * S * x - S * (1.0 - np.exp(-1j * x)))
    return out


def rabi_population(t, E0, E1, V):
    """Population transferred out of the initially occupied level of a
    two-level system [[E0, V], [V, E1]]."""
    dE = E1 - E0
    W2 = dE * dE + 4.0 * V * V
    return 4.0 * V * V / W2 * np.sin(np.sqrt(W2) * np.asarray(t) / (2.0 * HBAR)) ** 2


def electronic_populations(Hel, i0, t):
    """|<i| exp(-i Hel t/hbar) |i0>|^2 by diagonalising the small matrix."""
    lam, Z = np.linalg.eigh(Hel)
    out = []
    for tt in np.atleast_1d(t):
        psi = Z @ (np.exp(-1j * lam * tt / HBAR) * Z[i0, :].conj())
        out.append(np.abs(psi) ** 2)
    return np.array(out)
