"""Global time integrators on whole MPS (paper Section 2.1.1: the 4th-order
Runge-Kutta update, eqs. runge kutta 1-4 and runge kutta, the global
Krylov method, eqs. Krylov subspace and global Krylov, and the Taylor
expansion of the propagator that Section 3.1 runs at second order), complex128, written
for clarity.  Test infrastructure: the oracle of the library's global step.

Building blocks (the paper applies H to the compressed MPS and compresses
the intermediates; it does not fix how):
  apply_mpo    exact MPO x MPS product, bonds multiplied by the MPO bonds
               (the direct procedure of Section 2.1.1);
  apply_mpo_variational
               the MPO x MPS product fitted by sweeping two-site updates
               (the variational procedure, eq. variational app), bonds
               capped by the DBSS rule;
  lincomb      sum_k c_k |x_k> by block-diagonal bond concatenation;
  compress     left-to-right orthonormalisation (reduced SVD, every value
               kept), then right-to-left SVD truncation with the DBSS rule
               of the two-site sweep (tdvp.choose_rank) capped at D_max; the
               result is right-canonical with its centre on site 0.
Readings:
  * with apply="direct" H|x> is the direct product compressed and a sum the
    bond concatenation compressed; with apply="variational" both are fitted
    (fit_variational), so no bond D*w or sum_k D_k is ever formed;
  * RK4 applies the compression after every H application and after every
    sum (K_i and the stage arguments are compressed MPS);
  * the Taylor step of order p is sum_{k<=p} T_k with T_0 = psi and
    T_k = (-i dt/hbar / k) H T_{k-1}, each T_k compressed after its H
    application as in RK4, the sum compressed once;
  * the global Krylov basis is built by Lanczos on compressed MPS (three-term
    recurrence, alpha_j = Re<v_j|H v_j>, beta_j = |w_j|) and the new state is
    beta_0 sum_k c_k v_k with c = exp(-i dt/hbar T_m) e_1, compressed; it
    stops when beta_m |c_m| <= tol or at m_max vectors.
"""
import numpy as np

from . import HBAR
from .tdvp import choose_rank, heff2, svd_truncate, tridiag_expm_e1
from .observables import overlap, expectation


def apply_mpo(W, mps):
    """(W mps)[a w, s, b w'] = sum_s' W[w, w', s, s'] A[a, s', b]."""
    out = []
    for A, w in zip(mps, W):
        Dl, d, Dr = A.shape
        wl, wr = w.shape[0], w.shape[1]
        B = np.einsum("xyst,atb->axsby", w, A)
        out.append(B.reshape(Dl * wl, d, Dr * wr))
    return out


def lincomb(coeffs, states):
    """sum_k c_k |x_k> with bonds concatenated (first site along its right
    bond, last along its left bond, block-diagonal in between); c_k scales
    the first site of x_k."""
    n = len(states[0])
    out = []
    for s in range(n):
        if n == 1:
            out.append(sum(c * x[0] for c, x in zip(coeffs, states)))
            continue
        if s == 0:
            out.append(np.concatenate([c * x[0] for c, x in zip(coeffs, states)], axis=2))
        elif s == n - 1:
            out.append(np.concatenate([x[s] for x in states], axis=0))
        else:
            Dl = sum(x[s].shape[0] for x in states)
            Dr = sum(x[s].shape[2] for x in states)
            d = states[0][s].shape[1]
            B = np.zeros((Dl, d, Dr), dtype=complex)
            a0 = b0 = 0
            for x in states:
                a, _, b = x[s].shape
                B[a0:a0 + a, :, b0:b0 + b] = x[s]
                a0 += a
                b0 += b
            out.append(B)
    return out


def compress(mps, D_max, eps, sv_mode=0, tie_rel=1e-12):
    """Left-orthonormalise (reduced SVD, all values kept, which also drops
    bonds larger than their blocks), then truncate right to left.  Returns
    (right-canonical MPS with centre on site 0, discarded weight)."""
    A = [a.copy() for a in mps]
    n = len(A)
    for s in range(n - 1):
        Dl, d, Dr = A[s].shape
        u, sv, vh = np.linalg.svd(A[s].reshape(Dl * d, Dr), full_matrices=False)
        A[s] = u.reshape(Dl, d, -1)
        A[s + 1] = np.tensordot(sv[:, None] * vh, A[s + 1], axes=([1], [0]))
    disc = 0.0
    for s in range(n - 1, 0, -1):
        Dl, d, Dr = A[s].shape
        u, sv, vh = np.linalg.svd(A[s].reshape(Dl, d * Dr), full_matrices=False)
        k = choose_rank(sv, eps, D_max, sv_mode, tie_rel)
        disc += float(np.sum(sv[k:] ** 2))
        A[s] = vh[:k].reshape(k, d, Dr)
        A[s - 1] = np.tensordot(A[s - 1], u[:, :k] * sv[:k], axes=([2], [0]))
    return A, disc


def _env_left_mixed(L, bra, ket, W):
    """L'[x, a, a'] = sum conj(bra[b,s,a]) L[w,b,b'] W[w,x,s,s'] ket[b',s',a']
    (the left block of <phi| W |psi>), one operand at a time."""
    X = np.einsum("wbB,BSA->wbSA", L, ket, optimize=True)
    X = np.einsum("wxsS,wbSA->xbsA", W, X, optimize=True)
    return np.einsum("bsa,xbsA->xaA", bra.conj(), X, optimize=True)


def _env_right_mixed(R, bra, ket, W):
    """R'[w, a, a'] = sum conj(bra[a,s,b]) W[w,x,s,s'] R[x,b,b'] ket[a',s',b']."""
    X = np.einsum("xbB,ASB->xASb", R, ket, optimize=True)
    X = np.einsum("wxsS,xASb->wAsb", W, X, optimize=True)
    return np.einsum("asb,wAsb->waA", bra.conj(), X, optimize=True)


def fit_variational(terms, D_max, eps, sweeps=16, tol=1e-15):
    """|phi> minimising || |phi> - sum_k c_k O_k |x_k> ||^2 (eq. variational
    app; for a sum of MPS the O_k are identities) by sweeping local
    updates.  terms: list of (c_k, O_k, x_k), O_k a list of MPO tensors or
    None for the identity.  Reading: two-site updates, so that the bonds of
    |phi> follow the DBSS rule (eps, D_max) as in the direct route's
    compression.  With |phi> in mixed-canonical form around the pair (i, i+1)
    the distance is minimal at
        Phi = sum_k c_k L_k[w][a][a'] O_k,i[w,x] O_k,i+1[x,y] R_k[y][b][b'] x_k,i[a'] x_k,i+1[b']
    (L_k, R_k the left and right blocks of <phi|O_k|x_k>), which is
    truncated by SVD; left to right the pair splits into U (left-orthonormal)
    and S V^H, right to left into U S and V^H.  A sweep is both directions;
    sweeping stops ("until convergence") when |phi|^2 (the squared norm of
    the last pair) changes by at most tol relative to itself (default 1e-15,
    about the rounding level of the norm), or after `sweeps` sweeps (16).
    The start is a right-canonical copy of x_0.  Returns (phi right-canonical
    with its centre on site 0, sweeps run)."""
    x0 = terms[0][2]
    n = len(x0)
    ops = []
    for c, O, x in terms:
        if O is None:
            O = [np.eye(a.shape[1], dtype=complex)[None, None, :, :] for a in x]
        ops.append(O)
    phi = [a.copy() for a in x0]
    for s in range(n - 1, 0, -1):  # right-canonical copy of x_0
        Dl, d, Dr = phi[s].shape
        q, r = np.linalg.qr(phi[s].reshape(Dl, d * Dr).conj().T)
        phi[s] = q.conj().T.reshape(-1, d, Dr)
        phi[s - 1] = np.tensordot(phi[s - 1], r.conj().T, axes=([2], [0]))
    one = np.ones((1, 1, 1), dtype=complex)
    nt = len(terms)
    L = [[one] + [None] * n for _ in range(nt)]
    R = [[None] * n + [one] for _ in range(nt)]
    for k, (c, _, x) in enumerate(terms):
        for s in range(n - 1, 1, -1):
            R[k][s] = _env_right_mixed(R[k][s + 1], phi[s], x[s], ops[k][s])

    def pair(i):
        Phi = 0.0
        for k, (c, _, x) in enumerate(terms):
            theta = np.tensordot(x[i], x[i + 1], axes=([2], [0]))
            Phi = Phi + c * heff2(L[k][i], ops[k][i], ops[k][i + 1], R[k][i + 2], theta)
        return Phi

    last = None
    for sweep in range(1, sweeps + 1):
        for i in range(n - 1):  # left to right
            U, S, Vh, _, _ = svd_truncate(pair(i), eps, D_max)
            phi[i], phi[i + 1] = U, S[:, None, None] * Vh
            for k, (_, _, x) in enumerate(terms):
                L[k][i + 1] = _env_left_mixed(L[k][i], phi[i], x[i], ops[k][i])
        for i in range(n - 2, -1, -1):  # right to left
            U, S, Vh, _, _ = svd_truncate(pair(i), eps, D_max)
            phi[i], phi[i + 1] = U * S[None, None, :], Vh
            for k, (_, _, x) in enumerate(terms):
                R[k][i + 1] = _env_right_mixed(R[k][i + 2], phi[i + 1], x[i + 1], ops[k][i + 1])
        nrm = float(np.sum(S ** 2))
        if last is not None and abs(nrm - last) <= tol * max(nrm, 1e-300):
            return phi, sweep
        last = nrm
    return phi, sweeps


def apply_mpo_variational(W, psi, D_max, eps, sweeps=16, tol=1e-15):
    """W|psi> by the variational procedure (fit_variational with one term)."""
    return fit_variational([(1.0, W, psi)], D_max, eps, sweeps, tol)


def norm(mps):
    return float(np.sqrt(overlap(mps, mps).real))


def _H(W, x, D_max, eps, apply):
    """H|x> compressed: the direct product then compress, or the variational fit."""
    if apply == "variational":
        return apply_mpo_variational(W, x, D_max, eps)[0]
    return compress(apply_mpo(W, x), D_max, eps)[0]


def _Hc(f, W, x, D_max, eps, apply):
    """f H|x>: the direct product compressed, scaled and compressed again, or
    the variational fit scaled (a rescaled compressed MPS)."""
    if apply == "variational":
        return lincomb([f], [apply_mpo_variational(W, x, D_max, eps)[0]])
    return compress(lincomb([f], [_H(W, x, D_max, eps, apply)]), D_max, eps)[0]


def _comb(coeffs, states, D_max, eps, apply):
    """sum_k c_k |x_k>: concatenated and compressed, or fitted variationally."""
    if apply == "variational":
        return fit_variational([(c, None, x) for c, x in zip(coeffs, states)], D_max, eps)[0]
    return compress(lincomb(coeffs, states), D_max, eps)[0]


def rk4_step(mps, W, dt, D_max, eps, apply="direct"):
    """|psi(t + dt)> by eqs. runge kutta 1-4 (every intermediate compressed)."""
    f = -1j * dt / HBAR

    def Hc(x):
        return _Hc(f, W, x, D_max, eps, apply)

    K1 = Hc(mps)
    K2 = Hc(_comb([1.0, 0.5], [mps, K1], D_max, eps, apply))
    K3 = Hc(_comb([1.0, 0.5], [mps, K2], D_max, eps, apply))
    K4 = Hc(_comb([1.0, 1.0], [mps, K3], D_max, eps, apply))
    return _comb([1.0, 1 / 6, 1 / 3, 1 / 3, 1 / 6], [mps, K1, K2, K3, K4], D_max, eps, apply)


def taylor_step(mps, W, dt, D_max, eps, order=2, apply="direct"):
    """|psi(t + dt)> by the order-p Taylor expansion of exp(-i dt H / hbar)
    (every term compressed, then their sum)."""
    f = -1j * dt / HBAR
    terms = [mps]
    for k in range(1, order + 1):
        terms.append(_Hc(f / k, W, terms[-1], D_max, eps, apply))
    return _comb([1.0] * (order + 1), terms, D_max, eps, apply)


def global_krylov_step(mps, W, dt, D_max, eps, m_max=12, tol=1e-10, apply="direct"):
    """|psi(t + dt)> by eq. global Krylov: Lanczos on compressed MPS, the
    exact propagator in the basis, the result compressed.  Returns (mps,
    number of basis vectors)."""
    tau = dt / HBAR
    beta0 = norm(mps)
    V = [lincomb([1.0 / beta0], [mps])]
    alpha, beta = [], []
    for j in range(m_max):
        w = _H(W, V[j], D_max, eps, apply)
        a = float(overlap(V[j], w).real)
        alpha.append(a)
        terms, coeffs = [w, V[j]], [1.0, -a]
        if j > 0:
            terms.append(V[j - 1])
            coeffs.append(-beta[j - 1])
        w = _comb(coeffs, terms, D_max, eps, apply)
        b = norm(w)
        c = tridiag_expm_e1(np.array(alpha), np.array(beta), tau)
        if b * abs(c[-1]) <= tol or j == m_max - 1 or b == 0.0:
            out = _comb(list(beta0 * c), V, D_max, eps, apply)
            return out, j + 1
        beta.append(b)
        V.append(lincomb([1.0 / b], [w]))
    raise AssertionError("unreachable")


def energy(mps, W):
    return expectation(mps, W).real
