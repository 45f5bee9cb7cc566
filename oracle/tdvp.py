"""Two-site TDVP (paper Section 2.1.2, eq. two-site Hamiltonian and the
procedure that follows it), complex128, written for clarity, not speed.

Index conventions (shared with the docstrings of the tests):
  MPS tensor   A[alpha_{i-1}, sigma_i, alpha_i]
  MPO tensor   W[w_{i-1}, w_i, sigma, sigma']          (sigma = bra/output)
  left env     L[w, a, a']   a = bra (output) index, a' = ket (input) index
  right env    R[w, b, b']   b = bra (output) index, b' = ket (input) index
  two-site     theta[a, s, t, b]

Readings of the paper (which states the left-to-right procedure only):
* one time step = a left-to-right half-sweep with exp(-i H dt/2hbar) on every
  pair followed by a right-to-left half-sweep, the one-site backward
  evolution exp(+i H_eff,1 dt/2hbar) (eq. backward TDVP) after every pair
  except the last of each half-sweep;
* the local exponentials are Lanczos (Krylov) approximations with full
  re-orthogonalisation; the Krylov method itself is described by the paper
  for the global propagator (eqs. Krylov subspace, global Krylov);
* DBSS truncation: eps is a threshold on the relative discarded weight
  sum_{j>k} s_j^2 <= eps * sum_j s_j^2, capped at D_max; no renormalisation.
"""
import numpy as np
import scipy.linalg

from . import HBAR


# --------------------------------------------------------------------------
# environments (projections of H on the block bases, eqs. one-/two-site H)
# --------------------------------------------------------------------------
def env_boundary():
    return np.ones((1, 1, 1), dtype=complex)


def env_left(L, A, W):
    """L_{i+1}[x, a, a'] = sum conj(A[b,s,a]) L_i[w,b,b'] W[w,x,s,s'] A[b',s',a'],
    summed one operand at a time (ket, MPO, bra)."""
    X = np.einsum("wbB,BSA->wbSA", L, A, optimize=True)
    X = np.einsum("wxsS,wbSA->xbsA", W, X, optimize=True)
    return np.einsum("bsa,xbsA->xaA", A.conj(), X, optimize=True)


def env_right(R, B, W):
    """R_i[w, a, a'] = sum conj(B[a,s,b]) W[w,x,s,s'] R_{i+1}[x,b,b'] B[a',s',b'],
    summed one operand at a time (ket, MPO, bra)."""
    X = np.einsum("xbB,ASB->xASb", R, B, optimize=True)
    X = np.einsum("wxsS,xASb->wAsb", W, X, optimize=True)
    return np.einsum("asb,wAsb->waA", B.conj(), X, optimize=True)


def heff2(L, W1, W2, R, theta):
    """y[a,s,t,b] = sum L[w,a,a'] W1[w,x,s,s'] W2[x,y,t,t'] R[y,b,b'] theta[a',s',t',b']
    (eq. two-site Hamiltonian), summed one operand at a time."""
    X = np.einsum("waA,ASTB->waSTB", L, theta, optimize=True)
    X = np.einsum("wxsS,waSTB->xasTB", W1, X, optimize=True)
    X = np.einsum("xytT,xasTB->yastB", W2, X, optimize=True)
    return np.einsum("ybB,yastB->astb", R, X, optimize=True)


def heff2_block(L, W1, W2, R, theta, a, b):
    """y[a,:,:,b] of heff2 for one left and one right bond index: the same
    sum (eq. two-site Hamiltonian) restricted to one output row a and column
    b, for sampled checks of products too large to form on the CPU."""
    X = np.einsum("wA,ASTB->wSTB", L[:, a, :], theta, optimize=True)
    X = np.einsum("yB,wSTB->wyST", R[:, b, :], X, optimize=True)
    X = np.einsum("wxsS,wyST->xysT", W1, X, optimize=True)
    return np.einsum("xytT,xysT->st", W2, X, optimize=True)


def heff1(L, W, R, M):
    """y[a,s,b] = sum L[w,a,a'] W[w,x,s,s'] R[x,b,b'] M[a',s',b']
    (eq. one-site Hamiltonian 1), summed one operand at a time."""
    X = np.einsum("waA,ASB->waSB", L, M, optimize=True)
    X = np.einsum("wxsS,waSB->xasB", W, X, optimize=True)
    return np.einsum("xbB,xasB->asb", R, X, optimize=True)


def heff0(L, R, C):
    """y[a,b] = sum L[w,a,a'] R[w,b,b'] C[a',b'] (eq. zero-site Hamiltonian:
    the MPO bond between the two blocks is the only index the two
    environments share), summed one operand at a time."""
    X = np.einsum("waA,AB->waB", L, C, optimize=True)
    return np.einsum("wbB,waB->ab", R, X, optimize=True)


def heff0_matrix(L, R):
    M = np.einsum("waA,wbB->abAB", L, R, optimize=True)
    n = int(np.sqrt(M.size))
    return M.reshape(n, n)


def heff2_matrix(L, W1, W2, R):
    """Explicit H_eff,2 as a matrix over (a,s,t,b) (small problems only)."""
    M = np.einsum("waA,wxsS,xytT,ybB->astbASTB", L, W1, W2, R, optimize="greedy")
    n = int(np.sqrt(M.size))
    return M.reshape(n, n)


def heff1_matrix(L, W, R):
    M = np.einsum("waA,wxsS,xbB->asbASB", L, W, R, optimize=True)
    n = int(np.sqrt(M.size))
    return M.reshape(n, n)


# --------------------------------------------------------------------------
# Lanczos exponential
# --------------------------------------------------------------------------
def tridiag_expm_e1(alpha, beta, tau):
    """exp(-i tau T) e_1 for the real symmetric tridiagonal T(alpha, beta)."""
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    lam, Z = np.linalg.eigh(T)
    return Z @ (np.exp(-1j * tau * lam) * Z[0, :])


def lanczos_expm(apply_h, v, tau, tol=1e-13, m_max=60):
    """Approximate exp(-i tau H) v in the Krylov space of (H, v).

    Steps: orthonormal Krylov basis by Lanczos with two classical
    Gram-Schmidt re-orthogonalisation passes against all previous vectors;
    T_m tridiagonal with alpha_j = Re<v_j, H v_j>, beta_j = ||w_j||;
    stop when beta_m |e_m^T exp(-i tau T_m) e_1| <= tol (relative to ||v||)
    or at m_max; result ||v|| V_m exp(-i tau T_m) e_1.
    Returns (result, number of H applications, converged flag).
    """
    shape = v.shape
    v = v.reshape(-1)
    beta0 = np.linalg.norm(v)
    if beta0 == 0.0:
        return v.reshape(shape).copy(), 0, True
    V = [v / beta0]
    alpha, beta = [], []
    for j in range(m_max):
        w = apply_h(V[j].reshape(shape)).reshape(-1)
        a = float(np.vdot(V[j], w).real)
        w = w - a * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        for _ in range(2):
            Vm = np.array(V)
            w = w - Vm.T @ (Vm.conj() @ w)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        c = tridiag_expm_e1(np.array(alpha), np.array(beta), tau)
        err = b * abs(c[-1])
        if err <= tol or j == m_max - 1:
            res = beta0 * (np.array(V).T @ c)
            return res.reshape(shape), j + 1, bool(err <= tol)
        beta.append(b)
        V.append(w / b)
    raise AssertionError("unreachable")


# --------------------------------------------------------------------------
# SVD truncation (Section 2.1.1, DBSS)
# --------------------------------------------------------------------------
def choose_rank(s, eps, D_max, sv_mode=0, tie_rel=1e-12):
    """Number of singular values kept.

    sv_mode 0: smallest k >= 1 with sum_{j>=k} s_j^2 <= eps * sum_j s_j^2;
    sv_mode 1: keep every s_j >= eps * s_0;
    sv_mode 2: keep all.  Then k <= D_max, and a near-degenerate multiplet at
    the cut (s_k >= (1 - tie_rel) s_{k-1} > 0) is kept whole while k < D_max.
    """
    n = len(s)
    if sv_mode == 2:
        k = n
    elif sv_mode == 1:
        k = int(np.sum(s >= eps * s[0])) if n else 0
    else:
        sq = s.astype(float) ** 2
        total = sq.sum()
        tail = np.zeros(n + 1)
        for j in range(n - 1, -1, -1):  # tail[j] = sum_{l >= j} s_l^2
            tail[j] = tail[j + 1] + sq[j]
        k = n
        for j in range(1, n + 1):
            if tail[j] <= eps * total:
                k = j
                break
    k = max(1, min(k, D_max, n))
    if sv_mode != 2:
        while k < min(n, D_max) and s[k] > 0 and s[k] >= (1.0 - tie_rel) * s[k - 1]:
            k += 1
    return k


def svd(mat):
    """Thin SVD mat = u diag(s) vh, s descending: LAPACK's divide-and-conquer
    driver, or the QR-iteration driver where that one does not converge.
    Both are backward stable (errors of about eps_mach |mat| in every s_j);
    the divide-and-conquer driver is some 40 times faster at the sizes of the
    two-site tensors (1700 x 1700 complex)."""
    try:
        return scipy.linalg.svd(mat, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        return scipy.linalg.svd(mat, full_matrices=False, lapack_driver="gesvd")


def svd_truncate(theta, eps, D_max, sv_mode=0, tie_rel=1e-12, k_fixed=None):
    """theta[a,s,t,b] -> (U[a,s,k], S[k], Vh[k,t,b], discarded weight).
    k_fixed, when given, replaces the rank rule (frozen-rank differences)."""
    Dl, d1, d2, Dr = theta.shape
    mat = theta.reshape(Dl * d1, d2 * Dr)
    u, s, vh = svd(mat)
    k = choose_rank(s, eps, D_max, sv_mode, tie_rel) if k_fixed is None else int(k_fixed)
    disc = float(np.sum(s[k:] ** 2))
    return u[:, :k].reshape(Dl, d1, k), s[:k], vh[:k].reshape(k, d2, Dr), disc, s


# --------------------------------------------------------------------------
# the 2TDVP sweep
# --------------------------------------------------------------------------
class TDVP2:
    """State of a 2TDVP propagation: MPS (right-canonical, centre on site 0
    between steps), MPO and the environments."""

    def __init__(self, mps, W, krylov_tol=1e-13, krylov_max=60, sv_mode=0, tie_rel=1e-12):
        self.mps = [a.copy() for a in mps]
        self.W = W
        self.n = len(mps)
        self.krylov_tol = krylov_tol
        self.krylov_max = krylov_max
        self.sv_mode = sv_mode
        self.tie_rel = tie_rel
        n = self.n
        self.L = [None] * (n + 1)
        self.R = [None] * (n + 1)
        self.L[0] = env_boundary()
        self.R[n] = env_boundary()
        for i in range(n - 1, 0, -1):
            self.R[i] = env_right(self.R[i + 1], self.mps[i], W[i])
        self.time = 0.0

    def _expm2(self, i, theta, tau):
        L, W1, W2, R = self.L[i], self.W[i], self.W[i + 1], self.R[i + 2]
        return lanczos_expm(lambda x: heff2(L, W1, W2, R, x), theta, tau,
                            self.krylov_tol, self.krylov_max)

    def _expm1(self, i, M, tau):
        L, W, R = self.L[i], self.W[i], self.R[i + 1]
        return lanczos_expm(lambda x: heff1(L, W, R, x), M, tau,
                            self.krylov_tol, self.krylov_max)

    def step(self, dt, D_max, eps, ranks=None):
        """One symmetric 2TDVP time step of length dt (fs).  ranks = (k_lr, k_rl),
        each indexed by pair, fixes the kept ranks instead of the rank rule."""
        tau = dt / (2.0 * HBAR)
        n, mps, W = self.n, self.mps, self.W
        stats = dict(k_lr=[], k_rl=[], disc=[], krylov=[], converged=True)
        for i in range(n - 1):  # left -> right
            theta = np.tensordot(mps[i], mps[i + 1], axes=([2], [0]))
            theta, it, ok = self._expm2(i, theta, tau)
            stats["krylov"].append(it); stats["converged"] &= ok
            U, S, Vh, disc, _ = svd_truncate(theta, eps, D_max, self.sv_mode, self.tie_rel,
                                             None if ranks is None else ranks[0][i])
            stats["k_lr"].append(len(S)); stats["disc"].append(disc)
            mps[i] = U
            mps[i + 1] = S[:, None, None] * Vh
            self.L[i + 1] = env_left(self.L[i], mps[i], W[i])
            if i < n - 2:
                mps[i + 1], it, ok = self._expm1(i + 1, mps[i + 1], -tau)
                stats["krylov"].append(it); stats["converged"] &= ok
        for i in range(n - 2, -1, -1):  # right -> left
            theta = np.tensordot(mps[i], mps[i + 1], axes=([2], [0]))
            theta, it, ok = self._expm2(i, theta, tau)
            stats["krylov"].append(it); stats["converged"] &= ok
            U, S, Vh, disc, _ = svd_truncate(theta, eps, D_max, self.sv_mode, self.tie_rel,
                                             None if ranks is None else ranks[1][i])
            stats["k_rl"].append(len(S)); stats["disc"].append(disc)
            mps[i] = U * S[None, None, :]
            mps[i + 1] = Vh
            self.R[i + 1] = env_right(self.R[i + 2], mps[i + 1], W[i + 1])
            if i > 0:
                mps[i], it, ok = self._expm1(i, mps[i], -tau)
                stats["krylov"].append(it); stats["converged"] &= ok
        self.time += dt
        return stats


# --------------------------------------------------------------------------
# the 1TDVP sweep (zero-site backward steps, no truncation)
# --------------------------------------------------------------------------
def split_left(M):
    """M[a,s,b] = A[a,s,c] C[c,b], A left-orthonormal (eq. l orthonormal):
    Householder QR of the (a s) x b matrix.  The bond keeps its dimension,
    so it must not exceed the row count."""
    Dl, d, Dr = M.shape
    assert Dr <= Dl * d, "bond larger than its left block"
    q, r = np.linalg.qr(M.reshape(Dl * d, Dr))
    return q.reshape(Dl, d, Dr), r


def split_right(M):
    """M[a,s,b] = C[a,c] B[c,s,b], B right-orthonormal (eq. r orthonormal):
    Householder QR of the conjugate transpose of the a x (s b) matrix."""
    Dl, d, Dr = M.shape
    assert Dl <= d * Dr, "bond larger than its right block"
    q, r = np.linalg.qr(M.reshape(Dl, d * Dr).conj().T)
    return r.conj().T, q.conj().T.reshape(Dl, d, Dr)


class TDVP1:
    """One-site TDVP (Section 2.1.2, the 1TDVP scheme): every site is
    evolved forward with the one-site effective Hamiltonian, split into an
    orthonormal tensor and a bond matrix, and the bond matrix is evolved
    backward with the zero-site effective Hamiltonian before it is absorbed
    into the next site.  Bond dimensions never change and nothing is
    truncated, so norm and energy are conserved up to the Krylov tolerance.

    One time step (the same reading as the two-site scheme): a left-to-right
    half-sweep with tau = dt/2hbar and its mirror image from right to left;
    no backward step after the last site of either half-sweep.  The MPS
    enters right-canonical with the centre on site 0 and leaves that way."""

    def __init__(self, mps, W, krylov_tol=1e-13, krylov_max=60):
        self.mps = [a.copy() for a in mps]
        self.W = W
        self.n = len(mps)
        self.krylov_tol = krylov_tol
        self.krylov_max = krylov_max
        n = self.n
        self.L = [None] * (n + 1)
        self.R = [None] * (n + 1)
        self.L[0] = env_boundary()
        self.R[n] = env_boundary()
        for i in range(n - 1, 0, -1):
            self.R[i] = env_right(self.R[i + 1], self.mps[i], W[i])
        self.time = 0.0

    def _expm1(self, i, M, tau):
        L, W, R = self.L[i], self.W[i], self.R[i + 1]
        return lanczos_expm(lambda x: heff1(L, W, R, x), M, tau, self.krylov_tol, self.krylov_max)

    def _expm0(self, b, C, tau):
        """Bond b sits between sites b-1 and b: L[b] and R[b] meet there."""
        L, R = self.L[b], self.R[b]
        return lanczos_expm(lambda x: heff0(L, R, x), C, tau, self.krylov_tol, self.krylov_max)

    def step(self, dt):
        tau = dt / (2.0 * HBAR)
        n, mps, W = self.n, self.mps, self.W
        stats = dict(krylov=[], converged=True)

        def note(it, ok):
            stats["krylov"].append(it)
            stats["converged"] &= ok

        for i in range(n):  # left -> right
            mps[i], it, ok = self._expm1(i, mps[i], tau)
            note(it, ok)
            if i < n - 1:
                mps[i], C = split_left(mps[i])
                self.L[i + 1] = env_left(self.L[i], mps[i], W[i])
                C, it, ok = self._expm0(i + 1, C, -tau)
                note(it, ok)
                mps[i + 1] = np.tensordot(C, mps[i + 1], axes=([1], [0]))
        for i in range(n - 1, -1, -1):  # right -> left
            mps[i], it, ok = self._expm1(i, mps[i], tau)
            note(it, ok)
            if i > 0:
                C, mps[i] = split_right(mps[i])
                self.R[i] = env_right(self.R[i + 1], mps[i], W[i])
                C, it, ok = self._expm0(i, C, -tau)
                note(it, ok)
                mps[i - 1] = np.tensordot(mps[i - 1], C, axes=([2], [0]))
        self.time += dt
        return stats
