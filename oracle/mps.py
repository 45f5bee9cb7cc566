"""Matrix product states (paper eqs. MPS tensor / MPS matrix).

A state is a list of complex128 tensors A[s] with index order
(alpha_{s-1}, sigma_s, alpha_s); boundary bonds have dimension 1.
"""
import numpy as np


def product_state(dims, occ):
    """|occ_0> x |occ_1> x ... with all bond dimensions 1 (trivially
    right-canonical, orthogonality centre on site 0)."""
    out = []
    for d, k in zip(dims, occ):
        a = np.zeros((1, d, 1), dtype=complex)
        a[0, k, 0] = 1.0
        out.append(a)
    return out


def to_dense(mps):
    v = mps[0]
    for a in mps[1:]:
        v = np.tensordot(v, a, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


def from_dense_full_rank(psi, dims):
    """Exact MPS of a dense vector with every bond at full rank
    min(prod d_left, prod d_right), right-canonical with the centre on site 0.

    Successive SVDs from the right keep *all* singular values, zeros
    included, so every block basis is complete."""
    n = len(dims)
    rest = psi.reshape(-1, 1)
    tensors = [None] * n
    right_dim = 1
    for s in range(n - 1, 0, -1):
        mat = rest.reshape(-1, dims[s] * right_dim)
        u, sv, vh = np.linalg.svd(mat, full_matrices=False)
        k = min(mat.shape)
        tensors[s] = vh[:k].reshape(k, dims[s], right_dim)
        rest = u[:, :k] * sv[:k]
        right_dim = k
    tensors[0] = rest.reshape(1, dims[0], right_dim)
    return tensors


def full_rank_caps(dims):
    """Largest useful bond dimension on every bond 0..n."""
    n = len(dims)
    caps = []
    for b in range(n + 1):
        left = int(np.prod(dims[:b], dtype=object)) if b > 0 else 1
        right = int(np.prod(dims[b:], dtype=object)) if b < n else 1
        caps.append(min(left, right))
    return caps


def bond_dims(mps):
    return [mps[0].shape[0]] + [a.shape[2] for a in mps]


def mps_size(mps):
    """Number of stored coefficients sum_i m_{i-1} d_i m_i (Section 3.1)."""
    return int(sum(a.size for a in mps))


def left_orth_error(a):
    """|| sum_{s,alpha_{i-1}} A^* A - 1 || (eq. l orthonormal)."""
    m = a.reshape(-1, a.shape[2])
    return float(np.abs(m.conj().T @ m - np.eye(m.shape[1])).max())


def right_orth_error(b):
    """|| sum_{s,alpha_i} B B^* - 1 || (eq. r orthonormal)."""
    m = b.reshape(b.shape[0], -1)
    return float(np.abs(m @ m.conj().T - np.eye(m.shape[0])).max())
