"""GPU parity of one whole local 2TDVP update at the benchmark's saturated
bond dimension (IC-shaped 24-mode model, D = 128), called through the C ABI,
against the oracle on identical inputs.

The procedure after eq. two-site Hamiltonian (Section 2.1.2), for one pair
(i, i+1) of a left-to-right half-sweep: theta = M_i B_{i+1}, theta <-
exp(-i tau H_eff,2) theta, DBSS truncation theta = U S V^H (Section 2.1.1),
A_i = U, M_{i+1} = S V^H, the environment L_{i+1} from L_i, W_i and A_i, and
the backward one-site step M_{i+1} <- exp(+i tau H_eff,1) M_{i+1} (eq.
backward TDVP).

The state around the pair is a seeded synthetic MPS with every bond at its
saturated value min(128, full-rank cut): random isometries made left- or
right-orthonormal by the oracle's QR splits, and a centre whose singular
values fall geometrically over ten decades across the 128 kept values, as
in a state grown to D_max under eps = 1e-8.  The environments are the
oracle's chains over those tensors, so H_eff is Hermitian and has the
benchmark's operators.  (The state grown by the GPU's own warm-up steps is
not used: no oracle input may come from the path under test, and the oracle
needs hours per step at this bond dimension.)

Every step is compared twice: on identical inputs (the oracle's result of
the previous step uploaded), element by element where the result is unique
and on gauge-invariant quantities where it is not; and chained (the GPU's
own results passed on), through the gauge-invariant two-site tensor
A_i M'_{i+1} after the backward step."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

D = 128
EPS = 1e-8
TAU = 0.5 / (2 * 0.6582119569)  # dt = 0.5 fs, half a step
PAIRS = [3, 0]  # a bulk pair (d 17 x 18, bonds 128 | 128, subspace SVD route) and the chain's left end


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1908_10588_amd as T
    return T


@pytest.fixture(scope="module")
def ctx(T):
    return T.Ctx(0)


def _cg(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def state():
    return build_state()


def build_state():
    """Synthetic saturated state: sites 0..i-1 left-orthonormal for every
    pair i tested, sites 2.. right-orthonormal; L_i and R_{i+2} by the
    oracle's environment chains; the centre M_i of each pair."""
    from oracle import hamiltonian as ham
    from oracle import mpo as ompo
    from oracle import tdvp as ot
    model = synth.config2_model(0, D_max=D)
    W = ompo.build_mpo(model)
    dims = ham.site_dims(model)
    n = len(dims)
    bonds = [min(D, int(np.prod(dims[:k], dtype=float)), int(np.prod(dims[k:], dtype=float))) for k in range(n + 1)]
    rng = np.random.default_rng(2024)
    imax = max(PAIRS)
    left = []
    for j in range(imax):
        A, _ = ot.split_left(_cg(rng, bonds[j], dims[j], bonds[j + 1]))
        left.append(A)
    right = {}
    for j in range(n - 1, min(PAIRS), -1):
        _, B = ot.split_right(_cg(rng, bonds[j], dims[j], bonds[j + 1]))
        right[j] = B
    L = [ot.env_boundary()]
    for j in range(imax):
        L.append(ot.env_left(L[-1], left[j], W[j]))
    R = {n: ot.env_boundary()}
    for j in range(n - 1, min(PAIRS) + 1, -1):
        R[j] = ot.env_right(R[j + 1], right[j], W[j])
    centres = {}
    for i in PAIRS:
        Dl, d, Dr = bonds[i], dims[i], bonds[i + 1]
        k = min(Dl * d, Dr)
        X, _ = np.linalg.qr(_cg(rng, Dl * d, k))
        Y, _ = np.linalg.qr(_cg(rng, Dr, k))
        s = 10.0 ** (-5.0 * np.arange(k) / D) * (1.0 + 0.05 * rng.uniform(size=k))
        s = np.sort(s)[::-1] / np.linalg.norm(s)
        centres[i] = ((X * s) @ Y.conj().T).reshape(Dl, d, Dr)
    return dict(model=model, W=W, dims=dims, bonds=bonds, L=L, R=R, right=right, centres=centres)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _svd_gpu(T, ctx, theta_dev, shape, kcap):
    import torch
    Dl, d1, d2, Dr = shape
    U = torch.zeros(2, Dl, d1, kcap, dtype=torch.float64, device="cuda")
    S = torch.zeros(kcap, dtype=torch.float64, device="cuda")
    Vh = torch.zeros(2, kcap, d2, Dr, dtype=torch.float64, device="cuda")
    k, disc = T.tdmrg_svd_truncate(ctx, Dl, d1, d2, Dr, theta_dev, EPS, D, 0, 1e-12, kcap, U, S, Vh)
    rows, cols = Dl * d1, d2 * Dr
    Ug = T.from_planar(U.cpu().numpy().reshape(-1)[:2 * rows * k].reshape(2, rows, k))
    Vg = T.from_planar(Vh.cpu().numpy().reshape(-1)[:2 * k * cols].reshape(2, k, cols))
    return k, disc, Ug, S.cpu().numpy()[:k], Vg


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("i", PAIRS)
def test_saturated_local_update_parity(T, ctx, state, i):
    import torch
    from oracle import tdvp as ot
    W, dims, bonds = state["W"], state["dims"], state["bonds"]
    Dl, d1, Dm, d2, Dr = bonds[i], dims[i], bonds[i + 1], dims[i + 1], bonds[i + 2]
    wl, wc, wr = W[i].shape[0], W[i].shape[1], W[i + 1].shape[1]
    shape2 = (Dl, d1, d2, Dr, wl, wc, wr)
    print("saturated pair", i, "shape", shape2, flush=True)
    Lh, Rh = state["L"][i], state["R"][i + 2]
    M, B = state["centres"][i], state["right"][i + 1]
    W1, W2 = T.Wop(ctx, W[i]), T.Wop(ctx, W[i + 1])
    Ld, Rd = T.to_device(Lh), T.to_device(Rh)

    # theta formation
    th_ref = np.tensordot(M, B, axes=([2], [0]))
    th = torch.empty(2, Dl, d1, d2, Dr, dtype=torch.float64, device="cuda")
    T.tdmrg_theta_form(ctx, Dl, d1, Dm, d2, Dr, T.to_device(M), T.to_device(B), th)
    assert _rel(T.from_device(th), th_ref) < 1e-13

    # forward two-site exponential (the sweep's tolerance and step limit)
    th_ref, it_ref, ok = ot.lanczos_expm(lambda x: ot.heff2(Lh, W[i], W[i + 1], Rh, x), th_ref, TAU, 1e-13, 60)
    assert ok
    it, ok = T.tdmrg_local_expm(ctx, shape2, True, Ld, W1, W2, Rd, th, TAU, tol=1e-12, m_max=40)
    print("Lanczos steps GPU", it, "oracle", it_ref, flush=True)
    assert ok
    th_gpu = T.from_device(th)
    assert _rel(th_gpu, th_ref) < 1e-10

    # truncated SVD on identical input (the oracle's theta), GPU auto route
    U_ref, S_ref, Vh_ref, disc_ref, s_all = ot.svd_truncate(th_ref, EPS, D)
    kcap = min(Dl * d1, d2 * Dr, D)
    k, disc, Ug, Sg, Vg = _svd_gpu(T, ctx, T.to_device(th_ref), (Dl, d1, d2, Dr), kcap)
    s0 = s_all[0]
    print("k", k, len(S_ref), "disc", disc, disc_ref, "s_k/s_0", S_ref[-1] / s0, flush=True)
    assert k == len(S_ref)
    assert abs(disc - disc_ref) < 5e-13 * s0 ** 2
    assert np.abs(Sg ** 2 - S_ref ** 2).max() < 5e-13 * s0 ** 2
    trunc_ref = (U_ref.reshape(-1, k) * S_ref) @ Vh_ref.reshape(k, -1)
    assert np.abs((Ug * Sg) @ Vg - trunc_ref).max() < 1e-12 * s0
    assert np.abs(Ug.conj().T @ Ug - np.eye(k)).max() < 1e-12

    # environment update on identical input (the oracle's A_i)
    A_ref = U_ref
    L1_ref = ot.env_left(Lh, A_ref, W[i])
    L1 = torch.empty(2, wc, k, k, dtype=torch.float64, device="cuda")
    T.tdmrg_env_update_left(ctx, Dl, d1, k, Ld, W1, T.to_device(A_ref), L1)
    assert _rel(T.from_device(L1), L1_ref) < 1e-12

    # backward one-site step on identical input
    M1_ref = S_ref[:, None, None] * Vh_ref
    M1_back, _, ok = ot.lanczos_expm(lambda x: ot.heff1(L1_ref, W[i + 1], Rh, x), M1_ref, -TAU, 1e-13, 60)
    assert ok
    shape1 = (k, d2, 0, Dr, wc, 0, wr)
    M1 = T.to_device(M1_ref)
    it1, ok = T.tdmrg_local_expm(ctx, shape1, False, T.to_device(L1_ref), W2, None, Rd, M1, -TAU, tol=1e-12,
                                 m_max=40)
    assert ok
    assert _rel(T.from_device(M1), M1_back) < 1e-10

    # chained: the GPU's own SVD factors, environment and backward step
    kc, _, Uc, Sc, Vc = _svd_gpu(T, ctx, th, (Dl, d1, d2, Dr), kcap)
    assert kc == k
    A_c = T.to_device(Uc.reshape(Dl, d1, kc))
    L1c = torch.empty(2, wc, kc, kc, dtype=torch.float64, device="cuda")
    T.tdmrg_env_update_left(ctx, Dl, d1, kc, Ld, W1, A_c, L1c)
    M1c = T.to_device((Sc[:, None] * Vc).reshape(kc, d2, Dr))
    T.tdmrg_local_expm(ctx, shape1, False, L1c, W2, None, Rd, M1c, -TAU, tol=1e-12, m_max=40)
    two_site_gpu = np.tensordot(Uc.reshape(Dl, d1, kc), T.from_device(M1c), axes=([2], [0]))
    two_site_ref = np.tensordot(A_ref, M1_back, axes=([2], [0]))
    err = _rel(two_site_gpu, two_site_ref)
    print("chained A_i M'_{i+1} relative error", err, flush=True)
    assert err < 1e-10
