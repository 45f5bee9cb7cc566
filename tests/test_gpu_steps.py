"""GPU parity of the single steps of the 2TDVP hot path, called through the
C ABI, against the oracle on the same seeded inputs.

Shapes span several 64x64 GEMM tiles with ragged tails; the floating-point
bar is 1e-12 relative (FP64 arithmetic, different summation order) and 1e-5
relative for the FP32 contraction form."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SHAPES2 = [  # Dl, d1, d2, Dr, wl, wc, wr
    (1, 2, 8, 8, 1, 5, 5),
    (5, 3, 2, 7, 2, 3, 2),
    (37, 4, 5, 29, 3, 4, 5),
    (64, 6, 6, 64, 5, 5, 5),
    (70, 5, 3, 66, 4, 6, 3),
    (129, 2, 3, 17, 3, 2, 4),
]


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1908_10588_amd as T
    return T


@pytest.fixture(scope="module")
def ctx(T):
    return T.Ctx(0)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# channel stages: sparse pass, fused two-site pass as its own kernel, the
# fused pass inside the last GEMM's A loader, dense GEMMs
CHANNELS = {"sparse": (0, 0, 0), "fused": (0, 2, 0), "fused_in_gemm": (0, 2, 1), "gemm": (2, 0, 0)}


@pytest.mark.parametrize("shape", SHAPES2)
@pytest.mark.parametrize("density", [1.0, 0.4])
@pytest.mark.parametrize("channels", list(CHANNELS))
def test_heff2_parity(T, ctx, shape, density, channels):
    from oracle import tdvp as ot
    seed = (sum(shape) * 7 + int(density * 10)) % 1000
    print("heff2", shape, density, "channels", channels, "seed", seed, flush=True)
    p = synth.heff_problem(seed, *shape, w_density=density)
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    L, R, th = T.to_device(p["L"]), T.to_device(p["R"]), T.to_device(p["theta"])
    import torch
    gemm_mode, fusion, mix_in_gemm = CHANNELS[channels]
    ctx.set_channel_gemm(gemm_mode)
    T.lib().tdmrg_ctx_set_fusion(ctx.h, fusion)
    ctx.set_mix_in_gemm(mix_in_gemm)
    try:
        y = torch.empty_like(th)
        T.tdmrg_heff2_apply(ctx, shape, L, W1, W2, R, th, y)
        got = T.from_device(y)
        ref = ot.heff2(p["L"], p["W1"], p["W2"], p["R"], p["theta"])
        assert _rel(got, ref) < 1e-12
        y32 = torch.empty_like(th)
        T.tdmrg_heff2_apply(ctx, shape, L, W1, W2, R, th, y32, precision=T.FP32)
        assert _rel(T.from_device(y32), ref) < 2e-5
    finally:
        T.lib().tdmrg_ctx_set_fusion(ctx.h, 1)
        ctx.set_channel_gemm(1)
        ctx.set_mix_in_gemm(0)


def test_vibronic_mpo_pair_fusion(T, ctx):
    """The real MPO tensors of the benchmark model (sparse channel blocks), with
    and without the fused channel stage."""
    import torch
    from oracle import tdvp as ot
    model = synth.config2_model(0)
    mpo = T.MPO(ctx, model)
    i = 3
    W1n, W2n = mpo.site_tensor(i), mpo.site_tensor(i + 1)
    Dl, Dr = 9, 11
    shape = (Dl, W1n.shape[2], W2n.shape[2], Dr, W1n.shape[0], W1n.shape[1], W2n.shape[1])
    rng = np.random.default_rng(2)
    L = rng.standard_normal((shape[4], Dl, Dl)) + 1j * rng.standard_normal((shape[4], Dl, Dl))
    R = rng.standard_normal((shape[6], Dr, Dr)) + 1j * rng.standard_normal((shape[6], Dr, Dr))
    th = rng.standard_normal((Dl, shape[1], shape[2], Dr)) + 1j * rng.standard_normal((Dl, shape[1], shape[2], Dr))
    ref = ot.heff2(L, W1n, W2n, R, th)
    for fusion, mix in ((0, 1), (1, 1), (2, 1), (2, 0)):
        T.lib().tdmrg_ctx_set_fusion(ctx.h, fusion)
        ctx.set_mix_in_gemm(mix)
        y = torch.empty(2, *th.shape, dtype=torch.float64, device="cuda")
        T.tdmrg_heff2_apply(ctx, shape, T.to_device(L), mpo.wop(i), mpo.wop(i + 1), T.to_device(R),
                            T.to_device(th), y)
        assert _rel(T.from_device(y), ref) < 1e-12, (fusion, mix)
    T.lib().tdmrg_ctx_set_fusion(ctx.h, 1)
    ctx.set_mix_in_gemm(0)


@pytest.mark.parametrize("shape", [(1, 8, 0, 8, 1, 0, 5), (37, 4, 0, 29, 3, 0, 5),
                                   (80, 7, 0, 66, 5, 0, 4)])
def test_heff1_parity(T, ctx, shape):
    from oracle import tdvp as ot
    import torch
    Dl, d, _, Dr, wl, _, wr = shape
    p = synth.heff_problem(11, Dl, d, 1, Dr, wl, 1, wr, two_site=False)
    W = T.Wop(ctx, p["W"])
    L, R, M = T.to_device(p["L"]), T.to_device(p["R"]), T.to_device(p["theta"])
    y = torch.empty_like(M)
    T.tdmrg_heff1_apply(ctx, (Dl, d, 1, Dr, wl, 1, wr), L, W, R, M, y)
    ref = ot.heff1(p["L"], p["W"], p["R"], p["theta"])
    assert _rel(T.from_device(y), ref) < 1e-12


def test_heff2_hermitian_and_deterministic(T, ctx):
    import torch
    shape = (37, 4, 5, 29, 3, 4, 5)
    p = synth.heff_problem(3, *shape)
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    L, R = T.to_device(p["L"]), T.to_device(p["R"])
    rng = np.random.default_rng(0)
    x = rng.standard_normal(p["theta"].shape) + 1j * rng.standard_normal(p["theta"].shape)
    z = rng.standard_normal(p["theta"].shape) + 1j * rng.standard_normal(p["theta"].shape)
    hx, hz = torch.empty(2, *x.shape, dtype=torch.float64, device="cuda"), None
    hz = torch.empty_like(hx)
    T.tdmrg_heff2_apply(ctx, shape, L, W1, W2, R, T.to_device(x), hx)
    T.tdmrg_heff2_apply(ctx, shape, L, W1, W2, R, T.to_device(z), hz)
    a = np.vdot(z, T.from_device(hx))
    b = np.vdot(T.from_device(hz), x)
    assert abs(a - b) < 1e-12 * abs(a)
    hx2 = torch.empty_like(hx)
    T.tdmrg_heff2_apply(ctx, shape, L, W1, W2, R, T.to_device(x), hx2)
    assert torch.equal(hx, hx2)  # bitwise reproducible


@pytest.mark.parametrize("two_site,shape,tau", [
    (True, (5, 3, 2, 7, 2, 3, 2), 0.7),
    (True, (37, 4, 5, 29, 3, 4, 5), -0.4),
    (False, (40, 6, 1, 33, 4, 1, 5), 0.9),
])
def test_local_expm_parity(T, ctx, two_site, shape, tau):
    from oracle import tdvp as ot
    Dl, d1, d2, Dr, wl, wc, wr = shape
    p = synth.heff_problem(21, *shape, two_site=two_site)
    if two_site:
        W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
        ref, it_ref, _ = ot.lanczos_expm(lambda x: ot.heff2(p["L"], p["W1"], p["W2"], p["R"], x),
                                         p["theta"], tau)
    else:
        W1, W2 = T.Wop(ctx, p["W"]), None
        ref, it_ref, _ = ot.lanczos_expm(lambda x: ot.heff1(p["L"], p["W"], p["R"], x),
                                         p["theta"], tau)
    L, R, th = T.to_device(p["L"]), T.to_device(p["R"]), T.to_device(p["theta"])
    it, ok = T.tdmrg_local_expm(ctx, shape, two_site, L, W1, W2, R, th, tau, tol=1e-13, m_max=60)
    got = T.from_device(th)
    assert ok
    assert abs(it - it_ref) <= 1
    assert np.linalg.norm(got - ref) < 1e-11 * np.linalg.norm(ref)
    assert abs(np.linalg.norm(got) - np.linalg.norm(p["theta"])) < 1e-12


@pytest.mark.parametrize("tau", [0.8, 40.0, -300.0])
def test_local_expm_small_exact(T, ctx, tau):
    """Against scipy's expm of the explicit effective Hamiltonian (dimension
    36, so the Krylov space is exhausted by 36 vectors at any tau).  The
    spectrum spans +-1.19, so tau 40 takes the small tridiagonal exponential
    through a long Chebyshev expansion and tau -300 through the QR route."""
    import scipy.linalg
    from oracle import tdvp as ot
    shape = (3, 2, 3, 2, 2, 2, 3)
    p = synth.heff_problem(5, *shape)
    H = ot.heff2_matrix(p["L"], p["W1"], p["W2"], p["R"])
    ref = (scipy.linalg.expm(-1j * tau * H) @ p["theta"].reshape(-1)).reshape(p["theta"].shape)
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    th = T.to_device(p["theta"])
    print("local expm small exact, tau", tau, flush=True)
    T.tdmrg_local_expm(ctx, shape, True, T.to_device(p["L"]), W1, W2, T.to_device(p["R"]), th,
                       tau, tol=1e-14, m_max=40)
    # rounding of the phases exp(-i tau lambda) grows with |tau|
    assert np.abs(T.from_device(th) - ref).max() < 1e-12 * max(1.0, abs(tau))


@pytest.mark.parametrize("Dl,d1,d2,Dr,eps,D_max,mode", [
    (8, 4, 3, 10, 1e-6, 64, 0),
    (37, 5, 6, 29, 1e-8, 40, 0),
    (16, 8, 8, 16, 1e-3, 128, 1),
    (6, 2, 3, 5, 0.0, 100, 2),
    (50, 3, 3, 70, 1e-10, 20, 0),
    (16, 8, 1, 8, 1e-10, 64, 0),    # 128 x 8: Jacobi on the 8 columns, U by division + Cholesky QR
])
def test_svd_truncate_parity(T, ctx, Dl, d1, d2, Dr, eps, D_max, mode):
    import torch
    from oracle import tdvp as ot
    rng = np.random.default_rng(Dl + Dr)
    # graded spectrum so that the DBSS threshold actually selects a rank
    rows, cols = Dl * d1, d2 * Dr
    k0 = min(rows, cols)
    U, _ = np.linalg.qr(rng.standard_normal((rows, k0)) + 1j * rng.standard_normal((rows, k0)))
    V, _ = np.linalg.qr(rng.standard_normal((cols, k0)) + 1j * rng.standard_normal((cols, k0)))
    s = np.exp(-0.35 * np.arange(k0))
    th = ((U * s) @ V.conj().T).reshape(Dl, d1, d2, Dr)
    Ur, Sr, Vr, disc_r, _ = ot.svd_truncate(th, eps, D_max, mode)
    kcap = min(rows, cols, D_max)
    Ud = torch.zeros(2, Dl, d1, kcap, dtype=torch.float64, device="cuda")
    Sd = torch.zeros(kcap, dtype=torch.float64, device="cuda")
    Vd = torch.zeros(2, kcap, d2, Dr, dtype=torch.float64, device="cuda")
    k, disc = T.tdmrg_svd_truncate(ctx, Dl, d1, d2, Dr, T.to_device(th), eps, D_max, mode, 1e-12,
                                   kcap, Ud, Sd, Vd)
    assert k == len(Sr)
    assert abs(disc - disc_r) <= 1e-13 * max(1.0, np.sum(s ** 2))
    # outputs are packed at the kept rank: U [2][rows][k], Vh [2][k][cols]
    Ug = T.from_planar(Ud.cpu().numpy().reshape(-1)[:2 * rows * k].reshape(2, rows, k))
    Vg = T.from_planar(Vd.cpu().numpy().reshape(-1)[:2 * k * cols].reshape(2, k, cols))
    Sg = Sd.cpu().numpy()[:k]
    # singular values come from Gram eigenvalues: s^2 is exact to ~eps_mach * s_0^2
    assert np.abs(Sg ** 2 - Sr ** 2).max() < 1e-13 * s[0] ** 2
    # gauge-invariant comparison: the truncated matrix
    got = (Ug * Sg) @ Vg
    ref = (Ur.reshape(-1, k) * Sr) @ Vr.reshape(k, -1)
    assert np.abs(got - ref).max() < 1e-12
    assert np.abs(Ug.conj().T @ Ug - np.eye(k)).max() < 1e-12
    # Vh = S^-1 U^H theta, so (Vh Vh^H)_ij = (U^H theta theta^H U)_ij / (s_i s_j):
    # orthonormal to a few ulps of s_0^2 / (s_i s_j) for any accurate eigenbasis
    assert np.abs(Vg @ Vg.conj().T - np.eye(k)).max() < max(1e-12, 1e-15 * (s[0] / Sr[-1]) ** 2)


def test_theta_form_and_envs(T, ctx):
    import torch
    from oracle import tdvp as ot
    rng = np.random.default_rng(4)

    def cg(*s):
        return rng.standard_normal(s) + 1j * rng.standard_normal(s)

    Dl, d1, Dm, d2, Dr = 19, 5, 33, 4, 23
    M, B = cg(Dl, d1, Dm), cg(Dm, d2, Dr)
    th = torch.empty(2, Dl, d1, d2, Dr, dtype=torch.float64, device="cuda")
    T.tdmrg_theta_form(ctx, Dl, d1, Dm, d2, Dr, T.to_device(M), T.to_device(B), th)
    assert _rel(T.from_device(th), np.tensordot(M, B, axes=([2], [0]))) < 1e-13
    for dens in (1.0, 0.5):
        p = synth.heff_problem(8, Dl, d1, 1, Dm, 4, 1, 6, two_site=False, w_density=dens)
        W = T.Wop(ctx, p["W"])
        A = cg(Dl, d1, Dm)
        Lout = torch.empty(2, 6, Dm, Dm, dtype=torch.float64, device="cuda")
        T.tdmrg_env_update_left(ctx, Dl, d1, Dm, T.to_device(p["L"][:4]), W, T.to_device(A), Lout)
        assert _rel(T.from_device(Lout), ot.env_left(p["L"][:4], A, p["W"])) < 1e-12
        Rin = p["R"]  # (6, Dm, Dm)
        Rout = torch.empty(2, 4, Dl, Dl, dtype=torch.float64, device="cuda")
        T.tdmrg_env_update_right(ctx, Dl, d1, Dm, T.to_device(Rin), W, T.to_device(A), Rout)
        assert _rel(T.from_device(Rout), ot.env_right(Rin, A, p["W"])) < 1e-12


def test_envs_benchmark_size(T, ctx):
    """Environment updates at the benchmark's largest site: D 128 on both
    bonds, d 30, MPO bonds 15 x 15 with the block sparsity of a vibronic
    channel operator (half the blocks zero)."""
    import torch
    from oracle import tdvp as ot
    D, d, w = 128, 30, 15
    p = synth.heff_problem(9, D, d, 1, D, w, 1, w, two_site=False, w_density=0.5)
    rng = np.random.default_rng(30)
    A = rng.standard_normal((D, d, D)) + 1j * rng.standard_normal((D, d, D))
    W = T.Wop(ctx, p["W"])
    print("env update at D 128, d 30, w 15", flush=True)
    Lout = torch.empty(2, w, D, D, dtype=torch.float64, device="cuda")
    T.tdmrg_env_update_left(ctx, D, d, D, T.to_device(p["L"]), W, T.to_device(A), Lout)
    assert _rel(T.from_device(Lout), ot.env_left(p["L"], A, p["W"])) < 1e-12
    Rout = torch.empty(2, w, D, D, dtype=torch.float64, device="cuda")
    T.tdmrg_env_update_right(ctx, D, d, D, T.to_device(p["R"]), W, T.to_device(A), Rout)
    assert _rel(T.from_device(Rout), ot.env_right(p["R"], A, p["W"])) < 1e-12


def test_gemm_autotune_is_bitwise_neutral(T):
    """Tile autotuning only changes the workgroup tiling: H_eff,2 * theta with
    tuning on (every variant timed on the first call) equals the untuned
    product bitwise, and the tuned classes are reported."""
    import torch
    # the L and R stages (M x N x K x batch = 120 * 7*8*100 * 120 * 4 = 3.2e8)
    # are above the tuning threshold of 2e8; ragged tiles on every side
    shape = (120, 7, 8, 100, 4, 5, 4)
    p = synth.heff_problem(5, *shape)
    outs = []
    for tune in (0, 1):
        c = T.Ctx(0)
        c.set_autotune(tune)
        W1, W2 = T.Wop(c, p["W1"]), T.Wop(c, p["W2"])
        L, R, th = T.to_device(p["L"]), T.to_device(p["R"]), T.to_device(p["theta"])
        y = torch.empty_like(th)
        for _ in range(2):  # second call runs the tuned variant
            T.tdmrg_heff2_apply(c, shape, L, W1, W2, R, th, y)
        torch.cuda.synchronize()
        outs.append(y.clone())
        if tune:
            table = c.tile_table()
            print("tuned classes", table, flush=True)
            assert len(table) >= 1 and all(0 <= r["variant"] < 6 for r in table)
        c.close()
    assert torch.equal(outs[0], outs[1])


def test_lanczos_step_graphs_are_bitwise_eager(T):
    """With step graphs on, the first call captures one Lanczos step after its
    first eager step and replays it; a second call with the same operands
    replays from the start.  Both equal the all-eager result bitwise, and a
    graph-replayed sweep equals an eager one bitwise."""
    import torch
    shape = (37, 4, 5, 29, 3, 4, 5)
    p = synth.heff_problem(21, *shape)
    outs = []
    for graphs in (0, 1):
        c = T.Ctx(0)
        c.set_graphs(graphs)
        W1, W2 = T.Wop(c, p["W1"]), T.Wop(c, p["W2"])
        L, R = T.to_device(p["L"]), T.to_device(p["R"])
        for call in range(2):
            th = T.to_device(p["theta"])
            it, ok = T.tdmrg_local_expm(c, shape, True, L, W1, W2, R, th, 0.4, tol=1e-13, m_max=40)
            assert ok and it > 3
            outs.append(th.clone())
        cnt = c.graph_counters()
        print("graphs", graphs, cnt, flush=True)
        if graphs:
            assert cnt["captured"] == 1 and cnt["replayed"] == 2 * it - 1 and cnt["eager"] == 1
        else:
            assert cnt["captured"] == 0 and cnt["replayed"] == 0
        c.close()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    # whole sweeps: config 1, a few steps with and without graphs
    model = synth.config1_model(0)
    pops = []
    for graphs in (0, 1):
        c = T.Ctx(0)
        c.set_graphs(graphs)
        mpo = T.MPO(c, model)
        mps = T.MPS(c, mpo, model["occ"], model["D_max"])
        for _ in range(3):
            T.tdmrg_tdvp2_sweep(c, mps, mpo, model["dt_fs"], model["D_max"], model["eps"])
        pops.append(T.tdmrg_observables(c, mps, mpo)["pops"].copy())
        cnt = c.graph_counters()
        print("sweep graphs", graphs, cnt, flush=True)
        if graphs:
            assert cnt["replayed"] > cnt["eager"]
        del mps, mpo
        c.close()
    assert np.array_equal(pops[0], pops[1])


def test_heff2_benchmark_pair_full_size_sampled(T, ctx):
    """H_eff,2 * theta at the benchmark's full size: the heaviest pair of the
    IC-shaped 24-mode model (its MPO tensors, d up to 29 x 29, w up to 15) at
    D = 128 with Hermitian random environments, in the benchmark's launch
    configuration (default context: autotuned tiles, automatic channel-stage
    form), sampled output blocks y[a,:,:,b] against the oracle computed one
    block at a time."""
    import torch
    from oracle import mpo as ompo
    from oracle import tdvp as ot
    model = synth.config2_model(0, D_max=128)
    Ws = ompo.build_mpo(model)
    D = 128
    cost = [Ws[i].shape[2] * Ws[i + 1].shape[2] * (Ws[i].shape[0] + Ws[i + 1].shape[1]) for i in range(len(Ws) - 1)]
    i = int(np.argmax(cost))
    W1, W2 = Ws[i], Ws[i + 1]
    shape = (D, W1.shape[2], W2.shape[2], D, W1.shape[0], W1.shape[1], W2.shape[1])
    print("benchmark pair", i, shape, flush=True)
    p = synth.heff_problem(7, *shape)
    L, R, th = T.to_device(p["L"]), T.to_device(p["R"]), T.to_device(p["theta"])
    y = torch.empty_like(th)
    T.tdmrg_heff2_apply(ctx, shape, L, T.Wop(ctx, W1), T.Wop(ctx, W2), R, th, y)
    torch.cuda.synchronize()
    yh = T.from_device(y)
    for a, b in ((0, D - 1), (77, 5), (D - 1, 64)):
        ref = ot.heff2_block(p["L"], W1, W2, p["R"], p["theta"], a, b)
        err = np.abs(yh[a, :, :, b] - ref).max()
        print("block", a, b, "err", err, flush=True)
        assert err < 1e-12 * max(1.0, np.abs(ref).max()), (a, b)


def test_benchmark_steps_full_size_invariants(T, ctx):
    """The benchmark's workload at full size (IC-shaped 24-mode model, D_max
    128, warm-up steps of 2 fs that grow the bonds, then steps of 0.5 fs):
    the norm equals one minus every discarded weight (no renormalisation,
    unitary local exponentials), the populations sum to the norm, and the
    bonds reach D_max."""
    model = synth.config2_model(0, D_max=128)
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], 128)
    disc = 0.0
    for k, dt in enumerate([2.0] * 4 + [0.5] * 2):
        st = T.tdmrg_tdvp2_sweep(ctx, mps, mpo, dt, 128, model["eps"])
        disc += st.sum_disc
        print("full-size step", k, "max bond", max(mps.bond_dims()), "disc", st.sum_disc, flush=True)
    obs = T.tdmrg_observables(ctx, mps, mpo)
    bonds = mps.bond_dims()
    assert max(bonds) == 128
    assert abs(obs["norm2"] - (1.0 - disc)) < 1e-9, (obs["norm2"], disc)
    assert abs(obs["pops"].sum() - obs["norm2"]) < 1e-12


@pytest.mark.parametrize("shape", SHAPES2)
@pytest.mark.parametrize("form", ["bf16x3", "bf16x6"])
def test_heff2_bf16_split_parity(T, ctx, shape, form):
    """BF16-split contractions (operands split into two or three bfloat16
    pieces, FP32 accumulation on the BF16 MFMA): H_eff,2 theta against the
    oracle's FP64 product on the same operands, with the sparse channel pass
    and with the channel stages as GEMMs.  Bars from the split's
    representation error: three pieces reach the FP32 level (2e-5 relative to
    the largest output, as the FP32 form), two pieces about 2^-16 per
    product (1e-4; measured up to 1.3e-5)."""
    import torch
    from oracle import tdvp as ot
    prec, bar = (T.BF16X3, 1e-4) if form == "bf16x3" else (T.BF16X6, 2e-5)
    seed = (sum(shape) * 5 + 3) % 1000
    p = synth.heff_problem(seed, *shape, w_density=0.5)
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    L, R, th = T.to_device(p["L"]), T.to_device(p["R"]), T.to_device(p["theta"])
    ref = ot.heff2(p["L"], p["W1"], p["W2"], p["R"], p["theta"])
    try:
        for gemm_mode in (0, 2):
            ctx.set_channel_gemm(gemm_mode)
            y = torch.empty_like(th)
            T.tdmrg_heff2_apply(ctx, shape, L, W1, W2, R, th, y, precision=prec)
            err = _rel(T.from_device(y), ref)
            print("heff2", form, shape, "channel gemm", gemm_mode, "relative error", err, flush=True)
            assert err < bar, (gemm_mode, err)
    finally:
        ctx.set_channel_gemm(1)


@pytest.mark.parametrize("form", ["bf16x3", "bf16x6"])
def test_envs_and_batched_bf16_split(T, ctx, form):
    """Environment updates and the grouped (batched) product in the
    BF16-split forms against the oracle."""
    import torch
    from oracle import tdvp as ot
    prec, bar = (T.BF16X3, 1e-4) if form == "bf16x3" else (T.BF16X6, 2e-5)
    rng = np.random.default_rng(12)
    Dl, d, Dr = 37, 6, 45
    p = synth.heff_problem(13, Dl, d, 1, Dr, 4, 1, 5, two_site=False, w_density=0.6)
    W = T.Wop(ctx, p["W"])
    A = rng.standard_normal((Dl, d, Dr)) + 1j * rng.standard_normal((Dl, d, Dr))
    Lout = torch.empty(2, 5, Dr, Dr, dtype=torch.float64, device="cuda")
    T.tdmrg_env_update_left(ctx, Dl, d, Dr, T.to_device(p["L"]), W, T.to_device(A), Lout, precision=prec)
    assert _rel(T.from_device(Lout), ot.env_left(p["L"], A, p["W"])) < bar
    shapes = [(33, 4, 5, 29, 3, 4, 2), (70, 3, 2, 65, 2, 5, 3), (8, 7, 6, 9, 4, 2, 4)]
    probs = [synth.heff_problem(40 + k, *s, w_density=0.7) for k, s in enumerate(shapes)]
    Ws1 = [T.Wop(ctx, q["W1"]) for q in probs]
    Ws2 = [T.Wop(ctx, q["W2"]) for q in probs]
    Ls = [T.to_device(q["L"]) for q in probs]
    Rs = [T.to_device(q["R"]) for q in probs]
    ths = [T.to_device(q["theta"]) for q in probs]
    ys = [torch.empty_like(t) for t in ths]
    T.tdmrg_heff2_apply_batched(ctx, shapes, Ls, Ws1, Ws2, Rs, ths, ys, precision=prec)
    for q, y in zip(probs, ys):
        assert _rel(T.from_device(y), ot.heff2(q["L"], q["W1"], q["W2"], q["R"], q["theta"])) < bar
