"""GPU parity of the truncated SVD routes (Jacobi, Gram + eigensolver,
subspace iteration) against the oracle's LAPACK SVD and DBSS rank rule, on
matrices with a prescribed singular spectrum."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1908_10588_amd as T
    return T


@pytest.fixture()
def ctx(T):
    c = T.Ctx(0)
    yield c
    c.close()


def _matrix(seed, rows, cols, s):
    rng = np.random.default_rng(seed)
    r = len(s)
    U, _ = np.linalg.qr(rng.standard_normal((rows, r)) + 1j * rng.standard_normal((rows, r)))
    V, _ = np.linalg.qr(rng.standard_normal((cols, r)) + 1j * rng.standard_normal((cols, r)))
    return (U * s) @ V.conj().T


def _run(T, ctx, th, eps, D_max, sv_mode=0, tie_rel=1e-12):
    import torch
    rows, cols = th.shape
    kcap = min(rows, cols, D_max)
    Ud = torch.zeros(2, rows, kcap, dtype=torch.float64, device="cuda")
    Sd = torch.zeros(kcap, dtype=torch.float64, device="cuda")
    Vd = torch.zeros(2, kcap, cols, dtype=torch.float64, device="cuda")
    k, disc = T.tdmrg_svd_truncate(ctx, rows, 1, 1, cols, T.to_device(th.reshape(rows, 1, 1, cols)), eps,
                                   D_max, sv_mode, tie_rel, kcap, Ud, Sd, Vd)
    Ug = T.from_planar(Ud.cpu().numpy().reshape(-1)[:2 * rows * k].reshape(2, rows, k))
    Vg = T.from_planar(Vd.cpu().numpy().reshape(-1)[:2 * k * cols].reshape(2, k, cols))
    return k, disc, Ug, Sd.cpu().numpy()[:k], Vg


def _check(th, eps, D_max, got, s0, tie_rel=1e-12):
    from oracle import tdvp as ot
    k, disc, Ug, Sg, Vg = got
    rows, cols = th.shape
    Ur, Sr, Vr, disc_r, _ = ot.svd_truncate(th.reshape(rows, 1, 1, cols), eps, D_max, 0, tie_rel)
    assert k == len(Sr)
    assert abs(disc - disc_r) <= 1e-13 * s0 ** 2
    # s_j^2 to a few hundred ulps of s_0^2 (Gram routes square; Jacobi rotates
    # a few hundred vectors over tens of sweeps)
    assert np.abs(Sg ** 2 - Sr ** 2).max() < 5e-13 * s0 ** 2
    ref = (Ur.reshape(rows, k) * Sr) @ Vr.reshape(k, cols)
    assert np.abs((Ug * Sg) @ Vg - ref).max() < 1e-12 * s0
    assert np.abs(Ug.conj().T @ Ug - np.eye(k)).max() < 1e-12


@pytest.mark.parametrize("rows,cols,decay,D_max,eps", [
    (420, 390, 15.0, 64, 1e-8),     # Schmidt-like decay, cap reached
    (300, 520, 40.0, 64, 1e-10),    # slow decay: many iterations, wide matrix
    (384, 400, 4.0, 128, 1e-8),     # numerically rank deficient (s_j < 1e-16 s_0 beyond j ~ 150)
    (260, 250, 8.0, 96, 1e-3),      # threshold cut well below the cap
    (1100, 1300, 20.0, 64, 1e-8),   # Gram products with K >= 1024: split K, ragged last chunk
])
@pytest.mark.parametrize("schedule", [0, 1])
def test_subspace_svd_parity(T, ctx, rows, cols, decay, D_max, eps, schedule):
    """Both first-check schedules; schedule 0 runs the problem twice, the
    second time with its first check at the first run's converged iteration."""
    r = min(rows, cols)
    s = np.exp(-np.arange(r) / decay)
    th = _matrix(rows + cols, rows, cols, s)
    ctx.set_svd_method("subspace")
    ctx.set_svd_schedule(schedule)
    print("subspace SVD", rows, cols, decay, D_max, eps, "schedule", schedule, flush=True)
    runs = 2 if schedule == 0 else 1
    for _ in range(runs):
        got = _run(T, ctx, th, eps, D_max)
        _check(th, eps, D_max, got, s[0])
    c = ctx.svd_counters()
    assert c["subspace"] == runs and c["gram"] == 0 and c["subspace_factor_fail"] == 0, c


@pytest.mark.timeout(600)
def test_subspace_svd_benchmark_size(T, ctx):
    """The largest truncation of the benchmark's timed steps, (128*29) x
    (29*128) = 3712 x 3712 at D_max 128 and eps 1e-8, on the default (auto)
    route, which takes the subspace iteration here; the spectrum falls like
    the evolved two-site tensors of the saturated state (s_128 ~ 2e-3 s_0, so
    the D_max cap binds)."""
    rows = cols = 3712
    s = np.exp(-np.arange(800) / 20.0)
    th = _matrix(3712, rows, cols, s)
    print("subspace SVD at the benchmark size", rows, cols, flush=True)
    got = _run(T, ctx, th, 1e-8, 128)
    assert got[0] == 128
    assert ctx.svd_counters()["subspace"] == 1
    _check(th, 1e-8, 128, got, s[0])


def test_subspace_svd_keeps_tie_at_cut(T, ctx):
    """An exactly degenerate pair straddling the DBSS cut is kept whole."""
    rows, cols, D_max = 200, 260, 40
    s = np.exp(-np.arange(rows) / 6.0)
    s[21] = s[20]
    th = _matrix(5, rows, cols, s)
    sq = s ** 2
    eps = sq[21:].sum() / sq.sum() * (1 + 1e-9)  # natural cut k = 21, inside the pair
    ctx.set_svd_method("subspace")
    got = _run(T, ctx, th, eps, D_max)
    assert got[0] == 22
    assert ctx.svd_counters()["subspace"] == 1
    _check(th, eps, D_max, got, s[0])


def test_svd_routes_agree(T, ctx):
    """Jacobi, Gram + eigensolver and subspace iteration give the same
    truncated matrix on one problem all three accept."""
    rows, cols, D_max, eps = 240, 200, 48, 1e-9
    s = np.exp(-np.arange(cols) / 10.0)
    th = _matrix(17, rows, cols, s)
    outs = {}
    for m in ("jacobi", "gram", "subspace"):
        ctx.set_svd_method(m)
        outs[m] = _run(T, ctx, th, eps, D_max)
        _check(th, eps, D_max, outs[m], s[0])
    c = ctx.svd_counters()
    assert (c["jacobi"], c["gram"], c["subspace"]) == (1, 1, 1), c
    recon = {m: (o[2] * o[3]) @ o[4] for m, o in outs.items()}
    assert np.abs(recon["jacobi"] - recon["subspace"]).max() < 1e-12
    assert np.abs(recon["gram"] - recon["subspace"]).max() < 1e-12


def test_subspace_svd_rejects_keep_all(T, ctx):
    th = _matrix(3, 200, 200, np.exp(-np.arange(200) / 5.0))
    ctx.set_svd_method("subspace")
    with pytest.raises(T.TdmrgError):
        _run(T, ctx, th, 0.0, 32, sv_mode=2)


@pytest.mark.parametrize("n,spectrum", [
    (1, "graded"), (2, "graded"), (3, "degenerate"), (17, "graded"), (80, "graded"), (81, "degenerate"),
    (150, "rank_deficient"), (240, "degenerate"), (241, "graded"),
])
def test_gram_route_eigensolvers(T, ctx, n, spectrum):
    """The Gram route (G = theta theta^H of order n = rows) with both Hermitian
    eigensolvers: the library's Householder reduction + tridiagonal divide and
    conquer (n <= 240; 241 takes zheevd) and rocSOLVER zheevd.  Both
    match the oracle's SVD and each other on the truncated matrix; spectra
    with an exactly threefold degenerate triplet, a zero tail beyond rank 20,
    or a plain exponential fall."""
    rows, cols = n, n + 37
    r = min(rows, cols)
    s = np.exp(-np.arange(r) / max(r / 12.0, 1.0))
    if spectrum == "degenerate" and r >= 6:
        s[4] = s[5] = s[3]
    if spectrum == "rank_deficient":
        s[20:] = 0.0
    th = _matrix(1000 + n, rows, cols, s)
    D_max, eps = min(n, 64), 1e-10
    ctx.set_svd_method("gram")
    recon = {}
    for eig in ("reduction", "zheevd"):
        ctx.set_eigensolver(eig)
        print("Gram route", n, spectrum, eig, flush=True)
        got = _run(T, ctx, th, eps, D_max)
        _check(th, eps, D_max, got, s[0])
        recon[eig] = (got[2] * got[3]) @ got[4]
    assert np.abs(recon["reduction"] - recon["zheevd"]).max() < 1e-12 * s[0]
    assert ctx.svd_counters()["gram"] == 2


@pytest.mark.parametrize("eig", ["reduction", "zheevd"])
def test_subspace_svd_eigensolvers(T, ctx, eig):
    """The subspace iteration's Rayleigh-Ritz step with either eigensolver
    (block b = 96 for D_max 64)."""
    rows, cols, D_max, eps = 700, 650, 64, 1e-9
    s = np.exp(-np.arange(cols) / 12.0)
    s[10] = s[11] = s[9]
    th = _matrix(23, rows, cols, s)
    ctx.set_svd_method("subspace")
    ctx.set_eigensolver(eig)
    got = _run(T, ctx, th, eps, D_max)
    _check(th, eps, D_max, got, s[0])
    assert ctx.svd_counters()["subspace"] == 1
