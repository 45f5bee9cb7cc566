"""GPU adjoints (vector-Jacobian products) of H_eff,2*theta and of the local
exponential, called through the C ABI, against central finite differences of
the CPU oracle (the oracle gradient) and through torch.autograd."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1908_10588_amd as T
    return T


@pytest.fixture(scope="module")
def ctx(T):
    return T.Ctx(0)


def _cg(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rdot(a, b):
    """Real inner product Re sum conj(a) b of complex arrays."""
    return float(np.real(np.vdot(a, b)))


def _fd(fun, args, name, E, h):
    plus = dict(args)
    minus = dict(args)
    plus[name] = args[name] + h * E
    minus[name] = args[name] - h * E
    return (fun(**plus) - fun(**minus)) / (2 * h)


SHAPE = (5, 3, 2, 7, 2, 3, 2)
# Large enough that the library cuts the long reductions of the operator
# cotangents into chunks: the W2 products (65 blocks of K 37) and the W1
# products (13 blocks of K 111) into runs of whole blocks with a shorter last
# run, the L product (K 555) into K ranges.
SHAPE_SPLIT = (13, 5, 3, 37, 3, 4, 3)


def _operands(seed, shape, hermitian):
    p = synth.heff_problem(seed, *shape)
    if not hermitian:  # break the per-channel Hermiticity: general operators
        rng = np.random.default_rng(seed + 1)
        for k in ("L", "W1", "W2", "R"):
            p[k] = p[k] + 0.3 * _cg(rng, p[k].shape) / np.sqrt(p[k].size)
    return p


@pytest.mark.parametrize("shape,hermitian", [(SHAPE, True), (SHAPE, False), (SHAPE_SPLIT, False)])
def test_heff2_vjp_against_oracle_fd(T, ctx, shape, hermitian):
    import torch
    from oracle import tdvp as ot
    p = _operands(3, shape, hermitian)
    rng = np.random.default_rng(11)
    c = _cg(rng, p["theta"].shape)  # f = Re<c, y>, so ybar = c

    def f(L, W1, W2, R, theta):
        return _rdot(c, ot.heff2(L, W1, W2, R, theta))

    dev = {k: T.to_device(p[k]) for k in ("L", "R", "theta")}
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    bars = {k: torch.zeros(2, *p[k].shape, dtype=torch.float64, device="cuda")
            for k in ("L", "W1", "W2", "R", "theta")}
    T.tdmrg_heff2_apply_vjp(ctx, shape, dev["L"], W1, W2, dev["R"], dev["theta"], T.to_device(c),
                            bars["L"], bars["W1"], bars["W2"], bars["R"], bars["theta"])
    args = {k: p[k] for k in ("L", "W1", "W2", "R", "theta")}
    for name in args:
        E = _cg(rng, p[name].shape)
        fd = _fd(f, args, name, E, 1e-4)  # f is linear in each operand: exact up to rounding
        got = _rdot(T.from_device(bars[name]), E)
        assert abs(got - fd) <= 1e-10 * max(1.0, abs(fd)), (name, got, fd)


def _herm(E):
    """Project a direction onto operators Hermitian per channel (last two axes)."""
    return 0.5 * (E + np.conj(np.swapaxes(E, -1, -2)))


def test_local_expm_vjp_against_oracle_fd(T, ctx):
    """The Lanczos exponential is defined for Hermitian H_eff only, so operand
    directions are projected onto per-channel Hermitian ones; theta moves freely."""
    import torch
    from oracle import tdvp as ot
    shape = (4, 3, 2, 5, 2, 3, 2)
    p = _operands(5, shape, hermitian=True)
    tau = 0.7
    rng = np.random.default_rng(12)
    c = _cg(rng, p["theta"].shape)

    def f(L, W1, W2, R, theta):
        y, _, _ = ot.lanczos_expm(lambda x: ot.heff2(L, W1, W2, R, x), theta, tau, tol=1e-15)
        return _rdot(c, y)

    dev = {k: T.to_device(p[k]) for k in ("L", "R", "theta")}
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    bars = {k: torch.zeros(2, *p[k].shape, dtype=torch.float64, device="cuda")
            for k in ("L", "W1", "W2", "R", "theta")}
    T.tdmrg_local_expm_vjp(ctx, shape, dev["L"], W1, W2, dev["R"], dev["theta"], tau, T.to_device(c),
                           bars["L"], bars["W1"], bars["W2"], bars["R"], bars["theta"], nquad=10,
                           tol=1e-15, m_max=60)
    args = {k: p[k] for k in ("L", "W1", "W2", "R", "theta")}
    for name in args:
        E = _cg(rng, p[name].shape)
        if name != "theta":
            E = _herm(E)
        h = 1e-5
        fd = _fd(f, args, name, E, h)
        fd2 = _fd(f, args, name, E, h / 2)
        fd = (4 * fd2 - fd) / 3  # Richardson: O(h^4)
        got = _rdot(T.from_device(bars[name]), E)
        assert abs(got - fd) <= 1e-7 * max(1.0, abs(fd)), (name, got, fd)


def test_autograd_function(T, ctx):
    """torch.autograd through the hand-written adjoint passes torch's gradcheck
    on a tiny problem; L and R enter through a per-channel Hermitian
    parametrisation, since the exponential is defined for Hermitian H_eff."""
    import torch
    from paper_1908_10588_amd import autograd as A
    shape = (2, 2, 2, 3, 2, 2, 2)
    p = _operands(7, shape, hermitian=True)
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    L = T.to_device(p["L"]).requires_grad_(True)
    R = T.to_device(p["R"]).requires_grad_(True)
    th = T.to_device(p["theta"]).requires_grad_(True)

    def herm(X):  # planar [2, w, D, D] -> (X + X^H)/2 per channel
        re = 0.5 * (X[0] + X[0].transpose(-1, -2))
        im = 0.5 * (X[1] - X[1].transpose(-1, -2))
        return torch.stack([re, im])

    def fn(L, R, th):
        return A.local_expm(ctx, shape, herm(L), W1, W2, herm(R), th, 0.5)

    assert torch.autograd.gradcheck(fn, (L, R, th), eps=1e-6, atol=1e-7, rtol=1e-6)


def _unit_dirs(shape):
    """Every real and imaginary unit direction of a complex array."""
    n = int(np.prod(shape))
    for e in range(n):
        for ph in (1.0, 1j):
            E = np.zeros(n, dtype=complex)
            E[e] = ph
            yield E.reshape(shape)


def _herm_dirs(shape):
    """A basis of the directions Hermitian per channel (last two axes): e_aa,
    e_ab + e_ba and i (e_ab - e_ba) for a < b in every channel."""
    lead, n = shape[:-2], shape[-1]
    for idx in np.ndindex(*lead):
        for a in range(n):
            for b in range(a, n):
                for ph in ((1.0,) if a == b else (1.0, 1j)):
                    E = np.zeros(shape, dtype=complex)
                    E[idx + (a, b)] += ph
                    if a != b:
                        E[idx + (b, a)] += np.conj(ph)
                    yield E


def test_heff2_vjp_elementwise(T, ctx):
    """Every element of every cotangent (L, W_i, W_{i+1}, R, theta) of
    H_eff,2 theta with general operands against the oracle's central
    difference along that element's real and imaginary unit directions
    (f = Re<c, y> is linear in each operand, so the differences are exact up
    to rounding)."""
    import torch
    from oracle import tdvp as ot
    shape = (3, 2, 2, 3, 2, 2, 2)
    p = _operands(21, shape, hermitian=False)
    rng = np.random.default_rng(22)
    c = _cg(rng, p["theta"].shape)

    def f(L, W1, W2, R, theta):
        return _rdot(c, ot.heff2(L, W1, W2, R, theta))

    dev = {k: T.to_device(p[k]) for k in ("L", "R", "theta")}
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    bars = {k: torch.zeros(2, *p[k].shape, dtype=torch.float64, device="cuda")
            for k in ("L", "W1", "W2", "R", "theta")}
    T.tdmrg_heff2_apply_vjp(ctx, shape, dev["L"], W1, W2, dev["R"], dev["theta"], T.to_device(c),
                            bars["L"], bars["W1"], bars["W2"], bars["R"], bars["theta"])
    args = {k: p[k] for k in ("L", "W1", "W2", "R", "theta")}
    for name in args:
        got = T.from_device(bars[name])
        ref = np.zeros(p[name].shape, dtype=complex)
        for E in _unit_dirs(p[name].shape):
            ref += _fd(f, args, name, E, 1e-3) * E  # E is 1 or i at one element
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() <= 1e-11 * scale, (name, np.abs(got - ref).max())


def test_local_expm_vjp_elementwise(T, ctx):
    """The local exponential's cotangents along every basis direction: every
    element of theta, and every Hermitian-per-channel basis direction of L,
    W_i, W_{i+1} and R (the exponential is defined for Hermitian H_eff), each
    against Richardson-extrapolated central differences of the oracle."""
    import torch
    from oracle import tdvp as ot
    shape = (3, 2, 2, 3, 2, 2, 2)
    p = _operands(23, shape, hermitian=True)
    tau = 0.6
    rng = np.random.default_rng(24)
    c = _cg(rng, p["theta"].shape)

    def f(L, W1, W2, R, theta):
        y, _, _ = ot.lanczos_expm(lambda x: ot.heff2(L, W1, W2, R, x), theta, tau, tol=1e-15)
        return _rdot(c, y)

    dev = {k: T.to_device(p[k]) for k in ("L", "R", "theta")}
    W1, W2 = T.Wop(ctx, p["W1"]), T.Wop(ctx, p["W2"])
    bars = {k: torch.zeros(2, *p[k].shape, dtype=torch.float64, device="cuda")
            for k in ("L", "W1", "W2", "R", "theta")}
    T.tdmrg_local_expm_vjp(ctx, shape, dev["L"], W1, W2, dev["R"], dev["theta"], tau, T.to_device(c),
                           bars["L"], bars["W1"], bars["W2"], bars["R"], bars["theta"], nquad=10,
                           tol=1e-15, m_max=60)
    args = {k: p[k] for k in ("L", "W1", "W2", "R", "theta")}
    worst = 0.0
    for name in args:
        got = T.from_device(bars[name])
        dirs = _unit_dirs(p[name].shape) if name == "theta" else _herm_dirs(p[name].shape)
        for E in dirs:
            h = 1e-4
            fd = (4 * _fd(f, args, name, E, h / 2) - _fd(f, args, name, E, h)) / 3
            g = _rdot(got, E)
            worst = max(worst, abs(g - fd) / max(1.0, abs(fd)))
            assert abs(g - fd) <= 1e-7 * max(1.0, abs(fd)), (name, g, fd)
    print("largest relative deviation over all directions", worst, flush=True)
