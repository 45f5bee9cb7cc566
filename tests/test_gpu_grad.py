"""GPU gradient of an electronic population after a 2TDVP evolution with
respect to every coupling constant (reverse mode through the whole
evolution), against central differences of the CPU oracle's evolution at
the same (frozen) truncation ranks."""
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


def small_model(seed=3, n_modes=3, nbasis=4):
    """The first modes of a config-5 draw (linear, quadratic and bilinear
    couplings, V = 0) on a small basis, electronic site second."""
    m = synth.config5_model(seed)
    mm = dict(n_el=m["n_el"], E=m["E"].copy(), V=np.array([[0.0, 0.03], [0.03, 0.0]]),
              omega=m["omega"][:n_modes].copy(), nbasis=np.full(n_modes, nbasis, dtype=np.int64),
              g1=m["g1"][:n_modes].copy())
    sel = [k for k in range(len(m["g2_val"])) if m["g2_I"][k] < n_modes and m["g2_J"][k] < n_modes]
    for key in ("g2_I", "g2_J", "g2_i", "g2_j", "g2_val"):
        mm[key] = np.asarray(m[key])[sel].copy()
    mm["order"] = [1, -1] + [0] + list(range(2, n_modes))
    return synth.vibronic._finish(mm, 1, dt_fs=0.5, D_max=4, eps=1e-12, steps=3)


def oracle_pop(model, steps, D_max, eps, state, ranks=None):
    from oracle import hamiltonian as ham
    from oracle import mpo as ompo
    from oracle import mps as omps
    from oracle import observables as oobs
    from oracle import tdvp as ot
    st = ot.TDVP2(omps.product_state(ham.site_dims(model), model["occ"]), ompo.build_mpo(model),
                  krylov_tol=1e-15)
    rk = []
    for t in range(steps):
        s = st.step(model["dt_fs"], D_max, eps, None if ranks is None else ranks[t])
        rk.append((list(s["k_lr"]), list(s["k_rl"])[::-1]))
    return oobs.populations(model, st.mps)[state], rk


def params(model):
    """(name, index, setter) of every coupling constant, in the library's convention."""
    ne, nm = model["n_el"], len(model["omega"])
    out = [("E", (i,)) for i in range(ne)]
    out += [("V", (i, j)) for i in range(ne) for j in range(i + 1, ne)]
    out += [("omega", (I,)) for I in range(nm)]
    out += [("g1", (I, i, j)) for I in range(nm) for i in range(ne) for j in range(i, ne)]
    out += [("g2", (k,)) for k in range(len(model["g2_val"]))]
    return out


def bumped(model, name, idx, h):
    m = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in model.items()}
    key = "g2_val" if name == "g2" else name
    m[key] = np.array(m[key], dtype=float, copy=True)
    m[key][idx] += h
    if name in ("V", "g1") and idx[-1] != idx[-2]:  # symmetric pair: one constant
        sw = idx[:-2] + (idx[-1], idx[-2])
        m[key][sw] += h
    return m


@pytest.mark.parametrize("D_max,svd", [(4, "auto"), (16, "auto"), (4, "gram")])
def test_population_gradient_against_oracle_fd(T, ctx, D_max, svd):
    """D_max 4 truncates the middle bond (8 -> 4), so the adjoint of the
    truncation matters; D_max 16 is full rank.  svd "gram" forces the Gram +
    eigensolver route everywhere, including the full SVD inside the
    truncation adjoint (taken there automatically beyond small sizes)."""
    model = small_model()
    steps, eps, state = 3, 1e-12, 0
    print("gradient", D_max, svd, flush=True)
    ctx.set_svd_method(svd)
    try:
        g = T.tdmrg_tdvp2_population_grad(ctx, model, model["occ"], D_max, steps, model["dt_fs"], D_max, eps,
                                          state, nquad=10, krylov_tol=1e-15, krylov_max=60)
    finally:
        ctx.set_svd_method("auto")
    p0, rk = oracle_pop(model, steps, D_max, eps, state)
    # the Gram route's singular values carry an absolute error of eps s_0^2
    assert abs(g["pop"] - p0) < (1e-12 if svd == "auto" else 1e-10)
    for t in range(steps):
        assert list(g["ranks"][t, 0]) == rk[t][0] and list(g["ranks"][t, 1]) == rk[t][1], (t, g["ranks"][t], rk[t])
    if D_max == 4:
        assert min(min(a) for a, _ in rk) < 8 or max(max(a) for a, _ in rk) == 4  # truncation active
    h = 1e-5
    worst = 0.0
    for name, idx in params(model):
        fp, _ = oracle_pop(bumped(model, name, idx, h), steps, D_max, eps, state, rk)
        fm, _ = oracle_pop(bumped(model, name, idx, -h), steps, D_max, eps, state, rk)
        fd = (fp - fm) / (2 * h)
        got = g[name][idx]
        worst = max(worst, abs(got - fd) / max(1.0, abs(fd)))
        assert abs(got - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx, got, fd)
    print("max relative deviation from the oracle differences", worst, flush=True)


def two_site_model():
    """Electronic site + one mode (d = 5) with every kind of coupling: on two
    sites a 2TDVP step is one exponential of the whole H per half-sweep, so
    the evolution (and its gradient) is exact."""
    mm = dict(n_el=2, E=np.array([-0.3, 0.25]), V=np.array([[0.0, 0.04], [0.04, 0.0]]),
              omega=np.array([0.12]), nbasis=np.array([5], dtype=np.int64),
              g1=np.array([[[0.08, 0.03], [0.03, -0.05]]]),
              g2_I=np.array([0, 0]), g2_J=np.array([0, 0]), g2_i=np.array([0, 0]), g2_j=np.array([0, 1]),
              g2_val=np.array([0.01, 0.006]), order=[-1, 0])
    return synth.vibronic._finish(mm, 1, dt_fs=0.5, D_max=8, eps=0.0, steps=4)


def test_gradient_equals_exact_dynamics_gradient(T, ctx):
    """Two sites, no truncation: dP/dc = 2 Re <psi(T)| Pi |dpsi(T)> with dpsi
    the Frechet derivative of exp(-i H T / hbar) along -i (dH/dc) T / hbar
    (scipy.linalg.expm_frechet on the dense H; H is affine in every c)."""
    import scipy.linalg
    from oracle import HBAR
    from oracle import exact as oex
    from oracle import hamiltonian as ham
    model = two_site_model()
    steps, state = model["steps"], 0
    Tt = steps * model["dt_fs"]
    # eps 1e-14 drops only rounding-level singular values (none here: both
    # values of the el-mode cut are of order 0.1)
    g = T.tdmrg_tdvp2_population_grad(ctx, model, model["occ"], 8, steps, model["dt_fs"], 8, 1e-14, state,
                                      nquad=12, krylov_tol=1e-15, krylov_max=60)
    assert g["ranks"].min() == 2
    H0 = ham.dense_hamiltonian(model).toarray()
    psi0 = oex.product_vector(model)
    dims = ham.site_dims(model)
    el = list(model["order"]).index(-1)
    proj = np.zeros(dims)
    idx = [slice(None)] * len(dims)
    idx[el] = state
    proj[tuple(idx)] = 1.0
    proj = proj.reshape(-1)
    A = -1j * (Tt / HBAR) * H0
    U = scipy.linalg.expm(A)
    psi = U @ psi0
    assert abs(g["pop"] - np.sum(proj * np.abs(psi) ** 2)) < 1e-12
    worst = 0.0
    for name, idx_ in params(model):
        dH = ham.dense_hamiltonian(bumped(model, name, idx_, 1.0)).toarray() - H0
        _, L = scipy.linalg.expm_frechet(A, -1j * (Tt / HBAR) * dH)
        dpsi = L @ psi0
        ref = 2.0 * np.real(np.vdot(psi, proj * dpsi))
        got = g[name][idx_]
        worst = max(worst, abs(got - ref) / max(1e-3, abs(ref)))
        assert abs(got - ref) <= 1e-9 * max(1e-3, abs(ref)), (name, idx_, got, ref)
    print("max relative deviation from the exact gradient", worst, flush=True)


def test_rabi_gradient_closed_form(T, ctx):
    """Two levels coupled by V, one uncoupled mode: P_0(t) = 4V^2/W^2
    sin^2(W t / 2 hbar), W^2 = dE^2 + 4V^2, dE = E1 - E0, so dP/dV, dP/dE1 =
    -dP/dE0 are closed forms; the mode and the (zero) couplings do not move
    P_0 to first order (parity), and neither does omega."""
    from oracle import HBAR
    model = synth.rabi_model()
    steps, state = model["steps"], 0
    t = steps * model["dt_fs"]
    # the state stays a product (rank 1); eps 1e-14 drops the rounding-level
    # second singular value, which the truncation adjoint would divide by
    g = T.tdmrg_tdvp2_population_grad(ctx, model, model["occ"], 4, steps, model["dt_fs"], 4, 1e-14, state,
                                      nquad=12, krylov_tol=1e-15, krylov_max=60)
    assert g["ranks"].max() == 1
    E0, E1, V = model["E"][0], model["E"][1], model["V"][0, 1]
    dE = E1 - E0
    W = np.sqrt(dE * dE + 4 * V * V)
    x = W * t / (2 * HBAR)
    P = 4 * V * V / W ** 2 * np.sin(x) ** 2
    dP_dV = 8 * V * dE * dE / W ** 4 * np.sin(x) ** 2 + 4 * V * V / W ** 2 * np.sin(2 * x) * (t / (2 * HBAR)) * (4 * V / W)
    dP_ddE = -8 * V * V * dE / W ** 4 * np.sin(x) ** 2 + 4 * V * V / W ** 2 * np.sin(2 * x) * (t / (2 * HBAR)) * (dE / W)
    assert abs(g["pop"] - P) < 1e-12
    print("rabi gradient", g["V"][0, 1], dP_dV, g["E"], dP_ddE, flush=True)
    assert abs(g["V"][0, 1] - dP_dV) <= 1e-9 * abs(dP_dV)
    assert abs(g["E"][1] - dP_ddE) <= 1e-9 * abs(dP_ddE)
    assert abs(g["E"][0] + dP_ddE) <= 1e-9 * abs(dP_ddE)
    assert abs(g["omega"][0]) < 1e-12 and np.abs(g["g1"]).max() < 1e-12


def test_population_autograd_function(T, ctx):
    """The population gradient behind torch.autograd.Function: backward of
    P_2(T) gives the library's gradient of every coupling constant, and a
    central difference of the function itself in one inter-state constant
    agrees with it."""
    import torch

    from paper_1908_10588_amd import autograd as A
    model = small_model()
    steps, D, eps = 3, 4, 1e-12
    ts = {k: torch.tensor(np.asarray(model[k], dtype=np.float64), requires_grad=True)
          for k in ("E", "V", "omega", "g1", "g2_val")}
    P = A.population(ctx, model, ts["E"], ts["V"], ts["omega"], ts["g1"], ts["g2_val"], steps,
                     model["dt_fs"], D, eps, state=1)
    P.backward()
    ref = T.tdmrg_tdvp2_population_grad(ctx, model, model["occ"], D, steps, model["dt_fs"], D, eps, 1)
    assert abs(P.item() - ref["pop"]) < 1e-14
    for k, r in (("E", "E"), ("V", "V"), ("omega", "omega"), ("g1", "g1"), ("g2_val", "g2")):
        assert np.abs(ts[k].grad.numpy() - np.asarray(ref[r]).reshape(ts[k].shape)).max() < 1e-14, k
    h = 1e-5
    vals = []
    for sgn in (1, -1):
        m2 = dict(model)
        m2["g1"] = np.array(model["g1"], dtype=np.float64).copy()
        m2["g1"][0, 0, 1] += sgn * h  # the pair constant lambda of mode 0, both entries
        m2["g1"][0, 1, 0] += sgn * h
        vals.append(T.tdmrg_tdvp2_population_grad(ctx, m2, model["occ"], D, steps, model["dt_fs"], D, eps,
                                                  1)["pop"])
    fd = (vals[0] - vals[1]) / (2 * h)
    print("dP2/dlambda_0: autograd", ts["g1"].grad[0, 0, 1].item(), "central difference", fd, flush=True)
    assert abs(ts["g1"].grad[0, 0, 1].item() - fd) < 1e-6 * max(1.0, abs(fd))


@pytest.mark.timeout(900)
def test_population_gradient_full_config5_spot_check(T, ctx):
    """The whole config-5 model (2 states, 12 modes at d = 10, linear,
    quadratic and bilinear couplings; 13 sites) over 3 steps of 0.5 fs at its
    own D_max 64 and eps 1e-10: the GPU gradient of P_0 against central
    differences of the oracle's evolution at the GPU's truncation ranks, for
    three coupling constants (an electronic energy, the largest linear and the
    largest second-order coupling)."""
    model = synth.config5_model(0)
    steps, D_max, eps, state = 3, 64, 1e-10, 0
    g = T.tdmrg_tdvp2_population_grad(ctx, model, model["occ"], D_max, steps, model["dt_fs"], D_max, eps,
                                      state, nquad=12, krylov_tol=1e-15, krylov_max=60)
    p0, rk = oracle_pop(model, steps, D_max, eps, state)
    print("config 5: P_0", g["pop"], p0, "max bond", int(g["ranks"].max()), flush=True)
    assert abs(g["pop"] - p0) < 1e-10
    for t in range(steps):
        assert list(g["ranks"][t, 0]) == rk[t][0] and list(g["ranks"][t, 1]) == rk[t][1], (t, g["ranks"][t], rk[t])
    g1 = np.asarray(model["g1"])
    i1 = np.unravel_index(np.argmax(np.abs(g1)), g1.shape)
    k2 = int(np.argmax(np.abs(np.asarray(model["g2_val"]))))
    h = 1e-5
    for name, idx in (("E", (1,)), ("g1", tuple(int(x) for x in i1)), ("g2", (k2,))):
        fp, _ = oracle_pop(bumped(model, name, idx, h), steps, D_max, eps, state, rk)
        fm, _ = oracle_pop(bumped(model, name, idx, -h), steps, D_max, eps, state, rk)
        fd = (fp - fm) / (2 * h)
        got = g[name][idx]
        print("d P_0 / d", name, idx, "GPU", got, "oracle differences", fd, flush=True)
        assert abs(got - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx, got, fd)
