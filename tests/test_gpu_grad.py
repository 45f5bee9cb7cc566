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
    assert abs(g["pop"] - p0) < 1e-12
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
