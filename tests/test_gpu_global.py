"""GPU global integrators (tdmrg_global_step: global Krylov, RK4 and Taylor
on the whole MPS) against the oracle's, exact propagation and the Taylor
polynomial; and the paper's use of global steps to grow the bonds before
two-site steps."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import HBAR, exact
from oracle import globalprop as gp
from oracle import hamiltonian as ham
from oracle import mpo as ompo
from oracle import mps as omps
from oracle import observables as oobs
from oracle import tdvp as ot

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


def _grown(seed=0, nbasis=(3, 3, 3, 3)):
    model = synth.config1_model(seed)
    model["nbasis"] = np.array(nbasis)
    W = ompo.build_mpo(model)
    st = ot.TDVP2(omps.product_state(ham.site_dims(model), model["occ"]), W)
    for _ in range(2):
        st.step(1.0, 6, 1e-12)
    return model, W, st.mps


def _load(T, ctx, model, sites, cap):
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], cap)
    for s, A in enumerate(sites):
        mps.set_site(s, A)
    return mps, mpo


@pytest.mark.parametrize("method", ["krylov", "rk4"])
def test_global_step_parity(T, ctx, method):
    model, W, psi = _grown()
    print("global step", method, "bonds", omps.bond_dims(psi), flush=True)
    mps, mpo = _load(T, ctx, model, psi, 64)
    dt = 0.6
    st = T.tdmrg_global_step(ctx, mps, mpo, dt, 64, 1e-15, method=method, m_max=24, tol=1e-12)
    got = omps.to_dense(mps.tensors())
    if method == "krylov":
        ref = omps.to_dense(gp.global_krylov_step(psi, W, dt, 64, 1e-15, m_max=24, tol=1e-12)[0])
        H = ham.dense_hamiltonian(model).toarray()
        exact_v = scipy.linalg.expm(-1j * dt / HBAR * H) @ omps.to_dense(psi)
        assert np.linalg.norm(got - exact_v) < 1e-9
    else:
        ref = omps.to_dense(gp.rk4_step(psi, W, dt, 64, 1e-15))
        assert st.vectors == 4
    assert np.linalg.norm(got - ref) < 1e-9
    assert st.max_intermediate_bond >= max(omps.bond_dims(psi))
    for A in mps.tensors()[1:]:
        assert omps.right_orth_error(A) < 1e-10


@pytest.mark.parametrize("order", [2, 8])
def test_global_taylor_parity(T, ctx, order):
    """Taylor of order p against the oracle's; at order 2 (the paper's) the
    norm grows by tau^4 |H^2 psi|^2 / 4, as the closed form says."""
    model, W, psi = _grown()
    print("global taylor order", order, "bonds", omps.bond_dims(psi), flush=True)
    mps, mpo = _load(T, ctx, model, psi, 64)
    dt = 0.6
    st = T.tdmrg_global_step(ctx, mps, mpo, dt, 64, 1e-15, method="taylor", m_max=order)
    got = omps.to_dense(mps.tensors())
    ref = omps.to_dense(gp.taylor_step(psi, W, dt, 64, 1e-15, order=order))
    assert np.linalg.norm(got - ref) < 1e-9
    assert st.vectors == order
    if order == 2:
        H = ham.dense_hamiltonian(model).toarray()
        v = omps.to_dense(psi)
        tau = dt / HBAR
        want = np.vdot(v, v).real + tau ** 4 * np.linalg.norm(H @ (H @ v)) ** 2 / 4
        assert abs(np.vdot(got, got).real - want) < 1e-10 * want
    for A in mps.tensors()[1:]:
        assert omps.right_orth_error(A) < 1e-10


def test_global_steps_grow_bonds_then_two_site_steps(T, ctx):
    """From |S2> x |0> in the per-state chain with the states first, two-site
    steps alone cannot start the inter-state coupling; three global Krylov
    steps grow the bonds, two-site steps continue, and the populations follow
    the oracle running the same protocol."""
    model = synth.lvc4_per_state_model(0, "default")
    model["nbasis"] = np.array([6, 5, 4, 5])
    W = ompo.build_mpo(model)
    psi = omps.product_state(ham.site_dims(model), model["occ"])
    dt, D, eps = model["dt_fs"], 32, 1e-10
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], D)
    for _ in range(3):
        psi, _ = gp.global_krylov_step(psi, W, dt, D, eps, m_max=16, tol=1e-10)
        T.tdmrg_global_step(ctx, mps, mpo, dt, D, eps, method="krylov", m_max=16, tol=1e-10)
    assert max(mps.bond_dims()) > 1
    ref = ot.TDVP2(psi, W)
    for _ in range(4):
        ref.step(dt, D, eps)
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, dt, D, eps)
    pops = T.tdmrg_observables(ctx, mps, mpo)["pops"]
    assert np.abs(pops - oobs.populations(model, ref.mps)).max() < 1e-8
    ex = exact.el_populations(model, exact.evolve(model, exact.product_vector(model), [7 * dt])[0])
    assert np.abs(pops - ex).max() < 1e-4
    assert pops[0] > 1e-4  # population transfer happened


def test_global_step_refuses_wide_intermediates(T, ctx):
    """An MPO x MPS product whose bonds would exceed the validated maximum
    (192) is refused with EUNSUPPORTED before anything is changed: a
    full-rank state of config 1 (bonds 2/16/64/8) times MPO bonds of 5."""
    model = synth.config1_model(0)
    dims = ham.site_dims(model)
    rng = np.random.default_rng(3)
    v = rng.normal(size=int(np.prod(dims))) + 1j * rng.normal(size=int(np.prod(dims)))
    psi = omps.from_dense_full_rank(v / np.linalg.norm(v), dims)
    print("wide-intermediate refusal, bonds", omps.bond_dims(psi), flush=True)
    assert max(omps.bond_dims(psi)) * 5 > 192
    mps, mpo = _load(T, ctx, model, psi, 64)
    before = omps.to_dense(mps.tensors())
    for method in ("krylov", "rk4", "taylor"):
        with pytest.raises(T.TdmrgError) as ei:
            T.tdmrg_global_step(ctx, mps, mpo, 0.5, 64, 1e-10, method=method, m_max=4, tol=1e-10)
        assert ei.value.status == 6, ei.value
        assert np.array_equal(omps.to_dense(mps.tensors()), before)


@pytest.mark.skip(reason="three global Krylov steps on the 4-mode per-state model at full size (boson bases "
                         "25/19/11/19, D_max 256) ended in an illegal memory access on the GPU; the cause is not "
                         "known, so intermediates above bond 192 are refused and this case stays off the GPU")
def test_global_steps_full_size_ordering_model(T, ctx):
    model = synth.lvc4_per_state_model(0, "default")
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], 256)
    for _ in range(3):
        T.tdmrg_global_step(ctx, mps, mpo, model["dt_fs"], 256, 1e-8, method="krylov", m_max=16, tol=1e-10)
    assert max(mps.bond_dims()) > 1


def _full_rank_config1(seed=3, nbasis=None):
    model = synth.config1_model(0)
    if nbasis is not None:
        model["nbasis"] = np.array(nbasis)
    dims = ham.site_dims(model)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=int(np.prod(dims))) + 1j * rng.normal(size=int(np.prod(dims)))
    return model, omps.from_dense_full_rank(v / np.linalg.norm(v), dims)


def test_variational_apply_lifts_the_size_limit(T, ctx):
    """The variational procedure (eq. variational app) never forms the D*w
    products or the summed bonds: the global Krylov step on the full-rank
    config-1 state (bonds 2/16/64/8), which the direct route refuses, runs
    and equals exact propagation and the oracle's variational step."""
    model, psi = _full_rank_config1()
    W = ompo.build_mpo(model)
    mps, mpo = _load(T, ctx, model, psi, 64)
    ctx.set_mpo_apply(1)
    try:
        dt = 0.3
        print("variational global Krylov on bonds", omps.bond_dims(psi), flush=True)
        st = T.tdmrg_global_step(ctx, mps, mpo, dt, 64, 0.0, method="krylov", m_max=24, tol=1e-12)
    finally:
        ctx.set_mpo_apply(0)
    got = omps.to_dense(mps.tensors())
    H = ham.dense_hamiltonian(model).toarray()
    exact_v = scipy.linalg.expm(-1j * dt / HBAR * H) @ omps.to_dense(psi)
    assert np.linalg.norm(got - exact_v) < 1e-9
    ref, _ = gp.global_krylov_step(psi, W, dt, 64, 0.0, m_max=24, tol=1e-12, apply="variational")
    assert np.linalg.norm(got - omps.to_dense(ref)) < 1e-9
    assert st.max_intermediate_bond <= 64


@pytest.mark.parametrize("method", ["krylov", "rk4", "taylor"])
def test_variational_global_steps_truncated_parity(T, ctx, method):
    """With bonds capped below full rank (D_max 5), the GPU's variational
    steps (every product and every sum fitted) follow the oracle's with the
    same bonds, to the bar of the other global steps (measured 1e-14 to
    6e-12)."""
    model, W, psi = _grown()
    mps, mpo = _load(T, ctx, model, psi, 64)
    dt, D = 0.6, 5
    ctx.set_mpo_apply(1)
    try:
        kw = dict(m_max=2) if method == "taylor" else dict(m_max=24, tol=1e-12)
        T.tdmrg_global_step(ctx, mps, mpo, dt, D, 1e-14, method=method, **kw)
    finally:
        ctx.set_mpo_apply(0)
    got = omps.to_dense(mps.tensors())
    if method == "krylov":
        ref = gp.global_krylov_step(psi, W, dt, D, 1e-14, m_max=24, tol=1e-12, apply="variational")[0]
    elif method == "rk4":
        ref = gp.rk4_step(psi, W, dt, D, 1e-14, apply="variational")
    else:
        ref = gp.taylor_step(psi, W, dt, D, 1e-14, order=2, apply="variational")
    print(method, "variational D 5: GPU-oracle distance", np.linalg.norm(got - omps.to_dense(ref)), flush=True)
    assert mps.bond_dims() == omps.bond_dims(ref)
    assert np.linalg.norm(got - omps.to_dense(ref)) < 1e-9
