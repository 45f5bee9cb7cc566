"""GPU 2TDVP with one chain site per electronic state (the representation of
the paper's ordering study) against the oracle and exact propagation.
Populations must agree with the oracle to 1e-10."""
import numpy as np
import pytest

import synth
from oracle import exact
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


def _small(seed, nbasis, order):
    m = synth.config1_model(seed)
    m["nbasis"] = np.array(nbasis)
    return synth.per_state_model(m, order=order)


@pytest.mark.parametrize("order", [None, [0, -1, 1, -2, 2, 3]])
def test_per_state_sweep_parity_with_oracle(T, ctx, order):
    model = _small(0, (5, 4, 5, 4), order)
    D, eps = 10, 1e-10
    print("per-state sweep, order", model["order"], flush=True)
    W = ompo.build_mpo(model)
    ref = ot.TDVP2(omps.product_state(ham.site_dims(model), model["occ"]), W)
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], D)
    psi0 = mps.copy()
    for _ in range(8):
        ref.step(model["dt_fs"], D, eps)
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, model["dt_fs"], D, eps)
        ob = T.tdmrg_observables(ctx, mps, mpo, psi0)
        assert mps.bond_dims() == omps.bond_dims(ref.mps)
        assert np.abs(ob["pops"] - oobs.populations(model, ref.mps)).max() < 1e-10
        assert abs(ob["energy"] - oobs.energy(ref.mps, W)) < 1e-9
        assert abs(ob["pops"].sum() - ob["norm2"]) < 1e-12


def test_per_state_full_rank_exact(T, ctx):
    model = _small(1, (3, 3, 3, 3), [0, -1, 1, -2, 2, 3])
    psi0 = exact.product_vector(model)
    full = omps.from_dense_full_rank(psi0, ham.site_dims(model))
    cap = max(omps.bond_dims(full))
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], cap)
    for s, A in enumerate(full):
        mps.set_site(s, A)
    for _ in range(5):
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, model["dt_fs"], cap, 0.0, sv_mode=2)
    ref = exact.evolve(model, psi0, [5 * model["dt_fs"]])[0]
    assert np.linalg.norm(omps.to_dense(mps.tensors()) - ref) < 1e-10
    pops = T.tdmrg_observables(ctx, mps, mpo)["pops"]
    assert np.abs(pops - exact.el_populations(model, ref)).max() < 1e-10


@pytest.mark.parametrize("order", ["default", "optimized", "worst"])
def test_ordering_study_model_short_parity(T, ctx, order):
    """The 4-mode ordering-study model (boson bases 25, 19, 11, 19) from a
    superposition of the two electronic states: the first steps against the
    oracle, in three chain orders."""
    model = synth.lvc4_per_state_model(0, order)
    psi = synth.superposed_excitation_state(model, (np.sin(0.3), np.cos(0.3)))
    D, eps = 48, 1e-8
    print("lvc4", order, flush=True)
    W = ompo.build_mpo(model)
    ref = ot.TDVP2(psi, W)
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], D)
    for s, A in enumerate(psi):
        mps.set_site(s, A)
    for _ in range(4):
        ref.step(model["dt_fs"], D, eps)
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, model["dt_fs"], D, eps)
    assert mps.bond_dims() == omps.bond_dims(ref.mps)
    ob = T.tdmrg_observables(ctx, mps, mpo)
    assert np.abs(ob["pops"] - oobs.populations(model, ref.mps)).max() < 1e-10
    assert abs(ob["energy"] - oobs.energy(ref.mps, W)) < 1e-9
