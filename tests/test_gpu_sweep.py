"""GPU 2TDVP time steps (tdmrg_tdvp2_sweep) and observables against the
oracle, exact propagation and closed forms.  Populations must agree with the
oracle to 1e-10 relative (populations sum to ~1, so absolute = relative)."""
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


def _oracle_run(model, steps, D_max, eps, sv_mode=0, mps=None):
    dims = ham.site_dims(model)
    W = ompo.build_mpo(model)
    st = ot.TDVP2(mps if mps is not None else omps.product_state(dims, model["occ"]), W,
                  sv_mode=sv_mode)
    psi0 = [a.copy() for a in st.mps]
    out = []
    for _ in range(steps):
        stats = st.step(model["dt_fs"], D_max, eps)
        out.append(dict(pops=oobs.populations(model, st.mps), norm2=oobs.norm2(st.mps),
                        energy=oobs.energy(st.mps, W), C=oobs.overlap(psi0, st.mps),
                        bonds=omps.bond_dims(st.mps), k_rl=stats["k_rl"]))
    return st, out


def _gpu_run(T, ctx, model, steps, D_max, eps, D_cap=None, sv_mode=0, sites=None, precision=0):
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], D_cap or D_max)
    if sites is not None:
        for s, A in enumerate(sites):
            mps.set_site(s, A)
    psi0 = mps.copy()
    out = []
    for _ in range(steps):
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, model["dt_fs"], D_max, eps, sv_mode=sv_mode,
                            precision=precision)
        ob = T.tdmrg_observables(ctx, mps, mpo, psi0)
        ob["bonds"] = mps.bond_dims()
        out.append(ob)
    return mps, mpo, out


def test_config1_parity_with_oracle(T, ctx):
    model = synth.config1_model(0)
    print("config1 seed 0, 20 steps", flush=True)
    _, ref = _oracle_run(model, 20, model["D_max"], model["eps"])
    _, _, got = _gpu_run(T, ctx, model, 20, model["D_max"], model["eps"])
    for r, g in zip(ref, got):
        assert g["bonds"] == r["bonds"]
        assert np.abs(g["pops"] - r["pops"]).max() < 1e-10
        assert abs(g["norm2"] - r["norm2"]) < 1e-10
        assert abs(g["energy"] - r["energy"]) < 1e-9
        assert abs(g["C"] - r["C"]) < 1e-10


def test_config1_full_rank_exact(T, ctx):
    """Full-rank MPS, nothing truncated: the GPU sweep reproduces exact
    propagation in the 8192-dimensional product space."""
    model = synth.config1_model(1)
    dims = ham.site_dims(model)
    psi0 = exact.product_vector(model)
    full = omps.from_dense_full_rank(psi0, dims)
    mps, mpo, got = _gpu_run(T, ctx, model, 20, 64, 0.0, D_cap=64, sv_mode=2, sites=full)
    ref = exact.evolve(model, psi0, [20 * model["dt_fs"]])[0]
    v = omps.to_dense(mps.tensors())
    assert np.linalg.norm(v - ref) < 1e-10
    assert np.abs(got[-1]["pops"] - exact.el_populations(model, ref)).max() < 1e-10


def test_displaced_oscillator_closed_form(T, ctx):
    om, ka = np.array([0.12, 0.2, 0.07]), np.array([0.09, -0.14, 0.05])
    model = synth.single_mode_model(om, ka, nbasis=30, E=(0.3, -0.2), state=0)
    _, _, got = _gpu_run(T, ctx, model, 8, 4, 1e-14)
    for k, g in enumerate(got, start=1):
        ref = exact.displaced_autocorrelation(0.5 * k, 0.3, om, ka)
        assert abs(g["C"] - ref) < 1e-12
        assert max(g["bonds"]) == 1


def test_rabi_and_table1(T, ctx):
    model = synth.rabi_model(E0=0.0, E1=0.4, V01=0.05)
    _, _, got = _gpu_run(T, ctx, model, 10, 4, 1e-14)
    for k, g in enumerate(got, start=1):
        assert abs(g["pops"][0] - exact.rabi_population(0.5 * k, 0.0, 0.4, 0.05)) < 1e-12
    model = synth.sf_table1_model()
    H = np.diag(model["E"]) + model["V"]
    _, _, got = _gpu_run(T, ctx, model, 10, 6, 1e-14)
    for k, g in enumerate(got, start=1):
        ref = exact.electronic_populations(H, 0, 0.5 * k)[0]
        assert np.abs(g["pops"] - ref).max() < 1e-12


@pytest.mark.timeout(900)
@pytest.mark.parametrize("cfg", ["config5", "config3B", "config2"])
def test_short_horizon_parity(T, ctx, cfg):
    """First steps from the product state of the larger configurations (the
    oracle needs hours per step once the bonds saturate): 3 steps of config
    5, 4 of config 3 (ordering B, 4 modes per bath), 5 of config 2 (bonds up
    to 23 of 128 after the fifth)."""
    if cfg == "config5":
        model, steps, D = synth.config5_model(0), 3, 64
    elif cfg == "config3B":
        model = synth.config3_model(0, ordering="B", modes_per_bath=4)
        steps, D = 4, 32
    else:
        model, steps, D = synth.config2_model(0), 5, 128
    print(cfg, "steps", steps, "D", D, flush=True)
    _, ref = _oracle_run(model, steps, D, model["eps"])
    _, _, got = _gpu_run(T, ctx, model, steps, D, model["eps"])
    for r, g in zip(ref, got):
        assert g["bonds"] == r["bonds"]
        assert np.abs(g["pops"] - r["pops"]).max() < 1e-10
        assert abs(g["C"] - r["C"]) < 1e-10


def test_fp32_contractions_error_stated(T, ctx):
    """Mixed form: FP32 contractions, FP64 Lanczos/SVD; the population error
    against the FP64 oracle stays below 1e-5 on config 1."""
    model = synth.config1_model(0)
    _, ref = _oracle_run(model, 20, model["D_max"], model["eps"])
    _, _, got = _gpu_run(T, ctx, model, 20, model["D_max"], model["eps"], precision=1)
    err = max(np.abs(g["pops"] - r["pops"]).max() for g, r in zip(got, ref))
    print("FP32 population error", err, flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("form", ["bf16x3", "bf16x6"])
def test_bf16_split_error_stated(T, ctx, form):
    """Mixed form with BF16-split contractions (FP64 Lanczos, tridiagonal
    exponential and SVD): the population error against the FP64 oracle over
    20 steps of config 1, stated; both stay within the 1e-5 bar of the mixed
    forms (measured 2.4e-6 with two pieces, 1.1e-7 with three)."""
    model = synth.config1_model(0)
    prec = T.BF16X3 if form == "bf16x3" else T.BF16X6
    _, ref = _oracle_run(model, 20, model["D_max"], model["eps"])
    _, _, got = _gpu_run(T, ctx, model, 20, model["D_max"], model["eps"], precision=prec)
    err = max(np.abs(g["pops"] - r["pops"]).max() for g, r in zip(got, ref))
    print(form, "population error", err, flush=True)
    assert err < 1e-5


@pytest.mark.timeout(900)
@pytest.mark.parametrize("ordering,steps", [("A", 20), ("B", 36)])
def test_config3_full_model_parity(T, ctx, ordering, steps):
    """The whole config-3 model (3 states, three Debye baths of 40 modes,
    boson basis 6: 121 sites) from its product state at dt 0.25 fs, D_max 256,
    eps 1e-8: 5 fs (ordering A) and 9 fs (ordering B), while the oracle can
    still follow (bonds up to about 9); FP64 against the oracle step by step,
    and the FP32 contractions the configuration runs with against both."""
    model = synth.config3_model(0, ordering=ordering)
    D = 256
    print("config 3", ordering, "steps", steps, flush=True)
    _, ref = _oracle_run(model, steps, D, model["eps"])
    _, _, got = _gpu_run(T, ctx, model, steps, D, model["eps"])
    _, _, got32 = _gpu_run(T, ctx, model, steps, D, model["eps"], precision=T.FP32)
    err32 = 0.0
    for r, g, g32 in zip(ref, got, got32):
        assert g["bonds"] == r["bonds"]
        assert np.abs(g["pops"] - r["pops"]).max() < 1e-10
        assert abs(g["C"] - r["C"]) < 1e-10
        err32 = max(err32, float(np.abs(g32["pops"] - r["pops"]).max()))
    print("max bond", max(ref[-1]["bonds"]), "FP32 population error", err32, flush=True)
    assert err32 < 1e-5
