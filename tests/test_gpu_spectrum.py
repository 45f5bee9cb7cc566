"""GPU spectrum of a sampled autocorrelation (tdmrg_spectrum) against the
oracle's transform: element by element on energies spanning several
workgroups with a ragged tail, on a sample count spanning several LDS
chunks, and on the C(t) of a GPU 2TDVP run."""
import numpy as np
import pytest

import synth
from oracle import HBAR
from oracle import observables as oobs

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


def _gpu(T, ctx, C, dt, E, tau):
    import torch
    Cd = T.to_device(np.asarray(C, dtype=complex))
    Ed = torch.from_numpy(np.asarray(E, dtype=np.float64)).cuda()
    sd = torch.zeros(len(E), dtype=torch.float64, device="cuda")
    T.tdmrg_spectrum(ctx, Cd, dt, Ed, tau, sd)
    return sd.cpu().numpy()


@pytest.mark.parametrize("N,M,tau", [(1300, 700, 30.0), (2, 5, 50.0), (513, 257, 1e300)])
def test_spectrum_parity(T, ctx, N, M, tau):
    rng = np.random.default_rng(N + M)
    C = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    E = np.linspace(-0.5, 1.5, M)
    ref = oobs.absorption_spectrum(C, 0.5, E, tau)
    got = _gpu(T, ctx, C, 0.5, E, tau)
    assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300) + 1e-300


def test_spectrum_of_a_gpu_run(T, ctx):
    """C(t) of 60 GPU 2TDVP steps of config 1, transformed on the device and
    by the oracle; the sum rule over one period of the sampled transform
    (Re C(0) = 1) holds on the device result."""
    model = synth.config1_model(0)
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], model["D_max"])
    psi0 = mps.copy()
    C = [1.0 + 0j]
    for _ in range(60):
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, model["dt_fs"], model["D_max"], model["eps"])
        C.append(T.tdmrg_observables(ctx, mps, mpo, psi0)["C"])
    C = np.array(C)
    dt = model["dt_fs"]
    period = 2 * np.pi * HBAR / dt
    M = 128
    E = -2.0 + period * np.arange(M) / M
    got = _gpu(T, ctx, C, dt, E, 30.0)
    ref = oobs.absorption_spectrum(C, dt, E, 30.0)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    assert abs(got.sum() * period / M - 1.0) < 1e-11
