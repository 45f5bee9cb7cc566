"""Caller-owned workspace arena (tdmrg_ctx_create with an arena, sized by
tdmrg_workspace_query), through the C ABI: sweeps and observables on a
context whose workspace is carved from a torch.empty buffer give the results
of a context that allocates its own; an arena that is too small makes the
sweep return ENOMEM before it changes the state."""
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


def _run(T, ctx, model, steps, D, dt=None):
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], D)
    pops = []
    for _ in range(steps):
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, dt or model["dt_fs"], D, model["eps"])
        pops.append(T.tdmrg_observables(ctx, mps, mpo)["pops"].copy())
    return np.array(pops), mps.bond_dims()


@pytest.mark.parametrize("cfg", ["config1", "config2"])
def test_arena_sweeps_match_own_workspace(T, cfg):
    import torch
    if cfg == "config1":
        model, steps, D, dt = synth.config1_model(0), 10, 16, None
    else:
        model, steps, D, dt = synth.config2_model(0), 3, 64, 2.0
    need = T.tdmrg_workspace_query(model, D, 40)
    print(cfg, "arena bytes", need, flush=True)
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    ca = T.Ctx(0, arena=arena)
    got, bonds_a = _run(T, ca, model, steps, D, dt)
    cb = T.Ctx(0)
    ref, bonds_b = _run(T, cb, model, steps, D, dt)
    print(cfg, "max population difference", np.abs(got - ref).max(), "bonds", bonds_a, flush=True)
    assert bonds_a == bonds_b
    assert np.abs(got - ref).max() < 1e-13
    ca.close()
    cb.close()


def test_arena_too_small_is_enomem(T):
    import torch
    model = synth.config1_model(0)
    D = 16
    need = T.tdmrg_workspace_query(model, D, 40)
    arena = torch.empty(need // 8, dtype=torch.uint8, device="cuda")
    ctx = T.Ctx(0, arena=arena)
    mpo = T.MPO(ctx, model)
    mps = T.MPS(ctx, mpo, model["occ"], D)
    before = [A.copy() for A in mps.tensors()]
    with pytest.raises(T.TdmrgError) as ei:
        T.tdmrg_tdvp2_sweep(ctx, mps, mpo, model["dt_fs"], D, model["eps"])
    assert ei.value.status == 2, ei.value  # ENOMEM
    assert mps.bond_dims() == [1] * (len(before) + 1)
    for a, b in zip(mps.tensors(), before):
        assert np.array_equal(a, b)
    ctx.close()


def test_arena_rejects_host_memory(T):
    import ctypes
    buf = (ctypes.c_char * 4096)()
    h = ctypes.c_void_p()
    st = T.lib().tdmrg_ctx_create(0, None, ctypes.cast(buf, ctypes.c_void_p), 4096, ctypes.byref(h))
    assert st == 1  # EINVAL: not device memory
