"""GPU parity of the batched/persistent form: many uneven two-site problems
in grouped launches, against the oracle problem by problem."""
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


def _problems(T, ctx, seed, n, scale):
    shapes = synth.heff_batch_shapes(seed, n=n, Dlo=3, Dhi=40, dlo=2, dhi=7, wlo=1, whi=6, scale=scale)
    probs = []
    for k, s in enumerate(shapes):
        p = synth.heff_problem(seed * 1000 + k, *s, w_density=0.6 if k % 2 else 1.0)
        dev = dict(L=T.to_device(p["L"]), R=T.to_device(p["R"]), th=T.to_device(p["theta"]),
                   W1=T.Wop(ctx, p["W1"]), W2=T.Wop(ctx, p["W2"]))
        probs.append((s, p, dev))
    return probs


@pytest.mark.parametrize("gemm_mode", [0, 1, 2])
def test_heff2_batched_parity(T, ctx, gemm_mode):
    """Channel stages as the sparse pass (0), by the cost model (1, a mix of
    both within one batch) or as dense GEMMs (2)."""
    import torch
    from oracle import tdvp as ot
    probs = _problems(T, ctx, 7, 13, 1.0)
    ys = [torch.empty_like(d["th"]) for _, _, d in probs]
    print("batched heff2 shapes", [s for s, _, _ in probs], "channel GEMM mode", gemm_mode, flush=True)
    ctx.set_channel_gemm(gemm_mode)
    try:
        T.tdmrg_heff2_apply_batched(ctx, [s for s, _, _ in probs], [d["L"] for _, _, d in probs],
                                    [d["W1"] for _, _, d in probs], [d["W2"] for _, _, d in probs],
                                    [d["R"] for _, _, d in probs], [d["th"] for _, _, d in probs], ys)
    finally:
        ctx.set_channel_gemm(1)
    for (s, p, d), y in zip(probs, ys):
        ref = ot.heff2(p["L"], p["W1"], p["W2"], p["R"], p["theta"])
        got = T.from_device(y)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), s


@pytest.mark.parametrize("gemm_mode", [0, 2])
def test_heff2_batched_fp32_parity(T, ctx, gemm_mode):
    """The grouped product with FP32 contractions (FP32 MFMA products with
    FP32 intermediates, FP64 operands and output) against the oracle, with
    sparse (0) and dense (2) channel stages."""
    import torch
    from oracle import tdvp as ot
    probs = _problems(T, ctx, 5, 11, 1.0)
    ys = [torch.empty_like(d["th"]) for _, _, d in probs]
    ctx.set_channel_gemm(gemm_mode)
    try:
        T.tdmrg_heff2_apply_batched(ctx, [s for s, _, _ in probs], [d["L"] for _, _, d in probs],
                                    [d["W1"] for _, _, d in probs], [d["W2"] for _, _, d in probs],
                                    [d["R"] for _, _, d in probs], [d["th"] for _, _, d in probs], ys,
                                    precision=T.FP32)
    finally:
        ctx.set_channel_gemm(1)
    worst = 0.0
    for (s, p, d), y in zip(probs, ys):
        ref = ot.heff2(p["L"], p["W1"], p["W2"], p["R"], p["theta"])
        err = np.abs(T.from_device(y) - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err < 2e-5, (s, err)
    print("FP32 grouped product, worst relative error", worst, flush=True)


def test_heff2_batched_waves_match_single_launches(T, ctx):
    """A tiny batch budget forces one problem per wave; results must not change."""
    import torch
    probs = _problems(T, ctx, 9, 6, 1.0)
    args = ([s for s, _, _ in probs], [d["L"] for _, _, d in probs], [d["W1"] for _, _, d in probs],
            [d["W2"] for _, _, d in probs], [d["R"] for _, _, d in probs],
            [d["th"] for _, _, d in probs])
    y1 = [torch.empty_like(d["th"]) for _, _, d in probs]
    T.tdmrg_heff2_apply_batched(ctx, *args, y1)
    T.lib().tdmrg_ctx_set_batch_budget(ctx.h, 1)
    try:
        y2 = [torch.empty_like(d["th"]) for _, _, d in probs]
        T.tdmrg_heff2_apply_batched(ctx, *args, y2)
    finally:
        T.lib().tdmrg_ctx_set_batch_budget(ctx.h, 0)
    T.lib().tdmrg_ctx_set_fusion(ctx.h, 0)  # the grouped form runs the channel stages separately
    try:
        for a, b, (s, _, d) in zip(y1, y2, probs):
            y3 = torch.empty_like(d["th"])
            T.tdmrg_heff2_apply(ctx, s, d["L"], d["W1"], d["W2"], d["R"], d["th"], y3)
            assert torch.equal(a, b)
            assert torch.equal(a, y3)  # grouped launch == single launch, bitwise
    finally:
        T.lib().tdmrg_ctx_set_fusion(ctx.h, 1)


def test_local_expm_batched_parity(T, ctx):
    from oracle import tdvp as ot
    probs = _problems(T, ctx, 11, 9, 0.7)
    tau = 0.6
    its, ok = T.tdmrg_local_expm_batched(
        ctx, [s for s, _, _ in probs], [d["L"] for _, _, d in probs],
        [d["W1"] for _, _, d in probs], [d["W2"] for _, _, d in probs],
        [d["R"] for _, _, d in probs], [d["th"] for _, _, d in probs], tau, tol=1e-13, m_max=60)
    assert ok
    for (s, p, d), it in zip(probs, its):
        ref, it_ref, _ = ot.lanczos_expm(lambda x: ot.heff2(p["L"], p["W1"], p["W2"], p["R"], x),
                                         p["theta"], tau)
        got = T.from_device(d["th"])
        assert abs(it - it_ref) <= 1, s
        assert np.linalg.norm(got - ref) < 1e-11 * np.linalg.norm(ref), s


@pytest.mark.timeout(600)
def test_heff2_batched_full_size_sampled(T, ctx):
    """The 256-problem uneven batch at full size (the benchmark's launch
    configuration): output blocks y[a,:,:,b] of 16 problems spread evenly
    over the size order (the smallest and the largest included) against the
    oracle, computed one block at a time."""
    import torch
    import synth
    from oracle import tdvp as ot
    from synth import device as sdev
    shapes = synth.heff_batch_shapes(0, n=256)
    print("full-size batch, total complex", sum(s[0] * s[1] * s[2] * s[3] for s in shapes), flush=True)
    ops = sdev.batch_operands(0, shapes)
    W1 = [T.Wop(ctx, o["W1"]) for o in ops]
    W2 = [T.Wop(ctx, o["W2"]) for o in ops]
    ys = [torch.empty_like(o["theta"]) for o in ops]
    T.tdmrg_heff2_apply_batched(ctx, shapes, [o["L"] for o in ops], W1, W2, [o["R"] for o in ops],
                                [o["theta"] for o in ops], ys)
    torch.cuda.synchronize()
    size = [s[0] * s[1] * s[2] * s[3] * (s[4] + s[6]) for s in shapes]
    order = sorted(range(len(shapes)), key=lambda p: size[p])
    rng = np.random.default_rng(3)
    picks = sorted(set(order[round(q * (len(order) - 1) / 15)] for q in range(16)), key=lambda p: size[p])
    assert len(picks) == 16
    for p in picks:
        s = shapes[p]
        L, R, th = (T.from_device(ops[p][k]) for k in ("L", "R", "theta"))
        y = T.from_device(ys[p])
        for a, b in ((0, s[3] - 1), (int(rng.integers(s[0])), int(rng.integers(s[3])))):
            ref = ot.heff2_block(L, ops[p]["W1"], ops[p]["W2"], R, th, a, b)
            err = np.abs(y[a, :, :, b] - ref).max()
            print("problem", p, s, "block", a, b, "err", err, flush=True)
            assert err < 1e-12 * max(1.0, np.abs(ref).max()), (p, s, a, b)
