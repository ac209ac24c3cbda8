"""Call graphs: repeated device-output marginal/zexpect calls are captured on
their second occurrence and replayed.  Every replay must equal the eager
result bit for bit, with eager work, host-output calls and synchronizations
between the replays."""
import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return cc.Context()


def _eager(ctx, fn):
    ctx.call_graphs(False)
    try:
        return fn()
    finally:
        ctx.call_graphs(True)


@pytest.mark.parametrize("shots", [0, 3000])
def test_replays_match_eager_mid(ctx, shots):
    import torch
    w = W.mid(shots=shots)
    print(f"mid circuit, shots={shots}", flush=True)
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    masks = w.zmask_words()
    ref_m = _eager(ctx, lambda: plan.marginal(w.qubits, shots=shots, seed=w.seed))
    ref_z = _eager(ctx, lambda: plan.zexpect(masks, shots=shots, seed=w.seed))
    other = W.tiny()
    po = cc.Plan(ctx, other.n, other.ops, other.cuts)
    ref_o = po.marginal(other.qubits, seed=1)
    om = torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda")
    oz = torch.empty(masks.shape[0], dtype=torch.float64, device="cuda")
    for rep in range(5):
        om.fill_(float("nan"))
        oz.fill_(float("nan"))
        plan.marginal(w.qubits, shots=shots, seed=w.seed, out=om)
        plan.zexpect(masks, shots=shots, seed=w.seed, out=oz)
        # eager work of another plan and of this plan (host output) in between
        assert np.array_equal(po.marginal(other.qubits, seed=1), ref_o)
        if rep == 2:
            assert np.array_equal(plan.marginal(w.qubits, shots=shots, seed=w.seed), ref_m)
        torch.cuda.synchronize()
        assert np.array_equal(om.cpu().numpy(), ref_m), rep
        assert np.array_equal(oz.cpu().numpy(), ref_z), rep


def test_new_key_runs_its_own_request(ctx):
    import torch
    w = W.mid(shots=1000)
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    om = torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda")
    for seed in (11, 12):
        ref = _eager(ctx, lambda: plan.marginal(w.qubits, shots=1000, seed=seed))
        for rep in range(3):
            om.zero_()
            plan.marginal(w.qubits, shots=1000, seed=seed, out=om)
            torch.cuda.synchronize()
            assert np.array_equal(om.cpu().numpy(), ref), (seed, rep)
    # another output buffer and another qubit subset are other keys
    om2 = torch.empty(1 << 6, dtype=torch.float64, device="cuda")
    ref2 = _eager(ctx, lambda: plan.marginal(w.qubits[:6], shots=1000, seed=11))
    for rep in range(3):
        plan.marginal(w.qubits[:6], shots=1000, seed=11, out=om2)
        torch.cuda.synchronize()
        assert np.array_equal(om2.cpu().numpy(), ref2), rep


def test_fp32_exact_replays(ctx):
    import torch
    w = W.tiny()
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    q = list(range(w.n))
    ref = _eager(ctx, lambda: plan.marginal(q, precision=cc.CCUT_FP32_MFMA_FP64SUM))
    out = torch.empty(1 << w.n, dtype=torch.float64, device="cuda")
    for rep in range(4):
        out.fill_(-1.0)
        plan.marginal(q, precision=cc.CCUT_FP32_MFMA_FP64SUM, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep


def test_timing_forces_eager(ctx):
    import torch
    w = W.mid(shots=500)
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    om = torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda")
    ref = _eager(ctx, lambda: plan.marginal(w.qubits, shots=500, seed=3))
    for _ in range(3):
        plan.marginal(w.qubits, shots=500, seed=3, out=om)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_reset()
    try:
        plan.marginal(w.qubits, shots=500, seed=3, out=om)
        torch.cuda.synchronize()
        times = ctx.kernel_times()
    finally:
        ctx.timing(False)
    assert times["sv_kernel"][0] >= 1  # launched eagerly, so timed
    assert np.array_equal(om.cpu().numpy(), ref)
