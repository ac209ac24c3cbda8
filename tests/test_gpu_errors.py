"""Failure handling forced from the host, through the C ABI: an allocator
that refuses (CCUT_E_OOM) and a cancellation requested while an evaluation
runs (CCUT_E_CANCELLED, the request made from inside the allocator callback
that the evaluation calls).  No kernel is made to fail: the evaluation stops
at its own checks, and the context stays usable afterwards."""
import ctypes

import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C

pytestmark = pytest.mark.gpu


def _ctx_with(alloc_py):
    """A context on device 0 whose device allocations go through alloc_py
    (size -> pointer or None); frees go to torch's caching allocator."""
    import torch
    torch.cuda.set_device(0)
    opts = cc.ccut_opts()
    opts.device = 0
    opts.hip_stream = ctypes.c_void_p(torch.cuda.current_stream(0).cuda_stream)

    def _free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    a, f = cc.ALLOC_FN(lambda size, user: alloc_py(size)), cc.FREE_FN(_free)
    opts.alloc, opts.free = a, f
    return cc.ccut_ctx_create(opts), (a, f)


def _torch_alloc(size):
    import torch
    return torch.cuda.caching_allocator_alloc(size, 0, torch.cuda.current_stream(0))


def test_refusing_allocator_gives_oom_then_recovers():
    w = W.tiny()
    state = {"refuse": True}
    handle, keep = _ctx_with(lambda size: None if state["refuse"] else _torch_alloc(size))
    try:
        plan = cc.ccut_plan_create(handle, w.n, w.ops, w.cuts)
        eo = cc._eval_opts()
        out = np.zeros(1 << len(w.qubits))
        with pytest.raises(cc.CcutError) as e:
            cc.ccut_marginal(plan, handle, eo, w.qubits, out)
        assert e.value.status == cc.CCUT_E_OOM
        assert "allocation" in cc.ccut_last_error(handle)
        state["refuse"] = False
        cc.ccut_marginal(plan, handle, eo, w.qubits, out)
        assert np.abs(out - C.marginal(w.n, w.ops, w.cuts, w.qubits)).max() <= 1e-10
        cc.ccut_plan_destroy(plan)
    finally:
        cc.ccut_ctx_destroy(handle)


def test_cancel_during_evaluation_then_recovers():
    w = W.tiny()
    holder = {}

    def alloc(size):
        if holder.get("cancel"):
            holder["cancel"] = False
            cc.ccut_cancel(holder["ctx"])  # the evaluation that asked for memory is running
        return _torch_alloc(size)

    handle, keep = _ctx_with(alloc)
    holder["ctx"] = handle
    try:
        plan = cc.ccut_plan_create(handle, w.n, w.ops, w.cuts)
        eo = cc._eval_opts(shots=1000, seed=3)
        out = np.zeros(1 << len(w.qubits))
        holder["cancel"] = True
        with pytest.raises(cc.CcutError) as e:
            cc.ccut_marginal(plan, handle, eo, w.qubits, out)
        assert e.value.status == cc.CCUT_E_CANCELLED
        # the flag is cleared when the next evaluation starts
        cc.ccut_marginal(plan, handle, eo, w.qubits, out)
        ref = C.marginal(w.n, w.ops, w.cuts, w.qubits, shots=1000, seed=3)
        assert np.abs(out - ref).max() <= 1e-10
        cc.ccut_plan_destroy(plan)
    finally:
        cc.ccut_ctx_destroy(handle)
