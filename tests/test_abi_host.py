"""The C ABI without a GPU: the library loads, exports every symbol the
header declares, and plans on a host-only context exactly as the oracle's
fragmenter does (fragments, local qubit order, cut axes, variant counts),
with the documented error codes."""
import os
import re

import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "ccut.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ccut_status|void|const char \*)\s*(ccut_\w+)\s*\(", txt, re.M)))


def test_every_declared_symbol_is_exported_and_bound():
    names = _declared()
    assert len(names) >= 20
    L = cc.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in cc.SIGNATURES, n


def test_struct_layouts_match_header():
    import ctypes
    assert ctypes.sizeof(cc.ccut_op) == 24
    assert ctypes.sizeof(cc.ccut_cut) == 8
    assert ctypes.sizeof(cc.ccut_eval_opts) == 32


def _host_ctx(**kw):
    return cc.Context(-1, **kw)


def _compare(n, ops, cuts):
    ctx = _host_ctx()
    plan = cc.Plan(ctx, n, ops, cuts)
    frags = C.fragment_circuit(n, ops, cuts)
    got = plan.fragments()
    assert len(got) == len(frags)
    for g, f in zip(got, frags):
        assert g["m"] == f.m
        assert g["clifford"] == f.clifford
        assert g["segments"] == [tuple(s) for s in f.segments]
        assert g["axes"] == [(a.cut, a.side, a.local) for a in f.axes]
        assert g["n_variants"] == f.n_variants
    nf, nv, nt = plan.info()
    assert nt == 4 ** len(cuts) and nv == sum(f.n_variants for f in frags)


def test_plans_match_oracle_on_configs():
    for w in (W.tiny(), W.mid(), W.precision(), W.learned_circuit(200000)):
        _compare(w.n, w.ops, w.cuts)
    for i in range(8):
        w = W.batching_circuit(i)
        _compare(w.n, w.ops, w.cuts)


@pytest.mark.parametrize("seed", range(40))
def test_plans_match_oracle_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    ops = W.random_circuit(n, int(rng.integers(1, 40)), seed)
    k = int(rng.integers(0, min(6, len(ops)) + 1))
    cuts = W.random_cuts(n, ops, k, seed) if k else []
    _compare(n, ops, cuts)


def test_error_codes():
    ctx = _host_ctx(max_nc_qubits=4, max_cuts=2)
    ops = [("H", 0, -1, 0.0), ("CX", 0, 1, 0.0)]
    cases = [
        (2, ops, [(1, 0)], cc.CCUT_E_INVALID),            # op 0 not on qubit 1
        (2, ops, [(0, 0), (0, 0)], cc.CCUT_E_INVALID),    # duplicate
        (2, [("CX", 1, 1, 0.0)], [], cc.CCUT_E_INVALID),  # q0 == q1
        (2, [("H", 5, -1, 0.0)], [], cc.CCUT_E_INVALID),  # out of range
        (2, ops, [(0, 5)], cc.CCUT_E_INVALID),            # after_op out of range
    ]
    for n, o, c, st in cases:
        with pytest.raises(cc.CcutError) as e:
            cc.Plan(ctx, n, o, c)
        assert e.value.status == st
    wide = [("T", q, -1, 0.0) for q in range(5)] + [("CX", q, q + 1, 0.0) for q in range(4)]
    with pytest.raises(cc.CcutError) as e:
        cc.Plan(ctx, 5, wide, [])
    assert e.value.status == cc.CCUT_E_NC_TOO_WIDE
    many = [("H", 0, -1, 0.0)] * 3
    with pytest.raises(cc.CcutError) as e:
        cc.Plan(ctx, 1, many, [(0, 0), (0, 1), (0, 2)])
    assert e.value.status == cc.CCUT_E_TOO_MANY_CUTS


def test_host_only_context_refuses_evaluation():
    ctx = _host_ctx()
    w = W.tiny()
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    with pytest.raises(cc.CcutError) as e:
        plan.marginal(w.qubits)
    assert e.value.status == cc.CCUT_E_DEVICE


def test_shot_count_limit():
    """Shot counters and histogram counts are 32-bit per variant: 2^32 shots
    or more is refused before anything reaches a device."""
    ctx = _host_ctx()
    w = W.tiny()
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    with pytest.raises(cc.CcutError) as e:
        plan.marginal(w.qubits, shots=1 << 32)
    assert e.value.status == cc.CCUT_E_INVALID and "2^32" in str(e.value)
    with pytest.raises(cc.CcutError) as e:
        plan.marginal(w.qubits, shots=(1 << 32) - 1)  # valid: only the host-only context refuses
    assert e.value.status == cc.CCUT_E_DEVICE


def test_plan_outlives_destroyed_context():
    """Destroying a context while a plan made from it is alive defers the
    context's release to the plan's destruction."""
    ctx = cc.Context(-1)
    w = W.tiny()
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    ctx.close()
    assert plan.info()[0] == 2
    plan.close()
