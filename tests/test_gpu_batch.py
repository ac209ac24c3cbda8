"""Batched evaluation (autotuned affine-model launch + HIP graph) against
per-plan evaluation and the oracle, graph replays, device outputs written
in place by a replay, and the tuning cache."""
import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C, statevector as SV

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return cc.Context()


def _plans(ctx, ws):
    return [cc.Plan(ctx, w.n, w.ops, w.cuts) for w in ws]


@pytest.mark.parametrize("shots", [0, 2000])
def test_batch_equals_per_plan(ctx, shots):
    ws = [W.batching_circuit(i, shots=shots) for i in range(24)]
    print(f"batch of {len(ws)} circuits, shots={shots}", flush=True)
    plans = _plans(ctx, ws)
    b = cc.Batch(ctx, plans, [w.qubits for w in ws], shots=shots, seed=7, method=cc.CCUT_METHOD_VARIANTS)
    info = b.info()
    assert info["n_items"] > 0 and info["graphed"]
    outs = b.run()
    for i, (p, w) in enumerate(zip(plans, ws)):
        ref = p.marginal(w.qubits, shots=shots, seed=7, circuit=i, method=cc.CCUT_METHOD_VARIANTS)
        assert np.array_equal(outs[i], ref), i
        assert abs(outs[i].sum() - 1.0) < 1e-9


def test_batch_against_oracle_small(ctx):
    ws = [W.batching_circuit(i, shots=200) for i in (2, 6)]
    qs = [w.qubits[:6] for w in ws]
    plans = _plans(ctx, ws)
    b = cc.Batch(ctx, plans, qs, shots=200, seed=3)
    outs = b.run()
    for i, w in enumerate(ws):
        exp = C.marginal(w.n, w.ops, w.cuts, qs[i], shots=200, seed=3, circuit=i)
        assert np.abs(outs[i] - exp).max() <= 1e-10, i


def test_graph_replays_match_eager(ctx):
    import torch
    ws = [W.batching_circuit(i, shots=1000) for i in range(12)]
    plans = _plans(ctx, ws)
    qs = [w.qubits for w in ws]
    eager = cc.Batch(ctx, plans, qs, shots=1000, seed=5, use_graph=False).run()
    g = cc.Batch(ctx, plans, qs, shots=1000, seed=5, use_graph=True)
    assert g.info()["graphed"]
    other = W.tiny()
    po = cc.Plan(ctx, other.n, other.ops, other.cuts)
    for rep in range(4):
        outs = g.run()
        for i in range(len(ws)):
            assert np.array_equal(outs[i], eager[i]), (rep, i)
        # unrelated eager work and synchronisation between replays
        po.marginal(other.qubits, shots=100, seed=rep)
        x = torch.randn(1 << 16, device="cuda")
        torch.cuda.synchronize()
        assert float(x.abs().sum()) > 0


@pytest.mark.parametrize("use_graph", [True, False])
def test_device_outputs_match_host(ctx, use_graph):
    """Device outputs: one gather launch that the caller's stream waits on
    (no host synchronization); repeated runs into the same tensors, then
    into new ones, read back on the caller's stream."""
    import torch
    ws = [W.batching_circuit(i, shots=1000) for i in range(12)]
    plans = _plans(ctx, ws)
    qs = [w.qubits for w in ws]
    b = cc.Batch(ctx, plans, qs, shots=1000, seed=9, use_graph=use_graph)
    host = b.run()
    print(f"device outputs, graph={use_graph}", flush=True)
    for rep in range(3):
        outs = [torch.full((1 << len(q),), float("nan"), dtype=torch.float64, device="cuda") for q in qs]
        for _ in range(2):  # same addresses twice: the copy list is reused
            b.run(outs)
        got = [o.cpu().numpy() for o in outs]  # ordered on the caller's stream
        for i in range(len(ws)):
            assert np.array_equal(got[i], host[i]), (rep, i)
        x = torch.randn(1 << 16, device="cuda")
        assert float(x.abs().sum()) > 0
    # back to host outputs after device ones (a replay's output table
    # points at the batch's own results again)
    again = b.run()
    for i in range(len(ws)):
        assert np.array_equal(again[i], host[i]), i


def test_tuning_cache(ctx, tmp_path, monkeypatch):
    """The model launch's shape is timed once per batch shape: a second
    batch of the same plans takes it from the process cache (same block and
    grid, same results); with CCUT_TUNE_CACHE set, a timed shape is appended
    to that file as 'key block per_cu ms'."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("CCUT_TUNE_CACHE", str(path))
    ws = [W.batching_circuit(i, shots=500) for i in range(40, 47)]
    plans = _plans(ctx, ws)
    qs = [w.qubits for w in ws]
    a = cc.Batch(ctx, plans, qs, shots=500, seed=4, use_graph=False)
    ia = a.info()
    b = cc.Batch(ctx, plans, qs, shots=500, seed=4, use_graph=False)
    ib = b.info()
    assert ib["tune_cached"]
    assert (ib["block"], ib["grid"]) == (ia["block"], ia["grid"])
    assert ib["models_ms"] == pytest.approx(ia["models_ms"])
    ra, rb = a.run(), b.run()
    for i in range(len(ws)):
        assert np.array_equal(ra[i], rb[i]), i
    if not ia["tune_cached"]:  # timed here: written to the file
        lines = path.read_text().split("\n")
        rows = [l.split() for l in lines if l.strip()]
        assert any(int(r[1]) == ia["block"] and float(r[3]) == pytest.approx(ia["models_ms"], rel=1e-5) for r in rows)
        assert all(len(r) == 4 and int(r[2]) >= 1 for r in rows)


def test_run_batch_one_shot(ctx):
    ws = [W.batching_circuit(i) for i in range(3)]
    plans = _plans(ctx, ws)
    outs = [np.zeros(1 << len(w.qubits)) for w in ws]
    cc.ccut_run_batch(ctx.handle, plans, cc._eval_opts(0, 0), [w.qubits for w in ws], outs)
    for i, (p, w) in enumerate(zip(plans, ws)):
        assert np.abs(outs[i] - p.marginal(w.qubits, circuit=i)).max() <= 1e-12


def test_skinny_contraction_vs_uncut_state_vector(ctx):
    """A 20-qubit circuit of the batching shape with 3 cuts and its 16-qubit
    marginal: 4^3 terms x 2^16 outputs with 8 rows on the non-Clifford side
    take the skinny fp64 contraction, per plan and in a batch; the uncut
    brute-force state vector is the reference."""
    w = W.batching_circuit(230, shots=0)
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    k, nq = len(w.cuts), len(w.qubits)
    reqs = [cc.ccut_request_info(plan.handle, w.qubits, f)[1] for f in range(len(plan.fragments()))]
    assert (4 ** k) << nq > (1 << 20) and 1 << (sum(reqs) - max(reqs)) <= 32
    print(f"skinny contraction: n={w.n} k={k} requested bits {reqs}", flush=True)
    ref = SV.uncut_marginal(w.n, w.ops, w.qubits)
    got = plan.marginal(w.qubits)
    assert np.abs(got - ref).max() <= 1e-10
    out = cc.Batch(ctx, [plan], [w.qubits]).run()[0]
    assert np.array_equal(out, got)
