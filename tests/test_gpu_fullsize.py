"""GPU results at the workloads' full sizes against the oracle.

The expected values are tests/golden/fullsize.npz, written by
tests/golden/make_fullsize.py from the oracle alone (the result the paper
defines in Sec. V-C: the recombined distribution of the fragment variants,
whose only error is Clifford sampling):

* the 400-qubit, 6-cut precision workload, exact: its 16-qubit marginal and
  64 Z strings, per result, in fp64 (<= 1e-10) and with fp32 matrix-core
  products (<= 1e-5);
* the 32-qubit, 2-cut workload at 1e5 shots per variant: its 12-qubit
  marginal and 64 Z strings (<= 1e-10), the shots being identical under the
  shared Philox keys;
* five circuits of the 256-circuit batch at 1e4 shots, 16-qubit marginals,
  evaluated in the whole batch as the benchmark runs it (<= 1e-10).

The 300-qubit, 10-cut learned workload is too large for the cut oracle
(4^10 terms); its Clifford-equivalent (every T replaced by T T = S in the
truth, kept as T T in the cut circuit) is checked against the uncut
stabilizer marginal through the dense, sparse and fp32 contractions.
"""
import os

import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import stabilizer as stab

from _helpers import stabilizer_rows, tt_substitute

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fullsize.npz")
BATCH_CIRCUITS = (0, 76, 77, 126, 151)


def _log(msg):
    print(f"[fullsize] {msg}", flush=True)


@pytest.fixture(scope="module")
def gold():
    return np.load(GOLD)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return cc.Context()


def _per_result(got, exp):
    err = np.abs(got - exp)
    return float(err.max()), float((err / np.maximum(np.abs(exp), 1e-300)).max())


def test_precision_full_workload_per_result(ctx, gold):
    w = W.precision()
    _log("precision: 400 qubits, 6 cuts, exact; marginal and 64 Z strings, fp64 and fp32 products")
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    masks = w.zmask_words()
    m64 = plan.marginal(w.qubits)
    z64 = plan.zexpect(masks)
    m32 = plan.marginal(w.qubits, precision=cc.CCUT_FP32_MFMA_FP64SUM)
    z32 = plan.zexpect(masks, precision=cc.CCUT_FP32_MFMA_FP64SUM)
    m3 = plan.marginal(w.qubits, precision=cc.CCUT_FP32X3_MFMA_FP64SUM)
    z3 = plan.zexpect(masks, precision=cc.CCUT_FP32X3_MFMA_FP64SUM)
    em = gold["precision_marginal"]
    ez = gold["precision_z"]
    for name, got, exp, tol in (("marginal fp64", m64, em, 1e-10), ("Z strings fp64", z64, ez, 1e-10),
                                ("marginal fp32", m32, em, 1e-5), ("Z strings fp32", z32, ez, 1e-5),
                                ("marginal fp32 hi/lo", m3, em, 1e-5), ("Z strings fp32 hi/lo", z3, ez, 1e-5)):
        a, r = _per_result(got, exp)
        _log(f"precision {name}: max abs err {a:.3e}, max rel err {r:.3e}")
        assert np.all(np.abs(got - exp) <= tol), name


def test_mid_full_workload_sampled(ctx, gold):
    w = W.mid()
    _log("mid: 32 qubits, 2 cuts, 1e5 shots per variant; marginal and 64 Z strings")
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    got = plan.marginal(w.qubits, shots=w.shots, seed=w.seed)
    assert np.abs(got - gold["mid_marginal"]).max() <= 1e-10
    zg = plan.zexpect(w.zmask_words(), shots=w.shots, seed=w.seed)
    assert np.abs(zg - gold["mid_z"]).max() <= 1e-10


def test_batch_full_size_circuits(ctx, gold):
    import torch
    ws = W.batching(256, shots=10_000)
    _log("batch: 256 circuits, 1e4 shots, graph replay; 5 circuits against the oracle")
    plans = [cc.Plan(ctx, w.n, w.ops, w.cuts) for w in ws]
    batch = cc.Batch(ctx, plans, [w.qubits for w in ws], shots=10_000, seed=2000, use_graph=True)
    outs = [torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda") for w in ws]
    for _ in range(2):  # replays after the capture
        batch.run(outs)
    torch.cuda.synchronize()
    for i in BATCH_CIRCUITS:
        got = outs[i].cpu().numpy()
        err = np.abs(got - gold[f"batch_{i}"]).max()
        _log(f"batch circuit {i} ({ws[i].n} qubits, {len(ws[i].cuts)} cuts): max abs err {err:.3e}")
        assert err <= 1e-10, i


def test_learned_workload_clifford_equivalent(ctx):
    w = W.learned_circuit(200000)
    ops, cuts, cl = tt_substitute(w.ops, w.cuts)
    _log("learned T T = S: 300 qubits, 10 cuts, dense / sparse / fp32 against the uncut stabilizer marginal")
    plan = cc.Plan(ctx, w.n, ops, cuts)
    assert plan.info()[2] == 4 ** 10
    xs, zs, ss = stabilizer_rows(w.n, cl)
    ref = stab.distribution(xs, zs, ss, w.qubits)
    dense = plan.marginal(w.qubits)
    assert np.abs(dense - ref).max() <= 1e-12
    sparse = plan.marginal(w.qubits, flags=cc.CCUT_FLAG_SPARSE)
    assert np.abs(sparse - ref).max() <= 1e-12
    f32 = plan.marginal(w.qubits, precision=cc.CCUT_FP32_MFMA_FP64SUM)
    assert np.abs(f32 - ref).max() <= 1e-5
