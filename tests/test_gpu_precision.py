"""The 400-qubit, 6-cut precision workload on the GPU.

Pins at full width: the same circuit with every T replaced by T T (= S) is
Clifford, so its uncut output statistics are exact from the oracle's
stabilizer elimination; the cut pipeline (Heisenberg-picture Clifford
tensors, state-vector fragments, 4096-term contraction) must reproduce them.
On the real (non-Clifford) workload the Heisenberg and per-variant paths
must agree, a few variants' exact tables are checked against the oracle's
literal tableau, and the FP32-MFMA contraction must stay within 1e-5 of
the FP64 one on every output.
"""
import sys

import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C, stabilizer as stab, statevector as SV

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from _helpers import stabilizer_rows, tt_substitute  # noqa: E402

pytestmark = pytest.mark.gpu


def _log(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return cc.Context()


def _structured_masks(xs, zs, ss, n, count, seed):
    """Z strings with expectation +-1: random products of the Z-type
    stabilizer subgroup's generators."""
    Cm, s = stab.z_constraints(xs, zs, ss, list(range(n)))
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        sel = rng.random(Cm.shape[0]) < 0.5
        row = np.bitwise_xor.reduce(Cm[sel], axis=0) if sel.any() else Cm[0]
        out.append(sum(1 << q for q in range(n) if row[q]))
    return out


def _words(masks, n):
    nw = (n + 63) // 64
    return np.array([[(m >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for w in range(nw)] for m in masks], dtype=np.uint64)


def test_precision_clifford_equivalent_full_width(ctx):
    w = W.precision()
    ops, cuts, cl = tt_substitute(w.ops, w.cuts)
    _log("precision T T = S: marginal + Z strings")
    plan = cc.Plan(ctx, w.n, ops, cuts)
    assert sorted(f["m"] for f in plan.fragments()) == [6, 6, 394]
    xs, zs, ss = stabilizer_rows(w.n, cl)
    ref = stab.distribution(xs, zs, ss, w.qubits)
    got = plan.marginal(w.qubits)
    assert np.abs(got - ref).max() <= 1e-12
    got32 = plan.marginal(w.qubits, precision=cc.CCUT_FP32_MFMA_FP64SUM)
    assert np.abs(got32 - ref).max() <= 1e-5
    masks = w.zmasks + _structured_masks(xs, zs, ss, w.n, 16, 5)
    zref = np.array(stab.z_expectations(xs, zs, ss, masks, w.n), dtype=float)
    assert np.count_nonzero(zref) >= 16
    zg = plan.zexpect(_words(masks, w.n))
    assert np.abs(zg - zref).max() <= 1e-12
    zg32 = plan.zexpect(_words(masks, w.n), precision=cc.CCUT_FP32_MFMA_FP64SUM)
    assert np.abs(zg32 - zref).max() <= 1e-5


@pytest.mark.parametrize("n_ops,seed", [(50, 32), (50, 9), (70, 0)])
def test_mfma_contraction_vs_uncut_state_vector(ctx, n_ops, seed):
    """6 cuts and a 16-qubit marginal: 4^6 terms x 2^16 outputs go through
    the MFMA contraction in both precisions; the uncut brute-force state
    vector of the 18-qubit circuit is the reference."""
    ops = W.random_circuit(18, n_ops, seed)
    cuts = W.random_cuts(18, ops, 6, seed)
    qubits = list(range(1, 17))
    _log(f"mfma contraction vs uncut state vector: n_ops={n_ops} seed={seed}")
    ref = SV.uncut_marginal(18, ops, qubits)
    plan = cc.Plan(ctx, 18, ops, cuts)
    got = plan.marginal(qubits)
    assert np.abs(got - ref).max() <= 1e-10
    got32 = plan.marginal(qubits, precision=cc.CCUT_FP32_MFMA_FP64SUM)
    assert np.abs(got32 - ref).max() <= 1e-5


def test_precision_workload_paths_and_fp32_error(ctx):
    w = W.precision()
    _log("precision workload: Heisenberg vs variants, fp32 vs fp64")
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    r64 = plan.marginal(w.qubits)
    assert abs(r64.sum() - 1.0) <= 1e-10
    rv = plan.marginal(w.qubits, method=cc.CCUT_METHOD_VARIANTS)
    assert np.abs(r64 - rv).max() <= 1e-12
    r32 = plan.marginal(w.qubits, precision=cc.CCUT_FP32_MFMA_FP64SUM)
    err = np.abs(r32 - r64)
    _log(f"fp32-mfma marginal: max abs err {err.max():.3e}, max rel err "
         f"{(err / np.maximum(np.abs(r64), 1e-300)).max():.3e}")
    assert err.max() <= 1e-5
    masks = w.zmask_words()
    z64 = plan.zexpect(masks)
    z32 = plan.zexpect(masks, precision=cc.CCUT_FP32_MFMA_FP64SUM)
    assert np.abs(z32 - z64).max() <= 1e-5


def test_precision_variant_tables_spot_check(ctx):
    """A few variants of the 394-qubit fragment: exact tables from the GPU's
    per-variant tableau path against the oracle's literal tableau."""
    w = W.precision()
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    f = [i for i, fr in enumerate(frags) if fr.clifford][0]
    fr = frags[f]
    req = C.make_request(fr, w.qubits)
    got = plan.variant_tables(w.qubits, f)
    for v in (0, 1, 1365, 4095):
        _log(f"precision variant {v}")
        exp = C.clifford_exact(fr, v, req.meas, method="elim")
        assert np.array_equal(got[v], exp), v
