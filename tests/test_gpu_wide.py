"""Clifford fragments with more than 64 measured qubits (Sec. V-B,
Clifford fragments sampled): sample models, shot records and Z-string
parities over several words per outcome vector.

Bars: shot records bit-exact against literal per-shot CHP measurement
(oracle/chp.c, the same Philox draw); sampled and exact Z-string
expectations within 1e-12 of the oracle (integer parity counts, the same
contraction up to rounding); the 400-qubit precision workload's 64 strings
at 1e4 shots within a statistical bound of their exact values."""
import os
import sys

import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C, philox as PX

pytestmark = pytest.mark.gpu

CLIFF = ["H", "S", "SDG", "X", "Y", "Z", "CX", "CZ"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize.npz")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return cc.Context()


def _circuit(m, seed):
    """A random Clifford circuit on m wires with an H on wire 0 cut right
    after it (the big fragment gets a quantum input) and wire m - 1 cut
    after its last operation (a quantum output on the big fragment)."""
    ops = [("H", 0, -1, 0.0)] + W.random_circuit(m, 5 * m, seed, kinds=CLIFF)
    last = max(i for i, o in enumerate(ops) if o[1] == m - 1 or o[2] == m - 1)
    return ops, [(0, 0), (m - 1, last)]


def _pack_words(rec_u8):
    shots, nm = rec_u8.shape
    rw = (nm + 63) // 64
    out = np.zeros((shots, rw), dtype=np.uint64)
    for j in range(nm):
        out[:, j // 64] |= rec_u8[:, j].astype(np.uint64) << np.uint64(j % 64)
    return out


@pytest.mark.parametrize("m", [70, 130, 260, 400])
def test_shot_records_bit_exact_wide(ctx, m):
    _log(f"wide records m={m}")
    ops, cuts = _circuit(m, 700 + m)
    plan = cc.Plan(ctx, m, ops, cuts)
    frags = C.fragment_circuit(m, ops, cuts)
    rng = np.random.default_rng(m)
    qubits = sorted(int(q) for q in rng.choice(m, size=m - 3, replace=False))
    shots = 37 if m <= 130 else 9
    seen = 0
    for f, fr in enumerate(frags):
        req = C.make_request(fr, qubits)
        if not fr.clifford or len(req.meas) <= 64:
            continue
        seen += 1
        nv = fr.n_variants
        assert any(a.side == 0 for a in fr.axes) and any(a.side == 1 for a in fr.axes)
        got = plan.shot_records(qubits, f, 0, nv, shots=shots, seed=41)
        assert got.shape == (nv, shots, (len(req.meas) + 63) // 64)
        for v in range(nv):
            t = C.clifford_tableau(fr, v)
            exp = _pack_words(t.sample(req.meas, 41, PX.variant_id(0, f, v), 0, shots))
            assert np.array_equal(got[v], exp), (m, f, v)
    assert seen == 1


def _masks(m, count, seed, lo, hi):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        q = rng.choice(m, size=int(rng.integers(lo, hi)), replace=False)
        out.append(sum(1 << int(x) for x in q))
    return out


def _mask_words(masks, n):
    nw = (n + 63) // 64
    return np.array([[(z >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for w in range(nw)] for z in masks], dtype=np.uint64)


@pytest.mark.parametrize("m,shots", [(100, 301), (200, 64)])
def test_zexpect_wide_sampled_matches_oracle(ctx, m, shots):
    _log(f"wide zexpect sampled m={m}")
    ops, cuts = _circuit(m, 900 + m)
    masks = _masks(m, 8, m, 20, m - 10)
    plan = cc.Plan(ctx, m, ops, cuts)
    nm = max(len(C.zstring_measured_set(f, masks)) for f in C.fragment_circuit(m, ops, cuts))
    assert nm > 64
    want = C.zexpect(m, ops, cuts, masks, shots=shots, seed=13)
    got = plan.zexpect(_mask_words(masks, m), shots=shots, seed=13)
    assert np.max(np.abs(got - want)) <= 1e-12
    # settled parities too
    want = C.zexpect(m, ops, cuts, masks, shots=shots, seed=13, settle=True)
    got = plan.zexpect(_mask_words(masks, m), shots=shots, seed=13, flags=cc.CCUT_FLAG_SETTLE)
    assert np.max(np.abs(got - want)) <= 1e-12


def test_zexpect_wide_exact_from_variants(ctx):
    m = 150
    _log("wide zexpect exact (variants)")
    ops, cuts = _circuit(m, 1150)
    masks = _masks(m, 8, 1150, 30, 140)
    plan = cc.Plan(ctx, m, ops, cuts)
    want = C.zexpect(m, ops, cuts, masks)
    got = plan.zexpect(_mask_words(masks, m), method=cc.CCUT_METHOD_VARIANTS)
    assert np.max(np.abs(got - want)) <= 1e-12
    heis = plan.zexpect(_mask_words(masks, m), method=cc.CCUT_METHOD_HEISENBERG)
    assert np.max(np.abs(heis - want)) <= 1e-12


def test_precision_zstrings_sampled(ctx):
    """The 400-qubit precision workload's 64 Z strings at 1e4 shots (the
    Clifford fragment measures about 390 qubits): within 0.1 of the exact
    values (the oracle's, from the golden file) for every string, and the
    two seeds' estimates differ (the shots are random) while their mean
    error stays small.  The bound: each variant's sampled parity has
    standard deviation at most 1e-2 at 1e4 shots, and the recombination
    weights the variants with coefficients of order one."""
    w = W.precision()
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    nm = max(len(C.zstring_measured_set(f, w.zmasks)) for f in frags if f.clifford)
    _log(f"precision zstrings sampled, {nm} measured")
    assert nm > 64
    exact = np.load(GOLDEN)["precision_z"]
    masks = _mask_words(w.zmasks, w.n)
    est = [plan.zexpect(masks, shots=10000, seed=s) for s in (1, 2)]
    for e in est:
        assert np.all(np.isfinite(e))
        assert np.max(np.abs(e - exact)) <= 0.1
        assert np.mean(np.abs(e - exact)) <= 0.02
    assert np.max(np.abs(est[0] - est[1])) > 0
