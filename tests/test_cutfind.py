"""Automatic cut placement (host code behind the C ABI, no device needed)
against the brute-force oracle: every cut list it returns isolates the
non-Clifford ops within the width limit, needs at most two cuts per
non-Clifford op (Sec. III-B), matches the brute-force minimum on structured
cases and stays close to it on random tiny circuits; reconstructions with
its cuts equal the uncut state vector."""
import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutfind as F, cutting as C, statevector as sv


def _ops(*spec):
    return [(k, a, b, 0.3 if k == "RZ" else 0.0) for k, a, b in spec]


STRUCTURED = [
    # (name, n, ops, width, minimum cuts)
    ("T mid-wire", 2, _ops(("H", 0, -1), ("CX", 0, 1), ("T", 0, -1), ("CX", 0, 1), ("H", 0, -1)), 1, 2),
    ("T first on its wire", 2, _ops(("T", 0, -1), ("CX", 0, 1), ("H", 1, -1)), 1, 1),
    ("T last on its wire", 2, _ops(("CX", 0, 1), ("H", 0, -1), ("T", 0, -1)), 1, 1),
    ("two T one run", 2, _ops(("CX", 0, 1), ("T", 0, -1), ("S", 0, -1), ("H", 0, -1), ("TDG", 0, -1),
                              ("CX", 0, 1)), 1, 2),
    ("whole circuit fits", 3, _ops(("H", 0, -1), ("T", 0, -1), ("CX", 0, 1), ("CX", 1, 2), ("T", 2, -1)), 3, 0),
    ("two wires, width 2", 3, _ops(("H", 0, -1), ("T", 0, -1), ("CX", 0, 1), ("T", 1, -1), ("CX", 1, 2),
                                   ("H", 2, -1), ("CX", 0, 2)), 2, 2),
]


@pytest.mark.parametrize("case", STRUCTURED, ids=[c[0] for c in STRUCTURED])
def test_structured_minimum(case):
    name, n, ops, width, k_min = case
    assert F.min_cuts(n, ops, width, 4) == k_min  # the oracle's own count
    cuts = cc.find_cuts(n, ops, width)
    assert F.isolates(n, ops, cuts, width)
    assert len(cuts) == k_min, cuts


def test_workload_shapes():
    # block-structured workloads: the finder needs no more cuts than the
    # hand-placed block cuts, and its fragments keep the width limit
    for w, width in ((W.tiny(), 4), (W.mid(), 12), (W.precision(), 12), (W.learned_circuit(200000), 12)):
        cuts = cc.find_cuts(w.n, w.ops, width)
        assert len(cuts) <= len(w.cuts), w.name
        frags = C.fragment_circuit(w.n, w.ops, cuts)
        assert all(f.m <= width for f in frags if not f.clifford), w.name
    total_found = total_given = 0
    for i in range(0, 256, 8):
        w = W.batching_circuit(i)
        cuts = cc.find_cuts(w.n, w.ops, 12)
        assert len(cuts) <= 2 * F.n_non_clifford(w.ops)
        total_found += len(cuts)
        total_given += len(w.cuts)
    assert total_found <= total_given


@pytest.mark.parametrize("seed", range(24))
def test_random_tiny_against_brute_force(seed):
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(2, 5))
    ops = W.random_circuit(n, int(rng.integers(6, 13)), seed)
    n_nc = F.n_non_clifford(ops)
    for width in range(1, n + 1):
        cuts = cc.find_cuts(n, ops, width)
        assert F.isolates(n, ops, cuts, width), (width, cuts)
        assert len(cuts) <= 2 * n_nc
        k_min = F.min_cuts(n, ops, width, len(cuts))
        assert k_min is not None and k_min <= len(cuts)
        # a greedy search: allowed one cut above the minimum on these sizes
        assert len(cuts) <= k_min + 1, (width, cuts, k_min)


@pytest.mark.parametrize("seed", range(6))
def test_reconstruction_with_found_cuts(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(3, 7))
    ops = W.random_circuit(n, int(rng.integers(10, 30)), seed)
    # the narrowest width whose cut list the oracle contracts in seconds (k <= 4)
    width = next(wd for wd in range(2, n + 1) if len(cc.find_cuts(n, ops, wd)) <= 4)
    cuts = cc.find_cuts(n, ops, width)
    qubits = list(range(n))
    R = C.marginal(n, ops, cuts, qubits)
    assert np.abs(R - sv.uncut_marginal(n, ops, qubits)).max() <= 1e-12


def test_errors():
    ops = _ops(("H", 0, -1), ("T", 0, -1))
    with pytest.raises(cc.CcutError) as e:
        cc.find_cuts(1, ops, 0)
    assert e.value.status == cc.CCUT_E_INVALID
    with pytest.raises(cc.CcutError) as e:
        cc.find_cuts(1, _ops(("CX", 0, 0)), 1)
    assert e.value.status == cc.CCUT_E_INVALID
    assert cc.find_cuts(2, _ops(("H", 0, -1), ("CX", 0, 1)), 1) == []  # nothing to isolate
