"""The paper's workload families (Sec. VI-B) as generated here: their
structure, the closed forms of their Clifford versions, and exact
reconstructions with automatically placed cuts against the uncut state
vector (oracle only, CPU)."""
import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C, statevector as sv

NC = ("T", "TDG", "RZ")


def _count(ops, kinds):
    return sum(1 for o in ops if o[0] in kinds)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_structure(n):
    h = W.hwea(n, rounds=5, seed=1)
    assert _count(h.ops, ("CX",)) == 5 * (n - 1) and _count(h.ops, NC) == 1
    q = W.qaoa_sk(n, seed=1)
    assert _count(q.ops, ("CX",)) == n * (n - 1) and _count(q.ops, NC) == 1
    p = W.phase_code(n, seed=1)
    assert p.n == 2 * n - 1 and _count(p.ops, ("CX",)) == 2 * (n - 1) and _count(p.ops, NC) == 1
    assert p.qubits == list(range(n, 2 * n - 1))


@pytest.mark.parametrize("n", [4, 6, 8])
def test_clifford_versions_closed_forms(n):
    # without the injected T: a stabilizer state, so every <Z_q> is -1, 0 or
    # +1; an error-free phase-code round has the all-zero syndrome
    for w in (W.hwea(n, seed=2, n_t=0), W.qaoa_sk(n, seed=2, n_t=0)):
        p = sv.probabilities(sv.run(w.n, w.ops))
        for q in range(w.n):
            z = sv.z_expectation(p, w.n, 1 << q)
            assert min(abs(z - v) for v in (-1.0, 0.0, 1.0)) <= 1e-12
    pc = W.phase_code(n, seed=2, n_t=0)
    syn = sv.uncut_marginal(pc.n, pc.ops, pc.qubits)
    assert abs(syn[0] - 1.0) <= 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_found_cuts_reconstruct(seed):
    for w in (W.hwea(7, seed=seed), W.qaoa_sk(6, seed=seed), W.phase_code(5, seed=seed)):
        cuts = cc.find_cuts(w.n, w.ops, 3)
        assert 1 <= len(cuts) <= 2
        frags = C.fragment_circuit(w.n, w.ops, cuts)
        assert all(f.m <= 3 for f in frags if not f.clifford)
        R = C.marginal(w.n, w.ops, cuts, w.qubits)
        assert np.abs(R - sv.uncut_marginal(w.n, w.ops, w.qubits)).max() <= 1e-12, w.name
