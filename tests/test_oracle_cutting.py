"""Pins for the cutting oracle: the uncut brute-force state vector, textbook
closed forms, Clifford-equivalent circuits at width, normalisation,
unbiasedness of sampled estimates, and planted mistakes that must be caught."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import chp, cutting as C, mlp as M, statevector as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "textbook_cuts.txt")


def _golden():
    cases = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, n, ops, cuts, qubits, expect = [s.strip() for s in line.split("|")]
        op_list = []
        for tok in ops.split():
            k, a, b = tok.split(":")
            op_list.append((k, int(a), int(b), 0.0))
        cut_list = [tuple(int(v) for v in tok.split("@")) for tok in cuts.split()]
        cases.append((name, int(n), op_list, cut_list, [int(q) for q in qubits.split()],
                      np.array([float(v) for v in expect.split()])))
    return cases


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[0])
def test_textbook_cases(case):
    name, n, ops, cuts, qubits, expect = case
    R = C.marginal(n, ops, cuts, qubits)
    assert np.allclose(R, expect, atol=1e-14)
    Rs = C.marginal(n, ops, cuts, qubits, shots=4000, seed=1)
    assert np.isclose(Rs.sum(), 1.0)


def test_tiny_config_against_uncut_state_vector():
    w = W.tiny()
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    assert [(f.m, f.clifford) for f in frags] == [(4, False), (5, True)]
    ref = sv.uncut_marginal(w.n, w.ops, w.qubits)
    for method in ("branch", "elim"):
        R = C.marginal(w.n, w.ops, w.cuts, w.qubits, exact_method=method)
        assert np.abs(R - ref).max() <= 1e-12


@pytest.mark.parametrize("seed", range(30))
def test_random_circuits_random_cuts_against_state_vector(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    ops = W.random_circuit(n, int(rng.integers(4, 30)), seed)
    k = int(rng.integers(1, min(3, len(ops)) + 1))
    cuts = W.random_cuts(n, ops, k, seed)
    qubits = [int(q) for q in rng.permutation(n)[: int(rng.integers(1, n + 1))]]
    ref = sv.uncut_marginal(n, ops, qubits)
    R = C.marginal(n, ops, cuts, qubits)
    assert np.abs(R - ref).max() <= 1e-12
    masks = [int(m) for m in rng.integers(0, 1 << n, size=6)]
    p = sv.probabilities(sv.run(n, ops))
    z = C.zexpect(n, ops, cuts, masks)
    zr = [sv.z_expectation(p, n, m) for m in masks]
    assert np.abs(z - zr).max() <= 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_recombine_loop_equals_matmul(seed):
    rng = np.random.default_rng(1000 + seed)
    n = 6
    ops = W.random_circuit(n, 25, 1000 + seed)
    cuts = W.random_cuts(n, ops, 3, 1000 + seed)
    qubits = list(range(n))
    R, parts = C.marginal(n, ops, cuts, qubits, return_parts=True)
    nf = len(parts["frags"])
    left = [f for f in range(nf) if f % 2 == 0]
    R2 = C.recombine_matmul(parts["frags"], parts["reqs"], parts["tensors"], len(cuts), n, left)
    assert np.allclose(R, R2, atol=1e-14)


def test_downstream_tensor_traces():
    """A fragment that only has quantum inputs implements a trace-preserving
    map: summed over its outcomes, the Pauli column P gives Tr(P) = 2 for I
    and 0 otherwise on each input."""
    w = W.mid()
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    cl = [f for f in frags if f.clifford][0]
    assert all(a.side == 1 for a in cl.axes)
    req = C.make_request(cl, [24, 25, 26, 27])
    d = C.variant_distributions(cl, req.meas)
    T = C.pauli_tensor(cl, req, d)
    s = T.sum(axis=0)
    expect = np.zeros(4 ** len(cl.axes))
    expect[0] = 2.0 ** len(cl.axes)
    assert np.allclose(s, expect, atol=1e-12)


def test_config_fragment_shapes():
    shapes = {
        "tiny": (W.tiny(), [4, 5]),
        "mid": (W.mid(), [10, 24]),
        "precision": (W.precision(), [6, 6, 394]),
        "learned": (W.learned_circuit(200000), [5, 5, 5, 5, 290]),
    }
    for name, (w, sizes) in shapes.items():
        frags = C.fragment_circuit(w.n, w.ops, w.cuts)
        assert sorted(f.m for f in frags) == sorted(sizes), name
        assert sum(1 for f in frags if not f.clifford) == len(sizes) - 1
    for i in range(16):
        w = W.batching_circuit(i)
        frags = C.fragment_circuit(w.n, w.ops, w.cuts)
        assert len(frags) == 2 and sum(f.clifford for f in frags) == 1
        assert max(f.m for f in frags if f.clifford) <= 200


def _clifford_equivalent(n, blocks, depth, t_c, seed, kind):
    """Block circuit whose T gates are replaced by a Clifford-equivalent
    non-Clifford pattern: 'tt' puts T T (= S) in place of each T."""
    ops, cuts = W.block_circuit(n, depth, blocks, t_c=t_c, p_cx=0.3, seed=seed, n_t=len(blocks) * 2)
    cut_ops = {}
    out, cl = [], []
    for i, op in enumerate(ops):
        if op[0] == "T" and kind == "tt":
            out.append(op)
            out.append(op)
            cl.append(("S", op[1], -1, 0.0))
        else:
            out.append(op)
            cl.append(op)
        cut_ops[i] = len(out) - 1
    new_cuts = [(q, cut_ops[a]) for q, a in cuts]
    return out, new_cuts, cl


@pytest.mark.parametrize("seed", range(3))
def test_clifford_equivalent_at_width(seed):
    """T T = S: the cut result must equal the uncut circuit's exact
    stabilizer marginal, at widths where no state vector fits."""
    n = 48
    blocks = [W.Block([5, 6, 7, 8], [7, 8]), W.Block([30, 31, 32, 33], [30, 31])]
    ops, cuts, cl = _clifford_equivalent(n, blocks, 16, 8, 40 + seed, "tt")
    qubits = [5, 6, 9, 10, 28, 29, 32, 33]
    R = C.marginal(n, ops, cuts, qubits)
    t = chp.Tableau(n)
    for k, a, b, _ in cl:
        t.gate(k, a, b)
    ref = t.exact(qubits)
    assert np.abs(R - ref).max() <= 1e-12


def test_t_on_z_eigenstate_and_zero_t_at_width():
    n = 40
    blocks = [W.Block([10, 11, 12, 13], [12, 13])]
    ops, cuts = W.block_circuit(n, 14, blocks, t_c=7, p_cx=0.3, seed=77, n_t=0)
    # (i) no T at all, cuts still placed; (iii) T on qubits still in |0>
    ops3 = [("T", 10, -1, 0.0), ("T", 11, -1, 0.0)] + ops
    cuts3 = [(q, a + 2) for q, a in cuts]
    qubits = [10, 11, 14, 15, 20]
    t = chp.Tableau(n)
    for k, a, b, _ in ops:
        t.gate(k, a, b)
    ref = t.exact(qubits)
    assert np.abs(C.marginal(n, ops, cuts, qubits) - ref).max() <= 1e-12
    assert np.abs(C.marginal(n, ops3, cuts3, qubits) - ref).max() <= 1e-12


def test_sampled_is_normalised_and_unbiased():
    w = W.tiny()
    exact = C.marginal(w.n, w.ops, w.cuts, w.qubits)
    shots, seeds = 400, 60
    acc = np.zeros_like(exact)
    runs = []
    for s in range(seeds):
        R = C.marginal(w.n, w.ops, w.cuts, w.qubits, shots=shots, seed=s)
        assert np.isclose(R.sum(), 1.0, atol=1e-12)
        runs.append(R)
    runs = np.array(runs)
    mean = runs.mean(axis=0)
    se = runs.std(axis=0, ddof=1) / np.sqrt(seeds)
    assert np.all(np.abs(mean - exact) <= 4 * se + 1e-12)


def test_sampled_z_strings_unbiased():
    w = W.tiny()
    exact = C.zexpect(w.n, w.ops, w.cuts, w.zmasks)
    runs = np.array([C.zexpect(w.n, w.ops, w.cuts, w.zmasks, shots=300, seed=s) for s in range(40)])
    se = runs.std(axis=0, ddof=1) / np.sqrt(len(runs))
    assert np.all(np.abs(runs.mean(axis=0) - exact) <= 4 * se + 1e-12)


# ------------------------------------------- Clifford-specific optimisations

def test_support_terms_are_the_nonzero_terms_and_sparse_sum_equals_dense():
    # brute force: every term outside the support is an all-zero vector, and
    # the support sum equals the full ascending sum bit for bit (the skipped
    # terms are exact zeros)
    for seed in range(8):
        rng = np.random.default_rng(100 + seed)
        n = int(rng.integers(3, 7))
        kinds = W.CLIFFORD_KINDS if seed % 2 else W.ALL_KINDS
        ops = W.random_circuit(n, int(rng.integers(10, 30)), seed, kinds=kinds)
        cuts = W.random_cuts(n, ops, int(rng.integers(1, 4)), seed)
        qubits = list(range(n))
        R, parts = C.marginal(n, ops, cuts, qubits, return_parts=True)
        frags, reqs, tens, k = parts["frags"], parts["reqs"], parts["tensors"], len(cuts)
        sup = set(C.support(frags, tens, k))
        for P in range(4 ** k):
            tv = M.term_vector(frags, parts["reqs"], tens, k, P, n)
            assert (P in sup) == bool(np.any(tv != 0.0)), P
        Rs = C.marginal(n, ops, cuts, qubits, sparse=True)
        assert np.array_equal(Rs, R)
        assert np.abs(Rs - sv.uncut_marginal(n, ops, qubits)).max() <= 1e-12


def test_stabilizer_state_on_a_cut_vanishes_in_two_paulis():
    # H, cut, H on one wire: the cut carries |+>, so <Y> = <Z> = 0 upstream
    # (a one-qubit stabilizer state sits on a vertex of the Bloch
    # octahedron), and downstream H maps the Y and Z preparations to
    # uniform outcomes; the support keeps only I and X of the 4 terms
    ops = [("H", 0, -1, 0.0), ("H", 0, -1, 0.0)]
    cuts = [(0, 0)]
    R, parts = C.marginal(1, ops, cuts, [0], return_parts=True)
    up, dn = parts["tensors"]
    assert np.allclose(up, [[1.0, 1.0, 0.0, 0.0]]) and np.allclose(dn[:, 2:], 0.0)
    assert C.support(parts["frags"], parts["tensors"], 1) == [0, 1]  # I, X
    assert np.abs(R - np.array([1.0, 0.0])).max() <= 1e-12


def test_settled_shots_give_exact_clifford_expectations():
    # all-Clifford circuits: with settlement a few dozen shots per variant
    # reproduce the exact expectations (a string with a random parity shows
    # both values unless all 48 shots agree, probability 2^-47), without it
    # the estimate carries sampling noise
    for seed in range(4):
        rng = np.random.default_rng(200 + seed)
        n = int(rng.integers(3, 7))
        ops = W.random_circuit(n, int(rng.integers(12, 30)), seed, kinds=W.CLIFFORD_KINDS)
        cuts = W.random_cuts(n, ops, 2, seed)
        masks = [int(m) for m in rng.integers(1, 1 << n, size=8)]
        exact = C.zexpect(n, ops, cuts, masks)
        settled = C.zexpect(n, ops, cuts, masks, shots=48, seed=seed, settle=True)
        assert np.array_equal(settled, exact)
        zr = [sv.z_expectation(sv.probabilities(sv.run(n, ops)), n, m) for m in masks]
        assert np.abs(settled - zr).max() <= 1e-12
    raw = C.zexpect(n, ops, cuts, masks, shots=48, seed=1)
    assert not np.allclose(raw, exact, atol=1e-3) or np.all(np.abs(exact) == 1)


def test_validation_errors():
    ops = [("H", 0, -1, 0.0), ("CX", 0, 1, 0.0)]
    with pytest.raises(C.CutError):
        C.fragment_circuit(2, ops, [(1, 0)])          # op 0 is not on qubit 1
    with pytest.raises(C.CutError):
        C.fragment_circuit(2, ops, [(0, 0), (0, 0)])  # duplicate
    with pytest.raises(C.CutError):
        C.fragment_circuit(2, [("CX", 1, 1, 0.0)], [])
    with pytest.raises(C.CutError):
        C.fragment_circuit(2, [("FOO", 0, -1, 0.0)], [])


# ---------------------------------------------------------- planted mistakes

def _two_block_case(seed):
    """Random non-Clifford circuit on wires 0-2, a cut on wire 2, then a
    random non-Clifford circuit on wires 2-4: both fragments are generic, so
    every Pauli column of the cut is populated."""
    a = W.random_circuit(3, 16, 800 + seed)
    a.append(("T", 2, -1, 0.0))
    b = [(k, q0 + 2, (q1 + 2) if q1 >= 0 else -1, th)
         for k, q0, q1, th in W.random_circuit(3, 16, 850 + seed)]
    ops = a + b
    return 5, ops, [(2, len(a) - 1)], list(range(5))


def _pin_error():
    """Largest error of the oracle over the tiny config, the textbook cases,
    two-block circuits and small random circuits with random cuts."""
    cases = []
    w = W.tiny()
    cases.append((w.n, w.ops, w.cuts, w.qubits, sv.uncut_marginal(w.n, w.ops, w.qubits)))
    for name, n, ops, cuts, qubits, expect in _golden():
        cases.append((n, ops, cuts, qubits, expect))
    for seed in range(4):
        n, ops, cuts, qubits = _two_block_case(seed)
        cases.append((n, ops, cuts, qubits, sv.uncut_marginal(n, ops, qubits)))
        n = 4
        ops = W.random_circuit(n, 18, 700 + seed)
        cases.append((n, ops, W.random_cuts(n, ops, 2, 700 + seed), list(range(n)),
                      sv.uncut_marginal(n, ops, list(range(n)))))
    err = 0.0
    for n, ops, cuts, qubits, ref in cases:
        err = max(err, np.abs(C.marginal(n, ops, cuts, qubits) - ref).max())
    return err


@pytest.mark.parametrize("mutation", ["prep_sign", "prep_x", "prep_plus_i", "basis_y",
                                      "i_term", "cut_scale", "p_index"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    assert _pin_error() <= 1e-12
    if mutation == "prep_sign":
        bad = C.PREP_COEF.copy()
        bad[3, 1] = 1.0                      # Z = p0 + p1 (dropped sign)
        monkeypatch.setattr(C, "PREP_COEF", bad)
    elif mutation == "prep_x":
        bad = C.PREP_COEF.copy()
        bad[1, 2] = 1.0                      # X = p+ - p0 - p1 (dropped factor 2)
        monkeypatch.setattr(C, "PREP_COEF", bad)
    elif mutation == "prep_plus_i":
        monkeypatch.setattr(C, "PREP_OPS", {0: [], 1: ["X"], 2: ["H"], 3: ["H", "SDG"]})
    elif mutation == "basis_y":
        monkeypatch.setattr(C, "BASIS_OPS", {0: ["H"], 1: ["S", "H"], 2: []})
    elif mutation == "i_term":
        monkeypatch.setattr(C, "BASIS_Z", C.BASIS_X)   # I and Z terms from the X variant
    elif mutation == "cut_scale":
        orig = C.recombine
        monkeypatch.setattr(C, "recombine", lambda *a, **kw: orig(*a, **kw) * 2.0)
    elif mutation == "p_index":
        monkeypatch.setattr(C.Fragment, "p_index",
                            lambda self, P: sum(((P >> (2 * a.cut)) & 3) << (2 * (len(self.axes) - 1 - j))
                                                for j, a in enumerate(self.axes)))
    assert _pin_error() > 1e-3
