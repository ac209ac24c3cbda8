"""Pins of the Sec. IX downstream-skipping oracle (fewer stitching
calculations: variants no supported cut term reads are never evaluated).

* Which variants a term reads is checked against the transform itself:
  perturbing one variant's table changes exactly the tensor columns that
  read it, so ``needed_variants`` must mark a variant iff some supported
  term's column changes.
* Exact data: the skipped sum equals the dense one and the uncut state
  vector (the terms outside the exact support vanish).
* Sampled data: the estimate does not depend on the skipped variants'
  tables at all, and it is the dense estimate restricted to the support.
* Planted mistakes in the read tables fail the perturbation pin."""
import numpy as np
import pytest

import workloads as W
from oracle import cutting as C
from oracle import statevector as SV

CLIFF = ("H", "S", "SDG", "X", "Y", "Z", "CX", "CZ")


def _cases(count=8):
    out = []
    for seed in range(60):
        n = 4 + seed % 4
        kinds = CLIFF if seed % 3 else C.KINDS
        ops = W.random_circuit(n, 8 + 3 * n, 500 + seed, kinds=tuple(sorted(kinds)))
        k = 1 + seed % 3
        cuts = W.random_cuts(n, ops, k, 500 + seed)
        frags = C.fragment_circuit(n, ops, cuts)
        if max(f.n_variants for f in frags) > 64:
            continue
        qubits = list(range(0, n, 1 + seed % 2))
        out.append((n, ops, cuts, qubits))
        if len(out) == count:
            break
    return out


def _changed_columns(f, r, d, v, rng):
    base = C.pauli_tensor(f, r, d)
    d2 = np.array(d, dtype=np.float64)
    d2[v] = d2[v] + rng.normal(size=d2.shape[1])
    pert = C.pauli_tensor(f, r, d2)
    return set(np.nonzero(np.any(pert != base, axis=0))[0].tolist())


@pytest.mark.parametrize("case", range(8))
def test_needed_variants_match_the_transform(case):
    n, ops, cuts, qubits = _cases()[case]
    frags = C.fragment_circuit(n, ops, cuts)
    reqs = [C.make_request(f, qubits) for f in frags]
    rng = np.random.default_rng(case)
    k = len(cuts)
    for trial in range(3):
        S = sorted(set(rng.integers(0, 4 ** k, size=max(1, 4 ** k // 3)).tolist()))
        for f, r in zip(frags, reqs):
            d = C.variant_distributions(f, r.meas)
            need = C.needed_variants(f, S)
            cols = {f.p_index(P) for P in S}
            for v in range(f.n_variants):
                reads = bool(_changed_columns(f, r, d, v, rng) & cols)
                assert need[v] == reads, (case, trial, f.index, v)


@pytest.mark.parametrize("case", range(8))
def test_exact_skip_equals_dense_and_uncut(case):
    n, ops, cuts, qubits = _cases()[case]
    got = C.marginal_skip(n, ops, cuts, qubits)
    dense = C.marginal(n, ops, cuts, qubits)
    assert np.abs(got - dense).max() <= 1e-12
    assert np.abs(got - SV.uncut_marginal(n, ops, qubits)).max() <= 1e-12


@pytest.mark.parametrize("case", range(8))
def test_sampled_skip_ignores_skipped_variants(case):
    n, ops, cuts, qubits = _cases()[case]
    R, parts = C.marginal_skip(n, ops, cuts, qubits, shots=300, seed=case, return_parts=True)
    frags, reqs, S = parts["frags"], parts["reqs"], parts["support"]
    rng = np.random.default_rng(100 + case)
    dense_dists = [C.variant_distributions(f, r.meas, shots=300, seed=case) for f, r in zip(frags, reqs)]
    garbage = []
    for f, d in zip(frags, dense_dists):
        g = np.array(d, dtype=np.float64)
        g[~C.needed_variants(f, S)] = rng.normal(size=(int((~C.needed_variants(f, S)).sum()), g.shape[1]))
        garbage.append(g)
    tensors = [C.pauli_tensor(f, r, g) for f, r, g in zip(frags, reqs, garbage)]
    alt = C.recombine(frags, reqs, tensors, len(cuts), len(qubits), terms=S)
    assert np.array_equal(alt, R)
    # the dense sampled estimate restricted to the support
    dense_t = [C.pauli_tensor(f, r, d) for f, r, d in zip(frags, reqs, dense_dists)]
    assert np.array_equal(C.recombine(frags, reqs, dense_t, len(cuts), len(qubits), terms=S), R)


def test_skipping_saves_variants_on_clifford_downstream():
    """A Clifford fragment downstream of an H-then-cut keeps only I and X on
    that cut (Sec. IX's Bloch-octahedron example): its |+i> preparation is
    never read."""
    ops = [("H", 0, -1, 0.0), ("CX", 0, 1, 0.0), ("H", 0, -1, 0.0), ("S", 1, -1, 0.0)]
    cuts = [(0, 0)]
    frags = C.fragment_circuit(2, ops, cuts)
    reqs = [C.make_request(f, [0, 1]) for f in frags]
    S = C.exact_support(frags, reqs, 1)
    assert set(S) <= {C.I_, C.X_, C.Z_}
    down = [f for f in frags if any(a.side == 1 for a in f.axes)][0]
    need = C.needed_variants(down, S)
    assert not need[down.variant_index([3])]
    assert np.abs(C.marginal_skip(2, ops, cuts, [0, 1]) - SV.uncut_marginal(2, ops, [0, 1])).max() <= 1e-12


@pytest.mark.parametrize("mistake", ["x_without_plus", "y_without_plus_i", "identity_from_x"])
def test_planted_mistakes_fail(monkeypatch, mistake):
    if mistake == "x_without_plus":
        monkeypatch.setitem(C.PREPS_READ, C.X_, (0, 1))
    elif mistake == "y_without_plus_i":
        monkeypatch.setitem(C.PREPS_READ, C.Y_, (0, 1, 2))
    else:
        monkeypatch.setitem(C.BASES_READ, C.I_, (C.BASIS_X,))
    failed = False
    for case in range(8):
        try:
            test_needed_variants_match_the_transform(case)
        except AssertionError:
            failed = True
            break
    assert failed, mistake
