"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on
the same seeded inputs.

Bars: shot records and exact Clifford tables bit-exact (integer / dyadic
work); floating results within 1e-10 of the fp64 oracle.
"""
import sys

import numpy as np
import pytest

import paper_2303_10788_amd as cc
import workloads as W
from oracle import cutting as C, philox as PX, statevector as sv

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_10788_amd as cc
    return cc.Context()


def _plan(ctx, n, ops, cuts):
    import paper_2303_10788_amd as cc
    return cc.Plan(ctx, n, ops, cuts)


def _pack(rec_u8):
    out = np.zeros(rec_u8.shape[0], dtype=np.uint64)
    for j in range(rec_u8.shape[1]):
        out |= rec_u8[:, j].astype(np.uint64) << np.uint64(j)
    return out


def _oracle_records(n, ops, cuts, qubits, f, v, seed, shots, circuit=0):
    frag = C.fragment_circuit(n, ops, cuts)[f]
    req = C.make_request(frag, qubits)
    t = C.clifford_tableau(frag, v)
    vid = PX.variant_id(circuit, f, v)
    return _pack(t.sample(req.meas, seed, vid, 0, shots))


# ------------------------------------------------------------ shot records

@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_shot_records_bit_exact_configs(ctx, name):
    w = W.tiny() if name == "tiny" else W.mid()
    _log(f"shot records {name}")
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    f = [i for i, fr in enumerate(frags) if fr.clifford][0]
    shots = 1027  # ragged: not a multiple of 4 or of a workgroup
    for qubits in (w.qubits, list(range(w.n))):
        nv = frags[f].n_variants
        got = plan.shot_records(qubits, f, 0, nv, shots=shots, seed=w.seed + 7)
        for v in range(nv):
            exp = _oracle_records(w.n, w.ops, w.cuts, qubits, f, v, w.seed + 7, shots)
            assert np.array_equal(got[v], exp), (name, v)


@pytest.mark.parametrize("m", [3, 40, 64, 65, 130, 200, 260])
def test_shot_records_bit_exact_widths(ctx, m):
    """Random Clifford fragments across row-word counts (W = 1, 2, 4, 8)
    and measured sets up to 64 qubits, with preparations and rotations from
    a cut on each side."""
    _log(f"shot records width {m}")
    rng = np.random.default_rng(500 + m)
    ops = W.random_circuit(m, 6 * m, 500 + m, kinds=["H", "S", "SDG", "X", "Y", "Z", "CX", "CZ"])
    # an H on wire 0 cut right after it: a one-qubit upstream fragment (a
    # quantum output) and the rest downstream of it (a quantum input)
    ops = [("H", 0, -1, 0.0)] + ops
    cuts = [(0, 0)]
    plan = _plan(ctx, m, ops, cuts)
    frags = C.fragment_circuit(m, ops, cuts)
    nmeas = min(m, 64)
    qubits = sorted(int(q) for q in rng.choice(m, size=min(nmeas - 1, m), replace=False))
    shots = 203 if m <= 64 else 21
    for f, fr in enumerate(frags):
        if not fr.clifford:
            continue
        req = C.make_request(fr, qubits)
        if len(req.meas) > 64:
            continue
        nv = fr.n_variants
        got = plan.shot_records(qubits, f, 0, nv, shots=shots, seed=99)
        for v in range(nv):
            exp = _oracle_records(m, ops, cuts, qubits, f, v, 99, shots)
            assert np.array_equal(got[v], exp), (m, f, v)


def test_shot_records_circuit_index_and_subrange(ctx):
    w = W.tiny()
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    got = plan.shot_records(w.qubits, 1, 2, 4, shots=64, seed=3, circuit=5)
    for i, v in enumerate((2, 3)):
        exp = _oracle_records(w.n, w.ops, w.cuts, w.qubits, 1, v, 3, 64, circuit=5)
        assert np.array_equal(got[i], exp)


# ------------------------------------------------------------ variant tables

@pytest.mark.parametrize("seed", range(12))
def test_variant_tables_random(ctx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 9))
    ops = W.random_circuit(n, int(rng.integers(4, 40)), 300 + seed)
    k = int(rng.integers(1, min(3, len(ops)) + 1))
    cuts = W.random_cuts(n, ops, k, 300 + seed)
    qubits = [int(q) for q in rng.permutation(n)[: int(rng.integers(0, n + 1))]]
    _log(f"variant tables seed={seed} n={n} k={k}")
    plan = _plan(ctx, n, ops, cuts)
    frags = C.fragment_circuit(n, ops, cuts)
    for f, fr in enumerate(frags):
        req = C.make_request(fr, qubits)
        exp = C.variant_distributions(fr, req.meas)
        got = plan.variant_tables(qubits, f)
        if fr.clifford:
            assert np.array_equal(got, exp), (seed, f)   # dyadic: bit-exact
        else:
            assert np.abs(got - exp).max() <= 1e-12, (seed, f)
        Te = C.pauli_tensor(fr, req, exp).T
        for method in (cc.CCUT_METHOD_AUTO, cc.CCUT_METHOD_VARIANTS):
            Tg = plan.fragment_tensor(qubits, f, method=method)
            if fr.clifford:
                assert np.array_equal(Tg, Te), (seed, f, method)   # dyadic either way
            else:
                assert np.abs(Tg - Te).max() <= 1e-12, (seed, f, method)


@pytest.mark.parametrize("m,mirrored", [(m, mir) for m in (5, 6, 7, 8, 9, 10, 11, 12) for mir in (False, True)])
def test_variant_tables_wide_nc(ctx, m, mirrored):
    """Non-Clifford fragments of every register/lane/wave layout (5 to 12
    qubits; from 9 qubits on some qubits sit on wave bits and are swapped
    in), with the cut wires as quantum outputs or, mirrored, as inputs."""
    n = m + 5
    exits = [1, m - 1] if m > 2 else [m - 1]
    blocks = [W.Block(list(range(m)), exits)]
    ops, cuts = W.block_circuit(n, 30, blocks, t_c=15, p_cx=0.4, seed=700 + m, n_t=5, mirrored=mirrored)
    qubits = [0, 2, m - 2, m, n - 1] if m > 3 else [0, m, n - 1]
    qubits = sorted(set(q for q in qubits if q < n))
    _log(f"wide NC m={m} mirrored={mirrored}")
    plan = _plan(ctx, n, ops, cuts)
    frags = C.fragment_circuit(n, ops, cuts)
    seen = 0
    for f, fr in enumerate(frags):
        if fr.clifford:
            continue
        seen = max(seen, fr.m)
        req = C.make_request(fr, qubits)
        exp = C.variant_distributions(fr, req.meas)
        got = plan.variant_tables(qubits, f)
        assert np.abs(got - exp).max() <= 1e-12, (m, mirrored, f)
    assert seen == m


# ------------------------------------------------------------ marginals

def test_tiny_exact_marginal(ctx):
    w = W.tiny()
    _log("tiny exact marginal")
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    got = plan.marginal(w.qubits)
    exp = C.marginal(w.n, w.ops, w.cuts, w.qubits)
    ref = sv.uncut_marginal(w.n, w.ops, w.qubits)
    assert np.abs(got - exp).max() <= TOL
    assert np.abs(got - ref).max() <= TOL


@pytest.mark.parametrize("shots", [1, 5, 1000, 4099])
def test_tiny_sampled_marginal(ctx, shots):
    w = W.tiny()
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    got = plan.marginal(w.qubits, shots=shots, seed=11)
    exp = C.marginal(w.n, w.ops, w.cuts, w.qubits, shots=shots, seed=11)
    assert np.abs(got - exp).max() <= TOL
    assert abs(got.sum() - 1.0) <= 1e-12


@pytest.mark.parametrize("seed", range(16))
def test_random_marginals(ctx, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 9))
    ops = W.random_circuit(n, int(rng.integers(4, 40)), 1000 + seed)
    k = int(rng.integers(1, min(3, len(ops)) + 1))
    cuts = W.random_cuts(n, ops, k, 1000 + seed)
    qubits = [int(q) for q in rng.permutation(n)[: int(rng.integers(1, n + 1))]]
    _log(f"random marginal seed={seed} n={n} k={k}")
    plan = _plan(ctx, n, ops, cuts)
    got = plan.marginal(qubits)
    exp = C.marginal(n, ops, cuts, qubits)
    assert np.abs(got - exp).max() <= TOL
    assert np.abs(got - sv.uncut_marginal(n, ops, qubits)).max() <= TOL
    gv = plan.marginal(qubits, method=cc.CCUT_METHOD_VARIANTS)
    assert np.abs(gv - exp).max() <= TOL
    gs = plan.marginal(qubits, shots=257, seed=seed)
    es = C.marginal(n, ops, cuts, qubits, shots=257, seed=seed)
    assert np.abs(gs - es).max() <= TOL


def test_mid_exact_marginal_and_sampled_small(ctx):
    w = W.mid()
    _log("mid exact + sampled (2000 shots)")
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    got = plan.marginal(w.qubits)
    exp = C.marginal(w.n, w.ops, w.cuts, w.qubits)
    assert np.abs(got - exp).max() <= TOL
    assert np.abs(plan.marginal(w.qubits, method=cc.CCUT_METHOD_VARIANTS) - exp).max() <= TOL
    gs = plan.marginal(w.qubits, shots=2000, seed=w.seed)
    es = C.marginal(w.n, w.ops, w.cuts, w.qubits, shots=2000, seed=w.seed)
    assert np.abs(gs - es).max() <= TOL


def test_mid_full_size_sampled(ctx):
    """Full size (1e5 shots per variant): sampled shot records against the
    oracle's per-shot tableau at spot indices, normalisation, and closeness
    to the exact answer."""
    w = W.mid()
    _log("mid full-size sampled")
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    got = plan.marginal(w.qubits, shots=w.shots, seed=w.seed)
    assert abs(got.sum() - 1.0) <= 1e-12
    exact = plan.marginal(w.qubits)
    tvd = 0.5 * np.abs(got - exact).sum()
    assert tvd < 0.25
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    f = [i for i, fr in enumerate(frags) if fr.clifford][0]
    rec = plan.shot_records(w.qubits, f, 0, frags[f].n_variants, shots=w.shots, seed=w.seed)
    for v in (0, 7, 15):
        exp = _oracle_records(w.n, w.ops, w.cuts, w.qubits, f, v, w.seed, 600)
        assert np.array_equal(rec[v, :600], exp)
    # the histograms behind the estimate are the records' counts (a table
    # entry is count x fl(1/shots))
    tab = plan.variant_tables(w.qubits, f, shots=w.shots, seed=w.seed)
    for v in (0, 15):
        counts = np.bincount(rec[v].astype(np.int64), minlength=tab.shape[1])
        assert np.array_equal(counts * (1.0 / w.shots), tab[v])


# ------------------------------------------------------------ Z strings

def test_tiny_zexpect(ctx):
    w = W.tiny()
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    masks = W.Workload.zmask_words(w)
    got = plan.zexpect(masks)
    exp = C.zexpect(w.n, w.ops, w.cuts, w.zmasks)
    assert np.abs(got - exp).max() <= TOL
    gs = plan.zexpect(masks, shots=513, seed=4)
    es = C.zexpect(w.n, w.ops, w.cuts, w.zmasks, shots=513, seed=4)
    assert np.abs(gs - es).max() <= TOL


def test_mid_zexpect(ctx):
    w = W.mid()
    _log("mid zexpect exact + sampled(300)")
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    masks = w.zmask_words()
    got = plan.zexpect(masks)
    exp = C.zexpect(w.n, w.ops, w.cuts, w.zmasks)
    assert np.abs(got - exp).max() <= TOL
    assert np.abs(plan.zexpect(masks, method=cc.CCUT_METHOD_VARIANTS) - exp).max() <= TOL
    gs = plan.zexpect(masks, shots=300, seed=w.seed)
    es = C.zexpect(w.n, w.ops, w.cuts, w.zmasks, shots=300, seed=w.seed)
    assert np.abs(gs - es).max() <= TOL


@pytest.mark.parametrize("seed", range(8))
def test_random_zexpect(ctx, seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(2, 8))
    ops = W.random_circuit(n, int(rng.integers(4, 30)), 2000 + seed)
    k = int(rng.integers(1, min(3, len(ops)) + 1))
    cuts = W.random_cuts(n, ops, k, 2000 + seed)
    masks = [int(m) for m in rng.integers(1, 1 << n, size=7)]
    plan = _plan(ctx, n, ops, cuts)
    words = np.array([[m] for m in masks], dtype=np.uint64)
    got = plan.zexpect(words)
    exp = C.zexpect(n, ops, cuts, masks)
    assert np.abs(got - exp).max() <= TOL
    gs = plan.zexpect(words, shots=101, seed=seed)
    es = C.zexpect(n, ops, cuts, masks, shots=101, seed=seed)
    assert np.abs(gs - es).max() <= TOL


# ------------------------------------------------------------ edge cases

def test_edge_cases(ctx):
    # empty request: one entry, the total probability
    w = W.tiny()
    plan = _plan(ctx, w.n, w.ops, w.cuts)
    assert np.allclose(plan.marginal([]), [1.0])
    # no cuts at all
    ops = W.random_circuit(5, 30, 4)
    p0 = _plan(ctx, 5, ops, [])
    assert np.abs(p0.marginal([0, 1, 2, 3, 4]) - sv.uncut_marginal(5, ops, [0, 1, 2, 3, 4])).max() <= TOL
    # a cut after the last op of a wire, two cuts on one wire, both sides in one fragment
    ops = [("H", 0, -1, 0.0), ("CX", 0, 1, 0.0), ("T", 1, -1, 0.0), ("CX", 1, 0, 0.0), ("H", 1, -1, 0.0),
           ("CX", 0, 2, 0.0), ("S", 2, -1, 0.0)]
    cuts = [(2, 6), (0, 1), (0, 3), (1, 2)]
    p = _plan(ctx, 3, ops, cuts)
    got = p.marginal([2, 0, 1])
    assert np.abs(got - C.marginal(3, ops, cuts, [2, 0, 1])).max() <= TOL
    assert np.abs(got - sv.uncut_marginal(3, ops, [2, 0, 1])).max() <= TOL
    # invalid requests
    import paper_2303_10788_amd as cc
    with pytest.raises(cc.CcutError) as e:
        plan.marginal([0, 0])
    assert e.value.status == cc.CCUT_E_INVALID
    with pytest.raises(cc.CcutError) as e:
        plan.marginal([9])
    assert e.value.status == cc.CCUT_E_INVALID
