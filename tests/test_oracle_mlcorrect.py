"""Pins of the maximum-likelihood fragment correction oracle (Sec. V-C,
distribution builder; the reading is stated in oracle/mlcorrect.py): the
simplex projection against closed forms and a generic constrained
minimiser, the one-qubit Bloch-ball closed form, a two-block hand example,
the fixed point on exact data, physicality, idempotence, optimality
against random physical models, and planted mistakes that must fail."""
import itertools

import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as W
from oracle import cutting as C
from oracle import mlcorrect as ML

CLIFF = ("H", "S", "SDG", "X", "Y", "Z", "CX", "CZ")


def test_simplex_projection_closed_forms():
    assert np.allclose(ML.simplex_projection([0.7, 0.5, -0.2]), [0.6, 0.4, 0.0], atol=1e-15)
    assert np.allclose(ML.simplex_projection([0.5, 0.5, 0.5]), [1 / 3] * 3, atol=1e-15)
    assert np.allclose(ML.simplex_projection([2.0, 0.0, 0.0]), [1.0, 0.0, 0.0], atol=1e-15)
    on = np.array([0.1, 0.2, 0.3, 0.4])
    assert np.allclose(ML.simplex_projection(on), on, atol=1e-15)
    assert np.allclose(ML.simplex_projection([0.25, -0.5, 0.25, 0.25]), [1 / 3, 0, 1 / 3, 1 / 3], atol=1e-15)


@pytest.mark.parametrize("seed", range(12))
def test_simplex_projection_matches_constrained_minimiser(seed):
    rng = np.random.default_rng(seed)
    mu = rng.normal(0.25, 0.6, size=int(rng.integers(2, 9)))
    got = ML.simplex_projection(mu)
    res = minimize(lambda l: np.sum((l - mu) ** 2), np.full(len(mu), 1.0 / len(mu)),
                   jac=lambda l: 2 * (l - mu), method="SLSQP",
                   bounds=[(0, None)] * len(mu), constraints=[{"type": "eq", "fun": lambda l: l.sum() - 1}],
                   options={"ftol": 1e-15, "maxiter": 500})
    assert res.success
    assert np.allclose(got, res.x, atol=1e-6)
    assert np.all(got >= 0) and abs(got.sum() - 1) < 1e-12


def _bloch_block(r):
    # p[b][o][x=0] = (1 + (-1)^o r_b) / 2 for the bases X, Y, Z
    return np.array([[[(1 + r[b]) / 2], [(1 - r[b]) / 2]] for b in range(3)])


@pytest.mark.parametrize("r", [(0.3, -0.2, 0.5), (0.0, 0.0, 1.0), (0.9, 0.6, -0.3), (1.2, 0.0, 0.0),
                               (-0.7, 0.8, 0.6)])
def test_one_qubit_bloch_ball(r):
    """One quantum output, no classical outcome: rho = (I + r.sigma)/2 is
    physical iff |r| <= 1; outside the ball the nearest physical state is
    the pure state r/|r| (eigenvalues (1 +- |r|)/2 -> 1, 0)."""
    r = np.array(r)
    q = ML.correct_block(_bloch_block(r))
    got = np.array([q[b, 0, 0] - q[b, 1, 0] for b in range(3)])
    want = r if np.linalg.norm(r) <= 1 else r / np.linalg.norm(r)
    assert np.allclose(got, want, atol=1e-12)
    assert np.allclose(q[:, 0, 0] + q[:, 1, 0], 1.0, atol=1e-12)


def test_two_block_hand_example():
    """rho_0 = diag(0.7, -0.1), rho_1 = diag(0.3, 0.1): the joint spectrum
    [0.7, 0.3, 0.1, -0.1] projects with tau = 1/30 to
    [0.7 - 1/30, 0.3 - 1/30, 0.1 - 1/30, 0]."""
    diag = {0: (0.7, -0.1), 1: (0.3, 0.1)}
    p = np.zeros((3, 2, 2))
    for x, (a, b) in diag.items():
        p[2, 0, x], p[2, 1, x] = a, b                  # Z basis: the diagonal
        for bb in (0, 1):                              # X, Y bases: half the trace each
            p[bb, 0, x] = p[bb, 1, x] = (a + b) / 2
    q = ML.correct_block(p)
    t = 1 / 30
    want = {0: (0.7 - t, 0.0), 1: (0.3 - t, 0.1 - t)}
    for x, (a, b) in want.items():
        assert np.allclose([q[2, 0, x], q[2, 1, x]], [a, b], atol=1e-12)
        for bb in (0, 1):
            assert np.allclose([q[bb, 0, x], q[bb, 1, x]], [(a + b) / 2] * 2, atol=1e-12)


def _cut_cases():
    """Circuits whose fragments have one or two quantum outputs: tiny (a
    non-Clifford upstream fragment) and random Clifford circuits."""
    out = []
    w = W.tiny()
    out.append((w.n, w.ops, w.cuts, [0, 1, 5]))
    for seed in range(4):
        n = 4
        ops = W.random_circuit(n, 22, 100 + seed, kinds=CLIFF)
        cuts = W.random_cuts(n, ops, 2, 100 + seed)
        out.append((n, ops, cuts, [0, 2, 3]))
    return out


def _frags_with_outputs(n, ops, cuts, qubits):
    frags = C.fragment_circuit(n, ops, cuts)
    reqs = [C.make_request(f, qubits) for f in frags]
    return [(f, r) for f, r in zip(frags, reqs) if any(a.side == 0 for a in f.axes)
            and sum(a.side == 0 for a in f.axes) <= 2]


@pytest.mark.parametrize("case", range(5))
def test_fixed_point_on_exact_tables(case):
    """Exact variant data is a physical model already: the correction leaves
    it unchanged."""
    n, ops, cuts, qubits = _cut_cases()[case]
    pairs = _frags_with_outputs(n, ops, cuts, qubits)
    assert pairs
    for f, r in pairs:
        d = C.variant_distributions(f, r.meas)
        assert np.allclose(ML.correct_tables(f, r, d), d, atol=1e-12)


def _blocks(f, r, d):
    """Per preparation combination: the raw-state blocks of tables d."""
    outs = [j for j, a in enumerate(f.axes) if a.side == 0]
    ins = [j for j, a in enumerate(f.axes) if a.side == 1]
    n = len(outs)
    nx = 1 << len(r.req_pos)
    res = []
    for s in itertools.product(range(4), repeat=len(ins)):
        p = np.zeros((3 ** n, 1 << n, nx))
        for bi in range(3 ** n):
            dg = [0] * len(f.axes)
            for j, v in zip(ins, s):
                dg[j] = v
            for i, j in enumerate(outs):
                dg[j] = (bi // 3 ** i) % 3
            row = d[f.variant_index(dg)]
            for o in range(1 << n):
                for x in range(nx):
                    idx = 0
                    for i, j in enumerate(outs):
                        idx |= ((o >> i) & 1) << r.out_pos[j]
                    for i, q in enumerate(r.req_pos):
                        idx |= ((x >> i) & 1) << q
                    p[bi, o, x] = row[idx]
        res.append(p)
    return res


@pytest.mark.parametrize("case", range(1, 5))
def test_physical_and_idempotent_on_sampled_tables(case):
    n, ops, cuts, qubits = _cut_cases()[case]
    for f, r in _frags_with_outputs(n, ops, cuts, qubits):
        d = C.variant_distributions(f, r.meas, shots=40, seed=7)
        c = ML.correct_tables(f, r, d)
        for p in _blocks(f, r, c):
            rho = ML.raw_states(p)
            w = np.linalg.eigvalsh(rho)
            assert w.min() > -1e-12
            assert abs(np.trace(rho, axis1=1, axis2=2).real.sum() - 1) < 1e-12
        assert np.allclose(ML.correct_tables(f, r, c), c, atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_nearest_physical_model(seed):
    """The corrected model is at least as close (Frobenius) to the raw one as
    any random physical model of the same shape."""
    rng = np.random.default_rng(seed)
    n, nx = 1 + seed % 2, 3
    d = 1 << n
    p = rng.uniform(-0.1, 1.0, size=(3 ** n, d, nx))
    p /= p.sum(axis=(1, 2), keepdims=True)
    raw = ML.raw_states(p)
    best = np.linalg.norm(raw - ML.project_states(raw))
    for _ in range(200):
        A = rng.normal(size=(nx, d, d)) + 1j * rng.normal(size=(nx, d, d))
        S = A @ A.conj().transpose(0, 2, 1) * rng.uniform(0, 1, size=(nx, 1, 1))
        S /= np.trace(S, axis1=1, axis2=2).real.sum()
        assert best <= np.linalg.norm(raw - S) + 1e-12


def test_planted_mistakes_fail(monkeypatch):
    """Each plausible slip in the oracle breaks a pin.  (A relabelling used
    consistently on the way in and on the way out, such as a swapped pair
    of basis letters, cancels and is no slip.)"""
    n, ops, cuts, qubits = _cut_cases()[2]
    pairs = _frags_with_outputs(n, ops, cuts, qubits)
    tabs = [(f, r, C.variant_distributions(f, r.meas)) for f, r in pairs]

    def fixed():
        try:
            return all(np.allclose(ML.correct_tables(f, r, d), d, atol=1e-9) for f, r, d in tabs)
        except (IndexError, ValueError):  # a slip that leaves a Pauli unmeasured
            return False

    def hand():
        try:
            test_two_block_hand_example()
            return True
        except AssertionError:
            return False

    assert fixed() and hand()
    good = dict(ML.BASIS_PAULI)
    monkeypatch.setattr(ML, "BASIS_PAULI", {**good, C.BASIS_Y: C.X_})   # Y basis read as X
    assert not fixed()
    monkeypatch.setattr(ML, "BASIS_PAULI", good)
    eye = ML.SIGMA[C.I_]
    monkeypatch.setitem(ML.SIGMA, C.I_, 2 * eye)                         # lost 1/2 of the identity
    assert not fixed()
    monkeypatch.setitem(ML.SIGMA, C.I_, eye)
    monkeypatch.setattr(ML, "simplex_projection",                       # clip and renormalise
                        lambda mu: np.maximum(np.asarray(mu), 0) / np.maximum(np.asarray(mu), 0).sum())
    assert not hand()


def test_exact_marginal_unchanged_and_sampled_closer():
    """End to end: exact data gives the uncorrected marginal; on sampled
    data the corrected marginal's mean distance to the exact one over seeds
    is smaller (the correction removes unphysical sampling noise)."""
    n, ops, cuts, qubits = _cut_cases()[1]
    exact = C.marginal(n, ops, cuts, qubits)
    assert np.allclose(C.marginal(n, ops, cuts, qubits, ml=True), exact, atol=1e-12)
    raw = [np.abs(C.marginal(n, ops, cuts, qubits, shots=30, seed=s) - exact).sum() for s in range(12)]
    cor = [np.abs(C.marginal(n, ops, cuts, qubits, shots=30, seed=s, ml=True) - exact).sum() for s in range(12)]
    assert np.mean(cor) < np.mean(raw)
