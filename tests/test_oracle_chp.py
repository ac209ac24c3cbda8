"""Pins for the literal CHP tableau and the elimination-based stabilizer
statistics: against the brute-force state vector, the tableau's symplectic
invariants, and each other."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import chp, stabilizer as stab, statevector as sv

CLIFF = ["H", "S", "SDG", "X", "Y", "Z", "CX", "CZ"]


def _tab(n, ops):
    t = chp.Tableau(n)
    for k, a, b, _ in ops:
        t.gate(k, a, b)
    return t


def _symplectic_ok(x, z, n):
    M = np.concatenate([x[:2 * n], z[:2 * n]], axis=1).astype(np.int64)
    J = np.zeros((2 * n, 2 * n), np.int64)
    J[:n, n:] = np.eye(n, dtype=np.int64)
    J[n:, :n] = np.eye(n, dtype=np.int64)
    G = (M @ J @ M.T) % 2
    return np.array_equal(G, J)


def _rows_stabilize(t, psi, n):
    x, z, r = t.dump()
    for i in range(n, 2 * n):
        P = stab.pauli_matrix(x[i], z[i], r[i])
        if not np.allclose(P @ psi, psi, atol=1e-10):
            return False
    return True


def test_exhaustive_two_qubit_depth4_against_state_vector():
    alphabet = [("H", 0, -1), ("H", 1, -1), ("S", 0, -1), ("S", 1, -1), ("CX", 0, 1), ("CX", 1, 0)]
    for depth in range(0, 5):
        for seq in itertools.product(alphabet, repeat=depth):
            ops = [(k, a, b, 0.0) for k, a, b in seq]
            psi = sv.run(2, ops)
            t = _tab(2, ops)
            assert np.allclose(t.exact([0, 1]), sv.probabilities(psi), atol=1e-12), seq
            assert _rows_stabilize(t, psi, 2), seq


@pytest.mark.parametrize("seed", range(40))
def test_random_cliffords_all_kinds(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 6))
    ops = W.random_circuit(n, int(rng.integers(1, 30)), seed, kinds=CLIFF)
    psi = sv.run(n, ops)
    t = chp.Tableau(n)
    for op in ops:
        t.gate(op[0], op[1], op[2])
        x, z, _ = t.dump()
        assert _symplectic_ok(x, z, n)
    assert _rows_stabilize(t, psi, n)
    meas = list(rng.permutation(n)[: int(rng.integers(1, n + 1))])
    ref = sv.marginal(sv.probabilities(psi), n, meas)
    assert np.allclose(t.exact(meas), ref, atol=1e-12)
    x, z, r = t.dump()
    el = stab.distribution(x[n:2 * n], z[n:2 * n], r[n:2 * n], meas)
    assert np.allclose(el, ref, atol=1e-12)
    # dyadic values on an affine support that sums to one
    nz = ref[ref > 1e-12]
    assert np.isclose(nz.sum(), 1.0)
    assert np.allclose(nz, nz[0]) and np.isclose(np.log2(1 / nz[0]) % 1, 0)
    assert (nz.size & (nz.size - 1)) == 0


@pytest.mark.parametrize("seed", range(12))
def test_z_expectations_are_minus_one_zero_or_one(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 7))
    ops = W.random_circuit(n, 25, 100 + seed, kinds=CLIFF)
    psi = sv.run(n, ops)
    p = sv.probabilities(psi)
    t = _tab(n, ops)
    x, z, r = t.dump()
    for mask in range(1, 1 << n):
        supp = [q for q in range(n) if (mask >> q) & 1]
        e = stab.z_expectation(x[n:2 * n], z[n:2 * n], r[n:2 * n], supp)
        assert e in (-1, 0, 1)
        assert np.isclose(e, sv.z_expectation(p, n, mask), atol=1e-12)


def test_measurement_collapses_like_projection():
    rng = np.random.default_rng(7)
    for trial in range(30):
        n = int(rng.integers(2, 6))
        ops = W.random_circuit(n, 20, 500 + trial, kinds=CLIFF)
        psi = sv.run(n, ops)
        t = _tab(n, ops)
        a = int(rng.integers(n))
        bit = int(rng.integers(2))
        o, rnd = t.measure(a, bit)
        idx = np.arange(1 << n)
        proj = np.where(((idx >> a) & 1) == o, psi, 0)
        pr = np.vdot(proj, proj).real
        assert pr > 1e-12
        if rnd:
            assert np.isclose(pr, 0.5) and o == bit
        else:
            assert np.isclose(pr, 1.0)
        assert _rows_stabilize(t, proj / np.sqrt(pr), n)


def test_sampled_histogram_matches_exact_and_random_bits_are_fair():
    n = 5
    ops = W.random_circuit(n, 40, 321, kinds=CLIFF)
    t = _tab(n, ops)
    meas = [0, 1, 2, 3, 4]
    exact = t.exact(meas)
    shots = 20000
    h = t.sample_hist(meas, seed=11, vid=5, nshots=shots).astype(float)
    assert h.sum() == shots
    assert np.all(h[exact == 0] == 0)
    exp = exact[exact > 0] * shots
    chi2 = ((h[exact > 0] - exp) ** 2 / exp).sum()
    dof = int((exact > 0).sum()) - 1
    # chi-square with dof degrees of freedom: mean dof, sd sqrt(2 dof)
    assert chi2 < dof + 6 * np.sqrt(2 * max(dof, 1))
    rec = t.sample(meas, seed=11, vid=5, shot0=0, nshots=shots)
    first_random = [j for j in range(n) if t.clone().is_random(meas[j])][:1]
    for j in first_random:
        assert abs(rec[:, j].mean() - 0.5) < 4 * 0.5 / np.sqrt(shots)


def test_per_shot_sampling_is_a_pure_function_of_the_key():
    n = 4
    ops = W.random_circuit(n, 30, 99, kinds=CLIFF)
    t = _tab(n, ops)
    a = t.sample([0, 1, 2, 3], seed=3, vid=9, shot0=0, nshots=64)
    b = t.sample([0, 1, 2, 3], seed=3, vid=9, shot0=16, nshots=16)
    assert np.array_equal(a[16:32], b)
    c = t.sample([0, 1, 2, 3], seed=4, vid=9, shot0=0, nshots=64)
    assert not np.array_equal(a, c) or t.exact([0, 1, 2, 3]).max() == 1.0


def test_many_string_expectations_match_single():
    rng = np.random.default_rng(77)
    for trial in range(6):
        n = int(rng.integers(3, 9))
        ops = W.random_circuit(n, 30, 900 + trial, kinds=CLIFF)
        t = _tab(n, ops)
        x, z, r = t.dump()
        masks = [int(m) for m in rng.integers(1, 1 << n, size=20)]
        many = stab.z_expectations(x[n:2 * n], z[n:2 * n], r[n:2 * n], masks, n)
        for mk, e in zip(masks, many):
            supp = [q for q in range(n) if (mk >> q) & 1]
            assert e == stab.z_expectation(x[n:2 * n], z[n:2 * n], r[n:2 * n], supp)
