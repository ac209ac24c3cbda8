"""Pins for the brute-force state vector: the paper's gate definitions and
textbook states."""
import numpy as np

from oracle import statevector as sv


def test_gate_definitions_from_the_paper():
    # Sec. II-A: Y = -i Z X ; Sec. II-C: H = (Z + X)/sqrt 2 ; T = Z^(1/4)
    assert np.allclose(sv.Y, np.array([[0, -1j], [1j, 0]]))
    assert np.allclose(sv.H @ sv.H, np.eye(2))
    assert np.allclose(sv.H, np.array([[1, 1], [1, -1]]) / np.sqrt(2))
    T4 = np.linalg.matrix_power(sv.T, 4)
    assert np.allclose(T4, sv.Z)
    assert np.allclose(sv.S, np.linalg.matrix_power(sv.T, 2))
    assert np.allclose(sv.rz(np.pi / 4), sv.T)


def test_bell_and_ghz():
    p = sv.probabilities(sv.run(2, [("H", 0, -1, 0.0), ("CX", 0, 1, 0.0)]))
    assert np.allclose(p, [0.5, 0, 0, 0.5])
    ops = [("H", 0, -1, 0.0)] + [("CX", i, i + 1, 0.0) for i in range(4)]
    p = sv.probabilities(sv.run(5, ops))
    assert np.isclose(p[0], 0.5) and np.isclose(p[31], 0.5) and np.isclose(p.sum(), 1)


def test_bit_order_is_little_endian():
    p = sv.probabilities(sv.run(3, [("X", 1, -1, 0.0)]))
    assert p[2] == 1.0
    m = sv.marginal(p, 3, [1, 0])
    assert m[1] == 1.0  # bit 0 of the marginal index = qubit 1


def test_t_plus_in_x_basis():
    p = sv.probabilities(sv.run(1, [("H", 0, -1, 0.0), ("T", 0, -1, 0.0), ("H", 0, -1, 0.0)]))
    assert np.isclose(p[0], (1 + np.cos(np.pi / 4)) / 2)


def test_cz_symmetric_and_equals_h_cx_h():
    rng = np.random.default_rng(0)
    psi = rng.normal(size=8) + 1j * rng.normal(size=8)
    psi /= np.linalg.norm(psi)
    a = sv.apply_op(psi, ("CZ", 0, 2, 0.0), 3)
    b = sv.apply_op(psi, ("CZ", 2, 0, 0.0), 3)
    c = sv.apply_1q(sv.apply_op(sv.apply_1q(psi, sv.H, 2, 3), ("CX", 0, 2, 0.0), 3), sv.H, 2, 3)
    assert np.allclose(a, b) and np.allclose(a, c)


def test_z_expectation_matches_parity_sum():
    ops = [("H", 0, -1, 0.0), ("CX", 0, 1, 0.0), ("T", 1, -1, 0.0), ("H", 1, -1, 0.0)]
    p = sv.probabilities(sv.run(2, ops))
    for mask in range(4):
        e = sum(p[x] * (-1) ** bin(x & mask).count("1") for x in range(4))
        assert np.isclose(sv.z_expectation(p, 2, mask), e)
