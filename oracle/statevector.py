"""Brute-force dense state vector in complex128 (the exact simulator the
paper uses for non-Clifford fragments and as its accuracy yardstick,
Secs. V-B and VI-A).

Basis index convention: bit q of the index is the value of qubit q.
Gate matrices follow the paper's definitions (Sec. II): Y = -i Z X,
H = (Z + X)/sqrt(2), T = Z^(1/4) = diag(1, e^{i pi/4}); RZ(theta) is
Z^(theta/pi) = diag(1, e^{i theta}), the arbitrary Z^a of Sec. VIII.
"""
from __future__ import annotations

import numpy as np

_I = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
Y = -1j * (Z @ X)
H = (Z + X) / np.sqrt(2.0)
S = np.diag([1.0, 1.0j]).astype(np.complex128)
SDG = S.conj().T
T = np.diag([1.0, np.exp(1j * np.pi / 4)]).astype(np.complex128)
TDG = T.conj().T


def rz(theta: float) -> np.ndarray:
    return np.diag([1.0, np.exp(1j * theta)]).astype(np.complex128)


ONE_Q = {"H": H, "S": S, "SDG": SDG, "X": X, "Y": Y, "Z": Z, "T": T, "TDG": TDG}


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply_1q(psi: np.ndarray, U: np.ndarray, q: int, n: int) -> np.ndarray:
    t = psi.reshape((2,) * n)
    ax = n - 1 - q  # C order: axis 0 is the most significant bit
    t = np.tensordot(U, t, axes=([1], [ax]))
    t = np.moveaxis(t, 0, ax)
    return np.ascontiguousarray(t).reshape(-1)


def apply_controlled(psi: np.ndarray, U: np.ndarray, c: int, q: int, n: int) -> np.ndarray:
    """Apply U to qubit q on the basis states where qubit c is 1."""
    idx = np.arange(1 << n)
    on = ((idx >> c) & 1) == 1
    sub = psi.copy()
    upd = apply_1q(psi, U, q, n)
    sub[on] = upd[on]
    return sub


def apply_op(psi: np.ndarray, op, n: int) -> np.ndarray:
    kind, a, b, theta = op
    if kind in ONE_Q:
        return apply_1q(psi, ONE_Q[kind], a, n)
    if kind == "RZ":
        return apply_1q(psi, rz(theta), a, n)
    if kind == "CX":
        return apply_controlled(psi, X, a, b, n)
    if kind == "CZ":
        return apply_controlled(psi, Z, a, b, n)
    raise ValueError(kind)


def run(n: int, ops) -> np.ndarray:
    psi = zero_state(n)
    for op in ops:
        psi = apply_op(psi, op, n)
    return psi


def probabilities(psi: np.ndarray) -> np.ndarray:
    return np.abs(psi) ** 2


def marginal(probs: np.ndarray, n: int, qubits) -> np.ndarray:
    """p(b) with bit i of b = outcome of qubits[i]."""
    idx = np.arange(1 << n)
    out_idx = np.zeros(1 << n, dtype=np.int64)
    for i, q in enumerate(qubits):
        out_idx |= ((idx >> q) & 1) << i
    return np.bincount(out_idx, weights=probs, minlength=1 << len(qubits))


def uncut_marginal(n: int, ops, qubits) -> np.ndarray:
    """Exact output marginal of the whole (uncut) circuit from |0^n>,
    measured in Z (Sec. V-B: circuit inputs in |0>, outputs in Z)."""
    return marginal(probabilities(run(n, ops)), n, qubits)


def z_expectation(probs: np.ndarray, n: int, mask: int) -> float:
    idx = np.arange(1 << n)
    par = np.zeros(1 << n, dtype=np.int64)
    m = mask
    q = 0
    while m:
        if m & 1:
            par ^= (idx >> q) & 1
        m >>= 1
        q += 1
    return float(np.sum(probs * (1 - 2 * par)))
