"""Exact measurement statistics of a stabilizer state by GF(2) elimination on
its stabilizer generators -- an implementation independent of the CHP
measurement procedure, used to pin it.

A Clifford circuit's output distribution on a set M of measured qubits is
uniform over an affine subspace: the state's stabilizer group contains a
subgroup of Z-type elements supported on M, each +-Z_c of which fixes the
parity c.x of the outcomes to its sign bit.  Clifford expectation values of
Pauli strings are therefore -1, 0 or +1 (Sec. IX of the paper).

Pauli products use the plain one-qubit multiplication table
(XY = iZ, YZ = iX, ZX = iY and the reversed products with -i), not the
Aaronson-Gottesman g function, so this module shares no arithmetic with chp.c.
"""
from __future__ import annotations

import itertools

import numpy as np

# one-qubit code: I = 0, X = 1, Z = 2, Y = 3  (code = x + 2 z)
# _E[a, b] = e such that sigma_a sigma_b = i^e sigma_{a xor b}
_E = np.zeros((4, 4), dtype=np.int64)
_E[1, 2], _E[2, 1] = 3, 1   # XZ = -iY, ZX = iY
_E[1, 3], _E[3, 1] = 1, 3   # XY = iZ,  YX = -iZ
_E[2, 3], _E[3, 2] = 3, 1   # ZY = -iX, YZ = iX


def _mul_into(xp, zp, sp, X, Z, S, rows):
    """Replace rows ``rows`` of (X, Z, S) by (pivot) * (row).  All rows
    commute with the pivot, so the product phase is +-1."""
    cp = xp.astype(np.int64) + 2 * zp.astype(np.int64)
    cr = X[rows].astype(np.int64) + 2 * Z[rows].astype(np.int64)
    e = _E[cp[None, :], cr].sum(axis=1) % 4
    if np.any(e % 2):
        raise ValueError("anticommuting generators")
    S[rows] = S[rows] ^ sp ^ (e // 2).astype(np.uint8)
    X[rows] ^= xp
    Z[rows] ^= zp


def z_constraints(xs, zs, ss, meas):
    """Generators of the Z-type stabilizer subgroup supported on ``meas``.

    ``xs, zs`` are the (m, n) stabilizer rows, ``ss`` their sign bits.
    Returns ``(C, s)``: each row c of C (over the measured qubits, in the
    order of ``meas``) with sign s says ``c . x = s (mod 2)`` for every
    outcome x that can occur.
    """
    X = np.array(xs, dtype=np.uint8, copy=True)
    Z = np.array(zs, dtype=np.uint8, copy=True)
    S = np.array(ss, dtype=np.uint8, copy=True)
    m, n = X.shape
    meas = list(meas)
    inM = np.zeros(n, dtype=bool)
    inM[meas] = True
    used = np.zeros(m, dtype=bool)
    cols = [("x", j) for j in range(n)] + [("z", j) for j in range(n) if not inM[j]]
    for kind, j in cols:
        col = X[:, j] if kind == "x" else Z[:, j]
        cand = np.nonzero((col == 1) & ~used)[0]
        if cand.size == 0:
            continue
        p = int(cand[0])
        used[p] = True
        others = np.nonzero(col == 1)[0]
        others = others[others != p]
        if others.size:
            _mul_into(X[p].copy(), Z[p].copy(), S[p], X, Z, S, others)
    free = np.nonzero(~used)[0]
    assert not X[free].any() and not Z[free][:, ~inM].any()
    C = Z[free][:, meas]
    return C, S[free]


def distribution(xs, zs, ss, meas) -> np.ndarray:
    """Exact outcome distribution over ``meas`` (bit j of the index is the
    outcome of meas[j]) by enumerating all outcome strings."""
    C, s = z_constraints(xs, zs, ss, meas)
    k = len(meas)
    idx = np.arange(1 << k, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(k)[None, :]) & 1).astype(np.int64)
    ok = np.ones(1 << k, dtype=bool)
    for c, sign in zip(C.astype(np.int64), s.astype(np.int64)):
        ok &= (bits @ c) % 2 == sign
    out = np.zeros(1 << k, dtype=np.float64)
    out[ok] = 1.0 / ok.sum()
    return out


def _gf2_solve_sign(C, s, target):
    """If ``target`` is in the GF(2) row span of C, return the xor of the
    signs of one combination that produces it; else None."""
    A = np.concatenate([C.astype(np.uint8), s.astype(np.uint8)[:, None]], axis=1)
    t = np.concatenate([target.astype(np.uint8), [0]]).astype(np.uint8)
    ncol = C.shape[1]
    r = 0
    rows = A.copy()
    piv = []
    for j in range(ncol):
        cand = [i for i in range(r, rows.shape[0]) if rows[i, j]]
        if not cand:
            continue
        i = cand[0]
        rows[[r, i]] = rows[[i, r]]
        for i2 in range(rows.shape[0]):
            if i2 != r and rows[i2, j]:
                rows[i2] ^= rows[r]
        piv.append(j)
        r += 1
    for i, j in enumerate(piv):
        if t[j]:
            t ^= rows[i]
    if t[:ncol].any():
        return None
    return int(t[ncol])


def z_expectation(xs, zs, ss, support) -> int:
    """<Z_support> of the stabilizer state: +1, -1 or 0."""
    support = list(support)
    if not support:
        return 1
    C, s = z_constraints(xs, zs, ss, support)
    sign = _gf2_solve_sign(C, s, np.ones(len(support), dtype=np.uint8))
    if sign is None:
        return 0
    return -1 if sign else 1


def z_expectations(xs, zs, ss, masks, n) -> list:
    """<Z_support> for many supports at once (each mask an int over qubits
    0..n-1): one elimination of the Z-type subgroup on all qubits, then for
    each mask a membership test by reduction against its row echelon form."""
    C, s = z_constraints(xs, zs, ss, list(range(n)))
    A = np.concatenate([C.astype(np.uint8), s.astype(np.uint8)[:, None]], axis=1)
    piv = []
    r = 0
    for j in range(n):
        cand = np.nonzero(A[r:, j])[0]
        if cand.size == 0:
            continue
        i = r + int(cand[0])
        A[[r, i]] = A[[i, r]]
        hit = np.nonzero(A[:, j])[0]
        hit = hit[hit != r]
        A[hit] ^= A[r]
        piv.append(j)
        r += 1
        if r == A.shape[0]:
            break
    out = []
    for mk in masks:
        t = np.array([(mk >> q) & 1 for q in range(n)] + [0], dtype=np.uint8)
        for i, j in enumerate(piv):
            if t[j]:
                t ^= A[i]
        if t[:n].any():
            out.append(0)
        else:
            out.append(-1 if t[n] else 1)
    return out


def pauli_matrix(x_row, z_row, sign) -> np.ndarray:
    """Dense matrix of (-1)^sign * prod_q sigma_q (bit q of the basis index =
    qubit q), for pinning tableau rows against a state vector."""
    from .statevector import X as PX, Y as PY, Z as PZ
    n = len(x_row)
    M = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):
        code = int(x_row[q]) + 2 * int(z_row[q])
        P = [np.eye(2), PX, PZ, PY][code]
        M = np.kron(M, P)
    return (-1.0) ** int(sign) * M


def all_strings(k):
    return list(itertools.product([0, 1], repeat=k))
