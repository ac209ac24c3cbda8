"""Cut placement checks (test infrastructure): whether a cut list isolates
the non-Clifford operations (Sec. V-A: the cutter places cuts so that the
non-Clifford elements sit in their own fragments), and the fewest cuts that
do so, by brute force over all cut subsets of tiny circuits.

A cut list isolates the non-Clifford ops within width W when every
fragment holding a non-Clifford op has at most W qubits (the fragments are
the oracle's own, `cutting.fragment_circuit`).  Sec. III-B bounds the cuts
needed by twice the number of T gates (a cut before and after each).
"""
from __future__ import annotations

import itertools
from typing import List, Optional, Sequence, Tuple

from . import cutting as C

NON_CLIFFORD = ("T", "TDG", "RZ")


def isolates(n: int, ops, cuts: Sequence[Tuple[int, int]], width: int) -> bool:
    frags = C.fragment_circuit(n, ops, list(cuts))
    return all(f.m <= width for f in frags if not f.clifford)


def candidate_cuts(n: int, ops) -> List[Tuple[int, int]]:
    """Every place a cut can go: after each op on each of its wires, except
    after a wire's last op."""
    last = {}
    on = []
    for i, (k, a, b, _) in enumerate(ops):
        for q in ((a, b) if k in ("CX", "CZ") else (a,)):
            on.append((q, i))
            last[q] = i
    return [(q, i) for q, i in on if last[q] != i]


def min_cuts(n: int, ops, width: int, kmax: int) -> Optional[int]:
    """Fewest cuts that isolate the non-Clifford ops within `width`, or None
    if more than kmax are needed."""
    cand = candidate_cuts(n, ops)
    for k in range(kmax + 1):
        for sub in itertools.combinations(cand, k):
            if isolates(n, ops, sub, width):
                return k
    return None


def n_non_clifford(ops) -> int:
    return sum(1 for o in ops if o[0] in NON_CLIFFORD)
