"""Seeded synthetic near-Clifford workloads.

This module only draws circuits, cut lists, requested qubits and Z-string
masks from seeded numpy generators.  It holds none of the circuit-cutting
arithmetic: no tableau, no amplitude, no Pauli transform, no contraction.
Both the CPU oracle and the HIP path consume the same op lists from here.

Op format: ``(kind, q0, q1, theta)`` with ``kind`` one of
``H S SDG X Y Z CX CZ T TDG RZ`` (``q1 = -1`` for one-qubit gates,
``theta`` only used by ``RZ``).  A cut is ``(qubit, after_op)``: the wire
``qubit`` is cut right after the global op index ``after_op``, which acts on
that wire (the paper's cut locations, Sec. III-B and Sec. V-A).

Circuit shape ("block construction"): a non-Clifford block B of w wires
starts at t = 0; c exit wires of B are cut at layer t_c.  Before t_c
two-qubit gates never cross the block boundary; after t_c the exit wires
interact only outside B and the other block wires only inside B.  T gates
sit on block wires (on an exit wire only before its cut).  Cutting the exit
wires therefore isolates the non-Clifford operations (Sec. V-A) and leaves
one w-qubit non-Clifford fragment per block plus one Clifford fragment of
n - sum(w) + sum(c) qubits.  "Mirrored" circuits are the same op list in
reverse order, so the Clifford fragment is upstream of the block.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ONE_QUBIT = ("H", "S", "SDG", "X", "Y", "Z", "T", "TDG", "RZ")
TWO_QUBIT = ("CX", "CZ")
CLIFFORD_KINDS = ("H", "S", "SDG", "X", "Y", "Z", "CX", "CZ")
ALL_KINDS = ("H", "S", "SDG", "X", "Y", "Z", "CX", "CZ", "T", "TDG", "RZ")

Op = Tuple[str, int, int, float]
Cut = Tuple[int, int]


@dataclass
class Workload:
    """One synthetic problem: circuit + cuts + what to reconstruct."""

    name: str
    n: int
    ops: List[Op]
    cuts: List[Cut]
    qubits: List[int]                 # marginal request, bit i = qubits[i]
    zmasks: List[int] = field(default_factory=list)  # Z-strings, bit q = qubit q
    seed: int = 0
    shots: int = 0                    # shots per Clifford variant, 0 = exact
    nc_output_wires: List[int] = field(default_factory=list)
    depth: int = 0

    def zmask_words(self) -> np.ndarray:
        """Masks as uint64 words, ``[n_strings][ceil(n/64)]``."""
        nw = (self.n + 63) // 64
        out = np.zeros((len(self.zmasks), nw), dtype=np.uint64)
        for i, m in enumerate(self.zmasks):
            for w in range(nw):
                out[i, w] = (m >> (64 * w)) & 0xFFFFFFFFFFFFFFFF
        return out


@dataclass
class Block:
    wires: List[int]
    exits: List[int]


def _one_qubit_clifford(rng) -> str:
    return "H" if rng.random() < 0.5 else "S"


def _layer_groups(n: int, blocks: Sequence[Block], phase: int) -> List[List[int]]:
    """Wire groups within which two-qubit gates may act in this phase."""
    in_block = set()
    exits = set()
    for b in blocks:
        in_block.update(b.wires)
        exits.update(b.exits)
    groups: List[List[int]] = []
    if phase == 0:
        for b in blocks:
            groups.append(sorted(b.wires))
        groups.append([q for q in range(n) if q not in in_block])
    else:
        for b in blocks:
            groups.append(sorted(q for q in b.wires if q not in exits))
        groups.append([q for q in range(n) if q not in in_block or q in exits])
    return [g for g in groups if g]


def _gen_layer(rng, group: List[int], p_cx: float, topology: str, layer: int,
               out: List[Tuple[str, int, int]]):
    if topology == "random":
        order = list(rng.permutation(group))
        i = 0
        while i < len(order):
            q = int(order[i])
            if i + 1 < len(order) and rng.random() < p_cx:
                a, b = q, int(order[i + 1])
                if rng.random() < 0.5:
                    a, b = b, a
                out.append(("CX", a, b))
                i += 2
            else:
                out.append((_one_qubit_clifford(rng), q, -1))
                i += 1
    elif topology == "nn":
        chain = sorted(group)
        used = set()
        for j in range(layer % 2, len(chain) - 1, 2):
            a, b = chain[j], chain[j + 1]
            if rng.random() < p_cx:
                if rng.random() < 0.5:
                    a, b = b, a
                out.append(("CX", a, b))
                used.update((a, b))
        for q in chain:
            if q not in used:
                out.append((_one_qubit_clifford(rng), q, -1))
    else:
        raise ValueError(topology)


class _DSU:
    def __init__(self):
        self.p = {}

    def find(self, a):
        self.p.setdefault(a, a)
        while self.p[a] != a:
            self.p[a] = self.p[self.p[a]]
            a = self.p[a]
        return a

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra != rb:
            self.p[ra] = rb


def block_circuit(n: int, depth: int, blocks: Sequence[Block], t_c: int, p_cx: float,
                  seed: int, *, t_fixed: Optional[Sequence[Tuple[int, int]]] = None,
                  n_t: int = 0, topology: str = "random", mirrored: bool = False,
                  max_attempts: int = 2000):
    """Draw a block-structured near-Clifford circuit.

    Returns ``(ops, cuts)``.  Draws are repeated with the sub-seed
    ``(seed, attempt)`` until every block's wires (exit wires before the cut)
    and the Clifford remainder (all other wires plus the exit wires after the
    cut) each form one interacting group, so the cut list yields exactly one
    fragment per block plus one Clifford fragment.  The interaction bookkeeping
    below only tracks which wires met in a two-qubit gate.
    """
    exits = set(q for b in blocks for q in b.exits)
    block_of = {}
    for bi, b in enumerate(blocks):
        for q in b.wires:
            block_of[q] = bi
        assert set(b.exits) <= set(b.wires)
    for attempt in range(max_attempts):
        rng = np.random.default_rng([seed, attempt])
        # T placement: (qubit, layer) pairs
        if t_fixed is not None:
            t_list = list(t_fixed)
        else:
            cand = []
            for b in blocks:
                for q in b.wires:
                    hi = t_c if q in exits else depth
                    cand.extend((q, L) for L in range(hi))
            idx = rng.choice(len(cand), size=n_t, replace=False) if n_t else []
            t_list = [cand[i] for i in sorted(idx)]
        t_at = {}
        for q, L in t_list:
            t_at.setdefault(L, []).append(q)
        ops: List[Op] = []
        phases: List[int] = []
        for L in range(depth):
            phase = 0 if L < t_c else 1
            layer: List[Tuple[str, int, int]] = []
            for g in _layer_groups(n, blocks, phase):
                _gen_layer(rng, g, p_cx, topology, L, layer)
            for kind, a, b in layer:
                ops.append((kind, a, b, 0.0))
                phases.append(phase)
            for q in t_at.get(L, []):
                ops.append(("T", q, -1, 0.0))
                phases.append(phase)
        # interaction bookkeeping (which wire groups met)
        dsu = _DSU()

        def node(q, ph):
            return (q, ph) if q in exits else (q, 0)

        for (kind, a, b, _), ph in zip(ops, phases):
            if b >= 0:
                dsu.union(node(a, ph), node(b, ph))
        ok = True
        for b in blocks:
            members = [node(q, 0) for q in b.wires]
            roots = {dsu.find(m) for m in members}
            if len(roots) != 1:
                ok = False
        cl = [node(q, 0) for q in range(n) if q not in block_of] + [(q, 1) for q in exits]
        if len({dsu.find(m) for m in cl}) != 1:
            ok = False
        # every exit wire needs an op on both sides of its cut
        for q in exits:
            ph_ops = {ph for (k, a, b2, _), ph in zip(ops, phases) if q in (a, b2)}
            if ph_ops != {0, 1}:
                ok = False
        if not ok:
            continue
        if mirrored:
            ops = ops[::-1]
            phases = phases[::-1]
        first_phase = 1 if mirrored else 0
        cuts: List[Cut] = []
        for q in sorted(exits):
            last = max(i for i, ((k, a, b2, _), ph) in enumerate(zip(ops, phases))
                       if q in (a, b2) and ph == first_phase)
            cuts.append((q, last))
        return ops, cuts
    raise RuntimeError("block_circuit: no connected draw found")


def _zmasks(n: int, count: int, seed: int) -> List[int]:
    rng = np.random.default_rng([seed, 7])
    out = []
    for _ in range(count):
        bits = rng.random(n) < 0.5
        out.append(sum(1 << q for q in range(n) if bits[q]))
    return out


def _nearest(candidates: Sequence[int], anchors: Sequence[int], count: int) -> List[int]:
    key = lambda q: (min(abs(q - a) for a in anchors), q)
    return sorted(candidates, key=key)[:count]


# ---------------------------------------------------------------- configs

def tiny() -> Workload:
    """8 qubits, 10 layers, T on qubit 0 at layers 3 and 7, block {0..3},
    exit wire 3 cut after layer 5: a 4-qubit non-Clifford fragment and a
    5-qubit Clifford fragment; full 256-entry distribution, exact mode."""
    blocks = [Block([0, 1, 2, 3], [3])]
    ops, cuts = block_circuit(8, 10, blocks, t_c=6, p_cx=1.0 / 3.0, seed=0,
                              t_fixed=[(0, 3), (0, 7)])
    return Workload("tiny", 8, ops, cuts, list(range(8)), _zmasks(8, 16, 0), seed=0,
                    shots=0, nc_output_wires=[0, 1, 2], depth=10)


def mid(shots: int = 100_000) -> Workload:
    """32 qubits, 40 layers (CX density 0.3), 4 T gates on qubits 0-9, exits
    8 and 9 cut after layer 19: a 10-qubit non-Clifford fragment and a
    24-qubit Clifford fragment; 12-qubit marginal over qubits 20-31 and 64
    random Z-strings."""
    blocks = [Block(list(range(10)), [8, 9])]
    ops, cuts = block_circuit(32, 40, blocks, t_c=20, p_cx=0.3, seed=1000, n_t=4)
    return Workload("mid", 32, ops, cuts, list(range(20, 32)), _zmasks(32, 64, 1000),
                    seed=1000, shots=shots, nc_output_wires=list(range(8)), depth=40)


def batching_circuit(i: int, shots: int = 10_000) -> Workload:
    """Circuit i of the 256-circuit batch: width U[20,200], depth U[20,60],
    1-4 cuts, 1-6 T gates in one block of at most 12 wires, half of them
    mirrored in time; a 16-qubit marginal straddling the fragments."""
    seed = 2000 + i
    rng = np.random.default_rng([seed, 99])
    n = int(rng.integers(20, 201))
    depth = int(rng.integers(20, 61))
    c = int(rng.integers(1, 5))
    n_t = int(rng.integers(1, 7))
    w = int(rng.integers(c, 13))
    start = int(rng.integers(0, n - w + 1))
    wires = list(range(start, start + w))
    exits = sorted(int(q) for q in rng.choice(wires, size=c, replace=False))
    mirrored = bool(rng.random() < 0.5)
    t_c = int(rng.integers(depth // 4, 3 * depth // 4 + 1))
    t_c = max(1, min(depth - 1, t_c))
    ops, cuts = block_circuit(n, depth, [Block(wires, exits)], t_c=t_c, p_cx=0.3,
                              seed=seed, n_t=n_t, mirrored=mirrored)
    nc_out = list(wires) if mirrored else [q for q in wires if q not in exits]
    req = nc_out[:8]
    cl = [q for q in range(n) if q not in nc_out]
    req = sorted(req + _nearest(cl, wires, 16 - len(req)))
    return Workload(f"batch{i}", n, ops, cuts, req, [], seed=seed, shots=shots,
                    nc_output_wires=nc_out, depth=depth)


def batching(count: int = 256, shots: int = 10_000) -> List[Workload]:
    return [batching_circuit(i, shots) for i in range(count)]


def precision(shots: int = 0) -> Workload:
    """400-qubit nearest-neighbour ladder, 30 layers, two 6-qubit blocks
    (qubits 100-105 and 300-305) with 4 T gates each and exits {j, j+4, j+5}:
    6 cuts, 4096 cut terms; 64 Z-strings and a 16-qubit marginal."""
    blocks = [Block(list(range(100, 106)), [100, 104, 105]),
              Block(list(range(300, 306)), [300, 304, 305])]
    rng = np.random.default_rng([3000, 5])
    t_list = []
    for b in blocks:
        nonexit = [q for q in b.wires if q not in b.exits]
        for _ in range(4):
            q = int(rng.choice(nonexit))
            t_list.append((q, int(rng.integers(0, 30))))
    t_list.sort(key=lambda t: (t[1], t[0]))
    ops, cuts = block_circuit(400, 30, blocks, t_c=15, p_cx=0.5, seed=3000,
                              t_fixed=t_list, topology="nn")
    nc_out = [101, 102, 103, 301, 302, 303]
    cl = [q for q in range(400) if q not in nc_out and not (100 <= q <= 105 and q not in (100, 104, 105))
          and not (300 <= q <= 305 and q not in (300, 304, 305))]
    req = sorted(nc_out + _nearest(cl, [100, 105, 300, 305], 10))
    return Workload("precision", 400, ops, cuts, req, _zmasks(400, 64, 3000), seed=3000,
                    shots=shots, nc_output_wires=nc_out, depth=30)


def learned_circuit(seed: int, tail: int = 25, near_exits: bool = False) -> Workload:
    """300 qubits, 25 + tail layers (CX density 0.3), four 5-qubit blocks at
    30 + 75 i with 3 T gates each and (3, 3, 2, 2) exit wires: 10 cuts,
    4^10 cut terms; 16-qubit marginal (10 block outputs + 6 Clifford qubits).
    near_exits: the marginal is over the first 6 block outputs and the 10
    exit wires themselves (measured tail layers after their cut), so the
    Clifford fragment's outputs sit in the cuts' light cone."""
    exit_counts = (3, 3, 2, 2)
    blocks = []
    for i, c in enumerate(exit_counts):
        wires = list(range(30 + 75 * i, 35 + 75 * i))
        blocks.append(Block(wires, wires[5 - c:]))
    depth = 25 + tail
    ops, cuts = block_circuit(300, depth, blocks, t_c=25, p_cx=0.3, seed=seed, n_t=12)
    nc_out = [q for b in blocks for q in b.wires if q not in b.exits]
    if near_exits:
        req = sorted(nc_out[:6] + [q for b in blocks for q in b.exits])
    else:
        cl = [q for q in range(300) if q not in nc_out and not any(q in b.wires and q not in b.exits for b in blocks)]
        req = sorted(nc_out + _nearest(cl, [b.wires[0] for b in blocks], 6))
    name = f"learned{seed}" if (tail, near_exits) == (25, False) else f"learned{seed}_t{tail}{'e' if near_exits else ''}"
    return Workload(name, 300, ops, cuts, req, [], seed=seed, shots=0, nc_output_wires=nc_out, depth=depth)


def random_circuit(n: int, n_ops: int, seed: int, *, kinds: Sequence[str] = ALL_KINDS,
                   p_two: float = 0.35) -> List[Op]:
    """Unstructured random circuit for tests (any gate anywhere)."""
    rng = np.random.default_rng([seed, 11])
    one = [k for k in kinds if k in ONE_QUBIT]
    two = [k for k in kinds if k in TWO_QUBIT]
    ops: List[Op] = []
    for _ in range(n_ops):
        if two and n >= 2 and rng.random() < p_two:
            a, b = rng.choice(n, size=2, replace=False)
            ops.append((str(rng.choice(two)), int(a), int(b), 0.0))
        else:
            k = str(rng.choice(one))
            th = float(rng.uniform(-np.pi, np.pi)) if k == "RZ" else 0.0
            ops.append((k, int(rng.integers(n)), -1, th))
    return ops


def random_cuts(n: int, ops: Sequence[Op], k: int, seed: int) -> List[Cut]:
    """k distinct random cut locations (each right after an op on its wire)."""
    rng = np.random.default_rng([seed, 13])
    cand = []
    for i, (kind, a, b, _) in enumerate(ops):
        cand.append((a, i))
        if b >= 0:
            cand.append((b, i))
    if k > len(cand):
        raise ValueError("not enough cut locations")
    idx = rng.choice(len(cand), size=k, replace=False)
    return sorted((cand[i] for i in idx), key=lambda c: (c[1], c[0]))


# ------------------------------------------- the paper's workloads (Sec. VI-B)
# Written from the paper's descriptions (no benchmark-suite code): each
# circuit is Clifford with `n_t` T gates injected at random op positions;
# its cuts are left to the automatic cutter (cuts = []).

# Clifford angles of the ansatz rotations: RZ(k pi/2) is I, S, Z, S^dag
_RZ_CLIFFORD = {0: [], 1: ["S"], 2: ["Z"], 3: ["SDG"]}


def _clifford_rz(rng, q: int) -> List[Op]:
    return [(g, q, -1, 0.0) for g in _RZ_CLIFFORD[int(rng.integers(4))]]


def _clifford_ry(rng, q: int) -> List[Op]:
    # RY(k pi/2) up to a global phase: S^dag H RZ(k pi/2) H S
    body = _clifford_rz(rng, q)
    if not body:
        return []
    return [("SDG", q, -1, 0.0), ("H", q, -1, 0.0)] + body + [("H", q, -1, 0.0), ("S", q, -1, 0.0)]


def _inject_t(rng, ops: List[Op], n_t: int, n: int) -> List[Op]:
    """Insert n_t T gates on random wires at random positions of the op list."""
    out = list(ops)
    for _ in range(n_t):
        pos = int(rng.integers(len(out) + 1))
        out.insert(pos, ("T", int(rng.integers(n)), -1, 0.0))
    return out


def hwea(n: int, rounds: int = 5, seed: int = 0, n_t: int = 1) -> Workload:
    """Near-Clifford hardware-efficient ansatz (Sec. VI-B): per round a layer
    of single-qubit rotations (RY then RZ at Clifford angles), a linear
    chain of CX entanglers, and a final single-qubit rotation layer."""
    rng = np.random.default_rng([seed, 31, n])
    ops: List[Op] = []
    for _ in range(rounds):
        for q in range(n):
            ops += _clifford_ry(rng, q) + _clifford_rz(rng, q)
        for q in range(n - 1):
            ops.append(("CX", q, q + 1, 0.0))
        for q in range(n):
            ops += _clifford_ry(rng, q) + _clifford_rz(rng, q)
    ops = _inject_t(rng, ops, n_t, n)
    return Workload(f"hwea{n}", n, ops, [], list(range(n)), [1 << q for q in range(n)], seed=seed, depth=rounds)


def qaoa_sk(n: int, seed: int = 0, n_t: int = 1) -> Workload:
    """One round of MaxCut QAOA on the Sherrington-Kirkpatrick model
    (complete graph, weights +-1; Sec. IV / VI-B) at Clifford angles: H on
    every qubit, exp(-i gamma w_ij Z_i Z_j) for every pair as CX, RZ, CX with
    gamma w_ij a multiple of pi/4 (RZ(2 gamma w) a Clifford), then the
    mixer RX(2 beta) = H RZ(2 beta) H."""
    rng = np.random.default_rng([seed, 37, n])
    g = int(rng.integers(1, 4))   # 2 gamma = g pi/2
    b = int(rng.integers(1, 4))   # 2 beta = b pi/2
    ops: List[Op] = [("H", q, -1, 0.0) for q in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            w = 1 if rng.random() < 0.5 else -1
            k = (g * w) % 4
            ops.append(("CX", i, j, 0.0))
            ops += [(gate, j, -1, 0.0) for gate in _RZ_CLIFFORD[k]]
            ops.append(("CX", i, j, 0.0))
    for q in range(n):
        ops += [("H", q, -1, 0.0)] + [(gate, q, -1, 0.0) for gate in _RZ_CLIFFORD[b]] + [("H", q, -1, 0.0)]
    ops = _inject_t(rng, ops, n_t, n)
    return Workload(f"qaoa{n}", n, ops, [], list(range(n)), [1 << q for q in range(n)], seed=seed, depth=1)


def phase_code(n_data: int, seed: int = 0, n_t: int = 1) -> Workload:
    """One round of the phase-flip repetition code (Sec. VI-B): data qubits
    0..d-1 prepared in |+>, ancilla d+i measures X_i X_{i+1} (H, CX from
    the ancilla to both data qubits, H), data measured in the X basis.  The
    request is the syndrome (the ancillas), a sparse distribution."""
    rng = np.random.default_rng([seed, 41, n_data])
    d = n_data
    n = 2 * d - 1
    ops: List[Op] = [("H", q, -1, 0.0) for q in range(d)]
    for i in range(d - 1):
        a = d + i
        ops += [("H", a, -1, 0.0), ("CX", a, i, 0.0), ("CX", a, i + 1, 0.0), ("H", a, -1, 0.0)]
    ops += [("H", q, -1, 0.0) for q in range(d)]
    ops = _inject_t(rng, ops, n_t, n)
    return Workload(f"phase{d}", n, ops, [], list(range(d, n)), [], seed=seed, depth=1)
