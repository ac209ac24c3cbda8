"""Circuit cutting, plainly: fragmenter, fragment variants, fragment
evaluation, Pauli-basis transform, recombination (paper Secs. III-B, V).

The identity behind it (Peng et al., cited in Sec. III-B): a wire carrying
rho can be replaced by
    rho = 1/2 sum_{P in {I,X,Y,Z}} Tr(P rho) P ,
so the uncut circuit's output probability is
    R[b] = 2^-k sum_{P in {I,X,Y,Z}^k} prod_f T_f[b_f; P|f]
with one tensor per fragment and one index per cut (Sec. V-C: a tensor
network with one tensor per fragment and one edge per cut, 4^k cost).

Readings where the paper is silent (its Fig. 2 is not available):
* preparations at quantum inputs are {|0>, |1>, |+>, |+i>}; measurement
  bases at quantum outputs are {X, Y, Z};
* a quantum input contributes  I = p0 + p1,  Z = p0 - p1,
  X = 2 p+ - p0 - p1,  Y = 2 p+i - p0 - p1  (the operator P written in
  the four prepared states);
* a quantum output contributes  I = Z0 + Z1 (the I term comes from the
  Z-basis variant),  Z = Z0 - Z1,  X = X0 - X1,  Y = Y0 - Y1;
* by default no maximum-likelihood correction: raw (possibly negative)
  estimates (the correction is ``mlcorrect``, ml=True);
* non-Clifford fragments are evaluated exactly, Clifford fragments either
  exactly ("strong simulation", Sec. V-C) or by sampling shots;
* variant index: mixed radix over the fragment's incident cut axes in
  cut-list order (the upstream side of a cut before its downstream side),
  the first axis least significant; preparations radix 4 in the order
  (0, 1, +, +i), bases radix 3 in the order (X, Y, Z);
* Pauli index of a cut: I = 0, X = 1, Y = 2, Z = 3; the full term index is
  P = sum_c P_c 4^c (cut 0 least significant);
* only the fragment's measured set is measured: its requested circuit
  outputs plus its quantum outputs, in ascending fragment-local order
  (local qubits are ordered by (wire, segment)); bit j of a fragment
  outcome index is measurement j;
* output bit i of a marginal is the outcome of qubits[i].
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import chp as _chp
from . import philox as _philox
from . import stabilizer as _stab
from . import statevector as _sv

CLIFFORD = {"H", "S", "SDG", "X", "Y", "Z", "CX", "CZ"}
KINDS = CLIFFORD | {"T", "TDG", "RZ"}
TWO_QUBIT = {"CX", "CZ"}

I_, X_, Y_, Z_ = 0, 1, 2, 3            # Pauli codes
PREP_OPS = {0: [], 1: ["X"], 2: ["H"], 3: ["H", "S"]}          # |0>,|1>,|+>,|+i>
BASIS_OPS = {0: ["H"], 1: ["SDG", "H"], 2: []}                 # X, Y, Z
BASIS_X, BASIS_Y, BASIS_Z = 0, 1, 2

# quantum input: operator P written in the prepared states (0, 1, +, +i)
PREP_COEF = np.array([[1, 1, 0, 0],     # I
                      [-1, -1, 2, 0],   # X
                      [-1, -1, 0, 2],   # Y
                      [1, -1, 0, 0]],   # Z
                     dtype=np.float64)


class CutError(ValueError):
    pass


@dataclass
class Axis:
    cut: int        # index in the cut list
    side: int       # 0 = quantum output (upstream of the cut), 1 = quantum input
    local: int      # fragment-local qubit

    @property
    def radix(self) -> int:
        return 3 if self.side == 0 else 4


@dataclass
class Fragment:
    index: int
    segments: List[Tuple[int, int]]                  # (wire, segment) in local order
    ops: List[Tuple[str, int, int, float]]           # local qubit indices
    clifford: bool
    axes: List[Axis]
    circuit_outputs: Dict[int, int] = field(default_factory=dict)  # wire -> local

    @property
    def m(self) -> int:
        return len(self.segments)

    @property
    def n_variants(self) -> int:
        v = 1
        for a in self.axes:
            v *= a.radix
        return v

    def digits(self, v: int) -> List[int]:
        out = []
        for a in self.axes:
            out.append(v % a.radix)
            v //= a.radix
        return out

    def variant_index(self, digits: Sequence[int]) -> int:
        v, mul = 0, 1
        for d, a in zip(digits, self.axes):
            v += d * mul
            mul *= a.radix
        return v

    def variant_ops(self, v: int):
        """Preparations, then the fragment's gates, then basis rotations."""
        out = []
        for d, a in zip(self.digits(v), self.axes):
            if a.side == 1:
                out += [(g, a.local, -1, 0.0) for g in PREP_OPS[d]]
        out += self.ops
        for d, a in zip(self.digits(v), self.axes):
            if a.side == 0:
                out += [(g, a.local, -1, 0.0) for g in BASIS_OPS[d]]
        return out

    def p_index(self, P: int) -> int:
        """Restriction of the full term index P to this fragment's axes."""
        p = 0
        for j, a in enumerate(self.axes):
            p += ((P >> (2 * a.cut)) & 3) << (2 * j)
        return p


def validate(n: int, ops, cuts) -> None:
    if n <= 0:
        raise CutError("no qubits")
    for i, (k, a, b, th) in enumerate(ops):
        if k not in KINDS:
            raise CutError(f"op {i}: unknown gate {k}")
        if not (0 <= a < n):
            raise CutError(f"op {i}: qubit out of range")
        if k in TWO_QUBIT:
            if not (0 <= b < n) or a == b:
                raise CutError(f"op {i}: bad two-qubit operands")
    seen = set()
    for c, (q, after) in enumerate(cuts):
        if not (0 <= q < n) or not (0 <= after < len(ops)):
            raise CutError(f"cut {c}: out of range")
        k, a, b, _ = ops[after]
        if q != a and not (k in TWO_QUBIT and q == b):
            raise CutError(f"cut {c}: op {after} does not act on qubit {q}")
        if (q, after) in seen:
            raise CutError(f"cut {c}: duplicate")
        seen.add((q, after))


def fragment_circuit(n: int, ops, cuts) -> List[Fragment]:
    """Split each cut wire into segments; fragments are the connected
    components of segments joined by two-qubit gates (Secs. III-B, V-A)."""
    validate(n, ops, cuts)
    wire_ops: List[List[int]] = [[] for _ in range(n)]
    for i, (k, a, b, _) in enumerate(ops):
        wire_ops[a].append(i)
        if k in TWO_QUBIT:
            wire_ops[b].append(i)
    pos = [{op: p for p, op in enumerate(wo)} for wo in wire_ops]
    cut_pos: List[List[Tuple[int, int]]] = [[] for _ in range(n)]   # (position, cut id)
    for c, (q, after) in enumerate(cuts):
        cut_pos[q].append((pos[q][after], c))
    for q in range(n):
        cut_pos[q].sort()
    # segment of (op, wire): number of cuts on the wire at or before an earlier position
    def seg_of(op: int, q: int) -> int:
        p = pos[q][op]
        return sum(1 for cp, _ in cut_pos[q] if cp < p)
    cut_segment = {}                  # cut id -> (wire, upstream segment)
    for q in range(n):
        for s, (_, c) in enumerate(cut_pos[q]):
            cut_segment[c] = (q, s)
    parent: Dict[Tuple[int, int], Tuple[int, int]] = {}

    def find(u):
        parent.setdefault(u, u)
        while parent[u] != u:
            parent[u] = parent[parent[u]]
            u = parent[u]
        return u

    all_segs = [(q, s) for q in range(n) for s in range(len(cut_pos[q]) + 1)]
    for u in all_segs:
        find(u)
    for i, (k, a, b, _) in enumerate(ops):
        if k in TWO_QUBIT:
            ua, ub = find((a, seg_of(i, a))), find((b, seg_of(i, b)))
            if ua != ub:
                parent[ua] = ub
    comps: Dict[Tuple[int, int], List[Tuple[int, int]]] = {}
    for u in all_segs:
        comps.setdefault(find(u), []).append(u)
    groups = sorted((sorted(v) for v in comps.values()), key=lambda g: g[0])
    frags = []
    for fi, segs in enumerate(groups):
        local = {u: j for j, u in enumerate(segs)}
        segset = set(segs)
        fops = []
        for i, (k, a, b, th) in enumerate(ops):
            ua = (a, seg_of(i, a))
            if ua in segset:
                lb = local[(b, seg_of(i, b))] if k in TWO_QUBIT else -1
                fops.append((k, local[ua], lb, th))
        axes = []
        for c in range(len(cuts)):
            q, s = cut_segment[c]
            if (q, s) in segset:
                axes.append(Axis(c, 0, local[(q, s)]))
            if (q, s + 1) in segset:
                axes.append(Axis(c, 1, local[(q, s + 1)]))
        outs = {q: local[(q, s)] for (q, s) in segs if s == len(cut_pos[q])}
        frags.append(Fragment(fi, segs, fops, all(o[0] in CLIFFORD for o in fops), axes, outs))
    return frags


# ------------------------------------------------------------------ requests

@dataclass
class Request:
    """Per-fragment view of a marginal request."""
    meas: List[int]                 # measured set (local qubits, ascending)
    req_pos: List[int]              # positions in meas of the requested outputs
    req_user: List[int]             # their index in the user's qubit list
    out_pos: Dict[int, int]         # axis number -> position in meas (quantum outputs)


def make_request(frag: Fragment, qubits: Sequence[int]) -> Request:
    wanted = {frag.circuit_outputs[q]: i for i, q in enumerate(qubits) if q in frag.circuit_outputs}
    outs = {a.local: j for j, a in enumerate(frag.axes) if a.side == 0}
    meas = sorted(set(wanted) | set(outs))
    req_pos = [p for p, l in enumerate(meas) if l in wanted]
    req_user = [wanted[meas[p]] for p in req_pos]
    out_pos = {outs[l]: p for p, l in enumerate(meas) if l in outs}
    return Request(meas, req_pos, req_user, out_pos)


# ------------------------------------------------------- fragment evaluation

def nc_distribution(frag: Fragment, v: int, meas) -> np.ndarray:
    psi = _sv.run(frag.m, frag.variant_ops(v))
    return _sv.marginal(_sv.probabilities(psi), frag.m, meas)


def clifford_tableau(frag: Fragment, v: int) -> _chp.Tableau:
    t = _chp.Tableau(frag.m)
    for k, a, b, _ in frag.variant_ops(v):
        t.gate(k, a, b)
    return t


def clifford_exact(frag: Fragment, v: int, meas, method: str = "branch") -> np.ndarray:
    t = clifford_tableau(frag, v)
    if method == "branch":
        return t.exact(meas)
    x, z, r = t.dump()
    m = frag.m
    return _stab.distribution(x[m:2 * m], z[m:2 * m], r[m:2 * m], meas)


def clifford_sampled(frag: Fragment, v: int, meas, seed: int, vid: int, shots: int) -> np.ndarray:
    t = clifford_tableau(frag, v)
    return t.sample_hist(meas, seed, vid, shots).astype(np.float64) / shots


def variant_distributions(frag: Fragment, meas, *, shots: int = 0, seed: int = 0,
                          circuit: int = 0, exact_method: str = "branch") -> np.ndarray:
    """``[n_variants][2^len(meas)]`` outcome distributions of every variant."""
    out = np.zeros((frag.n_variants, 1 << len(meas)))
    for v in range(frag.n_variants):
        if not frag.clifford:
            out[v] = nc_distribution(frag, v, meas)
        elif shots == 0:
            out[v] = clifford_exact(frag, v, meas, exact_method)
        else:
            vid = _philox.variant_id(circuit, frag.index, v)
            out[v] = clifford_sampled(frag, v, meas, seed, vid, shots)
    return out


# ------------------------------------------------------- Pauli-basis transform

def pauli_tensor(frag: Fragment, req: Request, dists: np.ndarray) -> np.ndarray:
    """T_f[b_f][p_f]: the variant data rewritten in the Pauli basis of each
    cut axis (b_f bit i = i-th requested output in measured order,
    p_f = sum_j P_j 4^j over the fragment's axes)."""
    a = len(frag.axes)
    M = len(req.meas)
    shape = [ax.radix for ax in frag.axes][::-1] + [2] * M
    t = dists.reshape(shape)
    t = np.transpose(t, list(range(a - 1, -1, -1)) + list(range(a + M - 1, a - 1, -1)))
    labels = [("d", j) for j in range(a)] + [("b", p) for p in range(M)]
    for j, ax in enumerate(frag.axes):
        d = labels.index(("d", j))
        if ax.side == 1:
            t = np.moveaxis(np.tensordot(PREP_COEF, t, axes=([1], [d])), 0, d)
        else:
            bpos = labels.index(("b", req.out_pos[j]))
            z0 = np.take(np.take(t, BASIS_Z, axis=d), 0, axis=bpos - 1 if bpos > d else bpos)
            z1 = np.take(np.take(t, BASIS_Z, axis=d), 1, axis=bpos - 1 if bpos > d else bpos)
            x0 = np.take(np.take(t, BASIS_X, axis=d), 0, axis=bpos - 1 if bpos > d else bpos)
            x1 = np.take(np.take(t, BASIS_X, axis=d), 1, axis=bpos - 1 if bpos > d else bpos)
            y0 = np.take(np.take(t, BASIS_Y, axis=d), 0, axis=bpos - 1 if bpos > d else bpos)
            y1 = np.take(np.take(t, BASIS_Y, axis=d), 1, axis=bpos - 1 if bpos > d else bpos)
            stacked = np.stack([z0 + z1, x0 - x1, y0 - y1, z0 - z1], axis=0)  # I, X, Y, Z
            # the bit axis is gone; the new Pauli axis goes where the digit was
            labels.pop(bpos)
            dd = labels.index(("d", j))
            t = np.moveaxis(stacked, 0, dd)
    # remaining: Pauli axes (a of them) and requested bit axes in measured order
    order_b = [labels.index(("b", p)) for p in req.req_pos]
    order_d = [labels.index(("d", j)) for j in range(a)]
    t = np.transpose(t, order_b[::-1] + order_d[::-1])
    return np.ascontiguousarray(t).reshape(1 << len(req.req_pos), 4 ** a)


def support(frags: Sequence[Fragment], tensors, k: int) -> List[int]:
    """Cut terms P whose column T_f[:, P|f] is nonzero in every fragment,
    ascending: the terms that can contribute to the recombination sum
    (Sec. IX, fewer stitching calculations: for Clifford fragments most
    Pauli expectations vanish)."""
    nz = [np.any(T != 0.0, axis=0) for T in tensors]
    return [P for P in range(4 ** k) if all(z[f.p_index(P)] for f, z in zip(frags, nz))]


def recombine(frags: Sequence[Fragment], reqs: Sequence[Request], tensors, k: int,
              nq: int, sparse: bool = False, terms=None) -> np.ndarray:
    """R[b] = 2^-k sum_P prod_f T_f[b_f; P|f], summed over P in ascending
    order (the contraction of Sec. V-C, written out).  sparse: only the
    terms of ``support`` are summed (the skipped terms are exact zeros);
    terms: only these (ascending)."""
    b = np.arange(1 << nq, dtype=np.int64)
    bidx = []
    for req in reqs:
        bi = np.zeros_like(b)
        for i, u in enumerate(req.req_user):
            bi |= ((b >> u) & 1) << i
        bidx.append(bi)
    R = np.zeros(1 << nq, dtype=np.float64)
    if terms is None:
        terms = support(frags, tensors, k) if sparse else range(4 ** k)
    for P in terms:
        term = np.ones(1 << nq, dtype=np.float64)
        for f, T, bi in zip(frags, tensors, bidx):
            term = term * T[bi, f.p_index(P)]
        R += term
    return R * 2.0 ** (-k)


def recombine_matmul(frags: Sequence[Fragment], reqs: Sequence[Request], tensors, k: int,
                     nq: int, left: Sequence[int]) -> np.ndarray:
    """The same sum as one matrix product: fragments in ``left`` form the
    row operand A[b_L; P], the others the column operand B[b_R; P], each the
    elementwise product of its fragments' tensor columns; R = A B^T 2^-k."""
    Pall = np.arange(4 ** k, dtype=np.int64)

    def operand(fs):
        bits = sum(len(reqs[f].req_pos) for f in fs)
        op = np.ones((1 << bits, 4 ** k))
        shift = 0
        users = []
        for f in fs:
            T = tensors[f]
            pf = np.zeros_like(Pall)
            for j, ax in enumerate(frags[f].axes):
                pf += ((Pall >> (2 * ax.cut)) & 3) << (2 * j)
            rb = len(reqs[f].req_pos)
            rows = np.arange(1 << bits)
            op = op * T[(rows >> shift) & ((1 << rb) - 1)][:, pf]
            users += reqs[f].req_user
            shift += rb
        return op, users

    right = [f for f in range(len(frags)) if f not in left]
    A, uL = operand(list(left))
    B, uR = operand(right)
    C = (A @ B.T) * 2.0 ** (-k)
    out = np.zeros(1 << nq)
    rl = np.arange(C.shape[0])
    rr = np.arange(C.shape[1])
    bL = np.zeros_like(rl)
    for i, u in enumerate(uL):
        bL |= ((rl >> i) & 1) << u
    bR = np.zeros_like(rr)
    for i, u in enumerate(uR):
        bR |= ((rr >> i) & 1) << u
    out[bL[:, None] | bR[None, :]] = C
    return out


# ------------------------------------------------------------------ Sec. IX: fewer downstream evaluations

# The variants a cut term's column reads, per axis (from the transform above):
# on a quantum input, I and Z combine |0> and |1>, X also |+>, Y also |+i>;
# on a quantum output, I and Z come from the Z basis, X from X, Y from Y.
PREPS_READ = {I_: (0, 1), Z_: (0, 1), X_: (0, 1, 2), Y_: (0, 1, 3)}
BASES_READ = {I_: (BASIS_Z,), Z_: (BASIS_Z,), X_: (BASIS_X,), Y_: (BASIS_Y,)}


def exact_support(frags: Sequence[Fragment], reqs: Sequence[Request], k: int) -> List[int]:
    """Cut terms whose column is nonzero in every Clifford fragment's exact
    Pauli tensor, ascending.  A Clifford fragment's exact tensor is known
    before any of its variants is sampled (its expectations are 0 or +-1,
    Sec. IX); non-Clifford fragments do not restrict the set."""
    nz = []
    for f, r in zip(frags, reqs):
        if f.clifford:
            T = pauli_tensor(f, r, variant_distributions(f, r.meas))
            nz.append(np.any(T != 0.0, axis=0))
        else:
            nz.append(None)
    return [P for P in range(4 ** k) if all(z is None or z[f.p_index(P)] for f, z in zip(frags, nz))]


def needed_variants(frag: Fragment, terms) -> np.ndarray:
    """need[v]: some term of ``terms`` reads variant v of ``frag`` (every
    axis's preparation or basis is one the term's Pauli on that cut reads)."""
    need = np.zeros(frag.n_variants, dtype=bool)
    seen = set()
    for P in terms:
        key = frag.p_index(P)
        if key in seen:
            continue
        seen.add(key)
        opts = [PREPS_READ[(P >> (2 * ax.cut)) & 3] if ax.side == 1 else BASES_READ[(P >> (2 * ax.cut)) & 3]
                for ax in frag.axes]
        for digits in itertools.product(*opts):
            need[frag.variant_index(digits)] = True
    return need


def marginal_skip(n: int, ops, cuts, qubits, *, shots: int = 0, seed: int = 0, circuit: int = 0,
                  return_parts: bool = False):
    """The marginal with Sec. IX's downstream skipping: the support S is
    fixed from the Clifford fragments' exact tensors, the variants no term of
    S reads are never evaluated (their tables are zero), and only the terms
    of S are summed.  Exact data: the full sum (the other terms vanish)."""
    qubits = list(qubits)
    frags = fragment_circuit(n, ops, cuts)
    reqs = [make_request(f, qubits) for f in frags]
    S = exact_support(frags, reqs, len(cuts))
    dists = []
    for f, r in zip(frags, reqs):
        d = variant_distributions(f, r.meas, shots=shots, seed=seed, circuit=circuit)
        d = np.array(d, dtype=np.float64)
        d[~needed_variants(f, S)] = 0.0
        dists.append(d)
    tensors = [pauli_tensor(f, r, d) for f, r, d in zip(frags, reqs, dists)]
    R = recombine(frags, reqs, tensors, len(cuts), len(qubits), terms=S)
    if return_parts:
        return R, dict(frags=frags, reqs=reqs, dists=dists, tensors=tensors, support=S)
    return R


# ------------------------------------------------------------------ end to end

def marginal(n: int, ops, cuts, qubits, *, shots: int = 0, seed: int = 0, circuit: int = 0,
             exact_method: str = "branch", return_parts: bool = False, sparse: bool = False,
             ml: bool = False):
    """Reconstructed output marginal over ``qubits`` (bit i = qubits[i]).
    ml: the variant tables first go through the maximum-likelihood fragment
    correction (``mlcorrect``)."""
    qubits = list(qubits)
    if len(set(qubits)) != len(qubits) or any(not (0 <= q < n) for q in qubits):
        raise CutError("bad qubit request")
    frags = fragment_circuit(n, ops, cuts)
    reqs = [make_request(f, qubits) for f in frags]
    dists = [variant_distributions(f, r.meas, shots=shots, seed=seed, circuit=circuit,
                                   exact_method=exact_method) for f, r in zip(frags, reqs)]
    if ml:
        from . import mlcorrect
        dists = [mlcorrect.correct_tables(f, r, d) for f, r, d in zip(frags, reqs, dists)]
    tensors = [pauli_tensor(f, r, d) for f, r, d in zip(frags, reqs, dists)]
    R = recombine(frags, reqs, tensors, len(cuts), len(qubits), sparse=sparse)
    if return_parts:
        return R, dict(frags=frags, reqs=reqs, dists=dists, tensors=tensors)
    return R


# ------------------------------------------------------------------ Z strings

def zstring_measured_set(frag: Fragment, masks: Sequence[int]) -> List[int]:
    """Circuit outputs of the fragment that occur in any mask, plus its
    quantum outputs, ascending."""
    anymask = 0
    for m in masks:
        anymask |= m
    outs = {a.local for a in frag.axes if a.side == 0}
    req = {l for q, l in frag.circuit_outputs.items() if (anymask >> q) & 1}
    return sorted(req | outs)


def _variant_state(frag, v, meas, *, shots, seed, circuit):
    """What a variant's parity expectations are computed from: the exact
    outcome distribution (non-Clifford), the final stabilizer rows (exact
    Clifford) or the literal per-shot records (sampled Clifford)."""
    if not frag.clifford:
        return ("dist", nc_distribution(frag, v, meas))
    t = clifford_tableau(frag, v)
    if shots == 0:
        xs, zs, rs = t.dump()
        m = frag.m
        return ("stab", (xs[m:2 * m], zs[m:2 * m], rs[m:2 * m]))
    vid = _philox.variant_id(circuit, frag.index, v)
    return ("shots", t.sample(meas, seed, vid, 0, shots).astype(np.int64))


def _parity_expectation(state, meas, mk, settle=False):
    """E_v[(-1)^{mask . x}] for one mask (bitmask over measured positions).
    settle (sampled Clifford variants, Sec. IX fewer shots): the expectation
    of a Pauli on a stabilizer state is -1, 0 or +1, so shots that show both
    parities give 0 and shots that agree give their common sign."""
    kind, data = state
    sel = [j for j in range(len(meas)) if (mk >> j) & 1]
    if kind == "dist":
        x = np.arange(data.size, dtype=np.int64)
        par = np.zeros_like(x)
        for j in sel:
            par ^= (x >> j) & 1
        return float(np.sum(data * (1 - 2 * par)))
    if kind == "stab":
        xs, zs, rs = data
        return float(_stab.z_expectation(xs, zs, rs, [meas[j] for j in sel]))
    par = data[:, sel].sum(axis=1) % 2 if sel else np.zeros(data.shape[0], np.int64)
    if settle:
        odd = int(np.sum(par))
        return 1.0 if odd == 0 else -1.0 if odd == data.shape[0] else 0.0
    return float(np.sum(1 - 2 * par)) / data.shape[0]


def zstring_local_masks(frag: Fragment, meas, masks: Sequence[int]) -> List[int]:
    """Each mask restricted to the fragment's circuit outputs, as a bitmask
    over measured positions."""
    pos = {l: j for j, l in enumerate(meas)}
    zloc = []
    for mk in masks:
        bits = 0
        for q, l in frag.circuit_outputs.items():
            if (mk >> q) & 1:
                bits |= 1 << pos[l]
        zloc.append(bits)
    return zloc


def zstring_variant_expectations(frag: Fragment, meas, masks: Sequence[int], v: int, extras: Sequence[int], *,
                                 shots=0, seed=0, circuit=0, settle=False):
    """{extra: [E_v[(-1)^(z_f.b + extra.b)] for each mask z]} for variant v
    (extra: a bitmask of quantum-output positions)."""
    state = _variant_state(frag, v, meas, shots=shots, seed=seed, circuit=circuit)
    zloc = zstring_local_masks(frag, meas, masks)
    return {e: [_parity_expectation(state, meas, z | e, settle) for z in zloc] for e in extras}


def zstring_tensor(frag: Fragment, meas, masks: Sequence[int], *, shots=0, seed=0, circuit=0, settle=False,
                   expect=None):
    """t_f[z][p_f] = sum over the contributing variants of the coefficient
    times the variant's expectation of (-1)^(z_f.b + sum of the quantum-output
    bits of the axes with P != I).  expect: optional precomputed
    {(v, extra): expectations} (zstring_variant_expectations) used in place
    of evaluating variants here."""
    a = len(frag.axes)
    pos = {l: j for j, l in enumerate(meas)}
    zloc = zstring_local_masks(frag, meas, masks)
    # all (variant, extra-mask) pairs that can be needed
    out_bit = {j: 1 << pos[ax.local] for j, ax in enumerate(frag.axes) if ax.side == 0}
    states = {}
    cache = {} if expect is None else expect

    def E(v, extra):
        key = (v, extra)
        if key not in cache:
            if v not in states:
                states[v] = _variant_state(frag, v, meas, shots=shots, seed=seed, circuit=circuit)
            cache[key] = [_parity_expectation(states[v], meas, z | extra, settle) for z in zloc]
        return cache[key]

    t = np.zeros((len(masks), 4 ** a))
    for pf in range(4 ** a):
        Ps = [(pf >> (2 * j)) & 3 for j in range(a)]
        choices = []
        for j, (P, ax) in enumerate(zip(Ps, frag.axes)):
            if ax.side == 1:
                choices.append([(s, PREP_COEF[P, s], 0) for s in range(4) if PREP_COEF[P, s] != 0])
            else:
                basis = {I_: BASIS_Z, Z_: BASIS_Z, X_: BASIS_X, Y_: BASIS_Y}[P]
                choices.append([(basis, 1.0, 0 if P == I_ else out_bit[j])])
        for combo in itertools.product(*choices):
            digits = [c[0] for c in combo]
            coef = float(np.prod([c[1] for c in combo]))
            extra = 0
            for c in combo:
                extra |= c[2]
            t[:, pf] += coef * np.asarray(E(frag.variant_index(digits), extra))
    return t


def zexpect(n: int, ops, cuts, masks: Sequence[int], *, shots: int = 0, seed: int = 0,
            circuit: int = 0, return_parts: bool = False, settle: bool = False, expect=None):
    """<Z_z> for every mask z (bit q = qubit q):
    2^-k sum_P prod_f t_f[z; P|f].  expect: optional per-fragment
    precomputed variant expectations (see zstring_tensor)."""
    frags = fragment_circuit(n, ops, cuts)
    k = len(cuts)
    tens = []
    for f in frags:
        meas = zstring_measured_set(f, masks)
        tens.append(zstring_tensor(f, meas, masks, shots=shots, seed=seed, circuit=circuit, settle=settle,
                                   expect=None if expect is None else expect.get(f.index)))
    out = np.zeros(len(masks))
    for P in range(4 ** k):
        term = np.ones(len(masks))
        for f, t in zip(frags, tens):
            term = term * t[:, f.p_index(P)]
        out += term
    out *= 2.0 ** (-k)
    if return_parts:
        return out, dict(frags=frags, tensors=tens)
    return out
