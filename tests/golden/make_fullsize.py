"""Writes tests/golden/fullsize.npz: the oracle's results at full workload
size, the expected values of tests/test_gpu_fullsize.py.  It calls only the
oracle (oracle/) and the seeded input generators (workloads/); the fragment
variants of a circuit are spread over a process pool, then transformed and
recombined exactly as oracle.cutting.marginal / zexpect do.

    python tests/golden/make_fullsize.py [--workers 8]

Contents (fp64):
  precision_marginal   the 400-qubit, 6-cut workload, exact, 16-qubit marginal
  precision_z          the same, its 64 Z strings, exact
  mid_marginal         the 32-qubit, 2-cut workload, 1e5 shots per variant,
                       seed 1000, 12-qubit marginal over qubits 20-31
  mid_z                the same, its 64 Z strings
  batch_<i>            circuit i of the 256-circuit batch, 1e4 shots per
                       variant, seed 2000, circuit index i, 16-qubit marginal
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cutting as C  # noqa: E402
from oracle import philox as Ph  # noqa: E402

BATCH_CIRCUITS = (0, 76, 77, 126, 151)  # small; 256 variants at 197 qubits; 16 measured bits; mirrored 4 cuts; widest
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize.npz")


def _workload(name):
    if name == "precision":
        return W.precision()
    if name == "mid":
        return W.mid()
    return W.batching_circuit(int(name.split("_")[1]))


def _variants(task):
    """Distributions (marginal request) or parity states (Z strings) of
    variants [v0, v1) of fragment f."""
    name, mode, f, v0, v1, shots, seed, circuit = task
    w = _workload(name)
    frag = C.fragment_circuit(w.n, w.ops, w.cuts)[f]
    if mode == "marginal":
        meas = C.make_request(frag, w.qubits).meas
        out = []
        for v in range(v0, v1):
            if not frag.clifford:
                out.append(C.nc_distribution(frag, v, meas))
            elif shots == 0:
                out.append(C.clifford_exact(frag, v, meas, "elim"))
            else:
                out.append(C.clifford_sampled(frag, v, meas, seed, Ph.variant_id(circuit, frag.index, v), shots))
        return task, np.array(out)
    return task, None


def marginal(pool, name, shots, seed, circuit):
    w = _workload(name)
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    tasks = []
    for f in frags:
        step = max(1, f.n_variants // 64)
        for v0 in range(0, f.n_variants, step):
            tasks.append((name, "marginal", f.index, v0, min(f.n_variants, v0 + step), shots, seed, circuit))
    parts = {}
    for task, d in pool.imap_unordered(_variants, tasks):
        parts[(task[2], task[3])] = d
    reqs = [C.make_request(f, w.qubits) for f in frags]
    dists = [np.concatenate([parts[k] for k in sorted(k for k in parts if k[0] == f.index)]) for f in frags]
    tensors = [C.pauli_tensor(f, r, d) for f, r, d in zip(frags, reqs, dists)]
    return C.recombine(frags, reqs, tensors, len(w.cuts), len(w.qubits))


def _zvariant(task):
    name, f, v, shots, seed = task
    w = _workload(name)
    frag = C.fragment_circuit(w.n, w.ops, w.cuts)[f]
    meas = C.zstring_measured_set(frag, w.zmasks)
    pos = {l: j for j, l in enumerate(meas)}
    outs = [1 << pos[ax.local] for ax in frag.axes if ax.side == 0]
    extras = sorted({sum(b for j, b in enumerate(outs) if (s >> j) & 1) for s in range(1 << len(outs))})
    return f, v, C.zstring_variant_expectations(frag, meas, w.zmasks, v, extras, shots=shots, seed=seed)


def zexpect(pool, name, shots, seed):
    w = _workload(name)
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    tasks = [(name, f.index, v, shots, seed) for f in frags for v in range(f.n_variants)]
    expect = {f.index: {} for f in frags}
    for f, v, table in pool.imap_unordered(_zvariant, tasks, chunksize=4):
        for e, vals in table.items():
            expect[f][(v, e)] = vals
    return C.zexpect(w.n, w.ops, w.cuts, w.zmasks, shots=shots, seed=seed, expect=expect)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    res = dict(np.load(OUT)) if os.path.exists(OUT) else {}
    jobs = [("precision_marginal", lambda p: marginal(p, "precision", 0, 0, 0)),
            ("precision_z", lambda p: zexpect(p, "precision", 0, 0)),
            ("mid_marginal", lambda p: marginal(p, "mid", 100_000, 1000, 0)),
            ("mid_z", lambda p: zexpect(p, "mid", 100_000, 1000))]
    jobs += [(f"batch_{i}", (lambda i: lambda p: marginal(p, f"batch_{i}", 10_000, 2000, i))(i))
             for i in BATCH_CIRCUITS]
    with mp.get_context("fork").Pool(args.workers) as pool:
        for key, fn in jobs:
            if args.only is not None and key not in args.only:
                continue
            t0 = time.time()
            res[key] = np.asarray(fn(pool), dtype=np.float64)
            print(f"{key}: {res[key].shape} in {time.time() - t0:.1f} s", flush=True)
            np.savez_compressed(OUT, **res)


if __name__ == "__main__":
    main()
