"""Benchmark of the Clifford-based circuit-cutting hot path on one MI355X.

Default workload (the largest single-GPU configuration): 256 near-Clifford
circuits of uneven shape (width 20-200, depth 20-60, 1-6 T gates in one
block of at most 12 wires, 1-4 cuts, half of them mirrored in time), 1e4
shots per Clifford fragment variant, a 16-qubit marginal per circuit.  One
step = one replay of the captured batch: every fragment variant of every
circuit (affine sample models, Philox shots, state vectors), the Pauli transforms
and the 4^k recombinations.

Prints one JSON line.  value = fragment-variant shots per second of the
whole step; recombination term-products per second sit beside it, with the
dominant kernel's roofline (work per launch over its HIP-event-timed
launches), the fractions of the other modelled kernels, and the CPU oracle
timed on this host (single-threaded and on all cores) on a bounded sample
of the same circuits as cpu_baseline.

Other workloads (--workload): mid (32 qubits, 2 cuts, 1e5 shots), precision
(400 qubits, 6 cuts, fp32 matrix-core products), learned (300 qubits, 10
cuts, learned term proposal), scan (the paper's workload families).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fragment-variant shots/s + recombination terms/s; end-to-end vs plain at TVD≤1e-2"
PEAK_INT32_OPS = 256 * 64 * 2.4e9       # 256 CUs x 64 int32 VALU lanes/clk x 2.4 GHz
PEAK_HBM = 8.0e12
PEAK_FP64 = 78.6e12                     # fp64 vector (and MFMA) peak
PHILOX_OPS = 100                        # 10 rounds x (2 mul_lo + 2 mul_hi + 4 xor + 2 key add)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 2000 for mid, whose step takes about 0.1 ms; 20 for batching; "
                         "50 otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default: 200 for mid, 5 for batching, 10 otherwise)")
    ap.add_argument("--shots", type=int, default=None,
                    help="shots per Clifford variant (default: 1e5 for mid, 1e4 for batching)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 64 MiB elementwise copy first (the known-size kernel that scales the HBM "
                         "counters of a --pmc run)")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="instead of benchmarking: turn two rocprofv3 --pmc counter_collection.csv files "
                         "(FETCH_SIZE, WRITE_SIZE) of a --calibrate-copy run into profiles/<workload>_traffic.json")
    ap.add_argument("--traffic-kernel", default="sv_kernel")
    ap.add_argument("--contraction-only", action="store_true",
                    help="learned workload: only the held-out circuit's dense exhaustive contraction, fp64 and "
                         "fp32 (no training, few dispatches: for counter runs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", choices=["mid", "batching", "precision", "learned", "scan"], default="batching",
                    help="batching (default): 256 uneven circuits in one graph-captured batch; mid: the 32-qubit, "
                         "2-cut workload; precision: the 400-qubit, 6-cut workload with FP32-MFMA "
                         "recombination; learned: the 300-qubit, 10-cut workload, learned term proposal against "
                         "exhaustive recombination; scan: the paper's workload families with automatic cuts")
    args = ap.parse_args()
    short = args.workload == "mid"
    batch = args.workload == "batching"
    if args.steps is None:
        args.steps = 2000 if short else 20 if batch else 50
    if args.warmup is None:
        args.warmup = 200 if short else 5 if batch else 10
    if args.shots is None:
        args.shots = 10_000 if batch else 100_000
    return args


def cpu_baseline(w, target_s: float):
    """Time the oracle (single-threaded literal tableau per shot) on a bounded
    sample of the same workload: the sampled marginal and Z strings with
    fewer shots per variant; scaled to shots per second."""
    import numpy as np
    from oracle import cutting as C

    shots = 200
    while True:
        t0 = time.perf_counter()
        C.marginal(w.n, w.ops, w.cuts, w.qubits, shots=shots, seed=w.seed)
        C.zexpect(w.n, w.ops, w.cuts, w.zmasks, shots=shots, seed=w.seed)
        dt = time.perf_counter() - t0
        if dt >= target_s or shots >= w.shots:
            break
        shots = int(min(w.shots, max(shots * 2, shots * target_s / max(dt, 1e-3) * 1.1)))
    frags = C.fragment_circuit(w.n, w.ops, w.cuts)
    n_cliff_var = sum(f.n_variants for f in frags if f.clifford)
    total = 2 * n_cliff_var * shots
    return {"value": total / dt, "unit": "shots/s", "cores": 1, "kind": "oracle",
            "sample": f"mid workload with {shots} shots per Clifford variant (marginal + 64 Z strings), "
                      f"{total} shots in {dt:.1f} s, single-threaded literal per-shot tableau"}


# kernel name -> the source file whose contents its traffic figure belongs to
# (with common.hpp, which holds the launch shapes and job layouts)
KERNEL_SOURCES = {"sv_kernel": "k_sv.hip", "affine_kernel": "k_affine.hip", "carry_kernel": "k_heis.hip",
                  "parity": "k_sample.hip", "sample_kernel": "k_sample.hip"}
CALIB_BYTES = 64 << 20


def _source_hash(kernel):
    import hashlib
    for key, fname in KERNEL_SOURCES.items():
        if key in kernel:
            h = hashlib.sha256()
            for f in (fname, "common.hpp"):
                h.update(open(os.path.join(ROOT, "paper_2303_10788_amd", "csrc", f), "rb").read())
            return h.hexdigest()[:16]
    return None


def _kernel_base(name):
    """The kernel's own name: no return type, namespaces, template
    arguments or parameter list."""
    name = name.replace("void ", "").replace("(anonymous namespace)::", "")
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):  # the first '<' or '(' outside any bracket ends the qualified name
        if ch in "<(" and depth == 0:
            cut = i
            break
    return name[:cut].split("::")[-1]


def traffic_from_counters(args):
    """HBM bytes per launch of one kernel from a FETCH_SIZE and a WRITE_SIZE
    counter run, each scaled by the same counter on the 64 MiB copy
    (elementwise kernel reading and writing CALIB_BYTES)."""
    import csv
    out = {"workload": args.workload, "kernel": args.traffic_kernel, "source_sha": _source_hash(args.traffic_kernel)}
    # the batched launches of a kernel class count as its launches
    names = {"sv_kernel": ("sv_kernel", "sv_batch_kernel"), "sample_kernel": ("sample_kernel", "sample_batch_kernel")}
    names = names.get(args.traffic_kernel, (args.traffic_kernel,))
    for path, counter in zip(args.traffic, ("FETCH_SIZE", "WRITE_SIZE")):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        kern = [float(r["Counter_Value"]) for r in rows if _kernel_base(r["Kernel_Name"]) in names]
        calib = [float(r["Counter_Value"]) for r in rows if "elementwise" in r["Kernel_Name"]]
        calib = max(calib)  # the 64 MiB copy is the largest elementwise dispatch
        factor = (CALIB_BYTES / 1024.0) / calib
        key = counter.split("_")[0].lower()
        out[f"{key}_kib_per_launch"] = sum(kern) / len(kern)
        out[f"{key}_copy_kib"] = calib
        out[f"{key}_factor"] = factor
        out[f"{key}_bytes_per_launch"] = sum(kern) / len(kern) * 1024.0 * factor
        out["launches_sampled"] = len(kern)
    out["bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    dst = os.path.join(ROOT, "profiles", f"{args.workload}_traffic.json")
    with open(dst, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def traffic_for(workload, kernel):
    """HBM bytes per launch measured for this kernel, or None when there is
    no measurement or its source changed since."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != kernel or rec.get("source_sha") != _source_hash(kernel):
        return None
    return rec["bytes_per_launch"]


def main():
    args = parse()
    if args.traffic:
        return traffic_from_counters(args)
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batching":
        return bench_batching(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "scan":
        return bench_scan(args)
    import numpy as np
    import torch

    import paper_2303_10788_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    w = W.mid(shots=args.shots)
    ctx = cc.Context(0)
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    # the step's two requests are independent: the Z strings are served by a
    # second context on a stream of its own (default priority), so the two
    # calls overlap on the GPU
    side = torch.cuda.Stream(device=0)
    with torch.cuda.stream(side):
        ctx_z = cc.Context(0)
    plan_z = cc.Plan(ctx_z, w.n, w.ops, w.cuts)
    frags = plan.fragments()
    n_cliff_var = sum(f["n_variants"] for f in frags if f["clifford"])
    k = len(w.cuts)
    masks = w.zmask_words()
    out_m = torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda")
    out_z = torch.empty(masks.shape[0], dtype=torch.float64, device="cuda")

    def step():
        plan.marginal(w.qubits, shots=w.shots, seed=w.seed, out=out_m)
        plan_z.zexpect(masks, shots=w.shots, seed=w.seed, out=out_z)

    if args.calibrate_copy:
        a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
        b = a + 0.0
        torch.cuda.synchronize()
        del a, b
    dt = _timed(step, args.steps, args.warmup)
    # per-kernel breakdown from a separate pass with event timing on (the
    # events themselves cost time, so the timed steps above run without)
    times = _kernel_pass([ctx, ctx_z], step, args.steps)

    shots_per_step = 2 * n_cliff_var * w.shots
    terms_per_step = (4 ** k) * ((1 << len(w.qubits)) + masks.shape[0])
    ms_per_step = 1e3 * dt / args.steps
    value = shots_per_step / (dt / args.steps)

    # dominant kernel (among those with an algorithmic work model: the state
    # vector, the affine models, the sampler and the parity kernel) and its
    # algorithmic work per launch
    overall = max(times.items(), key=lambda kv: kv[1][1])[0]
    n_meas_z = 24
    n_ext = masks.shape[0]
    nc = [f for f in frags if not f["clifford"]]
    cl = [f for f in frags if f["clifford"]]
    # algorithmic work per step (both calls), as stated in the design notes
    # the marginal and the Z-string call each run the state-vector pass once
    sv_work = sv_flops(cc, plan, frags, w.qubits) + sv_flops(cc, plan, frags, _mask_qubits(masks, w.n))
    carry_ops = model_ops = 0.0
    for qs in (w.qubits, _mask_qubits(masks, w.n)):
        c_, m_ = affine_work(cc, plan, frags, qs)
        carry_ops += c_
        model_ops += m_
    work = {
        "sv_kernel": (sv_work, "fp64", PEAK_FP64, "GFLOP/s"),
        # one timer covers both: the carry-back and the per-variant elimination
        "affine_kernel": (carry_ops + model_ops, "alu", PEAK_INT32_OPS, "Gop/s"),
        # per shot: a Philox call per 4 shots and 32 measurement indices, then one
        # AND + POPCOUNT + accumulate per Z string
        "parity_kernel": (n_cliff_var * w.shots * (PHILOX_OPS / 4 * ((n_meas_z + 31) // 32) + 3 * n_ext),
                          "alu", PEAK_INT32_OPS, "Gop/s"),
        # per shot: Philox share + one select-and-xor per measurement + a histogram increment
        "sample_kernel": (n_cliff_var * w.shots * (PHILOX_OPS / 4 + 3 * len(w.qubits) + 1), "alu",
                          PEAK_INT32_OPS, "Gop/s"),
    }
    name, (launches, total_ms) = max(((k, v) for k, v in times.items() if k in work), key=lambda kv: kv[1][1])
    avg_s = total_ms / max(launches, 1) / 1e3
    units, bound, peak, unit = work[name]
    per_launch = units / max(launches / args.steps, 1)
    achieved = per_launch / avg_s
    roof = {"bound": bound, "kernel": name, "achieved": achieved / 1e9, "peak": peak / 1e9, "unit": unit,
            "frac": achieved / peak, "traffic": traffic_for("mid", name), "avg_launch_us": avg_s * 1e6,
            "work_per_launch": per_launch, "dominant_overall": overall}

    line = {
        "metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "mid: 32 qubits, 40 random Clifford layers (CX density 0.3), 4 T on qubits 0-9, "
                               "2 cuts (10-qubit non-Clifford + 24-qubit Clifford fragment), 1e5 shots per "
                               "variant, 12-qubit marginal over qubits 20-31 + 64 Z strings (the two requests "
                               "on two contexts / streams)",
                   "shots_per_step": shots_per_step, "clifford_variants": n_cliff_var, "cut_terms": 4 ** k},
        "recombination_terms_per_s": terms_per_step / (dt / args.steps),
        "kernels_ms_per_step": {kname: round(ms / args.steps, 5) for kname, (n, ms) in times.items() if n},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def sv_flops(cc, plan, frags, qubits):
    """Algorithmic fp64 flops of one state-vector pass over the non-Clifford
    fragments of a request: the gate program runs once per computational-
    basis input (2^n_in runs; 28 flops per amplitude pair of each fused
    one-qubit unitary); each of the 4^n_in preparation states is a sum of
    the run states it superposes (6^n_in terms over all preparations, 2 flops
    per amplitude each); per (preparation, basis) combination 3 flops per
    amplitude for |a|^2 and N/2 adds per unmeasured qubit."""
    total = 0.0
    for f, fr in enumerate(frags):
        if fr["clifford"]:
            continue
        n_in = sum(1 for a in fr["axes"] if a[1] == 1)
        n_out = len(fr["axes"]) - n_in
        N = 1 << fr["m"]
        n_meas, _ = cc.ccut_request_info(plan.handle, qubits, f)
        runs = 1 << n_in
        combine = 2 * N * (6 ** n_in) if n_in else 0
        total += runs * fr["n_one"] * 14 * N + combine + \
            (4 ** n_in) * (3 ** n_out) * (3 * N + (fr["m"] - n_meas) * N // 2)
    return total


def _mask_qubits(masks, n):
    """Circuit qubits that occur in any Z-string mask ([strings][words])."""
    import numpy as np
    anym = np.bitwise_or.reduce(np.asarray(masks, dtype=np.uint64), axis=0)
    return [q for q in range(n) if (int(anym[q >> 6]) >> (q & 63)) & 1]


def _kernel_pass(ctx, fn, steps):
    """{kernel: (launches, total ms)} over `steps` calls of fn with event
    timing, summed over the given context(s)."""
    import torch
    ctxs = ctx if isinstance(ctx, (list, tuple)) else [ctx]
    torch.cuda.synchronize()
    for c in ctxs:
        c.timing(True)
        c.timing_reset()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    times = {}
    for c in ctxs:
        for k, (n, ms) in c.kernel_times().items():
            n0, ms0 = times.get(k, (0, 0.0))
            times[k] = (n0 + n, ms0 + ms)
        c.timing(False)
    return times


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def host_info():
    """Host CPU: usable cores, nproc and the model name (as lscpu reports it)."""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cores": cores, "model": model}


def _oracle_fragment_task(task):
    """One pool task of the all-core oracle run: the variant distributions of
    variants [v0, v1) of fragment f of batch circuit i (the oracle's own
    per-variant functions, as oracle.cutting.variant_distributions calls them)."""
    import numpy as np
    import workloads as W
    from oracle import cutting as C
    from oracle import philox as Ph
    i, f, v0, v1, shots, seed = task
    w = W.batching_circuit(i, shots=shots)
    frag = C.fragment_circuit(w.n, w.ops, w.cuts)[f]
    meas = C.make_request(frag, w.qubits).meas
    out = np.zeros((v1 - v0, 1 << len(meas)))
    for v in range(v0, v1):
        if not frag.clifford:
            out[v - v0] = C.nc_distribution(frag, v, meas)
        else:
            out[v - v0] = C.clifford_sampled(frag, v, meas, seed, Ph.variant_id(i, frag.index, v), shots)
    return i, f, v0, out


def _oracle_batch_sample(idx, shots, seed, pool=None):
    """The oracle's sampled marginals of batch circuits idx (circuit index =
    batch position, as the GPU batch numbers its variant ids).  pool: a
    process pool that evaluates the fragment variants in parallel; the
    transform and recombination run in this process as in
    oracle.cutting.marginal."""
    import numpy as np
    import workloads as W
    from oracle import cutting as C
    res, n_shots = {}, 0
    if pool is None:
        for i in idx:
            w = W.batching_circuit(i, shots=shots)
            res[i] = C.marginal(w.n, w.ops, w.cuts, w.qubits, shots=shots, seed=seed, circuit=i)
            n_shots += shots * sum(f.n_variants for f in C.fragment_circuit(w.n, w.ops, w.cuts) if f.clifford)
        return res, n_shots
    tasks, parts = [], {}
    for i in idx:
        w = W.batching_circuit(i, shots=shots)
        frags = C.fragment_circuit(w.n, w.ops, w.cuts)
        for f in frags:
            step = max(1, f.n_variants // 16)
            for v0 in range(0, f.n_variants, step):
                tasks.append((i, f.index, v0, min(f.n_variants, v0 + step), shots, seed))
            if f.clifford:
                n_shots += shots * f.n_variants
    for i, f, v0, d in pool.imap_unordered(_oracle_fragment_task, tasks, chunksize=1):
        parts[(i, f, v0)] = d
    for i in idx:
        w = W.batching_circuit(i, shots=shots)
        frags = C.fragment_circuit(w.n, w.ops, w.cuts)
        reqs = [C.make_request(f, w.qubits) for f in frags]
        dists = [np.concatenate([parts[key] for key in sorted(k for k in parts if k[0] == i and k[1] == f.index)])
                 for f in frags]
        tensors = [C.pauli_tensor(f, r, d) for f, r, d in zip(frags, reqs, dists)]
        res[i] = C.recombine(frags, reqs, tensors, len(w.cuts), len(w.qubits))
    return res, n_shots


def cpu_baseline_batching(target_s: float, full_shots: int, seed: int):
    """The oracle (literal per-shot CHP tableau, fp64 state vectors, plain
    transform and ascending recombination) on a bounded sample of the batch:
    4 of its 256 circuits (every 64th), timed single-threaded and with the
    fragment variants spread over every usable host core, each at two shot
    counts.  The oracle's time is a per-variant part (building each
    variant's tableau gate by gate) plus a per-shot part (one literal
    tableau measurement sequence per shot), so the two timings give both,
    and the rate at the batch's own shots per variant follows; shots/s."""
    import multiprocessing as mp

    import numpy as np
    idx = list(range(0, 256, 64))
    lo = 8
    t0 = time.perf_counter()
    single_lo, n_lo = _oracle_batch_sample(idx, lo, seed)
    t1_lo = time.perf_counter() - t0
    # the larger sample: as many shots as fit the time target
    hi = lo
    while True:
        hi = int(max(2 * hi, min(full_shots, hi * target_s / max(t1_lo, 1e-3))))
        t0 = time.perf_counter()
        single_hi, n_hi = _oracle_batch_sample(idx, hi, seed)
        t1_hi = time.perf_counter() - t0
        if t1_hi >= 0.5 * target_s or hi >= full_shots:
            break
    n_var = n_lo // lo
    host = host_info()
    workers = max(1, min(16, host["usable_cores"]))
    ctx = mp.get_context("spawn")  # this process holds a GPU context: no fork
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_fragment_task, [(0, 0, 0, 1, 1, seed)] * workers)  # workers up and imported
        t0 = time.perf_counter()
        par_lo, _ = _oracle_batch_sample(idx, lo, seed, pool)
        tn_lo = time.perf_counter() - t0
        t0 = time.perf_counter()
        par_hi, _ = _oracle_batch_sample(idx, hi, seed, pool)
        tn_hi = time.perf_counter() - t0
    same = all(np.array_equal(single_lo[i], par_lo[i]) and np.array_equal(single_hi[i], par_hi[i]) for i in idx)

    def at_full(t_lo, t_hi):
        per_shot = max(t_hi - t_lo, 0.0) / (n_var * (hi - lo))
        per_var = max(t_lo - per_shot * n_var * lo, 0.0) / n_var
        return n_var * full_shots / (n_var * (per_var + per_shot * full_shots)), per_shot, per_var

    rate_n, shot_n, var_n = at_full(tn_lo, tn_hi)
    rate_1, shot_1, var_1 = at_full(t1_lo, t1_hi)
    sample = (f"batch circuits {idx} (4 of 256, {n_var} Clifford variants) timed at {lo} and {hi} shots per "
              f"variant; value = the rate at the batch's {full_shots} shots per variant from the per-variant "
              f"and per-shot times of those two runs (all-core: variants over a process pool of {workers}; "
              f"results equal to the single-threaded ones: {same})")
    return {"value": rate_n, "unit": "shots/s", "cores": workers, "kind": "oracle", "sample": sample,
            "measured": {"shots_lo": lo, "shots_hi": hi, "s_lo": tn_lo, "s_hi": tn_hi,
                         "rate_lo": n_lo / tn_lo, "rate_hi": n_hi / tn_hi,
                         "per_shot_us": shot_n * 1e6, "per_variant_ms": var_n * 1e3},
            "single_core": {"value": rate_1, "cores": 1, "s_lo": t1_lo, "s_hi": t1_hi, "rate_lo": n_lo / t1_lo,
                            "rate_hi": n_hi / t1_hi, "per_shot_us": shot_1 * 1e6, "per_variant_ms": var_1 * 1e3},
            "host": host}


def affine_work(cc, plan, frags, qubits):
    """Algorithmic int32 work of the affine sample models of a request's
    Clifford fragments, as (carry-back, elimination): the carry-back takes
    22 (fused one-qubit map) or 12 (CX, CZ) int32 operations per gate and 64
    carried rows (bit-sliced over rows; one row per requested output, two
    per quantum output); the elimination, per variant, step j and later
    measurement k > j, W = ceil(m/64) words of the constraint vector: three
    64-bit xors (6 int32 operations) and the cross-term popcount (2)."""
    carry = model = 0.0
    for f, fr in enumerate(frags):
        if not fr["clifford"]:
            continue
        nm, _ = cc.ccut_request_info(plan.handle, qubits, f)
        n_qout = sum(1 for a in fr["axes"] if a[1] == 0)
        rw = (nm + n_qout + 63) // 64
        carry += rw * (22 * fr["n_one"] + 12 * fr["n_two"])
        model += fr["n_variants"] * (nm * (nm - 1) // 2) * 8 * ((fr["m"] + 63) // 64)
    return carry, model


def batching_work(cc, plans, ws, shots):
    """Algorithmic work of one batch step per modelled kernel class:
    {kernel: (amount, kind)} with kind 'int' (int32 ops), 'fp64' (flops) or
    'bytes' (HBM bytes), as stated in the design notes."""
    sv = 0.0
    samp_ops = samp_bytes = 0.0
    tab_ops = base_ops = 0.0
    tr_bytes = 0.0
    rc_flops = rc_bytes = 0.0
    for p, w in zip(plans, ws):
        frags = p.fragments()
        sv += sv_flops(cc, p, frags, w.qubits)
        k = len(w.cuts)
        K = 4 ** k
        rows = []
        info = [cc.ccut_request_info(p.handle, w.qubits, f) for f in range(len(frags))]
        # the fold target (the fragment with the most requested bits, first
        # of equals, when all its cut axes are inputs) is read as its tables
        # and has no transform; sampled tables are read as 16-bit counts
        g = max(range(len(frags)), key=lambda f: (info[f][1], -f))
        if not frags[g]["axes"] or any(a[1] != 1 for a in frags[g]["axes"]):
            g = -1
        # sampled tables kept as 16-bit counts: the fold target's when a
        # matrix path contracts it, and every tiled fragment's
        plain = len(frags) > 2 and (K << len(w.qubits)) <= (1 << 20)
        c16 = set()
        if shots <= 0xFFFF:
            c16 = {f for f, fr in enumerate(frags)
                   if fr["clifford"] and ((f == g and not plain) or (f != g and fr["axes"]))}
        c_, m_ = affine_work(cc, p, frags, w.qubits)
        base_ops += c_
        tab_ops += m_
        for f, fr in enumerate(frags):
            nm, nr = info[f]
            nv = fr["n_variants"]
            rows.append(nr)
            if fr["axes"] and f != g:
                in_b = 2.0 if fr["clifford"] and shots <= 0xFFFF else 8.0
                tr_bytes += in_b * (nv << nm) + 8.0 * ((4 ** len(fr["axes"])) << nr)
            if not fr["clifford"]:
                continue
            # per shot: Philox share (100 per 4 shots and 32 indices), one
            # select-and-xor (3 ops) per measurement, one histogram increment;
            # the variant's fp64 table written once
            samp_ops += nv * shots * (PHILOX_OPS / 4 * ((nm + 31) // 32) + 3 * nm + 1)
            samp_bytes += (2.0 if f in c16 else 8.0) * (nv << nm)
        M = 1 << min(rows) if len(rows) > 1 else 1
        N = 1 << max(rows)
        rc_flops += 2.0 * M * N * K
        rc_bytes += 8.0 * K * M + (2.0 if g in c16 else 8.0) * K * N + 8.0 * M * N
    return {"sv_kernel": (sv, "fp64"), "affine_kernel": (tab_ops, "int"), "carry_kernel": (base_ops, "int"),
            "sample_kernel": (samp_ops, "int"), "sample_kernel:bytes": (samp_bytes, "bytes"),
            "transform_pass_kernel": (tr_bytes, "bytes"), "recombine_fp64_kernel": (rc_flops, "fp64"),
            "recombine_fp64_kernel:bytes": (rc_bytes, "bytes")}


PEAKS = {"int": (PEAK_INT32_OPS, "alu", "Gop/s"), "fp64": (PEAK_FP64, "fp64", "GFLOP/s"),
         "bytes": (PEAK_HBM, "hbm", "GB/s")}


def bench_batching(args):
    """256 circuits (width 20-200, depth 20-60, 1-4 cuts), 1e4 shots per
    variant, 16-qubit marginals; one step = one replay of the captured batch."""
    import torch

    import paper_2303_10788_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    shots = args.shots
    seed = 2000
    ws = W.batching(256, shots=shots)
    ctx = cc.Context(0)
    plans = [cc.Plan(ctx, w.n, w.ops, w.cuts) for w in ws]
    if args.calibrate_copy:
        a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
        b = a + 0.0
        torch.cuda.synchronize()
        del a, b
    t0 = time.perf_counter()
    batch = cc.Batch(ctx, plans, [w.qubits for w in ws], shots=shots, seed=seed, use_graph=True)
    t_create = time.perf_counter() - t0
    info = batch.info()
    outs = [torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda") for w in ws]
    dt = _timed(lambda: batch.run(outs), args.steps, args.warmup)
    eager = cc.Batch(ctx, plans, [w.qubits for w in ws], shots=shots, seed=seed, use_graph=False)
    dt_eager = _timed(lambda: eager.run(outs), args.steps, args.warmup)
    # per-kernel times from eager runs of the same launches with HIP events
    # on each launch's own stream (a graph replay records no events)
    times = _kernel_pass(ctx, lambda: eager.run(outs), args.steps)
    work = batching_work(cc, plans, ws, shots)
    fracs = {}
    for key, (amount, kind) in work.items():
        name = key.split(":")[0]
        launches, total_ms = times.get(name, (0, 0.0))
        if not launches:
            continue
        peak, bound, unit = PEAKS[kind]
        per_launch = amount / (launches / args.steps)
        avg_s = total_ms / launches / 1e3
        fracs[key] = {"bound": bound, "achieved": per_launch / avg_s / 1e9, "peak": peak / 1e9, "unit": unit,
                      "frac": per_launch / avg_s / peak, "avg_launch_us": avg_s * 1e6,
                      "launches_per_step": launches / args.steps, "work_per_launch": per_launch}
    # the dominant kernel: the modelled kernel class with the largest summed
    # launch time per step
    dom = max((k for k in fracs if ":" not in k), key=lambda k: times[k][1])
    roof = dict(fracs[dom], kernel=dom, traffic=traffic_for("batching", dom))
    n_var = sum(f["n_variants"] for p in plans for f in p.fragments() if f["clifford"])
    shots_per_step = n_var * shots
    terms = sum((4 ** len(w.cuts)) << len(w.qubits) for w in ws)
    line = {
        "metric": METRIC, "value": shots_per_step / (dt / args.steps), "unit": "shots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batching: 256 near-Clifford circuits, width 20-200, depth 20-60, 1-6 T in one block "
                               "of at most 12 wires, 1-4 cuts (half mirrored in time), 1e4 shots per variant, "
                               "16-qubit marginals, one graph-captured batch per step",
                   "clifford_variants": n_var, "shots_per_step": shots_per_step, "circuits": len(ws)},
        "recombination_terms_per_s": terms / (dt / args.steps),
        "batch": dict(info, create_s=t_create, eager_ms_per_step=1e3 * dt_eager / args.steps),
        "kernels_ms_per_step": {k: round(ms / args.steps, 5) for k, (n, ms) in times.items() if n},
        "roofline": roof,
        "kernel_fractions": fracs,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batching(args.cpu_seconds, shots, seed)
    print(json.dumps(line), flush=True)


def bench_precision(args):
    """400 qubits, 6 cuts (4096 terms): exact Clifford tensors, 16-qubit
    marginal and 64 Z strings recombined with fp32 matrix-core products and
    fp64 sums; the per-result error of both fp32 modes (fp32 operands, and
    hi/lo split operands) against the fp64 oracle's values (the committed
    full-size expected values, written by the oracle), else against the fp64
    contraction."""
    import numpy as np
    import torch

    import paper_2303_10788_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    w = W.precision()
    ctx = cc.Context(0)
    plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
    masks = w.zmask_words()
    out_m = torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda")
    out_z = torch.empty(masks.shape[0], dtype=torch.float64, device="cuda")
    f32 = cc.CCUT_FP32_MFMA_FP64SUM

    def step():
        plan.marginal(w.qubits, precision=f32, out=out_m)
        plan.zexpect(masks, precision=f32, out=out_z)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dt = _timed(step, args.steps, 0)
    times = _kernel_pass(ctx, step, args.steps)
    gold = os.path.join(ROOT, "tests", "golden", "fullsize.npz")
    if os.path.exists(gold):
        g = np.load(gold)
        ref_m, ref_z, ref_name = g["precision_marginal"], g["precision_z"], "fp64 oracle (tests/golden/fullsize.npz)"
    else:
        ref_m, ref_z, ref_name = plan.marginal(w.qubits), plan.zexpect(masks), "fp64 contraction on the GPU"

    def errs(m, z):
        em, ez = np.abs(m - ref_m), np.abs(z - ref_z)
        return {"marginal_max_abs": float(em.max()), "marginal_mean_abs": float(em.mean()),
                "zstring_max_abs": float(ez.max()), "zstring_mean_abs": float(ez.mean()),
                "marginal_max_rel_where_abs_gt_1e-3": float((em / np.abs(ref_m))[np.abs(ref_m) > 1e-3].max()
                                                            if np.any(np.abs(ref_m) > 1e-3) else 0.0)}

    per_result = {"reference": ref_name,
                  "fp32": errs(out_m.cpu().numpy(), out_z.cpu().numpy()),
                  "fp32_hi_lo": errs(plan.marginal(w.qubits, precision=cc.CCUT_FP32X3_MFMA_FP64SUM),
                                     plan.zexpect(masks, precision=cc.CCUT_FP32X3_MFMA_FP64SUM)),
                  "fp64": errs(plan.marginal(w.qubits), plan.zexpect(masks))}
    K = 4 ** len(w.cuts)
    M, N = 1 << 6, 1 << 10
    launches, gemm_ms = times["recombine_fp64_kernel"]
    per_launch_s = gemm_ms / max(launches, 1) / 1e3
    flops = 2.0 * M * N * K
    terms = K * ((1 << len(w.qubits)) + masks.shape[0])
    line = {
        "metric": METRIC, "value": terms / (dt / args.steps), "unit": "terms/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-mfma/f64", "data": "synthetic",
        "config": {"workload": "precision: 400-qubit nearest-neighbour ladder, 30 layers, 8 T in two 6-qubit blocks, "
                               "6 cuts (4096 terms), exact Clifford tensors, 16-qubit marginal + 64 Z strings"},
        "per_result_error": per_result,
        "kernels_ms_per_step": {k: round(ms / args.steps, 5) for k, (n, ms) in times.items() if n},
        "roofline": {"bound": "mfma", "kernel": "gemm_kernel<fp32>", "achieved": flops / per_launch_s / 1e12,
                     "peak": 157.3, "unit": "TFLOP/s", "frac": flops / per_launch_s / 157.3e12, "traffic": None,
                     "avg_launch_us": per_launch_s * 1e6},
    }
    print(json.dumps(line), flush=True)


PEAK_BF16 = 2.5e15


PEAK_FP32_MFMA = 157.3e12


def bench_learned(args):
    """300 qubits, 50 layers, four 5-qubit non-Clifford blocks, 10 cuts
    (4^10 terms), exact fragment tensors, 16-qubit marginal.  The network
    (64 -> 256 -> 256 -> 256 -> 1) is trained first on 64 other circuits of
    the same family (not timed in the steps; the TVD at 16 and 32 training
    circuits is reported too).  One step = the whole learned path on the
    held-out circuit: fragment tensors, network logits over all 4^10 terms,
    proposal, 16384 sampled terms contracted; against it the dense
    exhaustive path (fp64 and fp32 MFMA) and the Sec. IX sparse exhaustive
    path, and the network-free proposals on the same tensors: uniform,
    product of per-cut shares (the network's inputs) and the product of the
    fragments' column norms (the network's training labels, exact).  A
    second held-out circuit measures its exit wires after one Clifford layer
    (the Clifford fragment's outputs in the cuts' light cone).
    value = dense exhaustive time / learned time at the stated TVD."""
    import numpy as np
    import torch

    import paper_2303_10788_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    ctx = cc.Context(0)
    if args.contraction_only:
        w = W.learned_circuit(200000)
        plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
        buf = torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda")
        res = {}
        for name, prec in (("fp64", cc.CCUT_FP64), ("fp32", cc.CCUT_FP32_MFMA_FP64SUM)):
            L = cc.Learned(plan, w.qubits, precision=prec)
            res[name] = 1e3 * _timed(lambda: L.exhaustive(out=buf), args.steps, args.warmup) / args.steps
            L.close()
        print(json.dumps({"workload": "learned contraction", "exhaustive_ms": res}), flush=True)
        return
    n_samples = 16384
    n_train = 64
    t0 = time.perf_counter()
    xs, ys = [], []
    for s in range(100000, 100000 + n_train):
        w = W.learned_circuit(s)
        plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
        L = cc.Learned(plan, w.qubits)
        sup, _ = L.support(cap=1024)
        drawn = cc.sample_terms(ctx, cc.proposal(ctx, L.log_weights(kind=1)), 2048, seed=s, cid=1)
        uni = cc.sample_terms(ctx, cc.proposal(ctx, None, K=L.K), 1024, seed=s, cid=2)
        terms = torch.cat([sup, drawn, uni]).contiguous()
        xs.append(L.features(terms))
        ys.append(L.log_weights(terms, kind=2))
        L.close()
        plan.close()
    t_data = time.perf_counter() - t0
    nets, train = {}, {}
    for n in (16, 32, n_train):
        X = torch.cat(xs[:n]).contiguous()
        y = torch.cat(ys[:n]).contiguous()
        rows = (X.shape[0] // 64) * 64
        net = cc.Mlp(ctx, 64, 256)
        t0 = time.perf_counter()
        losses = net.train(X[:rows].contiguous(), y[:rows].contiguous(), batch=1024, steps=2000, lr=1e-3, seed=1)
        torch.cuda.synchronize()
        nets[n] = net
        train[n] = {"rows": rows, "loss_first": float(losses[:5].mean()), "loss_last": float(losses[-50:].mean()),
                    "train_s": time.perf_counter() - t0}
    net = nets[n_train]

    def tvd(a, b):
        return 0.5 * float(np.abs(a - b).sum())

    def evaluate(w, timed):
        plan = cc.Plan(ctx, w.n, w.ops, w.cuts)
        L = cc.Learned(plan, w.qubits)
        exact = L.exhaustive()
        _, n_support = L.support(cap=0)
        props = {"uniform": cc.proposal(ctx, None, K=L.K), "shares": cc.proposal(ctx, L.log_weights(kind=1)),
                 "norm_product": cc.proposal(ctx, L.log_weights(kind=0))}
        for n, nt in nets.items():
            props[f"learned_{n}"] = cc.proposal(ctx, L.logits(nt))
        tv = {k: tvd(L.estimate(q, n_samples, 9), exact) for k, q in props.items()}
        out = {"circuit": w.name, "support_terms": int(n_support), "tvd_at_16384_samples": tv}
        if timed:
            L32 = cc.Learned(plan, w.qubits, precision=cc.CCUT_FP32_MFMA_FP64SUM)
            buf = torch.empty(1 << len(w.qubits), dtype=torch.float64, device="cuda")

            def learned():
                Lx = cc.Learned(plan, w.qubits)
                Lx.estimate(cc.proposal(ctx, Lx.logits(net)), n_samples, 9, out=buf)
                Lx.close()

            fns = {"exhaustive_fp64": lambda: plan.marginal(w.qubits, out=buf),
                   "exhaustive_fp32": lambda: plan.marginal(w.qubits, out=buf, precision=cc.CCUT_FP32_MFMA_FP64SUM),
                   "sparse_exhaustive": lambda: plan.marginal(w.qubits, out=buf, flags=cc.CCUT_FLAG_SPARSE),
                   "learned": learned}
            out["ms"] = {k: 1e3 * _timed(f, args.steps, args.warmup) / args.steps for k, f in fns.items()}
            if w.name == "learned200000":
                # Sec. IX skipping in sampled mode: the marginal from 1000 shots per
                # variant with every Clifford variant sampled, and with only the
                # variants the exact support reads (the support is 1 term here)
                sfns = {"all_variants": lambda: plan.marginal(w.qubits, shots=1000, seed=5, out=buf),
                        "skip": lambda: plan.marginal(w.qubits, shots=1000, seed=5, out=buf,
                                                      flags=cc.CCUT_FLAG_SKIP)}
                out["sampled_1000_shots_ms"] = {k: 1e3 * _timed(f, 3, 1) / 3 for k, f in sfns.items()}
            # the contraction alone (tensors kept), with its kernel time
            con = {}
            for name, Lk in (("fp64", L), ("fp32", L32)):
                times = _kernel_pass(ctx, lambda: Lk.exhaustive(out=buf), args.steps)
                n_l, ms_l = times["recombine_fp64_kernel"]
                con[name] = ms_l / args.steps
            out["contraction_kernel_ms"] = con
            out["fp32_max_abs_err"] = float(np.abs(L32.exhaustive() - exact).max())
            L32.close()
        L.close()
        plan.close()
        return out

    held = [evaluate(W.learned_circuit(200000), True),
            evaluate(W.learned_circuit(200001, tail=1, near_exits=True), True)]
    main_ = held[0]
    ms = main_["ms"]
    w0 = W.learned_circuit(200000)
    p0 = cc.Plan(ctx, w0.n, w0.ops, w0.cuts)
    rbits = [cc.ccut_request_info(p0.handle, w0.qubits, f)[1] for f in range(p0.info()[0])]
    p0.close()
    K = 4 ** len(w0.cuts)
    N = 1 << max(rbits)                 # the column side: the fragment with the most requested bits
    M = 1 << (sum(rbits) - max(rbits))  # the row side: every other fragment
    flops = 2.0 * M * N * K
    c32 = main_["contraction_kernel_ms"]["fp32"]
    c64 = main_["contraction_kernel_ms"]["fp64"]
    line = {
        "metric": METRIC, "value": ms["exhaustive_fp64"] / ms["learned"],
        "unit": "x (dense exhaustive time / learned time, TVD<=1e-2)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms["learned"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16-mfma/f64",
        "data": "synthetic",
        "config": {"workload": "learned: 300 qubits, 50 layers (CX density 0.3), four 5-qubit blocks x 3 T, "
                               "exits (3,3,2,2) -> 10 cuts (4^10 terms), exact tensors, 16-qubit marginal; "
                               f"network trained on {n_train} circuits of the family, evaluated on held-out ones",
                   "samples": n_samples, "cut_terms": K},
        "held_out": held,
        "learned_vs_sparse_exhaustive_time": ms["learned"] / ms["sparse_exhaustive"],
        "train": {str(k): v for k, v in train.items()}, "dataset_s": t_data,
        "roofline": {"bound": "mfma", "kernel": f"gemm_kernel (dense exhaustive contraction, {M} x {N} x {K}, fp32)",
                     "achieved": flops / (c32 / 1e3) / 1e12, "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": flops / (c32 / 1e3) / PEAK_FP32_MFMA, "traffic": None, "avg_launch_us": 1e3 * c32},
        "contraction_fp64": {"achieved_tflops": flops / (c64 / 1e3) / 1e12, "peak_tflops": PEAK_FP64 / 1e12,
                             "frac": flops / (c64 / 1e3) / PEAK_FP64, "kernel_ms": c64},
    }
    print(json.dumps(line), flush=True)


def bench_scan(args):
    """The paper's workload families end to end (automatic cuts isolating
    the injected T gate within 4-qubit fragments, planning, exact GPU
    evaluation): near-Clifford HWEA (5 rounds), SK-model MaxCut QAOA (one
    round) and one round of the phase-flip repetition code, five seeded
    circuits per size.  Dense outputs are per-qubit marginals (from <Z_q>),
    the repetition code's the full syndrome distribution; their agreement
    with the uncut state vector is a test, not part of this timing.
    value = circuits per second over the whole scan."""
    import numpy as np
    import torch

    import paper_2303_10788_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    ctx = cc.Context(0)
    fams = [("hwea", lambda n, s: W.hwea(n, seed=s), [10, 20, 50, 100, 200, 300]),
            ("qaoa", lambda n, s: W.qaoa_sk(n, seed=s), [4, 8, 12, 16, 20, 26]),
            ("phase", lambda n, s: W.phase_code(n, seed=s), [5, 9, 13, 17, 21])]
    rows, total_s, total_c = [], 0.0, 0
    warm = W.hwea(10, seed=99)  # first-call costs (module loads, allocations) out of the scan
    cc.Plan(ctx, warm.n, warm.ops, cc.find_cuts(warm.n, warm.ops, 4)).zexpect(warm.zmask_words())
    for fam, make, sizes in fams:
        for n in sizes:
            times, ks = [], []
            for s in range(5):
                w = make(n, s)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                cuts = cc.find_cuts(w.n, w.ops, 4)
                plan = cc.Plan(ctx, w.n, w.ops, cuts)
                if fam == "phase":
                    plan.marginal(w.qubits)
                else:
                    plan.zexpect(w.zmask_words())
                dt = time.perf_counter() - t0
                times.append(dt)
                ks.append(len(cuts))
                plan.close()
            total_s += sum(times)
            total_c += len(times)
            rows.append({"family": fam, "qubits": w.n, "cuts": ks, "ms_mean": 1e3 * float(np.mean(times)),
                         "ms_max": 1e3 * float(np.max(times))})
    line = {
        "metric": METRIC, "value": total_c / total_s, "unit": "circuits/s (cut + plan + exact GPU evaluation)",
        "n_gpus": 1, "steps": total_c, "warmup": 1, "ms_per_step": 1e3 * total_s / total_c, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64/f64", "data": "synthetic",
        "config": {"workload": "scan: near-Clifford HWEA (5 rounds), SK MaxCut QAOA (1 round), phase-flip "
                               "repetition code (1 round), one T each, automatic cuts within 4-qubit fragments"},
        "scan": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
