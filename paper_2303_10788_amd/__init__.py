"""Clifford-based circuit cutting on MI355X: Python binding of libccut.so.

The functions named ``ccut_*`` mirror the C ABI in include/ccut.h one to
one (argument marshalling only; every step runs in the library's HIP
kernels).  ``Context`` and ``Plan`` are thin conveniences over them that
hand the library torch's current stream and caching allocator.

The library is loaded from this package directory; if it is missing the
import of the binding fails loudly (build it with
``python -m paper_2303_10788_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccut.so")

GATES = {"H": 0, "S": 1, "SDG": 2, "X": 3, "Y": 4, "Z": 5, "CX": 6, "CZ": 7, "T": 8, "TDG": 9, "RZ": 10}
CCUT_OK, CCUT_E_INVALID, CCUT_E_OOM, CCUT_E_DEVICE = 0, -1, -2, -3
CCUT_E_NC_TOO_WIDE, CCUT_E_TOO_MANY_CUTS, CCUT_E_CANCELLED, CCUT_E_UNSUPPORTED = -4, -5, -6, -7
CCUT_FP64, CCUT_FP32_MFMA_FP64SUM, CCUT_FP32X3_MFMA_FP64SUM = 0, 1, 2
CCUT_METHOD_AUTO, CCUT_METHOD_VARIANTS, CCUT_METHOD_HEISENBERG = 0, 1, 2
CCUT_FLAG_SPARSE, CCUT_FLAG_SETTLE, CCUT_FLAG_ML, CCUT_FLAG_SKIP = 1, 2, 4, 8
KERNELS = ("affine_kernel", "sample_kernel", "hist_reduce_kernel", "exact_kernel", "sv_kernel",
           "parity_kernel", "transform_pass_kernel", "recombine_fp64_kernel", "zrecombine_fp64_kernel",
           "heisenberg_kernels", "mlp_kernels", "term_kernels", "carry_kernel")
STATUS_NAMES = {0: "CCUT_OK", -1: "CCUT_E_INVALID", -2: "CCUT_E_OOM", -3: "CCUT_E_DEVICE",
                -4: "CCUT_E_NC_TOO_WIDE", -5: "CCUT_E_TOO_MANY_CUTS", -6: "CCUT_E_CANCELLED",
                -7: "CCUT_E_UNSUPPORTED"}


class ccut_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("q0", ctypes.c_uint32), ("q1", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("theta", ctypes.c_double)]


class ccut_cut(ctypes.Structure):
    _fields_ = [("qubit", ctypes.c_uint32), ("after_op", ctypes.c_uint32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class ccut_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("user", ctypes.c_void_p), ("max_nc_qubits", ctypes.c_uint32),
                ("max_cuts", ctypes.c_uint32)]


class ccut_eval_opts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("shots_per_variant", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("circuit", ctypes.c_uint32), ("method", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class CcutError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# exported symbols and their signatures (argtypes, restype)
_P = ctypes.c_void_p
_U32P = ctypes.POINTER(ctypes.c_uint32)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "ccut_ctx_create": ([ctypes.POINTER(ccut_opts), ctypes.POINTER(_P)], ctypes.c_int),
    "ccut_ctx_destroy": ([_P], None),
    "ccut_last_error": ([_P], ctypes.c_char_p),
    "ccut_cancel": ([_P], None),
    "ccut_plan_create": ([_P, ctypes.c_uint32, ctypes.POINTER(ccut_op), ctypes.c_size_t,
                          ctypes.POINTER(ccut_cut), ctypes.c_size_t, ctypes.POINTER(_P)], ctypes.c_int),
    "ccut_plan_destroy": ([_P], None),
    "ccut_plan_info": ([_P, _U32P, _U64P, _U64P], ctypes.c_int),
    "ccut_fragment_info": ([_P, ctypes.c_uint32, _U32P, _I32P, _U32P, _U64P], ctypes.c_int),
    "ccut_fragment_segments": ([_P, ctypes.c_uint32, _U32P, _U32P], ctypes.c_int),
    "ccut_fragment_axes": ([_P, ctypes.c_uint32, _U32P, _U32P, _U32P], ctypes.c_int),
    "ccut_marginal": ([_P, ctypes.POINTER(ccut_eval_opts), _U32P, ctypes.c_uint32, _P, ctypes.c_int],
                      ctypes.c_int),
    "ccut_zexpect": ([_P, ctypes.POINTER(ccut_eval_opts), _U64P, ctypes.c_uint32, _P, ctypes.c_int],
                     ctypes.c_int),
    "ccut_shot_records": ([_P, ctypes.POINTER(ccut_eval_opts), _U32P, ctypes.c_uint32, ctypes.c_uint32,
                           ctypes.c_uint64, ctypes.c_uint64, _P, ctypes.c_int], ctypes.c_int),
    "ccut_variant_tables": ([_P, ctypes.POINTER(ccut_eval_opts), _U32P, ctypes.c_uint32, ctypes.c_uint32,
                             _P, ctypes.c_int], ctypes.c_int),
    "ccut_fragment_tensor": ([_P, ctypes.POINTER(ccut_eval_opts), _U32P, ctypes.c_uint32, ctypes.c_uint32,
                              _P, ctypes.c_int], ctypes.c_int),
    "ccut_request_info": ([_P, _U32P, ctypes.c_uint32, ctypes.c_uint32, _U32P, _U32P], ctypes.c_int),
    "ccut_fragment_ops": ([_P, ctypes.c_uint32, _U32P, _U32P], ctypes.c_int),
    "ccut_batch_create": ([_P, ctypes.POINTER(_P), ctypes.c_size_t, ctypes.POINTER(ccut_eval_opts),
                           ctypes.POINTER(_U32P), _U32P, ctypes.c_int, ctypes.POINTER(_P)], ctypes.c_int),
    "ccut_batch_run": ([_P, ctypes.POINTER(_P), ctypes.c_int], ctypes.c_int),
    "ccut_batch_info": ([_P, _U64P, _U32P, _U32P, _I32P, _I32P, _DP], ctypes.c_int),
    "ccut_batch_destroy": ([_P], None),
    "ccut_run_batch": ([_P, ctypes.POINTER(_P), ctypes.c_size_t, ctypes.POINTER(ccut_eval_opts),
                        ctypes.POINTER(_U32P), _U32P, ctypes.POINTER(_P)], ctypes.c_int),
    "ccut_timing_enable": ([_P, ctypes.c_int], ctypes.c_int),
    "ccut_call_graphs": ([_P, ctypes.c_int], ctypes.c_int),
    "ccut_timing_reset": ([_P], ctypes.c_int),
    "ccut_timing_read": ([_P, ctypes.c_uint32, _U64P, _DP], ctypes.c_int),
    "ccut_kernel_name": ([ctypes.c_uint32], ctypes.c_char_p),
    "ccut_learned_create": ([_P, ctypes.POINTER(ccut_eval_opts), _U32P, ctypes.c_uint32, ctypes.POINTER(_P)],
                            ctypes.c_int),
    "ccut_learned_info": ([_P, _U32P, _U64P, _U32P], ctypes.c_int),
    "ccut_learned_features": ([_P, _P, ctypes.c_uint64, ctypes.c_uint64, _P], ctypes.c_int),
    "ccut_learned_log_weights": ([_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _P], ctypes.c_int),
    "ccut_learned_support": ([_P, ctypes.c_uint64, _P, _U64P], ctypes.c_int),
    "ccut_learned_logits": ([_P, _P, _P], ctypes.c_int),
    "ccut_learned_estimate": ([_P, _P, ctypes.c_uint64, ctypes.c_uint64, _P, ctypes.c_int, _P], ctypes.c_int),
    "ccut_learned_exhaustive": ([_P, _P, ctypes.c_int], ctypes.c_int),
    "ccut_learned_destroy": ([_P], None),
    "ccut_learned_marginal": ([_P, ctypes.POINTER(ccut_eval_opts), _P, ctypes.c_uint64, _U32P, ctypes.c_uint32, _P,
                               ctypes.c_int, _DP], ctypes.c_int),
    "ccut_proposal": ([_P, _P, ctypes.c_uint64, ctypes.c_double, _P], ctypes.c_int),
    "ccut_sample_terms": ([_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _P],
                          ctypes.c_int),
    "ccut_sample_terms_noalloc": ([_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                   _P], ctypes.c_int),
    "ccut_mlp_create": ([_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_P)], ctypes.c_int),
    "ccut_mlp_set_params": ([_P, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t], ctypes.c_int),
    "ccut_mlp_get_params": ([_P, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t], ctypes.c_int),
    "ccut_mlp_forward": ([_P, _P, ctypes.c_uint64, _P], ctypes.c_int),
    "ccut_mlp_gradients": ([_P, _P, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float), _DP], ctypes.c_int),
    "ccut_mlp_train": ([_P, _P, _P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_float,
                        ctypes.c_uint64, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "ccut_mlp_train_step": ([_P, _P, _P, ctypes.c_uint64, ctypes.c_float, ctypes.POINTER(ctypes.c_float)],
                            ctypes.c_int),
    "ccut_mlp_destroy": ([_P], None),
    "ccut_find_cuts": ([ctypes.c_uint32, ctypes.POINTER(ccut_op), ctypes.c_size_t, ctypes.c_uint32,
                        ctypes.POINTER(ccut_cut), ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libccut.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2303_10788_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(st: int, ctx) -> None:
    if st != CCUT_OK:
        msg = lib().ccut_last_error(ctx)
        raise CcutError(st, msg.decode() if msg else "")


# ----------------------------------------------------------- same-name calls

def ccut_ctx_create(opts: Optional[ccut_opts]):
    h = _P()
    st = lib().ccut_ctx_create(ctypes.byref(opts) if opts is not None else None, ctypes.byref(h))
    _check(st, None)
    return h


def ccut_ctx_destroy(ctx) -> None:
    lib().ccut_ctx_destroy(ctx)


def ccut_last_error(ctx) -> str:
    return (lib().ccut_last_error(ctx) or b"").decode()


def ccut_cancel(ctx) -> None:
    lib().ccut_cancel(ctx)


def _ops_array(ops):
    arr = (ccut_op * max(len(ops), 1))()
    for i, (k, a, b, th) in enumerate(ops):
        arr[i] = ccut_op(GATES[k] if isinstance(k, str) else int(k), int(a), int(b) if b >= 0 else 0, 0,
                         float(th))
    return arr


def _cuts_array(cuts):
    arr = (ccut_cut * max(len(cuts), 1))()
    for i, (q, a) in enumerate(cuts):
        arr[i] = ccut_cut(int(q), int(a))
    return arr


def ccut_find_cuts(n_qubits: int, ops, max_width: int = 12):
    """Cut locations [(qubit, after_op)] that put every non-Clifford op in
    a fragment of at most max_width qubits, with few cuts."""
    arr = _ops_array(ops)
    k = ctypes.c_size_t()
    cap = max(2 * len(ops), 1)
    out = (ccut_cut * cap)()
    _check(lib().ccut_find_cuts(n_qubits, arr, len(ops), max_width, out, cap, ctypes.byref(k)), None)
    return [(out[i].qubit, out[i].after_op) for i in range(k.value)]


find_cuts = ccut_find_cuts


def ccut_plan_create(ctx, n_qubits: int, ops, cuts):
    h = _P()
    st = lib().ccut_plan_create(ctx, n_qubits, _ops_array(ops), len(ops), _cuts_array(cuts), len(cuts),
                                ctypes.byref(h))
    _check(st, ctx)
    return h


def ccut_plan_destroy(plan) -> None:
    lib().ccut_plan_destroy(plan)


def ccut_plan_info(plan):
    nf, nv, nt = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    st = lib().ccut_plan_info(plan, ctypes.byref(nf), ctypes.byref(nv), ctypes.byref(nt))
    _check(st, None)
    return nf.value, nv.value, nt.value


def ccut_fragment_info(plan, f: int):
    m, cl, na, nv = ctypes.c_uint32(), ctypes.c_int32(), ctypes.c_uint32(), ctypes.c_uint64()
    st = lib().ccut_fragment_info(plan, f, ctypes.byref(m), ctypes.byref(cl), ctypes.byref(na), ctypes.byref(nv))
    _check(st, None)
    return m.value, bool(cl.value), na.value, nv.value


def ccut_fragment_segments(plan, f: int):
    m = ccut_fragment_info(plan, f)[0]
    w = (ctypes.c_uint32 * m)()
    s = (ctypes.c_uint32 * m)()
    _check(lib().ccut_fragment_segments(plan, f, w, s), None)
    return list(zip(list(w), list(s)))


def ccut_fragment_axes(plan, f: int):
    na = ccut_fragment_info(plan, f)[2]
    c, s, l = (ctypes.c_uint32 * max(na, 1))(), (ctypes.c_uint32 * max(na, 1))(), (ctypes.c_uint32 * max(na, 1))()
    _check(lib().ccut_fragment_axes(plan, f, c, s, l), None)
    return [(c[j], s[j], l[j]) for j in range(na)]


def _eval_opts(shots=0, seed=0, precision=CCUT_FP64, circuit=0, method=CCUT_METHOD_AUTO, flags=0):
    return ccut_eval_opts(int(seed) & 0xFFFFFFFFFFFFFFFF, int(shots), int(precision), int(circuit), int(method),
                          int(flags))


def _u32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return a, a.ctypes.data_as(_U32P)


def _out_ptr(out):
    """(pointer, on_device) for a numpy array or a torch tensor."""
    if isinstance(out, np.ndarray):
        return ctypes.c_void_p(out.ctypes.data), 0
    return ctypes.c_void_p(out.data_ptr()), 1 if out.is_cuda else 0


def ccut_marginal(plan, ctx, eo: ccut_eval_opts, qubits, out) -> None:
    q, qp = _u32(qubits)
    p, dev = _out_ptr(out)
    _check(lib().ccut_marginal(plan, ctypes.byref(eo), qp, len(q), p, dev), ctx)


def ccut_zexpect(plan, ctx, eo: ccut_eval_opts, masks: np.ndarray, out) -> None:
    m = np.ascontiguousarray(masks, dtype=np.uint64)
    p, dev = _out_ptr(out)
    _check(lib().ccut_zexpect(plan, ctypes.byref(eo), m.ctypes.data_as(_U64P), m.shape[0], p, dev), ctx)


def ccut_shot_records(plan, ctx, eo, qubits, fragment, v_begin, v_end, out) -> None:
    q, qp = _u32(qubits)
    p, dev = _out_ptr(out)
    _check(lib().ccut_shot_records(plan, ctypes.byref(eo), qp, len(q), fragment, v_begin, v_end, p, dev), ctx)


def ccut_variant_tables(plan, ctx, eo, qubits, fragment, out) -> None:
    q, qp = _u32(qubits)
    p, dev = _out_ptr(out)
    _check(lib().ccut_variant_tables(plan, ctypes.byref(eo), qp, len(q), fragment, p, dev), ctx)


def ccut_fragment_tensor(plan, ctx, eo, qubits, fragment, out) -> None:
    q, qp = _u32(qubits)
    p, dev = _out_ptr(out)
    _check(lib().ccut_fragment_tensor(plan, ctypes.byref(eo), qp, len(q), fragment, p, dev), ctx)


def ccut_fragment_ops(plan, f: int):
    one, two = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().ccut_fragment_ops(plan, f, ctypes.byref(one), ctypes.byref(two)), None)
    return one.value, two.value


def ccut_request_info(plan, qubits, fragment):
    q, qp = _u32(qubits)
    nm, nr = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().ccut_request_info(plan, qp, len(q), fragment, ctypes.byref(nm), ctypes.byref(nr)), None)
    return nm.value, nr.value


def _batch_args(plans, qubits):
    n = len(plans)
    ph = (_P * n)(*[p.handle for p in plans])
    qarrs = [np.ascontiguousarray(np.asarray(q, dtype=np.uint32)) for q in qubits]
    qp = (_U32P * n)(*[a.ctypes.data_as(_U32P) for a in qarrs])
    nq = (ctypes.c_uint32 * n)(*[len(q) for q in qubits])
    return ph, qarrs, qp, nq


def ccut_batch_create(ctx, plans, eo, qubits, use_graph=True):
    ph, keep, qp, nq = _batch_args(plans, qubits)
    h = _P()
    _check(lib().ccut_batch_create(ctx, ph, len(plans), ctypes.byref(eo), qp, nq, 1 if use_graph else 0,
                                   ctypes.byref(h)), ctx)
    return h


def ccut_batch_run(batch, ctx, outs) -> None:
    ptrs = [_out_ptr(o) for o in outs]
    arr = (_P * len(outs))(*[p for p, _ in ptrs])
    _check(lib().ccut_batch_run(batch, arr, ptrs[0][1] if ptrs else 0), ctx)


def ccut_batch_info(batch):
    n, blk, grid, reg, gr, ms = (ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int32(),
                                  ctypes.c_int32(), ctypes.c_double())
    _check(lib().ccut_batch_info(batch, ctypes.byref(n), ctypes.byref(blk), ctypes.byref(grid), ctypes.byref(reg),
                                 ctypes.byref(gr), ctypes.byref(ms)), None)
    return dict(n_items=n.value, block=blk.value, grid=grid.value, tune_cached=bool(reg.value),
                graphed=bool(gr.value), models_ms=ms.value)


def ccut_batch_destroy(batch) -> None:
    lib().ccut_batch_destroy(batch)


def ccut_run_batch(ctx, plans, eo, qubits, outs) -> None:
    ph, keep, qp, nq = _batch_args(plans, qubits)
    arr = (_P * len(outs))(*[o.ctypes.data for o in outs])
    _check(lib().ccut_run_batch(ctx, ph, len(plans), ctypes.byref(eo), qp, nq, arr), ctx)


def ccut_timing_enable(ctx, on: bool) -> None:
    _check(lib().ccut_timing_enable(ctx, 1 if on else 0), ctx)


def ccut_call_graphs(ctx, on: bool) -> None:
    _check(lib().ccut_call_graphs(ctx, 1 if on else 0), ctx)


def ccut_timing_reset(ctx) -> None:
    _check(lib().ccut_timing_reset(ctx), ctx)


def ccut_timing_read(ctx, kid: int):
    n, ms = ctypes.c_uint64(), ctypes.c_double()
    _check(lib().ccut_timing_read(ctx, kid, ctypes.byref(n), ctypes.byref(ms)), ctx)
    return n.value, ms.value


def ccut_kernel_name(kid: int) -> str:
    return lib().ccut_kernel_name(kid).decode()


# ----------------------------------------------------------- conveniences

class Context:
    """A library context on one device.  ``device=None`` uses torch's
    current device, stream and caching allocator; ``device=-1`` makes a
    host-only context (planning and validation only)."""

    def __init__(self, device: Optional[int] = None, *, max_nc_qubits: int = 0, max_cuts: int = 0,
                 use_torch: bool = True):
        self._keep = []
        opts = ccut_opts()
        opts.max_nc_qubits = max_nc_qubits
        opts.max_cuts = max_cuts
        if device is not None and device < 0:
            opts.device = -1
        else:
            import torch
            dev = torch.cuda.current_device() if device is None else int(device)
            opts.device = dev
            if use_torch:
                stream = torch.cuda.current_stream(dev)
                opts.hip_stream = ctypes.c_void_p(stream.cuda_stream)

                def _alloc(size, user, _dev=dev, _s=stream, _a=torch.cuda.caching_allocator_alloc):
                    try:
                        return _a(size, _dev, _s)
                    except Exception:
                        return None

                def _free(ptr, user, _d=torch.cuda.caching_allocator_delete):
                    try:
                        _d(ptr)
                    except Exception:  # interpreter shutdown: torch already torn down
                        pass

                a, f = ALLOC_FN(_alloc), FREE_FN(_free)
                self._keep += [a, f]
                opts.alloc, opts.free = a, f
        self.device = opts.device
        self.handle = ccut_ctx_create(opts)

    def close(self):
        if getattr(self, "handle", None):
            ccut_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing(self, on: bool = True):
        ccut_timing_enable(self.handle, on)

    def call_graphs(self, on: bool = True):
        """Replay repeated device-output marginal/zexpect calls as captured
        HIP graphs (on by default)."""
        ccut_call_graphs(self.handle, on)

    def timing_reset(self):
        ccut_timing_reset(self.handle)

    def kernel_times(self):
        """{kernel name: (launches, total ms)} since the last reset."""
        return {KERNELS[k]: ccut_timing_read(self.handle, k) for k in range(len(KERNELS))}


class Plan:
    """A planned circuit + cut list (fragments and variants fixed)."""

    def __init__(self, ctx: Context, n: int, ops: Sequence, cuts: Sequence):
        self.ctx = ctx
        self.n = n
        self.handle = ccut_plan_create(ctx.handle, n, ops, cuts)

    def close(self):
        if getattr(self, "handle", None):
            ccut_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return ccut_plan_info(self.handle)

    def fragments(self):
        nf = self.info()[0]
        out = []
        for f in range(nf):
            m, cl, na, nv = ccut_fragment_info(self.handle, f)
            one, two = ccut_fragment_ops(self.handle, f)
            out.append(dict(m=m, clifford=cl, n_variants=nv, segments=ccut_fragment_segments(self.handle, f),
                            axes=ccut_fragment_axes(self.handle, f), n_one=one, n_two=two))
        return out

    def marginal(self, qubits, *, shots=0, seed=0, precision=CCUT_FP64, circuit=0, method=CCUT_METHOD_AUTO,
                 out=None, flags=0):
        eo = _eval_opts(shots, seed, precision, circuit, method, flags)
        if out is None:
            out = np.zeros(1 << len(qubits), dtype=np.float64)
        ccut_marginal(self.handle, self.ctx.handle, eo, qubits, out)
        return out

    def learned_marginal(self, mlp, qubits, n_terms, *, shots=0, seed=0, circuit=0, method=CCUT_METHOD_AUTO,
                         out=None):
        """Importance-sampled marginal with `mlp` as the term proposal:
        (estimate, summed standard error of its entries)."""
        eo = _eval_opts(shots, seed, CCUT_FP64, circuit, method)
        if out is None:
            out = np.zeros(1 << len(qubits), dtype=np.float64)
        se = ccut_learned_marginal(self.handle, self.ctx.handle, eo, mlp.handle, n_terms, qubits, out)
        return out, se

    def zexpect(self, masks, *, shots=0, seed=0, precision=CCUT_FP64, circuit=0, method=CCUT_METHOD_AUTO,
                out=None, flags=0):
        masks = np.asarray(masks, dtype=np.uint64)
        if masks.ndim == 1:
            masks = masks[:, None]
        if out is None:
            out = np.zeros(masks.shape[0], dtype=np.float64)
        ccut_zexpect(self.handle, self.ctx.handle, _eval_opts(shots, seed, precision, circuit, method, flags), masks,
                     out)
        return out

    def shot_records(self, qubits, fragment, v_begin, v_end, *, shots, seed=0, circuit=0):
        """uint64 records [variant][shot] (at most 64 measurements), else
        [variant][shot][ceil(n_meas / 64)] (bit j of word w = measurement
        64 w + j)."""
        nm, _ = ccut_request_info(self.handle, qubits, fragment)
        rw = (nm + 63) // 64 if nm > 64 else 1
        out = np.zeros((v_end - v_begin) * shots * rw, dtype=np.uint64)
        ccut_shot_records(self.handle, self.ctx.handle, _eval_opts(shots, seed, 0, circuit), qubits, fragment,
                          v_begin, v_end, out)
        return out.reshape(v_end - v_begin, shots) if rw == 1 else out.reshape(v_end - v_begin, shots, rw)

    def variant_tables(self, qubits, fragment, *, shots=0, seed=0, circuit=0, flags=0):
        nm, _ = ccut_request_info(self.handle, qubits, fragment)
        nv = ccut_fragment_info(self.handle, fragment)[3]
        out = np.zeros(nv << nm, dtype=np.float64)
        ccut_variant_tables(self.handle, self.ctx.handle, _eval_opts(shots, seed, 0, circuit, flags=flags), qubits,
                            fragment, out)
        return out.reshape(nv, 1 << nm)

    def fragment_tensor(self, qubits, fragment, *, shots=0, seed=0, circuit=0, method=CCUT_METHOD_AUTO, flags=0):
        _, nr = ccut_request_info(self.handle, qubits, fragment)
        na = ccut_fragment_info(self.handle, fragment)[2]
        out = np.zeros((4 ** na) << nr, dtype=np.float64)
        ccut_fragment_tensor(self.handle, self.ctx.handle, _eval_opts(shots, seed, 0, circuit, method, flags), qubits,
                             fragment, out)
        return out.reshape(4 ** na, 1 << nr)


class Batch:
    """Many plans evaluated together: one persistent autotuned tableau
    launch for all Clifford variants, the rest per plan, captured once as a
    HIP graph (``use_graph``) and replayed by ``run``."""

    def __init__(self, ctx: Context, plans, qubits, *, shots=0, seed=0, precision=CCUT_FP64,
                 method=CCUT_METHOD_AUTO, use_graph=True):
        self.ctx = ctx
        self.plans = list(plans)
        self.qubits = [list(q) for q in qubits]
        self.handle = ccut_batch_create(ctx.handle, self.plans, _eval_opts(shots, seed, precision, 0, method),
                                        self.qubits, use_graph)

    def info(self):
        return ccut_batch_info(self.handle)

    def run(self, outs=None):
        if outs is None:
            outs = [np.zeros(1 << len(q), dtype=np.float64) for q in self.qubits]
        ccut_batch_run(self.handle, self.ctx.handle, outs)
        return outs

    def close(self):
        if getattr(self, "handle", None):
            ccut_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------- learned term proposal
# Device buffers are torch tensors on the context's device (bf16 rows are
# torch.bfloat16, labels/logits float32, q float64, term lists int64).

def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def ccut_learned_create(plan, ctx, eo, qubits):
    q, qp = _u32(qubits)
    h = _P()
    _check(lib().ccut_learned_create(plan, ctypes.byref(eo), qp, len(q), ctypes.byref(h)), ctx)
    return h


def ccut_learned_info(L):
    k, K, w = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
    _check(lib().ccut_learned_info(L, ctypes.byref(k), ctypes.byref(K), ctypes.byref(w)), None)
    return k.value, K.value, w.value


def ccut_learned_features(L, ctx, terms, first, n, x):
    _check(lib().ccut_learned_features(L, _dptr(terms), first, n, _dptr(x)), ctx)


def ccut_learned_log_weights(L, ctx, terms, first, n, kind, y):
    _check(lib().ccut_learned_log_weights(L, _dptr(terms), first, n, kind, _dptr(y)), ctx)


def ccut_learned_support(L, ctx, cap, terms):
    cnt = ctypes.c_uint64()
    _check(lib().ccut_learned_support(L, cap, _dptr(terms), ctypes.byref(cnt)), ctx)
    return cnt.value


def ccut_learned_logits(L, ctx, mlp, logits):
    _check(lib().ccut_learned_logits(L, mlp, _dptr(logits)), ctx)


def ccut_learned_estimate(L, ctx, q, n, seed, out, terms_out=None):
    p, dev = _out_ptr(out)
    _check(lib().ccut_learned_estimate(L, _dptr(q), n, int(seed) & 0xFFFFFFFFFFFFFFFF, p, dev, _dptr(terms_out)),
           ctx)


def ccut_learned_exhaustive(L, ctx, out):
    p, dev = _out_ptr(out)
    _check(lib().ccut_learned_exhaustive(L, p, dev), ctx)


def ccut_learned_destroy(L) -> None:
    lib().ccut_learned_destroy(L)


def ccut_learned_marginal(plan, ctx, eo, mlp, n_terms, qubits, out, want_stderr=True):
    q, qp = _u32(qubits)
    p, dev = _out_ptr(out)
    se = ctypes.c_double()
    _check(lib().ccut_learned_marginal(plan, ctypes.byref(eo), mlp, n_terms, qp, len(q), p, dev,
                                       ctypes.byref(se) if want_stderr else None), ctx)
    return se.value if want_stderr else None


def ccut_proposal(ctx, logits, K, eps, q):
    _check(lib().ccut_proposal(ctx, _dptr(logits), K, eps, _dptr(q)), ctx)


def ccut_sample_terms(ctx, q, K, n, seed, cid, out):
    _check(lib().ccut_sample_terms(ctx, _dptr(q), K, n, int(seed) & 0xFFFFFFFFFFFFFFFF,
                                   int(cid) & 0xFFFFFFFFFFFFFFFF, _dptr(out)), ctx)


def ccut_sample_terms_noalloc(stream, q, K, n, seed, cid, out):
    """The allocation-free term draw on the current device, enqueued on
    `stream` (a torch stream, a raw hipStream_t, or None for the null
    stream); out is valid in stream order."""
    raw = getattr(stream, "cuda_stream", stream)
    _check(lib().ccut_sample_terms_noalloc(raw, _dptr(q), K, n, int(seed) & 0xFFFFFFFFFFFFFFFF,
                                           int(cid) & 0xFFFFFFFFFFFFFFFF, _dptr(out)), None)


def ccut_mlp_create(ctx, F, H):
    h = _P()
    _check(lib().ccut_mlp_create(ctx, F, H, ctypes.byref(h)), ctx)
    return h


def ccut_mlp_set_params(M, ctx, params: np.ndarray):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().ccut_mlp_set_params(M, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size), ctx)


def ccut_mlp_get_params(M, ctx, count):
    a = np.zeros(count, dtype=np.float32)
    _check(lib().ccut_mlp_get_params(M, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), count), ctx)
    return a


def ccut_mlp_forward(M, ctx, x, n, y):
    _check(lib().ccut_mlp_forward(M, _dptr(x), n, _dptr(y)), ctx)


def ccut_mlp_gradients(M, ctx, x, t, n, count):
    g = np.zeros(count, dtype=np.float32)
    loss = ctypes.c_double()
    _check(lib().ccut_mlp_gradients(M, _dptr(x), _dptr(t), n, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    ctypes.byref(loss)), ctx)
    return g, loss.value


def ccut_mlp_train(M, ctx, x, t, n, batch, steps, lr, seed):
    losses = np.zeros(max(steps, 1), dtype=np.float32)
    _check(lib().ccut_mlp_train(M, _dptr(x), _dptr(t), n, batch, steps, lr, int(seed) & 0xFFFFFFFFFFFFFFFF,
                                losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), ctx)
    return losses[:steps]


def ccut_mlp_train_step(M, ctx, x, t, n, lr):
    loss = ctypes.c_float()
    _check(lib().ccut_mlp_train_step(M, _dptr(x), _dptr(t), n, lr, ctypes.byref(loss)), ctx)
    return loss.value


def ccut_mlp_destroy(M) -> None:
    lib().ccut_mlp_destroy(M)


def mlp_param_count(F: int, H: int) -> int:
    return H * F + 2 * H * H + 4 * H + 1


def mlp_pack(params) -> np.ndarray:
    """Flat parameter vector from [(W1, b1), (W2, b2), (W3, b3), (w4, b4)]."""
    return np.concatenate([np.ravel(a) for W, b in params for a in (W, b)]).astype(np.float32)


def mlp_unpack(flat, F: int, H: int):
    shapes = [((H, F), (H,)), ((H, H), (H,)), ((H, H), (H,)), ((1, H), (1,))]
    out, o = [], 0
    for sw, sb in shapes:
        nw, nb = int(np.prod(sw)), int(np.prod(sb))
        out.append((np.asarray(flat[o:o + nw]).reshape(sw), np.asarray(flat[o + nw:o + nw + nb]).reshape(sb)))
        o += nw + nb
    return out


class Mlp:
    """The F -> H -> H -> H -> 1 ReLU network on the device."""

    def __init__(self, ctx: Context, F: int = 64, H: int = 256):
        self.ctx, self.F, self.H = ctx, F, H
        self.count = mlp_param_count(F, H)
        self.handle = ccut_mlp_create(ctx.handle, F, H)

    def set_params(self, flat):
        ccut_mlp_set_params(self.handle, self.ctx.handle, flat)

    def get_params(self):
        return ccut_mlp_get_params(self.handle, self.ctx.handle, self.count)

    def forward(self, x, y=None):
        import torch
        if y is None:
            y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        ccut_mlp_forward(self.handle, self.ctx.handle, x, x.shape[0], y)
        return y

    def gradients(self, x, t):
        return ccut_mlp_gradients(self.handle, self.ctx.handle, x, t, x.shape[0], self.count)

    def train(self, x, t, *, batch, steps, lr=1e-3, seed=0):
        return ccut_mlp_train(self.handle, self.ctx.handle, x, t, x.shape[0], batch, steps, lr, seed)

    def train_step(self, x, t, lr=1e-3):
        """One Adam step on the whole batch x (fp32 [n][F], rounded to bf16), t [n]."""
        return ccut_mlp_train_step(self.handle, self.ctx.handle, x, t, x.shape[0], lr)

    def close(self):
        if getattr(self, "handle", None):
            ccut_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Learned:
    """Per-circuit term model: fragment tensors, column norms and share
    tables of one marginal request, kept on the device."""

    def __init__(self, plan: Plan, qubits, *, shots=0, seed=0, circuit=0, method=CCUT_METHOD_AUTO,
                 precision=CCUT_FP64):
        self.plan, self.ctx = plan, plan.ctx
        self.nq = len(qubits)
        self.handle = ccut_learned_create(plan.handle, self.ctx.handle,
                                          _eval_opts(shots, seed, precision, circuit, method), qubits)
        self.k, self.K, self.width = ccut_learned_info(self.handle)

    def features(self, terms=None, first=0, n=None):
        import torch
        n = (terms.shape[0] if terms is not None else self.K - first) if n is None else n
        x = torch.empty((n, self.width), dtype=torch.bfloat16, device="cuda")
        ccut_learned_features(self.handle, self.ctx.handle, terms, first, n, x)
        return x

    def log_weights(self, terms=None, first=0, n=None, kind=0):
        import torch
        n = (terms.shape[0] if terms is not None else self.K - first) if n is None else n
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        ccut_learned_log_weights(self.handle, self.ctx.handle, terms, first, n, kind, y)
        return y

    def support(self, cap=1 << 16):
        import torch
        t = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
        cnt = ccut_learned_support(self.handle, self.ctx.handle, cap, t)
        return t[:min(cnt, cap)], cnt

    def logits(self, mlp: Mlp):
        import torch
        y = torch.empty(self.K, dtype=torch.float32, device="cuda")
        ccut_learned_logits(self.handle, self.ctx.handle, mlp.handle, y)
        return y

    def estimate(self, q, n, seed, out=None, terms_out=None):
        if out is None:
            out = np.zeros(1 << self.nq)
        ccut_learned_estimate(self.handle, self.ctx.handle, q, n, seed, out, terms_out)
        return out

    def exhaustive(self, out=None):
        if out is None:
            out = np.zeros(1 << self.nq)
        ccut_learned_exhaustive(self.handle, self.ctx.handle, out)
        return out

    def close(self):
        if getattr(self, "handle", None):
            ccut_learned_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def proposal(ctx: Context, logits, K=None, eps=0.05):
    """q (float64 device tensor) from logits, or uniform when logits is None."""
    import torch
    K = logits.shape[0] if K is None else K
    q = torch.empty(K, dtype=torch.float64, device="cuda")
    ccut_proposal(ctx.handle, logits, K, eps, q)
    return q


def sample_terms(ctx: Context, q, n, seed, cid):
    import torch
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    ccut_sample_terms(ctx.handle, q, q.shape[0], n, seed, cid, out)
    return out
