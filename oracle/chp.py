"""ctypes wrapper around the literal Aaronson-Gottesman tableau in chp.c.

``build()`` compiles chp.c with gcc into ``oracle/_chp.so``; ``lib()`` loads
it (building first if it is missing or older than the source).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chp.c")
_SO = os.path.join(_HERE, "_chp.so")
_lib = None

GATE_CODE = {"H": 0, "S": 1, "SDG": 2, "X": 3, "Y": 4, "Z": 5, "CX": 6, "CZ": 7}


def build(force: bool = False) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        vp = ctypes.c_void_p
        L.chp_new.restype = vp
        L.chp_new.argtypes = [ctypes.c_int]
        L.chp_free.argtypes = [vp]
        L.chp_clone.restype = vp
        L.chp_clone.argtypes = [vp]
        L.chp_copy_into.argtypes = [vp, vp]
        L.chp_gate.restype = ctypes.c_int
        L.chp_gate.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.chp_is_random.restype = ctypes.c_int
        L.chp_is_random.argtypes = [vp, ctypes.c_int]
        L.chp_measure.restype = ctypes.c_int
        L.chp_measure.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.chp_dump.argtypes = [vp, vp, vp, vp]
        L.chp_philox.argtypes = [vp, vp, vp]
        L.chp_sample.argtypes = [vp, vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64, vp]
        L.chp_sample_hist.argtypes = [vp, vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint64, vp]
        L.chp_exact.argtypes = [vp, vp, ctypes.c_int, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Tableau:
    """Owning handle of one n-qubit CHP tableau, initially |0...0>."""

    def __init__(self, n: int, _handle=None):
        self.n = n
        self._h = _handle if _handle is not None else lib().chp_new(n)

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.chp_free(h)

    def clone(self) -> "Tableau":
        return Tableau(self.n, lib().chp_clone(self._h))

    def gate(self, kind: str, a: int, b: int = -1) -> None:
        if lib().chp_gate(self._h, GATE_CODE[kind], a, b) != 0:
            raise ValueError(kind)

    def is_random(self, a: int) -> bool:
        return bool(lib().chp_is_random(self._h, a))

    def measure(self, a: int, bit: int = 0):
        """Measure qubit a in Z; a random outcome equals ``bit``.
        Returns ``(outcome, was_random)``."""
        wr = ctypes.c_int(0)
        o = lib().chp_measure(self._h, a, int(bit), ctypes.byref(wr))
        return o, bool(wr.value)

    def dump(self):
        """``(x, z, r)`` uint8 arrays of shape (2n+1, n), (2n+1, n), (2n+1,)."""
        rows = 2 * self.n + 1
        x = np.zeros((rows, self.n), np.uint8)
        z = np.zeros((rows, self.n), np.uint8)
        r = np.zeros(rows, np.uint8)
        lib().chp_dump(self._h, _ptr(x), _ptr(z), _ptr(r))
        return x, z, r

    def sample(self, meas, seed: int, vid: int, shot0: int, nshots: int) -> np.ndarray:
        """Per-shot literal measurement of ``meas`` in order; returns uint8
        outcomes of shape (nshots, len(meas))."""
        m = np.ascontiguousarray(meas, dtype=np.int32)
        out = np.zeros((nshots, len(m)), np.uint8)
        lib().chp_sample(self._h, _ptr(m), len(m), seed, vid, shot0, nshots, _ptr(out))
        return out

    def sample_hist(self, meas, seed: int, vid: int, nshots: int) -> np.ndarray:
        m = np.ascontiguousarray(meas, dtype=np.int32)
        h = np.zeros(1 << len(m), np.uint64)
        lib().chp_sample_hist(self._h, _ptr(m), len(m), seed, vid, nshots, _ptr(h))
        return h

    def exact(self, meas) -> np.ndarray:
        """Exact distribution over the outcomes of ``meas`` (bit j = meas[j])."""
        m = np.ascontiguousarray(meas, dtype=np.int32)
        t = np.zeros(1 << len(m), np.float64)
        lib().chp_exact(self._h, _ptr(m), len(m), _ptr(t))
        return t


def philox_c(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().chp_philox(_ptr(c), _ptr(k), _ptr(o))
    return tuple(int(v) for v in o)
