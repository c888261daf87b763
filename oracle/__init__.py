"""CPU oracle of the T-odd triple-product pass -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

Two layers:
* ``tp_oracle.c``: plain float64 textbook evaluation (rest-frame boost, triple
  product, plane angle, invariant masses), OpenMP over events.  Events whose
  float64 decision lies within a generous margin of a boundary are flagged.
* ``exact.py``: flagged events are decided in exact rational arithmetic.

``run()`` returns counts and stats of the whole sample; ``brute_force()``
decides every event exactly (small inputs only).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

from . import exact

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CLS_NAMES = ("I", "II", "III", "IV", "zero", "invalid")


def build(force: bool = True) -> str:
    """Compile the float64 oracle (gcc, OpenMP, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.or_pass.restype = ctypes.c_int64
        lib.or_pass.argtypes = [
            ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p,
            ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_void_p),
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        lib.or_max_threads.restype = ctypes.c_int32
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().or_max_threads())


def _arrays(comps, tag):
    """comps: array-like [4][4][n] (float32 or float64), tag int8[n] -> contiguous numpy."""
    arr = [[np.ascontiguousarray(np.asarray(comps[s][c])) for c in range(4)] for s in range(4)]
    dt = arr[0][0].dtype
    if dt not in (np.float32, np.float64) or any(a.dtype != dt for row in arr for a in row):
        raise TypeError("components must all be float32 or all float64")
    return arr, np.ascontiguousarray(np.asarray(tag, dtype=np.int8))


def _axes_tuple(axes):
    return [(int(a.kind), int(a.slots), np.asarray(a.edges, dtype=np.float64)) for a in axes]


def _event_comps(arr, i):
    return [[float(arr[s][c][i]) for c in range(4)] for s in range(4)]


def _pass(arr, tag, triple, planes, ax, nthreads, want_events, cap, identical=None):
    lib = _load()
    n = tag.shape[0]
    nb_total = int(np.prod([len(e) - 1 for _, _, e in ax])) if ax else 0
    counts = np.zeros((nb_total + 1) * 4, dtype=np.uint64)
    stats = np.zeros(4, dtype=np.uint64)
    flagged = np.zeros(cap, dtype=np.int64)
    cls = np.zeros(n, dtype=np.int8) if want_events else None
    ct = np.zeros(n, dtype=np.float64) if want_events else None
    coord = np.zeros(2 * n, dtype=np.float64) if want_events else None
    ptrs = (ctypes.c_void_p * 16)(*[arr[s][c].ctypes.data for s in range(4) for c in range(4)])
    kinds = (ctypes.c_int32 * 2)(*([k for k, _, _ in ax] + [0, 0])[:2])
    nbins = (ctypes.c_int32 * 2)(*([len(e) - 1 for _, _, e in ax] + [0, 0])[:2])
    slots = (ctypes.c_int32 * 2)(*([s for _, s, _ in ax] + [0, 0])[:2])
    edge_arrs = [np.ascontiguousarray(e) for _, _, e in ax]
    eptr = (ctypes.c_void_p * 2)(*([e.ctypes.data for e in edge_arrs] + [None, None])[:2])
    ident = (ctypes.c_int32 * 2)(*identical) if identical is not None else None
    t0 = time.perf_counter()
    nflag = lib.or_pass(n, 0 if arr[0][0].dtype == np.float32 else 1, ptrs, tag.ctypes.data,
                        (ctypes.c_int32 * 3)(*triple), (ctypes.c_int32 * 4)(*planes),
                        ctypes.cast(ident, ctypes.c_void_p) if ident is not None else None, len(ax),
                        kinds, nbins, slots, eptr, counts.ctypes.data, stats.ctypes.data,
                        flagged.ctypes.data, cap,
                        cls.ctypes.data if cls is not None else None,
                        ct.ctypes.data if ct is not None else None,
                        coord.ctypes.data if coord is not None else None, int(nthreads))
    seconds = time.perf_counter() - t0
    if coord is not None:
        ct = (ct, coord.reshape(n, 2))
    return nb_total, counts, stats, flagged, int(nflag), cls, ct, seconds


def run(comps, tag, triple, planes, axes=(), nthreads: int = 0, want_events: bool = False,
        resolve: bool = True, identical=None):
    """Counts and stats of a whole sample.

    Returns dict(counts=[(nbins+1) x 4] python ints (row 0 = all classified
    events, row 1+b = bin b), stats=[events, zero, invalid, out_of_range],
    n_flagged, seconds (float64 pass only), seconds_exact), and with
    want_events also per-event class (int8, flagged events after resolution)
    and the float64 C_T values and axis coordinates (cos Phi, m^2, |cos theta|).
    Flagged events keep their float64 coordinates but the resolved class.
    ``identical`` = (fast slot, slow slot): two identical particles, ordered
    per event by rest-frame energy before anything else.
    """
    arr, tag = _arrays(comps, tag)
    ax = _axes_tuple(axes)
    cap = max(1024, tag.shape[0] // 1000)
    res = _pass(arr, tag, triple, planes, ax, nthreads, want_events, cap, identical)
    if res[4] > cap:
        res = _pass(arr, tag, triple, planes, ax, nthreads, want_events, res[4] + 16, identical)
    nb_total, counts, stats, flagged, nflag, cls, ct, seconds = res
    counts_l = [[int(v) for v in counts[r * 4:(r + 1) * 4]] for r in range(nb_total + 1)]
    stats_l = [int(v) for v in stats]
    fl = flagged[:nflag].copy()
    t1 = time.perf_counter()
    if resolve:
        for i in fl:
            c, b = exact.exact_decision(_event_comps(arr, i), int(tag[i]), triple, planes, ax, identical)
            exact.accumulate(counts_l, stats_l, c, b if ax else None)
            if cls is not None:
                cls[i] = c
    out = dict(counts=counts_l, stats=stats_l, n_flagged=nflag, flagged=fl,
               seconds=seconds, seconds_exact=time.perf_counter() - t1)
    if want_events:
        out["cls"] = cls
        out["ct"], out["coord"] = ct
    return out


def brute_force(comps, tag, triple, planes, axes=(), identical=None):
    """Decide every event in exact rational arithmetic (small inputs only)."""
    arr, tag = _arrays(comps, tag)
    ax = _axes_tuple(axes)
    nb_total = int(np.prod([len(e) - 1 for _, _, e in ax])) if ax else 0
    counts = [[0] * 4 for _ in range(nb_total + 1)]
    stats = [0, 0, 0, 0]
    cls = np.zeros(tag.shape[0], dtype=np.int8)
    for i in range(tag.shape[0]):
        c, b = exact.exact_decision(_event_comps(arr, i), int(tag[i]), triple, planes, ax, identical)
        exact.accumulate(counts, stats, c, b if ax else None)
        cls[i] = c
    return dict(counts=counts, stats=stats, cls=cls)


def asymmetries(counts):
    """Exact asymmetries of every row of counts (list of dicts, see exact.asym_row)."""
    return [exact.asym_row(row) for row in counts]
