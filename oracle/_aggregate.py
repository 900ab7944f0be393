"""Plain three-pass aggregation (oracle, TEST INFRASTRUCTURE ONLY).

`aggregate_py` states the algorithm as a plain Python loop; it is the
definition and is used directly on small graphs.  Large graphs go through
`oracle/csrc/plain_aggregation.c`, a line-by-line C transcription of the same
loops compiled with gcc (loaded with ctypes), which the CPU tests pin against
`aggregate_py` on random and structured graphs.

Passes (nodes visited in ascending order, Vanek, Mandel & Brezina 1996):
  1. unaggregated i with a non-empty strong neighbourhood N_i whose members
     are all unaggregated: new aggregate {i} + N_i;
  2. against a snapshot of pass 1, each unaggregated i with N_i non-empty
     joins the aggregate of the aggregated j in N_i with the largest weight
     w_ij (first such j in ascending order on ties);
  3. each still unaggregated i with N_i non-empty: new aggregate made of i
     and the members of N_i that are still unaggregated.
Nodes with empty N_i that no pass touched keep id -1.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "csrc", "liboracle_agg.so")
_SRC_PATH = os.path.join(_HERE, "csrc", "plain_aggregation.c")
_lib = None

# graphs up to this many nodes use the Python definition directly
PY_LIMIT = 20000


def aggregate_py(indptr, indices, weight, strong):
    n = len(indptr) - 1
    indptr = [int(v) for v in indptr]
    indices = [int(v) for v in indices]
    weight = [float(v) for v in weight]
    strong = [bool(v) for v in strong]
    nbr = []
    for i in range(n):
        nbr.append([(indices[k], weight[k]) for k in range(indptr[i], indptr[i + 1])
                    if strong[k]])
    agg = [-1] * n
    nagg = 0
    for i in range(n):                                   # pass 1
        if agg[i] != -1 or not nbr[i]:
            continue
        if all(agg[j] == -1 for j, _ in nbr[i]):
            agg[i] = nagg
            for j, _ in nbr[i]:
                agg[j] = nagg
            nagg += 1
    snap = list(agg)
    for i in range(n):                                   # pass 2
        if snap[i] != -1 or not nbr[i]:
            continue
        best, bestw = -1, 0.0
        for j, w in nbr[i]:
            if snap[j] != -1 and (best < 0 or w > bestw):
                best, bestw = j, w
        if best >= 0:
            agg[i] = snap[best]
    for i in range(n):                                   # pass 3
        if agg[i] != -1 or not nbr[i]:
            continue
        agg[i] = nagg
        for j, _ in nbr[i]:
            if agg[j] == -1:
                agg[j] = nagg
        nagg += 1
    return np.array(agg, dtype=np.int64), nagg


def build_c(force=False):
    """Compile the C transcription with gcc (oracle test infrastructure)."""
    import subprocess
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH):
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-std=c99",
                               "-o", _LIB_PATH, _SRC_PATH])
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build_c()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_plain_aggregation.restype = ctypes.c_int64
        lib.oracle_plain_aggregation.argtypes = [
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def aggregate_c(indptr, indices, weight, strong):
    lib = _load()
    n = len(indptr) - 1
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    s = np.ascontiguousarray(strong, dtype=np.uint8)
    agg = np.empty(n, dtype=np.int64)
    nagg = lib.oracle_plain_aggregation(n, ip.ctypes.data, ix.ctypes.data,
                                        w.ctypes.data, s.ctypes.data,
                                        agg.ctypes.data)
    return agg, int(nagg)


def aggregate(indptr, indices, weight, strong):
    if len(indptr) - 1 <= PY_LIMIT:
        return aggregate_py(indptr, indices, weight, strong)
    return aggregate_c(indptr, indices, weight, strong)
