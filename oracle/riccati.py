"""ctypes front end of the sequential FP64 tree Riccati oracle (tree_riccati.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The recursion follows
Sec. XI-A's sequential baseline with the local formulas of eqs. (FW),
(factor-local), (local-affine-solve), the affine message of Lemma 5,
eq. (xroot) and eq. (recover).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tree_riccati.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


# -O3 for an x86-64 level every current server CPU has (AVX2, FMA; the library
# is built here and run on other hosts, so not -march=native), with
# floating-point contraction off: each product and sum rounds as written, so
# the results do not depend on the instruction set chosen.
BUILD_FLAGS = "-O3 -march=x86-64-v3 -ffp-contract=off"


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no fast-math; BUILD_FLAGS)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc"] + BUILD_FLAGS.split() + ["-fPIC", "-shared", "-std=c99",
                               "-D_POSIX_C_SOURCE=200809L", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_tree_riccati.restype = ctypes.c_int
            lib.oracle_tree_riccati.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _ip] + \
                [_dp] * 9 + [_dp] * 5 + [_dp, _dp]
            lib.oracle_tree_riccati_batch.restype = ctypes.c_int
            lib.oracle_tree_riccati_batch.argtypes = [
                ctypes.c_int64, _ip, ctypes.c_int32, ctypes.c_int32,
                ctypes.POINTER(_ip), ctypes.POINTER(_dp), ctypes.POINTER(_dp), ctypes.c_int32]
            _lib = lib
    return _lib


_ORDER = ("Q", "q", "c", "Delta", "R", "S", "r", "A", "B")


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def tree_riccati(parent: np.ndarray, data: dict) -> dict:
    """Solve one tree-LQR instance; returns K, P, x, u, lam (= y), p, kff (= k_e)."""
    lib = _load()
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    N = parent.shape[0]
    n = data["Q"].shape[-1]
    m = data["R"].shape[-1]
    ins = [_c(data[k]) for k in _ORDER]
    out = {"K": np.zeros((N, m, n)), "P": np.zeros((N, n, n)), "x": np.zeros((N, n)),
           "u": np.zeros((N, m)), "lam": np.zeros((N, n)), "p": np.zeros((N, n)),
           "kff": np.zeros((N, m))}
    rc = lib.oracle_tree_riccati(N, n, m, parent.ctypes.data_as(_ip),
                                 *[a.ctypes.data_as(_dp) for a in ins],
                                 *[out[k].ctypes.data_as(_dp) for k in ("K", "P", "x", "u", "lam", "p", "kff")])
    if rc != 0:
        raise RuntimeError(f"oracle_tree_riccati failed with status {rc}")
    return out


def tree_riccati_batch(instances, nthreads: int):
    """Solve independent trees spread over `nthreads` POSIX threads.
    instances: list of (parent, data); returns a list of dicts (K, P, x, u, lam)."""
    lib = _load()
    count = len(instances)
    parents = [np.ascontiguousarray(p, dtype=np.int64) for p, _ in instances]
    ins = [[_c(d[k]) for k in _ORDER] for _, d in instances]
    outs = []
    for p, d in instances:
        N = p.shape[0]
        n = d["Q"].shape[-1]
        m = d["R"].shape[-1]
        outs.append({"K": np.zeros((N, m, n)), "P": np.zeros((N, n, n)), "x": np.zeros((N, n)),
                     "u": np.zeros((N, m)), "lam": np.zeros((N, n))})
    n = instances[0][1]["Q"].shape[-1]
    m = instances[0][1]["R"].shape[-1]
    Ns = np.array([p.shape[0] for p in parents], dtype=np.int64)
    par_arr = (_ip * count)(*[p.ctypes.data_as(_ip) for p in parents])
    dat_arr = (_dp * (9 * count))(*[a.ctypes.data_as(_dp) for row in ins for a in row])
    out_arr = (_dp * (5 * count))(*[o[k].ctypes.data_as(_dp) for o in outs
                                    for k in ("K", "P", "x", "u", "lam")])
    rc = lib.oracle_tree_riccati_batch(count, Ns.ctypes.data_as(_ip), n, m, par_arr, dat_arr, out_arr,
                                       int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_tree_riccati_batch failed with status {rc}")
    return outs
