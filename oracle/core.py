"""ctypes binding of ``ht_oracle.c`` (test infrastructure only).

Every function takes and returns numpy arrays; matrices are passed to C as
column-major FP64 copies, so callers' arrays are never modified.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ht_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lib = None


def oracle_lib_path():
    return _LIB


def build_oracle(force=True):
    """Compile ht_oracle.c with gcc (plain C, -O2, strict IEEE: no -ffast-math;
    OpenMP for the independent loops of the O(n^3) form)."""
    os.makedirs(_BUILD, exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fopenmp", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def build_planted_variant(out_dir, plant):
    """Compile a copy of the oracle with the deliberate mistake number
    `plant` (ORC_PLANT in ht_oracle.c) into out_dir and load it; used only
    by the tests that show the pins catch such mistakes."""
    path = os.path.join(str(out_dir), "liboracle_plant%d.so" % int(plant))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fopenmp", "-DORC_PLANT=%d" % int(plant), _SRC,
                           "-o", path, "-lm"])
    return _bind(ctypes.CDLL(path))


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_oracle()
    _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    lib.orc_house.restype = ctypes.c_double
    lib.orc_house.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.orc_basic_ht.restype = ctypes.c_int
    lib.orc_basic_ht.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, ctypes.c_uint64]
    lib.orc_ms_ht.restype = None
    lib.orc_ms_ht.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
    lib.orc_fast_ht.restype = ctypes.c_int
    lib.orc_fast_ht.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, ctypes.c_uint64,
                                ctypes.c_int, dp]
    lib.orc_fast_flops.restype = ctypes.c_double
    lib.orc_fast_flops.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.orc_normal.restype = ctypes.c_double
    lib.orc_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fcopy(M):
    return np.array(M, dtype=np.float64, order="F", copy=True)


def house(x):
    """Householder reflector of Golub & Van Loan Alg. 5.1.1 (cited in Lemma 2.1).

    Returns (v, beta, alpha) with v[0] = 1 and (I - beta v v^T) x = alpha e1,
    alpha = ||x||_2.
    """
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    v = np.zeros_like(x)
    beta = ctypes.c_double(0.0)
    alpha = lib.orc_house(len(x), _ptr(x), _ptr(v), ctypes.byref(beta))
    return v, beta.value, alpha


def basic_ht(A, B, ncols=None, seed=0):
    """Algorithm 2 (BasicHouseHT, Appendix A).  Returns (H, T, Q, Z, n_perturbed).

    ``ncols`` limits the reduction to the first ncols columns (default n-2);
    after c columns, H[:, :c], T[:, :c+1], Q[:, :c+1] and Z[:, :c+1] are final.
    """
    lib = _load()
    n = A.shape[0]
    H, T = _fcopy(A), _fcopy(B)
    Q = np.zeros((n, n), order="F")
    Z = np.zeros((n, n), order="F")
    if ncols is None:
        ncols = max(n - 2, 0)
    npert = lib.orc_basic_ht(n, _ptr(H), _ptr(T), _ptr(Q), _ptr(Z), int(ncols), int(seed))
    return H, T, Q, Z, npert


def ms_ht(A, B, ncols=None):
    """Moler-Stewart Givens HT reduction.  Returns (H, T, Q, Z)."""
    lib = _load()
    n = A.shape[0]
    H, T = _fcopy(A), _fcopy(B)
    Q = np.zeros((n, n), order="F")
    Z = np.zeros((n, n), order="F")
    if ncols is None:
        ncols = max(n - 2, 0)
    lib.orc_ms_ht(n, _ptr(H), _ptr(T), _ptr(Q), _ptr(Z), int(ncols))
    return H, T, Q, Z


def fast_ht(A, B, ncols=None, seed=0, threads=0, timing=None, lib=None):
    """O-fast: Algorithm 2's reflector pair per column with B kept triangular
    by rank-one QR updates (Givens), Theta(n^3).  Returns (H, T, Q, Z,
    n_perturbed).  ``threads`` OpenMP threads (0: the runtime default); the
    result does not depend on it.  The C call releases the GIL, so several
    pencils can be reduced from Python threads at once (threads=1 each).
    If ``timing`` is a dict, timing["loop_s"] receives the wall time of the
    column loop alone and timing["columns"] the columns reduced; a positive
    timing["limit_s"] on entry stops the loop after the first column that
    reaches that many seconds (a bounded sample of a large reduction).
    ``lib`` selects another build of the oracle (build_planted_variant)."""
    lib = lib or _load()
    n = A.shape[0]
    H, T = _fcopy(A), _fcopy(B)
    Q = np.zeros((n, n), order="F")
    Z = np.zeros((n, n), order="F")
    if ncols is None:
        ncols = max(n - 2, 0)
    tm = (ctypes.c_double * 2)(float(timing.get("limit_s", 0.0)) if timing else 0.0, 0.0)
    npert = lib.orc_fast_ht(n, _ptr(H), _ptr(T), _ptr(Q), _ptr(Z), int(ncols), int(seed),
                            int(threads), tm)
    if timing is not None:
        timing["loop_s"] = tm[0]
        timing["columns"] = int(tm[1])
    return H, T, Q, Z, npert


def fast_flops(n, ncols=None):
    """Modelled flop count of fast_ht's first ``ncols`` columns (all by
    default): about 33 n^3 for the whole reduction."""
    if ncols is None:
        ncols = max(n - 2, 0)
    return _load().orc_fast_flops(int(n), int(ncols))


def normal(seed, counter):
    """N(0,1) number `counter` of stream `seed` (splitmix64 + Box-Muller)."""
    return _load().orc_normal(int(seed), int(counter))
