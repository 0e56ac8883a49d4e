"""ctypes wrapper of the oracle's C node sums and pair sums (sums.c).

TEST INFRASTRUCTURE ONLY.  build() compiles sums.c with gcc into
oracle/liboracle_sums.so; nothing here touches the GPU library.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sums.c")
_LIB = os.path.join(_HERE, "liboracle_sums.so")
_lib = None

# Portable flags: the library may run on another x86-64 host than the one
# that built it.  No fast-math and no contraction of a*b+c into an FMA.
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-shared", "-std=gnu11"]


def build(force: bool = True) -> str:
    """Compile sums.c into liboracle_sums.so (always, when force is set)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_reconstruct.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, i64p,
                                           ctypes.c_int64, i32p, ctypes.c_int64,
                                           ctypes.c_double, dp, ctypes.c_int]
        lib.oracle_reconstruct.restype = ctypes.c_int
        lib.oracle_energies.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, i64p,
                                        ctypes.c_int64, i32p, dp, ctypes.c_int64,
                                        ctypes.c_double, dp, dp, ctypes.c_int]
        lib.oracle_energies.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _prep(tau, W, basis):
    """tau: [Q, nd, nd] (a cube) or [3, Q, nd, nd] (a box, one table per direction)."""
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    basis = np.ascontiguousarray(basis, dtype=np.int64)
    ndir = 3 if tau.ndim == 4 else 1
    if ndir == 3 and tau.shape[0] != 3:
        raise ValueError("a box takes three direction tables")
    Q, nd, nd2 = tau.shape[-3:]
    if nd != nd2 or nd % 2 != 1 or W.shape != (Q,):
        raise ValueError("tau must be [(3,) Q, 2K+1, 2K+1] and W [Q]")
    return tau, ndir, W, basis, Q, (nd - 1) // 2


def reconstruct(tau, W, basis, quads, L=1.0, nthreads=0):
    """<ij|kl> for each row (i, j, k, l) of quads, by Eq. 14 (FP64, compensated).
    For a box, tau holds the three direction tables and L is the reference
    length (box_tables)."""
    tau, ndir, W, basis, Q, K = _prep(tau, W, basis)
    quads = np.ascontiguousarray(quads, dtype=np.int32).reshape(-1, 4)
    out = np.empty(quads.shape[0])
    rc = _load().oracle_reconstruct(_ptr(tau, ctypes.c_double), ndir, _ptr(W, ctypes.c_double),
                                    Q, K, _ptr(basis, ctypes.c_int64), basis.shape[0],
                                    _ptr(quads, ctypes.c_int32), quads.shape[0],
                                    float(L), _ptr(out, ctypes.c_double), int(nthreads))
    if rc == 2:
        raise IndexError("quadruple index out of range")
    if rc:
        raise RuntimeError(f"oracle_reconstruct failed ({rc})")
    return out


def energies(tau, W, basis, occ, f=None, L=1.0, nthreads=0):
    """(E_H, E_x) per spin channel by literal double loops over ordered pairs."""
    tau, ndir, W, basis, Q, K = _prep(tau, W, basis)
    occ = np.ascontiguousarray(occ, dtype=np.int32).reshape(-1)
    fp = None
    if f is not None:
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if f.shape != occ.shape:
            raise ValueError("f must match occ")
        fp = _ptr(f, ctypes.c_double)
    eh = ctypes.c_double()
    ex = ctypes.c_double()
    rc = _load().oracle_energies(_ptr(tau, ctypes.c_double), ndir, _ptr(W, ctypes.c_double),
                                 Q, K, _ptr(basis, ctypes.c_int64), basis.shape[0],
                                 _ptr(occ, ctypes.c_int32), fp, occ.shape[0], float(L),
                                 ctypes.byref(eh), ctypes.byref(ex), int(nthreads))
    if rc == 2:
        raise IndexError("occupied index out of range")
    if rc:
        raise RuntimeError(f"oracle_energies failed ({rc})")
    return eh.value, ex.value
