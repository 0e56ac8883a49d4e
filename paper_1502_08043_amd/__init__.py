"""Python binding of libpwcoul: argument marshalling over the C ABI only.

Every step of the computation runs in the library's HIP kernels; this module
turns torch tensors into device pointers and the current torch stream into a
hipStream_t, and turns status codes into exceptions.  PyTorch provides device
memory and streams and nothing else.  There is no CPU fallback: if the
library is missing, importing the binding's entry points raises.

Names follow the C ABI in include/pwcoul.h (the pwc_ prefix dropped).
"""
import ctypes
import os

import numpy as np
import torch  # loaded first: libpwcoul binds to the HIP runtime torch carries

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpwcoul.so")

FP64 = 0
MIXED = 1
MESH_GEOMETRIC = 0
MESH_TWO_INTERVAL = 1
PAIR_AUTO, PAIR_NODESUM, PAIR_KTABLE = 0, 1, 2

OK, ERR_ARG, ERR_RANGE, ERR_NOMEM, ERR_DEVICE, ERR_BUSY, ERR_STATE = range(7)


class PwcError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class Mesh(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_sub", ctypes.c_int), ("ratio", ctypes.c_double),
                ("q_sub", ctypes.c_int), ("q_tail", ctypes.c_int), ("alpha_c", ctypes.c_double)]

    @classmethod
    def geometric(cls, q_sub, q_tail=8, n_sub=8, ratio=5.0, alpha_c=0.0):
        return cls(MESH_GEOMETRIC, n_sub, ratio, q_sub, q_tail, alpha_c)

    @classmethod
    def two_interval(cls, q_sub, q_tail=None, alpha_c=0.0):
        return cls(MESH_TWO_INTERVAL, 1, 5.0, q_sub, q_sub if q_tail is None else q_tail, alpha_c)


_lib = None


def lib():
    """The loaded libpwcoul (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1502_08043_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        sig = {
            "pwc_version": (ctypes.c_char_p, []),
            "pwc_status_str": (ctypes.c_char_p, [i32]),
            "pwc_mesh_default": (i32, [i32, ctypes.POINTER(Mesh)]),
            "pwc_mesh_count": (i32, [ctypes.POINTER(Mesh), ctypes.POINTER(i32)]),
            "pwc_table_create": (i32, [dbl, i32, i32, ctypes.POINTER(Mesh), vp,
                                       ctypes.POINTER(vp)]),
            "pwc_table_destroy": (i32, [vp]),
            "pwc_table_info": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)]),
            "pwc_basis": (i32, [vp, vp]),
            "pwc_mesh_nodes": (i32, [vp, vp, vp]),
            "pwc_table_copy": (i32, [vp, vp, vp]),
            "pwc_reconstruct": (i32, [vp, vp, i64, vp, i32, vp]),
            "pwc_energies_async": (i32, [vp, vp, vp, i64, i32, vp, vp]),
            "pwc_energies_ex": (i32, [vp, vp, vp, i64, i32, i32, vp, vp]),
            "pwc_energies": (i32, [vp, vp, vp, i64, i32, vp, vp]),
            "pwc_sync": (i32, [vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(s):
    return lib().pwc_status_str(int(s)).decode()


def version():
    return lib().pwc_version().decode()


def _check(s, what):
    if s != OK:
        raise PwcError(s, what)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def mesh_default(n_nodes):
    m = Mesh()
    _check(lib().pwc_mesh_default(int(n_nodes), ctypes.byref(m)), "pwc_mesh_default")
    return m


def mesh_count(mesh):
    q = ctypes.c_int()
    _check(lib().pwc_mesh_count(ctypes.byref(mesh), ctypes.byref(q)), "pwc_mesh_count")
    return q.value


class Table:
    """Owning handle of a pwc_table (tables for one box, cutoff and mesh)."""

    def __init__(self, L, n2max, n_nodes=0, mesh=None, stream=None):
        h = ctypes.c_void_p()
        mp = ctypes.byref(mesh) if mesh is not None else None
        _check(lib().pwc_table_create(float(L), int(n2max), int(n_nodes), mp, _stream(stream),
                                      ctypes.byref(h)), "pwc_table_create")
        self._h = h
        N, nmax, Q, nb = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib().pwc_table_info(h, ctypes.byref(N), ctypes.byref(nmax), ctypes.byref(Q),
                                    ctypes.byref(nb)), "pwc_table_info")
        self.L, self.n2max = float(L), int(n2max)
        self.N, self.nmax, self.Q, self.device_bytes = N.value, nmax.value, Q.value, nb.value
        self.nd = 4 * self.nmax + 1

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("table is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().pwc_table_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def basis(self):
        out = np.empty((self.N, 3), dtype=np.int32)
        _check(lib().pwc_basis(self.handle, out.ctypes.data_as(ctypes.c_void_p)), "pwc_basis")
        return out

    def mesh_nodes(self):
        beta = np.empty(self.Q)
        W = np.empty(self.Q)
        _check(lib().pwc_mesh_nodes(self.handle, beta.ctypes.data_as(ctypes.c_void_p),
                                    W.ctypes.data_as(ctypes.c_void_p)), "pwc_mesh_nodes")
        return beta, W

    def copy_tables(self, out=None, stream=None):
        """FP64 tables as a device tensor [Q, nd, nd]."""
        if out is None:
            out = torch.empty((self.Q, self.nd, self.nd), dtype=torch.float64, device="cuda")
        _check(lib().pwc_table_copy(self.handle, _dev_ptr(out, torch.float64, "out"),
                                    _stream(stream)), "pwc_table_copy")
        return out

    def reconstruct(self, quads, out=None, precision=FP64, stream=None):
        """<ij|kl> for an int32 device tensor [n, 4] of (i, j, k, l); async."""
        if quads.dim() != 2 or quads.shape[1] != 4:
            raise ValueError("quads must be [n, 4]")
        n = quads.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=quads.device)
        if out.numel() != n:
            raise ValueError("out must have n elements")
        _check(lib().pwc_reconstruct(self.handle, _dev_ptr(quads, torch.int32, "quads"), n,
                                     _dev_ptr(out, torch.float64, "out"), int(precision),
                                     _stream(stream)), "pwc_reconstruct")
        return out

    def energies_async(self, occ, f=None, precision=FP64, out=None, stream=None,
                       algo=PAIR_AUTO):
        """Enqueue (E_H, E_x) into a device tensor [2]."""
        M = occ.numel()
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=occ.device)
        fp = _dev_ptr(f, torch.float64, "f") if f is not None else None
        _check(lib().pwc_energies_ex(self.handle, _dev_ptr(occ, torch.int32, "occ"), fp, M,
                                     int(precision), int(algo),
                                     _dev_ptr(out, torch.float64, "out"), _stream(stream)),
               "pwc_energies_ex")
        return out

    def energies(self, occ, f=None, precision=FP64, stream=None, algo=PAIR_AUTO):
        """(E_H, E_x) of one spin channel for occupied basis indices occ (int32 device)."""
        if algo != PAIR_AUTO:
            out = self.energies_async(occ, f, precision, stream=stream, algo=algo)
            self.sync(stream)
            return tuple(float(v) for v in out.cpu().numpy())
        h = np.zeros(2)
        fp = _dev_ptr(f, torch.float64, "f") if f is not None else None
        _check(lib().pwc_energies(self.handle, _dev_ptr(occ, torch.int32, "occ"), fp, occ.numel(),
                                  int(precision), h.ctypes.data_as(ctypes.c_void_p),
                                  _stream(stream)), "pwc_energies")
        return float(h[0]), float(h[1])

    def sync(self, stream=None):
        """Wait for the stream and raise PwcError if a kernel saw a bad index."""
        _check(lib().pwc_sync(self.handle, _stream(stream)), "pwc_sync")
