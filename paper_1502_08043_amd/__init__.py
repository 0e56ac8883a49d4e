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
FP32 = 2
MESH_GEOMETRIC = 0
MESH_TWO_INTERVAL = 1
MESH_GEOMETRIC_ROOT = 2
PAIR_AUTO, PAIR_NODESUM, PAIR_KTABLE = 0, 1, 2

OK, ERR_ARG, ERR_RANGE, ERR_NOMEM, ERR_DEVICE, ERR_BUSY, ERR_STATE, ERR_IO, ERR_LIMIT = range(9)
NOALLOC_MAX_QUADS = 8388608     # PWC_NOALLOC_MAX_QUADS


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
    def geometric_root(cls, q_sub, q_tail=4, n_sub=4, ratio=7.0, alpha_c=0.0):
        """Pieces in sqrt(beta), tail exact for polynomials in t^2."""
        return cls(MESH_GEOMETRIC_ROOT, n_sub, ratio, q_sub, q_tail, alpha_c)

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
            "pwc_table_save": (i32, [vp, ctypes.c_char_p]),
            "pwc_table_create_box": (i32, [dbl, dbl, dbl, i32, i32, ctypes.POINTER(Mesh), vp,
                                           ctypes.POINTER(vp)]),
            "pwc_table_box": (i32, [vp, ctypes.POINTER(dbl)]),
            "pwc_table_params": (i32, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32),
                                       ctypes.POINTER(Mesh)]),
            "pwc_table_load": (i32, [ctypes.c_char_p, vp, ctypes.POINTER(vp)]),
            "pwc_table_info": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)]),
            "pwc_table_layout": (i32, [vp, i32] + [ctypes.POINTER(i32)] * 5),
            "pwc_table_fused": (i32, [vp, i32, ctypes.POINTER(i32)]),
            "pwc_table_set_layout": (i32, [vp, i32, i32]),
            "pwc_table_set_direct_max": (i32, [vp, i64]),
            "pwc_table_build_values": (i32, [vp, vp]),
            "pwc_mesh_build": (i32, [ctypes.POINTER(Mesh), dbl, vp, vp]),
            "pwc_basis_enumerate": (i32, [i32, vp, ctypes.POINTER(i64)]),
            "pwc_table_values_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)]),
            "pwc_table_free_values": (i32, [vp]),
            "pwc_release_cached_memory": (i32, []),
            "pwc_basis": (i32, [vp, vp]),
            "pwc_mesh_nodes": (i32, [vp, vp, vp]),
            "pwc_table_copy": (i32, [vp, vp, vp]),
            "pwc_reconstruct": (i32, [vp, vp, i64, vp, i32, vp]),
            "pwc_reconstruct_noalloc": (i32, [vp, vp, i64, vp, i32, vp]),
            "pwc_energies_async": (i32, [vp, vp, vp, i64, i32, vp, vp]),
            "pwc_energies_ex": (i32, [vp, vp, vp, i64, i32, i32, vp, vp]),
            "pwc_energies": (i32, [vp, vp, vp, i64, i32, vp, vp]),
            "pwc_sync": (i32, [vp, vp]),
            "pwc_reconstruct_profile": (i32, [vp, vp, i64, vp, i32, vp, vp, i32,
                                              ctypes.POINTER(i32)]),
            "pwc_table_create_gauss": (i32, [vp, vp, i32, dbl, dbl, i32, ctypes.POINTER(Mesh), vp,
                                             ctypes.POINTER(vp)]),
            "pwc_gauss_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(dbl)]),
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


def release_cached_memory():
    """Return the device blocks the library keeps from freed tables."""
    _check(lib().pwc_release_cached_memory(), "pwc_release_cached_memory")


def mesh_points(mesh, L=1.0):
    """Host-only: the (beta, W) nodes and weights a table of side L uses with this mesh."""
    Q = ctypes.c_int()
    _check(lib().pwc_mesh_count(ctypes.byref(mesh), ctypes.byref(Q)), "pwc_mesh_count")
    beta, W = np.empty(Q.value), np.empty(Q.value)
    _check(lib().pwc_mesh_build(ctypes.byref(mesh), float(L), beta.ctypes.data_as(ctypes.c_void_p),
                                W.ctypes.data_as(ctypes.c_void_p)), "pwc_mesh_build")
    return beta, W


def enumerate_basis(n2max):
    """Host-only: the canonical basis |n|^2 <= n2max, int32 [N, 3]."""
    N = ctypes.c_int64()
    _check(lib().pwc_basis_enumerate(int(n2max), None, ctypes.byref(N)), "pwc_basis_enumerate")
    out = np.empty((N.value, 3), dtype=np.int32)
    _check(lib().pwc_basis_enumerate(int(n2max), out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(N)),
           "pwc_basis_enumerate")
    return out


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

    def __init__(self, L, n2max, n_nodes=0, mesh=None, stream=None, _handle=None):
        if _handle is not None:
            h = _handle
        else:
            h = ctypes.c_void_p()
            mp = ctypes.byref(mesh) if mesh is not None else None
            _check(lib().pwc_table_create(float(L), int(n2max), int(n_nodes), mp, _stream(stream),
                                          ctypes.byref(h)), "pwc_table_create")
        self._h = h
        N, nmax, Q, nb = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib().pwc_table_info(h, ctypes.byref(N), ctypes.byref(nmax), ctypes.byref(Q),
                                    ctypes.byref(nb)), "pwc_table_info")
        Lv, n2v, mesh_v = ctypes.c_double(), ctypes.c_int(), Mesh()
        _check(lib().pwc_table_params(h, ctypes.byref(Lv), ctypes.byref(n2v), ctypes.byref(mesh_v)),
               "pwc_table_params")
        self.L, self.n2max, self.mesh = Lv.value, n2v.value, mesh_v
        self.N, self.nmax, self.Q, self.device_bytes = N.value, nmax.value, Q.value, nb.value
        sides = (ctypes.c_double * 3)()
        _check(lib().pwc_table_box(h, sides), "pwc_table_box")
        self.sides = tuple(sides)
        self.ndir = 1 if self.sides[0] == self.sides[1] == self.sides[2] else 3
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

    def save(self, path):
        """Write the mesh and the FP64 tables to `path` (see pwc_table_save)."""
        _check(lib().pwc_table_save(self.handle, os.fsencode(path)), "pwc_table_save")

    @classmethod
    def box(cls, Lx, Ly, Lz, n2max, n_nodes=0, mesh=None, stream=None):
        """Tables of a rectangular box with sides (Lx, Ly, Lz) (see pwc_table_create_box)."""
        h = ctypes.c_void_p()
        mp = ctypes.byref(mesh) if mesh is not None else None
        _check(lib().pwc_table_create_box(float(Lx), float(Ly), float(Lz), int(n2max), int(n_nodes),
                                          mp, _stream(stream), ctypes.byref(h)),
               "pwc_table_create_box")
        return cls(None, 0, _handle=h)

    @classmethod
    def load(cls, path, stream=None):
        """A table from a file written by save(), without recomputing the integrals."""
        h = ctypes.c_void_p()
        _check(lib().pwc_table_load(os.fsencode(path), _stream(stream), ctypes.byref(h)),
               "pwc_table_load")
        return cls(None, 0, _handle=h)

    def layout(self, precision=0):
        """Reconstruction layout of one precision:
        dict(lanes, words, nodes_per_pass, passes, entry_bytes)."""
        v = [ctypes.c_int() for _ in range(5)]
        _check(lib().pwc_table_layout(self.handle, int(precision), *[ctypes.byref(x) for x in v]),
               "pwc_table_layout")
        return dict(zip(("lanes", "words", "nodes_per_pass", "passes", "entry_bytes"),
                        (x.value for x in v)))

    def fused(self, precision=0):
        """True when node-pass reconstructions of this precision run as one
        fused launch (pwc_table_fused)."""
        v = ctypes.c_int()
        _check(lib().pwc_table_fused(self.handle, int(precision), ctypes.byref(v)), "pwc_table_fused")
        return bool(v.value)

    def set_layout(self, lanes=0, words=0):
        """Force the reconstruction layout, (lanes, words) in (16, 1), (8, 2), (8, 1),
        (4, 2), (2, 4), (1, 8), (4, 1); (0, 0) = default."""
        _check(lib().pwc_table_set_layout(self.handle, int(lanes), int(words)),
               "pwc_table_set_layout")

    def set_direct_max(self, n):
        """Lists of at most n quadruples skip the node passes (0: never)."""
        _check(lib().pwc_table_set_direct_max(self.handle, int(n)), "pwc_table_set_direct_max")

    def build_values(self, stream=None):
        """Evaluate every distinct integral once (the value table); FP64
        reconstructions then read one value per quadruple.  Asynchronous on
        the stream: later work on it sees the values."""
        _check(lib().pwc_table_build_values(self.handle, _stream(stream)), "pwc_table_build_values")
        self._refresh_bytes()

    def free_values(self):
        _check(lib().pwc_table_free_values(self.handle), "pwc_table_free_values")
        self._refresh_bytes()

    def values_info(self):
        """(built, bytes): whether the value table is built and its size."""
        b, n = ctypes.c_int(), ctypes.c_size_t()
        _check(lib().pwc_table_values_info(self.handle, ctypes.byref(b), ctypes.byref(n)),
               "pwc_table_values_info")
        return bool(b.value), n.value

    def _refresh_bytes(self):
        nb = ctypes.c_size_t()
        _check(lib().pwc_table_info(self.handle, None, None, None, ctypes.byref(nb)), "pwc_table_info")
        self.device_bytes = nb.value

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
        """FP64 tables as a device tensor [Q, nd, nd] (a cube) or [3, Q, nd, nd] (a box)."""
        if out is None:
            shape = (self.Q, self.nd, self.nd) if self.ndir == 1 else (3, self.Q, self.nd, self.nd)
            out = torch.empty(shape, dtype=torch.float64, device="cuda")
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

    def reconstruct_noalloc(self, quads, out, precision=FP64, stream=None):
        """pwc_reconstruct_noalloc: the node passes with the library's fixed
        scratch (no allocation by the library; the caller passes `out`);
        async.  Calls that may overlap on the device race."""
        if quads.dim() != 2 or quads.shape[1] != 4 or out.numel() != quads.shape[0]:
            raise ValueError("quads must be [n, 4] and out [n]")
        _check(lib().pwc_reconstruct_noalloc(self.handle, _dev_ptr(quads, torch.int32, "quads"),
                                             quads.shape[0], _dev_ptr(out, torch.float64, "out"),
                                             int(precision), _stream(stream)),
               "pwc_reconstruct_noalloc")
        return out

    def reconstruct_profile(self, quads, out=None, precision=FP64, stream=None):
        """Like reconstruct, then waits; returns (out, per-launch ms [decode, pass 1..P])."""
        n = quads.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=quads.device)
        ms = np.zeros(64)
        ns = ctypes.c_int()
        _check(lib().pwc_reconstruct_profile(self.handle, _dev_ptr(quads, torch.int32, "quads"), n,
                                             _dev_ptr(out, torch.float64, "out"), int(precision),
                                             _stream(stream), ms.ctypes.data_as(ctypes.c_void_p),
                                             64, ctypes.byref(ns)), "pwc_reconstruct_profile")
        return out, ms[:ns.value].copy()

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


class GaussTable(Table):
    """Tables of a separable s-type Gaussian basis (pwc_table_create_gauss):
    one-dimensional exponents `exps` and centers `centers` (host arrays [n1]),
    the same set along x, y and z; basis function (l n1 + m) n1 + n is
    f_l(x) f_m(y) f_n(z).  reconstruct / sync / copy_tables / mesh_nodes as
    for planewave tables."""

    def __init__(self, exps, centers, L, eps=1e-15, n_nodes=0, mesh=None, stream=None):
        a = np.ascontiguousarray(exps, dtype=np.float64)
        A = np.ascontiguousarray(centers, dtype=np.float64)
        if a.shape != A.shape or a.ndim != 1:
            raise ValueError("exps and centers must be 1-D arrays of one length")
        h = ctypes.c_void_p()
        mp = ctypes.byref(mesh) if mesh is not None else None
        _check(lib().pwc_table_create_gauss(a.ctypes.data_as(ctypes.c_void_p),
                                            A.ctypes.data_as(ctypes.c_void_p), len(a), float(L),
                                            float(eps), int(n_nodes), mp, _stream(stream),
                                            ctypes.byref(h)), "pwc_table_create_gauss")
        super().__init__(None, 0, _handle=h)
        n1, npair, e = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().pwc_gauss_info(h, ctypes.byref(n1), ctypes.byref(npair), ctypes.byref(e)),
               "pwc_gauss_info")
        self.n1, self.n_pairs, self.eps = n1.value, npair.value, e.value
        self.nd = self.n_pairs

    def copy_tables(self, out=None, stream=None):
        """FP64 tables as a device tensor [Q, P1, P1] over the kept pairs."""
        if out is None:
            out = torch.empty((self.Q, self.n_pairs, self.n_pairs), dtype=torch.float64, device="cuda")
        _check(lib().pwc_table_copy(self.handle, _dev_ptr(out, torch.float64, "out"),
                                    _stream(stream)), "pwc_table_copy")
        return out


# ---------------------------------------------------------------- serving ----

REQ_RECONSTRUCT, REQ_ENERGIES = 0, 1


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("L", ctypes.c_double), ("n2max", ctypes.c_int),
                ("n_nodes", ctypes.c_int), ("has_mesh", ctypes.c_int), ("mesh", Mesh),
                ("prec", ctypes.c_int), ("algo", ctypes.c_int), ("d_idx", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("d_f", ctypes.c_void_p), ("d_out", ctypes.c_void_p),
                ("ready_event", ctypes.c_void_p), ("Ly", ctypes.c_double), ("Lz", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("e_h", ctypes.c_double), ("e_x", ctypes.c_double),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("table_built", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("table_builds", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64), ("resident_tables", ctypes.c_int),
                ("resident_bytes", ctypes.c_size_t), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("integrals_per_s", ctypes.c_double),
                ("pairs_per_s", ctypes.c_double), ("launches", ctypes.c_uint64),
                ("batched", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _server_lib():
    L = lib()
    if not hasattr(L, "_server_sig"):
        vp = ctypes.c_void_p
        L.pwc_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(vp)]
        L.pwc_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.pwc_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
        L.pwc_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
        L.pwc_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.pwc_server_reset_stats.argtypes = [vp]
        L.pwc_server_destroy.argtypes = [vp]
        for n in ("pwc_server_create", "pwc_server_submit", "pwc_server_poll", "pwc_server_wait",
                  "pwc_server_get_stats", "pwc_server_reset_stats", "pwc_server_destroy"):
            getattr(L, n).restype = ctypes.c_int
        L._server_sig = True
    return L


class Server:
    """Continuous-batching request loop (pwc_server_*).  Keeps the tensors of
    every outstanding request alive until its result is collected."""

    def __init__(self, hbm_budget_bytes, max_inflight=4):
        h = ctypes.c_void_p()
        _check(_server_lib().pwc_server_create(int(hbm_budget_bytes), int(max_inflight),
                                               ctypes.byref(h)), "pwc_server_create")
        self._h = h
        self._keep = {}

    def _submit(self, req, keep):
        # The server's streams wait for the work queued so far on the current
        # stream (inputs being written, outputs being cleared).
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        req.ready_event = ev.cuda_event
        keep = keep + (ev,)
        t = ctypes.c_uint64()
        _check(_server_lib().pwc_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)),
               "pwc_server_submit")
        self._keep[t.value] = keep
        return t.value

    @staticmethod
    def _key(req, L, n2max, n_nodes, mesh):
        """L: a cube side, or the sides (Lx, Ly, Lz) of a rectangular box."""
        if isinstance(L, (tuple, list)):
            req.L, req.Ly, req.Lz = (float(v) for v in L)
        else:
            req.L = float(L)
        req.n2max, req.n_nodes = int(n2max), int(n_nodes)
        if mesh is not None:
            req.has_mesh, req.mesh = 1, mesh

    def submit_reconstruct(self, L, n2max, quads, out, precision=FP64, n_nodes=0, mesh=None):
        req = Request()
        req.kind = REQ_RECONSTRUCT
        self._key(req, L, n2max, n_nodes, mesh)
        req.prec = int(precision)
        req.d_idx = _dev_ptr(quads, torch.int32, "quads").value
        req.n = quads.shape[0]
        req.d_out = _dev_ptr(out, torch.float64, "out").value
        return self._submit(req, (quads, out))

    def submit_energies(self, L, n2max, occ, out, f=None, precision=FP64, algo=PAIR_AUTO,
                        n_nodes=0, mesh=None):
        req = Request()
        req.kind = REQ_ENERGIES
        self._key(req, L, n2max, n_nodes, mesh)
        req.prec, req.algo = int(precision), int(algo)
        req.d_idx = _dev_ptr(occ, torch.int32, "occ").value
        req.n = occ.numel()
        req.d_f = _dev_ptr(f, torch.float64, "f").value if f is not None else None
        req.d_out = _dev_ptr(out, torch.float64, "out").value
        return self._submit(req, (occ, out, f))

    def wait(self, ticket):
        r = Result()
        _check(_server_lib().pwc_server_wait(self._h, int(ticket), ctypes.byref(r)), "pwc_server_wait")
        self._keep.pop(ticket, None)
        return r

    def poll(self, ticket):
        r = Result()
        s = _server_lib().pwc_server_poll(self._h, int(ticket), ctypes.byref(r))
        if s == ERR_BUSY:
            return None
        _check(s, "pwc_server_poll")
        self._keep.pop(ticket, None)
        return r

    def stats(self):
        st = ServerStats()
        _check(_server_lib().pwc_server_get_stats(self._h, ctypes.byref(st)), "pwc_server_get_stats")
        return st.as_dict()

    def reset_stats(self):
        _check(_server_lib().pwc_server_reset_stats(self._h), "pwc_server_reset_stats")

    def close(self):
        if getattr(self, "_h", None) is not None:
            _server_lib().pwc_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
