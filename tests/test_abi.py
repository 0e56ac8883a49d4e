"""The C ABI library loads and exports every entry point declared in include/*.h.

CPU only: nothing here launches a kernel.  Argument checks that return before
any device work are exercised too.
"""
import ctypes
import glob
import os
import re

import pytest

from tests.conftest import ROOT

LIB = os.path.join(ROOT, "paper_1502_08043_amd", "libpwcoul.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1502_08043_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(pwc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_api():
    names = declared_symbols()
    for n in ("pwc_table_create", "pwc_reconstruct", "pwc_energies", "pwc_sync"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls(lib):
    lib.pwc_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.pwc_version()
    lib.pwc_status_str.restype = ctypes.c_char_p
    assert lib.pwc_status_str(2) == b"index out of range"
    assert lib.pwc_status_str(99) == b"unknown status"

    class Mesh(ctypes.Structure):
        _fields_ = [("kind", ctypes.c_int), ("n_sub", ctypes.c_int), ("ratio", ctypes.c_double),
                    ("q_sub", ctypes.c_int), ("q_tail", ctypes.c_int), ("alpha_c", ctypes.c_double)]

    m = Mesh()
    assert lib.pwc_mesh_default(96, ctypes.byref(m)) == 0
    assert (m.kind, m.n_sub, m.ratio, m.q_sub, m.q_tail) == (0, 8, 5.0, 11, 8)
    q = ctypes.c_int()
    assert lib.pwc_mesh_count(ctypes.byref(m), ctypes.byref(q)) == 0 and q.value == 96
    assert lib.pwc_mesh_default(50, ctypes.byref(m)) == 1
    bad = Mesh(0, 8, 1.0, 5, 8, 0.0)           # ratio must exceed 1
    assert lib.pwc_mesh_count(ctypes.byref(bad), ctypes.byref(q)) == 1
    mesh1 = Mesh(1, 1, 5.0, 90, 90, 0.0)
    assert lib.pwc_mesh_count(ctypes.byref(mesh1), ctypes.byref(q)) == 0 and q.value == 180


def test_create_rejects_bad_arguments_before_device_work(lib):
    lib.pwc_table_create.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert lib.pwc_table_create(0.0, 9, 48, None, None, ctypes.byref(h)) == 1      # L <= 0
    assert lib.pwc_table_create(-1.0, 9, 48, None, None, ctypes.byref(h)) == 1
    assert lib.pwc_table_create(1.0, 0, 48, None, None, ctypes.byref(h)) == 1      # n2max < 1
    assert lib.pwc_table_create(1.0, 625, 48, None, None, ctypes.byref(h)) == 1    # too large
    assert lib.pwc_table_create(1.0, 9, 50, None, None, ctypes.byref(h)) == 1      # Q % 8
    assert lib.pwc_table_create(1.0, 9, 48, None, None, None) == 1
    assert h.value is None
    lib.pwc_reconstruct.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64, ctypes.c_void_p,
                                                            ctypes.c_int, ctypes.c_void_p]
    assert lib.pwc_reconstruct(None, None, 0, None, 0, None) == 1
    lib.pwc_sync.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.pwc_sync(None, None) == 1
    lib.pwc_table_layout.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 5
    assert lib.pwc_table_layout(None, 0, None, None, None, None, None) == 1
    lib.pwc_table_set_layout.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    assert lib.pwc_table_set_layout(None, 8, 1) == 1
    lib.pwc_table_destroy.argtypes = [ctypes.c_void_p]
    assert lib.pwc_table_destroy(None) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1502_08043_amd as pw
    monkeypatch.setattr(pw, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pw, "_lib", None)
    with pytest.raises(ImportError):
        pw.lib()


def test_server_create_rejects_bad_arguments(lib):
    lib.pwc_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert lib.pwc_server_create(0, 4, ctypes.byref(h)) == 1
    assert lib.pwc_server_create(1 << 30, 0, ctypes.byref(h)) == 1
    assert lib.pwc_server_create(1 << 30, 65, ctypes.byref(h)) == 1
    assert lib.pwc_server_create(1 << 30, 4, None) == 1
    lib.pwc_server_destroy.argtypes = [ctypes.c_void_p]
    assert lib.pwc_server_destroy(None) == 0


def _table_header(version=2, n2max=2, Q=16, nd=5, ndir=1, N=19, payload_bytes=0, checksum=12345):
    """A table-file header (the layout pwc_table_save writes): magic, version,
    header size, the three box sides, n2max, Q, nd, mesh kind, N, n_sub,
    q_sub, q_tail, ndir, ratio, alpha_c, payload size and checksum."""
    import struct
    head = struct.pack("<8sIIdddiiiiqiiiiddQQ", b"PWCTABL1", version, 112, 1.0, 1.0, 1.0,
                       n2max, Q, nd, 0, N, 1, 8, 8, ndir, 5.0, 0.0, payload_bytes, checksum)
    assert len(head) == 112
    return head


def test_table_files_rejected_before_device_work(lib, tmp_path):
    """pwc_table_load refuses missing, foreign, corrupt, truncated and
    oversized files with PWC_ERR_IO before touching the device or sizing
    any buffer from the file."""
    import numpy as np
    lib.pwc_table_load.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.pwc_table_save.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    lib.pwc_status_str.restype = ctypes.c_char_p
    assert lib.pwc_status_str(7) == b"table file error"
    h = ctypes.c_void_p()

    def load(name, data):
        path = tmp_path / name
        path.write_bytes(data)
        return lib.pwc_table_load(str(path).encode(), None, ctypes.byref(h))

    assert lib.pwc_table_load(str(tmp_path / "missing.tab").encode(), None, ctypes.byref(h)) == 7
    assert h.value is None
    assert lib.pwc_table_load(None, None, ctypes.byref(h)) == 1
    assert lib.pwc_table_save(None, str(tmp_path / "x.tab").encode()) == 1
    assert load("foreign.tab", b"not a table file" * 16) == 7
    assert load("empty.tab", b"") == 7
    # n2max = 2: nmax = 1, nd = 5, E1 = 9 orbits; Q = 16 nodes (8 x 1 + 8)
    Q, E1 = 16, 9
    payload = np.arange(2 * Q + Q * E1, dtype=np.float64).tobytes() + bytes(2 * E1)
    assert load("bad_sum.tab", _table_header(payload_bytes=len(payload)) + payload) == 7
    assert load("trunc.tab", _table_header(payload_bytes=len(payload)) + payload[:-8]) == 7
    assert load("trail.tab", _table_header(payload_bytes=len(payload)) + payload + b"x") == 7
    assert load("v1.tab", _table_header(version=1, payload_bytes=len(payload)) + payload) == 7
    # sizes that would wrap or exhaust memory are refused from the header alone
    assert load("huge_q.tab", _table_header(Q=1 << 30, payload_bytes=(1 << 63) + 8) + payload) == 7
    assert load("huge_nd.tab", _table_header(nd=1 << 20, payload_bytes=1 << 62) + payload) == 7
    assert load("bad_nd.tab", _table_header(nd=7, payload_bytes=len(payload)) + payload) == 7
    assert load("bad_n2.tab", _table_header(n2max=100000, payload_bytes=len(payload)) + payload) == 7
    assert load("bad_dir.tab", _table_header(ndir=2, payload_bytes=len(payload)) + payload) == 7
    assert load("neg_q.tab", _table_header(Q=-4, payload_bytes=len(payload)) + payload) == 7
    assert h.value is None
