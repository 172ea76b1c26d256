"""CPU oracle for localized VT / VV / TT relation blocks (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's ``cpu_baseline`` leg, never by the library.  The oracle is
plain single-threaded C (``oracle.c``) written from the definitions of the
paper (Section 2.2, Table 1; Section 4.3 for the internal/external rule); it
shares no code with the GPU path.

Functions pinned against the paper and the mathematics by
``tests/test_oracle_pins.py``: VT, VV and TT blocks and the owner rule; by
``tests/test_oracle_simplices.py``: the edge and triangle lists E, F with their
interval arrays, and the VE, VF, EF, ET and FT blocks.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REL_VT, REL_VV, REL_TT = 1, 2, 4
REL_VE, REL_VF, REL_EF, REL_ET, REL_FT = 8, 16, 32, 64, 128
_COBOUND = REL_VE | REL_VF | REL_EF | REL_ET | REL_FT
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc -O2 into liboracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                        _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    i32p = C.POINTER(C.c_int32)
    lib.oracle_validate.argtypes = [C.c_int32, C.c_int64, i32p, i32p, C.c_int32]
    lib.oracle_validate.restype = C.c_int
    lib.oracle_create.argtypes = [C.c_int32, C.c_int64, i32p, i32p, C.c_int32, C.POINTER(C.c_void_p)]
    lib.oracle_create.restype = C.c_int
    lib.oracle_destroy.argtypes = [C.c_void_p]
    lib.oracle_destroy.restype = None
    lib.oracle_set_mutation.argtypes = [C.c_void_p, C.c_int]
    lib.oracle_set_mutation.restype = None
    lib.oracle_block.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.oracle_block.restype = C.c_int
    lib.oracle_block_copy.argtypes = [C.c_void_p, i32p, i32p, i32p]
    lib.oracle_block_copy.restype = None
    lib.oracle_owner.argtypes = [C.c_void_p, C.c_int64]
    lib.oracle_owner.restype = C.c_int32
    lib.oracle_vt_degree.argtypes = [C.c_void_p, C.c_int32]
    lib.oracle_vt_degree.restype = C.c_int64
    lib.oracle_buf_new.argtypes = []
    lib.oracle_buf_new.restype = C.c_void_p
    lib.oracle_buf_free.argtypes = [C.c_void_p]
    lib.oracle_buf_free.restype = None
    lib.oracle_block_into.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]
    lib.oracle_block_into.restype = C.c_int
    lib.oracle_buf_copy.argtypes = [C.c_void_p, i32p, i32p, i32p]
    lib.oracle_buf_copy.restype = None
    lib.oracle_enumerate.argtypes = [C.c_void_p]
    lib.oracle_enumerate.restype = C.c_int
    lib.oracle_num_edges.argtypes = [C.c_void_p]
    lib.oracle_num_edges.restype = C.c_int64
    lib.oracle_num_faces.argtypes = [C.c_void_p]
    lib.oracle_num_faces.restype = C.c_int64
    i64p = C.POINTER(C.c_int64)
    lib.oracle_simplices.argtypes = [C.c_void_p, i32p, i64p, i32p, i64p]
    lib.oracle_simplices.restype = None
    _lib = lib
    return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def validate(tets, cluster, nclusters) -> bool:
    lib = _load()
    t, tp = _i32(np.asarray(tets).reshape(-1))
    c, cp = _i32(cluster)
    return lib.oracle_validate(int(c.shape[0]), int(t.shape[0] // 4), tp, cp, int(nclusters)) == 0


class Oracle:
    """Oracle context over one mesh: ``block(k, rel)`` returns the CSR block
    (row_ids, offsets, entries) of cluster k for one relation (1=VT, 2=VV,
    4=TT) as int32 numpy arrays."""

    def __init__(self, tets, cluster, nclusters):
        lib = _load()
        self._lib = lib
        self._t, tp = _i32(np.asarray(tets).reshape(-1))
        self._c, cp = _i32(cluster)
        self.nv = int(self._c.shape[0])
        self.nt = int(self._t.shape[0] // 4)
        self.nclusters = int(nclusters)
        h = C.c_void_p()
        st = lib.oracle_create(self.nv, self.nt, tp, cp, self.nclusters, C.byref(h))
        if st != 0:
            raise ValueError("oracle_create failed with status %d (invalid mesh)" % st)
        self._h = h

    @classmethod
    def of(cls, mesh):
        return cls(mesh.tets, mesh.cluster, mesh.nclusters)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_mutation(self, m: int):
        self._lib.oracle_set_mutation(self._h, int(m))

    def enumerate(self):
        """Number the edges and triangles (Section 4.3, read through the
        example of Section 4.4); needed by the VE / VF / EF / ET / FT blocks."""
        st = self._lib.oracle_enumerate(self._h)
        if st != 0:
            raise MemoryError("oracle_enumerate failed with status %d" % st)

    def simplices(self):
        """(E as ne x 2, I_E as ncl + 1, F as nf x 3, I_F as ncl + 1)."""
        self.enumerate()
        ne = int(self._lib.oracle_num_edges(self._h))
        nf = int(self._lib.oracle_num_faces(self._h))
        e = np.empty((ne, 2), np.int32)
        f = np.empty((nf, 3), np.int32)
        ie = np.empty(self.nclusters + 1, np.int64)
        if_ = np.empty(self.nclusters + 1, np.int64)
        i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        self._lib.oracle_simplices(self._h, e.ctypes.data_as(i32p), ie.ctypes.data_as(i64p),
                                   f.ctypes.data_as(i32p), if_.ctypes.data_as(i64p))
        return e, ie, f, if_

    def block(self, k: int, rel: int):
        if rel & _COBOUND:
            self.enumerate()
        nr = C.c_int64()
        nz = C.c_int64()
        st = self._lib.oracle_block(self._h, int(k), int(rel), C.byref(nr), C.byref(nz))
        if st != 0:
            raise ValueError("oracle_block(%d, %d) failed with status %d" % (k, rel, st))
        rows = np.empty(nr.value, dtype=np.int32)
        offs = np.empty(nr.value + 1, dtype=np.int32)
        ents = np.empty(nz.value, dtype=np.int32)
        i32p = C.POINTER(C.c_int32)
        self._lib.oracle_block_copy(self._h, rows.ctypes.data_as(i32p), offs.ctypes.data_as(i32p),
                                    ents.ctypes.data_as(i32p))
        return rows, offs, ents

    def blocks(self, pairs, threads: int | None = None):
        """The blocks of many (cluster, relation) pairs, built by several
        threads sharing this context (each with its own buffer); returns a
        list of (row_ids, offsets, entries) in the order of ``pairs``.  The
        planted-mistake switch must be off."""
        import threading
        from concurrent.futures import ThreadPoolExecutor
        pairs = list(pairs)
        if any(r & _COBOUND for _, r in pairs):
            self.enumerate()
        threads = threads or min(16, os.cpu_count() or 1)
        local = threading.local()
        bufs = []
        lock = threading.Lock()
        i32p = C.POINTER(C.c_int32)

        def one(kr):
            b = getattr(local, "b", None)
            if b is None:
                b = local.b = self._lib.oracle_buf_new()
                with lock:
                    bufs.append(b)
            nr = C.c_int64()
            nz = C.c_int64()
            st = self._lib.oracle_block_into(self._h, b, int(kr[0]), int(kr[1]), C.byref(nr), C.byref(nz))
            if st != 0:
                raise ValueError("oracle_block_into(%d, %d) failed with status %d" % (kr[0], kr[1], st))
            rows = np.empty(nr.value, dtype=np.int32)
            offs = np.empty(nr.value + 1, dtype=np.int32)
            ents = np.empty(nz.value, dtype=np.int32)
            self._lib.oracle_buf_copy(b, rows.ctypes.data_as(i32p), offs.ctypes.data_as(i32p),
                                      ents.ctypes.data_as(i32p))
            return rows, offs, ents

        try:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                return list(ex.map(one, pairs))
        finally:
            for b in bufs:
                self._lib.oracle_buf_free(b)

    def owner(self, t: int) -> int:
        return int(self._lib.oracle_owner(self._h, int(t)))

    def vt_degree(self, v: int) -> int:
        return int(self._lib.oracle_vt_degree(self._h, int(v)))
