"""ctypes binding of the C ABI in include/gale.h (argument marshalling only).

Every relation is built by the HIP kernels inside libgale.so; this module only
converts numpy arrays to pointers and views back to numpy arrays.  Importing
it without the built library raises an error: there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgale.so")

REL_VT, REL_VV, REL_TT, REL_ALL = 1, 2, 4, 7
REL_VE, REL_VF, REL_EF, REL_ET, REL_FT, REL_EXT = 8, 16, 32, 64, 128, 248
FORM_PLAIN, FORM_BATCHED = 0, 1
MODE_DIRECT, MODE_SERVE = 0, 1
FRONT_SINGLE, FRONT_PER_RELATION = 0, 1

OK, EINVAL, ENOMEM, EAGAIN, ENOENT, ESTATE, EDEVICE = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EAGAIN", -4: "ENOENT", -5: "ESTATE", -6: "EDEVICE"}


class GaleConfig(C.Structure):
    _fields_ = [
        ("device", C.c_int32), ("mode", C.c_int32), ("form", C.c_int32), ("block_threads", C.c_int32),
        ("lds_bytes", C.c_int32), ("max_inflight", C.c_int32), ("cache_budget_bytes", C.c_uint64),
        ("max_queue", C.c_int32), ("launch_classes", C.c_int32), ("hip_stream", C.c_void_p),
        ("global_cu_share", C.c_double), ("dev_arena", C.c_void_p), ("arena_bytes", C.c_uint64),
        ("tune_table_path", C.c_char_p), ("prefetch_depth", C.c_int32), ("front_end", C.c_int32),
        ("simplex_lists", C.c_int32), ("tile_entries", C.c_int32),
    ]


class GaleCsr(C.Structure):
    _fields_ = [
        ("cluster", C.c_int32), ("rel", C.c_uint32), ("nrows", C.c_int32), ("pad", C.c_int32),
        ("nnz", C.c_int64), ("row_ids", C.POINTER(C.c_int32)), ("offsets", C.POINTER(C.c_int32)),
        ("entries", C.POINTER(C.c_int32)),
    ]


class GaleStats(C.Structure):
    _fields_ = [
        ("nv", C.c_int32), ("nclusters", C.c_int32), ("nt", C.c_int64), ("stream_tets", C.c_int64),
        ("device_mesh_bytes", C.c_uint64), ("load_seconds", C.c_double),
        ("requests", C.c_uint64), ("blocks_built", C.c_uint64), ("entries_built", C.c_uint64),
        ("kernel_launches", C.c_uint64), ("overflow_reruns", C.c_uint64), ("global_path_blocks", C.c_uint64),
        ("tt_exhaustive_blocks", C.c_uint64),
        ("cache_hits", C.c_uint64), ("cache_misses", C.c_uint64), ("evictions", C.c_uint64),
        ("cache_bytes_resident", C.c_uint64), ("cache_budget", C.c_uint64),
        ("entries_delivered", C.c_uint64), ("bytes_d2h", C.c_uint64), ("batches", C.c_uint64),
        ("mean_batch_clusters", C.c_double), ("queue_depth_mean", C.c_double),
        ("queue_depth_max", C.c_int32), ("pad", C.c_int32),
        ("lat_p50_us", C.c_double), ("lat_p99_us", C.c_double), ("lat_mean_us", C.c_double),
        ("lat_max_us", C.c_double), ("lat_count", C.c_uint64),
        ("stage_queue_us", C.c_double), ("stage_build_us", C.c_double), ("stage_copy_us", C.c_double),
        ("timed_launches", C.c_uint64), ("kernel_ms_total", C.c_double), ("hybrid_path_blocks", C.c_uint64),
        ("global_cu_share", C.c_double),
        ("stage_push_us", C.c_double), ("stage_prep_us", C.c_double), ("stage_kernel_copy_us", C.c_double),
        ("stage_integration_us", C.c_double),
        ("wait_push_s_max", C.c_double), ("wait_queue_s_max", C.c_double), ("wait_prep_s_max", C.c_double),
        ("wait_kernel_copy_s_max", C.c_double), ("wait_integration_s_max", C.c_double),
        ("prefetch_built", C.c_uint64), ("prefetch_hits", C.c_uint64), ("prefetch_evicted", C.c_uint64),
        ("demand_evictions", C.c_uint64), ("front_end", C.c_int32), ("tune_applied", C.c_int32),
    ]


class GaleSimplices(C.Structure):
    _fields_ = [
        ("ne", C.c_int64), ("nf", C.c_int64), ("ncl", C.c_int32), ("pad", C.c_int32),
        ("e", C.POINTER(C.c_int32)), ("f", C.POINTER(C.c_int32)), ("ie", C.POINTER(C.c_int64)),
        ("if_", C.POINTER(C.c_int64)),
    ]


class GaleClusterInfo(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("cluster", "nV", "nT", "ns", "nh", "L", "nnzVT", "cap_vv")]


class GaleConsumerCfg(C.Structure):
    _fields_ = [
        ("threads", C.c_int32), ("n_order", C.c_int32), ("cluster_order", C.POINTER(C.c_int32)),
        ("rel_mask", C.c_uint32), ("pad", C.c_int32), ("seed", C.c_uint64), ("zipf_s", C.c_double),
        ("tets", C.POINTER(C.c_int32)), ("nt", C.c_int64), ("field", C.POINTER(C.c_float)),
        ("nv", C.c_int32), ("pad2", C.c_int32),
    ]


class GaleConsumerResult(C.Structure):
    _fields_ = [
        ("accesses", C.c_uint64), ("reaccesses", C.c_uint64), ("mismatches", C.c_uint64), ("errors", C.c_uint64),
        ("clusters", C.c_uint64), ("minima", C.c_uint64), ("maxima", C.c_uint64), ("saddles", C.c_uint64),
        ("regular", C.c_uint64), ("wall_s", C.c_double), ("lat_p50_us", C.c_double), ("lat_p99_us", C.c_double),
        ("lat_mean_us", C.c_double), ("lat_max_us", C.c_double), ("first_error", C.c_int32), ("pad", C.c_int32),
    ]


class GaleGradientCfg(C.Structure):
    _fields_ = [
        ("threads", C.c_int32), ("n_order", C.c_int32), ("cluster_order", C.POINTER(C.c_int32)),
        ("tets", C.POINTER(C.c_int32)), ("nt", C.c_int64), ("field", C.POINTER(C.c_float)),
        ("nv", C.c_int32), ("pad", C.c_int32),
    ]


class GaleGradientResult(C.Structure):
    _fields_ = [
        ("clusters", C.c_uint64), ("errors", C.c_uint64), ("critical", C.c_uint64 * 4), ("pairs", C.c_uint64 * 3),
        ("wall_s", C.c_double), ("lat_p50_us", C.c_double), ("lat_p99_us", C.c_double),
        ("lat_mean_us", C.c_double), ("lat_max_us", C.c_double), ("request_s_max", C.c_double),
        ("compute_s_max", C.c_double), ("first_error", C.c_int32), ("pad", C.c_int32),
    ]


class GaleError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s: %s (%s) %s" % (where, _NAMES.get(status, status), status, detail))
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgale.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libgale.so is not built (%s); run __graft_entry__.build()" % path)
    # PyTorch ships its own HIP runtime under the same sonames as the system
    # one this library links to.  Loading torch first makes the library's
    # dependency resolve to the runtime already in the process, so the
    # library and torch (device memory, streams) share one runtime whatever
    # order the caller initialises them in.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    i32p = C.POINTER(C.c_int32)
    vp = C.c_void_p
    u64p = C.POINTER(C.c_uint64)
    sig = {
        "gale_create": ([C.POINTER(GaleConfig), C.POINTER(vp)], C.c_int32),
        "gale_load": ([vp, C.c_int32, C.c_int64, i32p, i32p, C.c_int32], C.c_int32),
        "gale_submit": ([vp, i32p, C.c_int32, C.c_uint32, u64p], C.c_int32),
        "gale_build": ([vp, i32p, C.c_int32, C.c_uint32, C.c_int32, u64p], C.c_int32),
        "gale_build_static": ([vp, i32p, C.c_int32, C.c_uint32, vp, C.c_int64, C.POINTER(C.c_int64)],
                              C.c_int32),
        "gale_poll": ([vp, C.c_uint64, C.c_int64], C.c_int32),
        "gale_block": ([vp, C.c_uint64, C.c_int32, C.c_uint32, C.POINTER(GaleCsr)], C.c_int32),
        "gale_block_device": ([vp, C.c_uint64, C.c_int32, C.c_uint32, C.POINTER(GaleCsr)], C.c_int32),
        "gale_release": ([vp, C.c_uint64], C.c_int32),
        "gale_get_stats": ([vp, C.POINTER(GaleStats)], C.c_int32),
        "gale_reset_stats": ([vp], C.c_int32),
        "gale_get_cluster_info": ([vp, C.c_int32, C.POINTER(GaleClusterInfo)], C.c_int32),
        "gale_get_simplices": ([vp, C.POINTER(GaleSimplices)], C.c_int32),
        "gale_stream": ([vp], vp),
        "gale_strerror": ([C.c_int32], C.c_char_p),
        "gale_last_error": ([], C.c_char_p),
        "gale_destroy": ([vp], None),
        "gale_graph_create": ([vp, i32p, C.c_int32, C.c_uint32, u64p], C.c_int32),
        "gale_graph_launch": ([vp, C.c_uint64, u64p], C.c_int32),
        "gale_graph_destroy": ([vp, C.c_uint64], C.c_int32),
        "gale_autotune": ([vp, i32p, C.c_int32, C.c_uint32, C.c_int32, i32p, C.POINTER(C.c_double)], C.c_int32),
        "gale_lowerstar_classify": ([C.c_int32, i32p, i32p, i32p, i32p, i32p, i32p, C.c_int64,
                                     C.POINTER(C.c_float), C.c_int32, i32p], C.c_int32),
        "gale_consumer_run": ([vp, C.POINTER(GaleConsumerCfg), C.POINTER(GaleConsumerResult)], C.c_int32),
        "gale_gradient_cluster": ([C.c_int32, i32p, i32p, i32p, i32p, i32p, i32p, i32p, i32p, C.c_int64, i32p,
                                   C.c_int64, i32p, C.c_int64, C.POINTER(C.c_float), C.c_int32, i32p, C.c_int64,
                                   C.POINTER(C.c_int64)], C.c_int32),
        "gale_gradient_run": ([vp, C.POINTER(GaleGradientCfg), C.POINTER(GaleGradientResult)], C.c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _check(st: int, where: str):
    if st != OK:
        raise GaleError(st, where, _lib.gale_last_error().decode(errors="replace"))


class Context:
    """One library context (one device).  ``mode`` is "direct" or "serve";
    ``form`` (direct mode) is "plain" or "batched"."""

    def __init__(self, device: int = 0, mode: str = "direct", form: str = "batched", block_threads: int = 0,
                 lds_bytes: int = 0, max_inflight: int = 0, cache_budget_bytes: int = 0, max_queue: int = 0,
                 stream=None, launch_classes: int = 0, global_cu_share: float = 0.0, dev_arena=None,
                 arena_bytes: int = 0, tune_table_path: str | None = None, prefetch_depth: int = 0,
                 front_end: str = "single", simplex_lists: bool = False, tile_entries: int = 0):
        lib = load_library()
        self._lib = lib
        cfg = GaleConfig()
        cfg.device = device
        cfg.mode = {"direct": MODE_DIRECT, "serve": MODE_SERVE}[mode]
        cfg.form = {"plain": FORM_PLAIN, "batched": FORM_BATCHED}[form]
        cfg.block_threads = block_threads
        cfg.lds_bytes = lds_bytes
        cfg.max_inflight = max_inflight
        cfg.cache_budget_bytes = cache_budget_bytes
        cfg.max_queue = max_queue
        cfg.launch_classes = launch_classes
        cfg.hip_stream = stream
        cfg.global_cu_share = global_cu_share
        cfg.dev_arena = dev_arena
        cfg.arena_bytes = arena_bytes
        self._tune_path = tune_table_path.encode() if tune_table_path else None
        cfg.tune_table_path = self._tune_path
        cfg.prefetch_depth = prefetch_depth
        cfg.front_end = {"single": FRONT_SINGLE, "per_relation": FRONT_PER_RELATION}[front_end]
        cfg.simplex_lists = 1 if simplex_lists else 0
        cfg.tile_entries = int(tile_entries)
        h = C.c_void_p()
        _check(lib.gale_create(C.byref(cfg), C.byref(h)), "gale_create")
        self._h = h
        self.mode = mode

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gale_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self) -> int:
        return int(self._lib.gale_stream(self._h) or 0)

    def load(self, tets, cluster, nclusters: int):
        t, tp = _i32(np.asarray(tets).reshape(-1))
        c, cp = _i32(cluster)
        _check(self._lib.gale_load(self._h, int(c.shape[0]), int(t.shape[0] // 4), tp, cp, int(nclusters)),
               "gale_load")

    def submit(self, ids, mask: int = REL_ALL) -> int:
        a, p = _i32(np.atleast_1d(ids))
        tk = C.c_uint64()
        _check(self._lib.gale_submit(self._h, p, int(a.shape[0]), int(mask), C.byref(tk)), "gale_submit")
        return tk.value

    def try_submit(self, ids, mask: int = REL_ALL):
        """Like submit, but returns the status instead of raising (for EAGAIN)."""
        a, p = _i32(np.atleast_1d(ids))
        tk = C.c_uint64()
        st = self._lib.gale_submit(self._h, p, int(a.shape[0]), int(mask), C.byref(tk))
        return st, tk.value

    def build(self, ids, mask: int = REL_ALL, form: str = "batched") -> int:
        a, p = _i32(np.atleast_1d(ids))
        tk = C.c_uint64()
        f = {"plain": FORM_PLAIN, "batched": FORM_BATCHED}[form]
        _check(self._lib.gale_build(self._h, p, int(a.shape[0]), int(mask), f, C.byref(tk)), "gale_build")
        return tk.value

    def build_static(self, ids, mask: int, dev_out: int, out_words: int):
        """gale_build_static: build into the device buffer at address dev_out
        (out_words int32 words) with no device allocation; returns (status,
        block_words) where block_words[i] is the word offset of ids[i]'s block
        and block_words[-1] the words needed (status ENOMEM: buffer too small,
        nothing built)."""
        a, p = _i32(np.atleast_1d(ids))
        bw = np.zeros(a.shape[0] + 1, np.int64)
        st = self._lib.gale_build_static(self._h, p, int(a.shape[0]), int(mask), dev_out or None, int(out_words),
                                         bw.ctypes.data_as(C.POINTER(C.c_int64)))
        if st not in (OK, ENOMEM):
            _check(st, "gale_build_static")
        return st, bw

    def poll(self, ticket: int, timeout_ns: int = -1) -> bool:
        st = self._lib.gale_poll(self._h, C.c_uint64(ticket), int(timeout_ns))
        if st == EAGAIN:
            return False
        _check(st, "gale_poll")
        return True

    def _view(self, fn, ticket, cluster, rel):
        v = GaleCsr()
        _check(fn(self._h, C.c_uint64(ticket), int(cluster), int(rel), C.byref(v)), fn.__name__)
        return v

    def block(self, ticket: int, cluster: int, rel: int):
        """Host block as numpy copies (row_ids, offsets, entries)."""
        v = self._view(self._lib.gale_block, ticket, cluster, rel)
        n, z = v.nrows, v.nnz
        rows = np.ctypeslib.as_array(v.row_ids, shape=(n,)).copy() if n else np.empty(0, np.int32)
        offs = np.ctypeslib.as_array(v.offsets, shape=(n + 1,)).copy()
        ents = np.ctypeslib.as_array(v.entries, shape=(z,)).copy() if z else np.empty(0, np.int32)
        return rows, offs, ents

    def block_device(self, ticket: int, cluster: int, rel: int) -> GaleCsr:
        """Device view: raw device pointers and sizes."""
        return self._view(self._lib.gale_block_device, ticket, cluster, rel)

    def release(self, ticket: int):
        _check(self._lib.gale_release(self._h, C.c_uint64(ticket)), "gale_release")

    def stats(self) -> dict:
        s = GaleStats()
        _check(self._lib.gale_get_stats(self._h, C.byref(s)), "gale_get_stats")
        return {name: getattr(s, name) for name, _ in GaleStats._fields_ if name != "pad"}

    def graph_create(self, cluster_ids, mask: int = 7) -> int:
        a = np.ascontiguousarray(cluster_ids, np.int32)
        g = C.c_uint64()
        _check(self._lib.gale_graph_create(self._h, a.ctypes.data_as(C.POINTER(C.c_int32)), int(a.shape[0]),
                                           int(mask), C.byref(g)), "gale_graph_create")
        return g.value

    def graph_launch(self, graph: int) -> int:
        tk = C.c_uint64()
        _check(self._lib.gale_graph_launch(self._h, int(graph), C.byref(tk)), "gale_graph_launch")
        return tk.value

    def graph_destroy(self, graph: int):
        _check(self._lib.gale_graph_destroy(self._h, int(graph)), "gale_graph_destroy")

    def autotune(self, cluster_ids, mask: int = 7, reps: int = 2):
        """Time the launch-class candidates (0, 2, 4, 6) on this request and keep
        the fastest (then the global launch's share of the CUs, see
        stats()["global_cu_share"]); returns (chosen, {candidate: mean ms})."""
        a = np.ascontiguousarray(cluster_ids, np.int32)
        p = a.ctypes.data_as(C.POINTER(C.c_int32))
        chosen = C.c_int32()
        ms = (C.c_double * 4)()
        _check(self._lib.gale_autotune(self._h, p, int(a.shape[0]), int(mask), int(reps), C.byref(chosen), ms),
               "gale_autotune")
        return chosen.value, dict(zip((0, 2, 4, 6), list(ms)))

    def cluster_info(self, cluster: int) -> dict:
        """Sizes of one cluster's prepared lists (nV, nT, ns, nh, L, nnzVT, cap_vv)."""
        ci = GaleClusterInfo()
        _check(self._lib.gale_get_cluster_info(self._h, int(cluster), C.byref(ci)), "gale_get_cluster_info")
        return {name: getattr(ci, name) for name, _ in GaleClusterInfo._fields_}

    def simplices(self):
        """(E as ne x 2, I_E, F as nf x 3, I_F) copied from the library's
        edge and triangle lists (gale_get_simplices)."""
        x = GaleSimplices()
        _check(self._lib.gale_get_simplices(self._h, C.byref(x)), "gale_get_simplices")
        ne, nf, ncl = x.ne, x.nf, x.ncl
        e = np.ctypeslib.as_array(x.e, shape=(2 * ne,)).reshape(ne, 2).copy() if ne else np.empty((0, 2), np.int32)
        f = np.ctypeslib.as_array(x.f, shape=(3 * nf,)).reshape(nf, 3).copy() if nf else np.empty((0, 3), np.int32)
        ie = np.ctypeslib.as_array(x.ie, shape=(ncl + 1,)).copy()
        if_ = np.ctypeslib.as_array(x.if_, shape=(ncl + 1,)).copy()
        return e, ie, f, if_

    def reset_stats(self):
        _check(self._lib.gale_reset_stats(self._h), "gale_reset_stats")


def strerror(status: int) -> str:
    return load_library().gale_strerror(int(status)).decode()


CP_REGULAR, CP_MINIMUM, CP_MAXIMUM, CP_SADDLE = 0, 1, 2, 3


def lowerstar_classify(rows, vt, vv, tets, field) -> np.ndarray:
    """Critical-point label of every row of one cluster from its VT and VV
    blocks (each a (row_ids, offsets, entries) triple as returned by
    Context.block), the mesh tetrahedra and a float32 field; see
    include/gale_lowerstar.h.  Runs on the calling thread (the GIL is released)."""
    lib = load_library()
    i32 = C.POINTER(C.c_int32)
    rows = np.ascontiguousarray(rows, np.int32)
    vt_off, vt_ent = (np.ascontiguousarray(a, np.int32) for a in vt[1:])
    vv_off, vv_ent = (np.ascontiguousarray(a, np.int32) for a in vv[1:])
    tets = np.ascontiguousarray(tets, np.int32)
    field = np.ascontiguousarray(field, np.float32)
    out = np.empty(rows.shape[0], np.int32)
    st = lib.gale_lowerstar_classify(int(rows.shape[0]), rows.ctypes.data_as(i32), vt_off.ctypes.data_as(i32),
                                     vt_ent.ctypes.data_as(i32), vv_off.ctypes.data_as(i32),
                                     vv_ent.ctypes.data_as(i32), tets.ctypes.data_as(i32), int(tets.shape[0]),
                                     field.ctypes.data_as(C.POINTER(C.c_float)), int(field.shape[0]),
                                     out.ctypes.data_as(i32))
    if st != 0:
        raise GaleError(EINVAL, "gale_lowerstar_classify", "invalid block or id out of range")
    return out


def consumer_run(ctx: "Context", tets, field, cluster_order, threads: int = 40, mask: int = 7, seed: int = 0,
                 zipf_s: float = 1.1) -> dict:
    """Run the consumer workload with native threads against ctx (see
    include/gale_lowerstar.h); returns the result fields as a dict."""
    lib = load_library()
    order = np.ascontiguousarray(cluster_order, np.int32)
    tets = np.ascontiguousarray(tets, np.int32)
    field = np.ascontiguousarray(field, np.float32)
    i32 = C.POINTER(C.c_int32)
    cfg = GaleConsumerCfg(threads=int(threads), n_order=int(order.shape[0]), cluster_order=order.ctypes.data_as(i32),
                          rel_mask=int(mask), seed=int(seed), zipf_s=float(zipf_s), tets=tets.ctypes.data_as(i32),
                          nt=int(tets.shape[0]), field=field.ctypes.data_as(C.POINTER(C.c_float)),
                          nv=int(field.shape[0]))
    res = GaleConsumerResult()
    st = lib.gale_consumer_run(ctx._h, C.byref(cfg), C.byref(res))
    if st != OK:
        raise GaleError(st, "gale_consumer_run", "bad argument")
    return {name: getattr(res, name) for name, _ in GaleConsumerResult._fields_ if not name.startswith("pad")}


def gradient_cluster(ve, vf, vt, edges, faces, tets, field) -> np.ndarray:
    """Discrete gradient of one cluster's lower stars (include/gale_gradient.h)
    from its VE, VF, VT blocks (each (row_ids, offsets, entries)), the edge and
    triangle lists, the mesh and a float32 field; returns the records as an
    (n, 3) int32 array of {dim, lower id, upper id} (upper -1: critical)."""
    lib = load_library()
    i32 = C.POINTER(C.c_int32)
    rows = np.ascontiguousarray(ve[0], np.int32)
    arrs = [np.ascontiguousarray(a, np.int32) for a in (ve[1], ve[2], vf[1], vf[2], vt[1], vt[2])]
    edges = np.ascontiguousarray(edges, np.int32).reshape(-1)
    faces = np.ascontiguousarray(faces, np.int32).reshape(-1)
    tets = np.ascontiguousarray(tets, np.int32).reshape(-1)
    field = np.ascontiguousarray(field, np.float32)
    cap = rows.shape[0] + arrs[1].shape[0] + arrs[3].shape[0] + arrs[5].shape[0]
    rec = np.empty((max(cap, 1), 3), np.int32)
    n = C.c_int64()
    p = [a.ctypes.data_as(i32) for a in arrs]
    st = lib.gale_gradient_cluster(int(rows.shape[0]), rows.ctypes.data_as(i32), p[0], p[1], p[2], p[3], p[4], p[5],
                                   edges.ctypes.data_as(i32), int(edges.shape[0] // 2), faces.ctypes.data_as(i32),
                                   int(faces.shape[0] // 3), tets.ctypes.data_as(i32), int(tets.shape[0] // 4),
                                   field.ctypes.data_as(C.POINTER(C.c_float)), int(field.shape[0]),
                                   rec.ctypes.data_as(i32), int(cap), C.byref(n))
    if st != 0:
        raise GaleError(EINVAL, "gale_gradient_cluster", "invalid block, id out of range or record space")
    return rec[: n.value].copy()


def gradient_run(ctx: "Context", tets, field, cluster_order, threads: int = 40) -> dict:
    """The DiscreteGradient workload with native threads against a DIRECT-mode
    context loaded with simplex_lists (include/gale_gradient.h)."""
    lib = load_library()
    order = np.ascontiguousarray(cluster_order, np.int32)
    tets = np.ascontiguousarray(tets, np.int32)
    field = np.ascontiguousarray(field, np.float32)
    i32 = C.POINTER(C.c_int32)
    cfg = GaleGradientCfg(threads=int(threads), n_order=int(order.shape[0]), cluster_order=order.ctypes.data_as(i32),
                          tets=tets.ctypes.data_as(i32), nt=int(tets.shape[0]),
                          field=field.ctypes.data_as(C.POINTER(C.c_float)), nv=int(field.shape[0]))
    res = GaleGradientResult()
    st = lib.gale_gradient_run(ctx._h, C.byref(cfg), C.byref(res))
    if st != OK:
        raise GaleError(st, "gale_gradient_run", "bad argument or context")
    out = {name: getattr(res, name) for name, _ in GaleGradientResult._fields_ if not name.startswith("pad")}
    out["critical"] = list(res.critical)
    out["pairs"] = list(res.pairs)
    return out
