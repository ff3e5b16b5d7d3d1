"""MI355X-native streaming graph-ANN hot path (SVFusion, arXiv 2601.08528).

Thin Python binding of the C ABI in ``include/svf.h``: argument marshalling
only.  Every step of search, insertion, deletion and repair runs in the HIP
kernels of ``libsvf.so``; importing the binding without that library raises.
Host arrays are numpy; device buffers are passed as raw pointers (for
example ``torch.Tensor.data_ptr()``) together with a stream handle.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsvf.so")

METRIC_L2, METRIC_IP = 0, 1
PREC_FP32, PREC_FP16, PREC_BF16, PREC_FP8 = 0, 1, 2, 3
OK, E_INVAL, E_NOMEM, E_DEVICE, E_NOTFOUND, E_BUSY, E_INTERNAL = 0, -1, -2, -3, -4, -5, -6

EXPORTED = [
    "svf_create", "svf_destroy", "svf_set_option", "svf_get_option", "svf_insert",
    "svf_insert_dev", "svf_build", "svf_delete", "svf_consolidate", "svf_consolidate_wait", "svf_search",
    "svf_search_dev", "svf_stats_get", "svf_export_graph", "svf_import_graph", "svf_last_error",
    "svf_search_listed", "svf_search_trace", "svf_model_get", "svf_model_fit", "svf_mlp_create", "svf_mlp_destroy",
    "svf_mlp_num_params", "svf_mlp_set_params", "svf_mlp_get_params", "svf_mlp_forward",
    "svf_mlp_loss_grad", "svf_mlp_train", "svf_mlp_last_error",
    "svf_serve_start", "svf_serve_stop", "svf_submit_search", "svf_submit_insert",
    "svf_submit_delete", "svf_wait", "svf_save", "svf_load", "svf_cache_slots",
    "svf_cache_calibrate", "svf_search_dev_noalloc",
]


class RequestInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("queue_ms", C.c_double), ("total_ms", C.c_double),
                ("batch_queries", C.c_int64), ("epoch", C.c_int64)]


class SvfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("svf status %d: %s" % (code, msg))
        self.code = code


class Stats(C.Structure):
    _fields_ = [
        ("n_slots", C.c_int64), ("n_alive", C.c_int64), ("capacity", C.c_int64),
        ("last_queries", C.c_int64), ("last_n_dist", C.c_int64), ("last_n_exp", C.c_int64),
        ("last_search_ms", C.c_double),
        ("ins_search_ms", C.c_double), ("ins_prune_ms", C.c_double),
        ("ins_reverse_ms", C.c_double), ("ins_commit_ms", C.c_double),
        ("del_mark_ms", C.c_double), ("del_repair_ms", C.c_double),
        ("last_repaired", C.c_int64), ("device_bytes", C.c_int64),
        ("cache_slots", C.c_int64), ("cache_gather_hits", C.c_int64),
        ("cache_gather_misses", C.c_int64), ("cache_last_trace_hits", C.c_int64),
        ("cache_last_placed", C.c_int64), ("cache_promotions", C.c_int64),
        ("cache_evictions", C.c_int64),
        ("consolidations", C.c_int64), ("last_model_fallback", C.c_int64),
        ("long_lists", C.c_int64),
        ("place_count_ms", C.c_double), ("place_indeg_ms", C.c_double),
        ("place_walk_ms", C.c_double), ("place_evict_ms", C.c_double),
        ("place_apply_ms", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libsvf.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsvf.so is not built: run python -m paper_2601_08528_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.svf_create.argtypes = [i32, i32, i32, C.POINTER(vp)]
        L.svf_destroy.argtypes = [vp]
        L.svf_set_option.argtypes = [vp, C.c_char_p, f64]
        L.svf_get_option.argtypes = [vp, C.c_char_p, C.POINTER(f64)]
        L.svf_insert.argtypes = [vp, vp, i64, vp]
        L.svf_insert_dev.argtypes = [vp, vp, i64, vp, vp]
        L.svf_build.argtypes = [vp, vp, i64]
        L.svf_delete.argtypes = [vp, vp, i64]
        L.svf_consolidate.argtypes = [vp]
        L.svf_consolidate_wait.argtypes = [vp]
        L.svf_search.argtypes = [vp, vp, i64, i32, i32, vp, vp]
        L.svf_search_dev.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, vp, vp]
        L.svf_search_dev_noalloc.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, vp, vp]
        L.svf_stats_get.argtypes = [vp, C.POINTER(Stats)]
        L.svf_export_graph.argtypes = [vp, vp, vp, vp, i64]
        L.svf_import_graph.argtypes = [vp, vp, i64, vp, vp, vp]
        L.svf_cache_slots.argtypes = [vp, vp, i64, C.POINTER(i64)]
        L.svf_cache_calibrate.argtypes = [vp, vp]
        L.svf_save.argtypes = [vp, C.c_char_p]
        L.svf_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.svf_search_listed.argtypes = [vp, vp, i64, i32, i32, vp, i32, vp, vp, vp]
        L.svf_search_trace.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp]
        L.svf_model_get.argtypes = [vp, vp, vp, vp, i64, vp, i64]
        L.svf_model_fit.argtypes = [vp, vp, i64, i32, i32, i32, i32, C.POINTER(C.c_float)]
        L.svf_mlp_create.argtypes = [i32, i32, i32, C.c_uint64, C.POINTER(vp)]
        L.svf_mlp_destroy.argtypes = [vp]
        L.svf_mlp_num_params.argtypes = [vp, C.POINTER(i64)]
        L.svf_mlp_set_params.argtypes = [vp, vp]
        L.svf_mlp_get_params.argtypes = [vp, vp]
        L.svf_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.svf_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i64, C.c_float, C.c_float,
                                        C.POINTER(C.c_float), vp]
        L.svf_mlp_train.argtypes = [vp, vp, vp, vp, i64, i32, i32, C.c_float, C.c_float,
                                    C.c_float, C.POINTER(C.c_float)]
        L.svf_serve_start.argtypes = [vp, i32, i64, i64]
        L.svf_serve_stop.argtypes = [vp]
        L.svf_submit_search.argtypes = [vp, vp, i64, i32, i32, vp, vp, C.POINTER(C.c_uint64)]
        L.svf_submit_insert.argtypes = [vp, vp, i64, vp, C.POINTER(C.c_uint64)]
        L.svf_submit_delete.argtypes = [vp, vp, i64, C.POINTER(C.c_uint64)]
        L.svf_wait.argtypes = [vp, C.c_uint64, f64, C.POINTER(RequestInfo)]
        L.svf_last_error.restype = C.c_char_p
        L.svf_mlp_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if not name.endswith("last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SvfError(rc, lib().svf_last_error().decode())
    return rc


def _p(a):
    return None if a is None else a.ctypes.data


class Index:
    """One index handle (``svf_create`` ... ``svf_destroy``)."""

    def __init__(self, dim: int, degree: int, metric: int = METRIC_L2, **options):
        h = C.c_void_p()
        _check(lib().svf_create(dim, degree, metric, C.byref(h)))
        self.h = h
        self.dim, self.degree, self.metric = dim, degree, metric
        for k, v in options.items():
            self.set_option(k, v)

    def close(self):
        if getattr(self, "h", None):
            lib().svf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key: str, value: float):
        _check(lib().svf_set_option(self.h, key.encode(), float(value)))

    def get_option(self, key: str) -> float:
        out = C.c_double()
        _check(lib().svf_get_option(self.h, key.encode(), C.byref(out)))
        return out.value

    def insert(self, vecs) -> np.ndarray:
        v = np.ascontiguousarray(vecs, dtype=np.float32).reshape(-1, self.dim)
        ids = np.empty(v.shape[0], np.int32)
        _check(lib().svf_insert(self.h, _p(v), v.shape[0], _p(ids)))
        return ids

    def insert_dev(self, d_vecs: int, n: int, d_out_ids: int | None = None, stream: int | None = None):
        _check(lib().svf_insert_dev(self.h, d_vecs, n, d_out_ids, stream))

    def build(self, vecs):
        v = np.ascontiguousarray(vecs, dtype=np.float32).reshape(-1, self.dim)
        _check(lib().svf_build(self.h, _p(v), v.shape[0]))

    def delete(self, ids):
        a = np.ascontiguousarray(ids, dtype=np.int32).reshape(-1)
        _check(lib().svf_delete(self.h, _p(a), a.shape[0]))

    def consolidate(self):
        _check(lib().svf_consolidate(self.h))

    def consolidate_wait(self):
        _check(lib().svf_consolidate_wait(self.h))

    def search(self, queries, k: int, beam: int):
        q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, self.dim)
        ids = np.empty((q.shape[0], k), np.int32)
        d = np.empty((q.shape[0], k), np.float32)
        _check(lib().svf_search(self.h, _p(q), q.shape[0], k, beam, _p(ids), _p(d)))
        return ids, d

    def search_dev(self, d_queries: int, nq: int, k: int, beam: int, d_ids: int, d_dists: int,
                   d_n_dist: int | None = None, d_n_exp: int | None = None, stream: int | None = None):
        _check(lib().svf_search_dev(self.h, d_queries, nq, k, beam, d_ids, d_dists, d_n_dist,
                                    d_n_exp, stream))

    def search_dev_noalloc(self, d_queries: int, nq: int, k: int, beam: int, d_ids: int,
                           d_dists: int, d_n_dist: int | None = None, d_n_exp: int | None = None,
                           stream: int | None = None):
        _check(lib().svf_search_dev_noalloc(self.h, d_queries, nq, k, beam, d_ids, d_dists,
                                            d_n_dist, d_n_exp, stream))

    def search_listed(self, queries, k: int, beam: int, entries, max_iters=None):
        q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, self.dim)
        e = np.ascontiguousarray(entries, dtype=np.int32).reshape(q.shape[0], -1)
        mi = None if max_iters is None else np.ascontiguousarray(max_iters, dtype=np.int32)
        ids = np.empty((q.shape[0], k), np.int32)
        d = np.empty((q.shape[0], k), np.float32)
        _check(lib().svf_search_listed(self.h, _p(q), q.shape[0], k, beam, _p(e), e.shape[1],
                                       _p(mi), _p(ids), _p(d)))
        return ids, d

    def search_trace(self, queries, k: int, beam: int):
        """Plain search plus, per query, the expansion count after which its
        top-k last changed."""
        q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, self.dim)
        ids = np.empty((q.shape[0], k), np.int32)
        d = np.empty((q.shape[0], k), np.float32)
        lc = np.empty(q.shape[0], np.int32)
        _check(lib().svf_search_trace(self.h, _p(q), q.shape[0], k, beam, _p(ids), _p(d), _p(lc)))
        return ids, d, lc

    def model_get(self, hidden: int = 256):
        """The trained predictor: (flat parameters, entry lists n_clusters x entry_cap)."""
        nc, ecap = C.c_int32(), C.c_int32()
        _check(lib().svf_model_get(self.h, C.byref(nc), C.byref(ecap), None, 0, None, 0))
        din, no = self.dim, nc.value + 1
        n = din * hidden + hidden + hidden * hidden + hidden + hidden * no + no
        params = np.empty(n, np.float32)
        lists = np.empty((nc.value, ecap.value), np.int32)
        _check(lib().svf_model_get(self.h, None, None, _p(params), n, _p(lists), lists.size))
        return params, lists

    def model_fit(self, train_queries, k: int, beam: int, n_clusters: int = 64, epochs: int = 10):
        q = np.ascontiguousarray(train_queries, dtype=np.float32).reshape(-1, self.dim)
        loss = C.c_float()
        _check(lib().svf_model_fit(self.h, _p(q), q.shape[0], k, beam, n_clusters, epochs,
                                   C.byref(loss)))
        return loss.value

    # ---- serving loop -----------------------------------------------------
    def serve_start(self, streams: int = 4, max_batch: int = 16384, hbm_budget: int = 0):
        _check(lib().svf_serve_start(self.h, streams, max_batch, hbm_budget))

    def serve_stop(self):
        _check(lib().svf_serve_stop(self.h))

    def submit_search(self, queries, k: int, beam: int):
        """Returns (ticket, ids, dists); the arrays fill in when the ticket
        completes (keep them alive until wait())."""
        q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, self.dim)
        ids = np.empty((q.shape[0], k), np.int32)
        d = np.empty((q.shape[0], k), np.float32)
        t = C.c_uint64()
        _check(lib().svf_submit_search(self.h, _p(q), q.shape[0], k, beam, _p(ids), _p(d),
                                       C.byref(t)))
        return t.value, ids, d

    def submit_insert(self, vecs):
        v = np.ascontiguousarray(vecs, dtype=np.float32).reshape(-1, self.dim)
        ids = np.empty(v.shape[0], np.int32)
        t = C.c_uint64()
        _check(lib().svf_submit_insert(self.h, _p(v), v.shape[0], _p(ids), C.byref(t)))
        return t.value, ids

    def submit_delete(self, ids):
        a = np.ascontiguousarray(ids, dtype=np.int32).reshape(-1)
        t = C.c_uint64()
        _check(lib().svf_submit_delete(self.h, _p(a), a.shape[0], C.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0) -> dict:
        info = RequestInfo()
        rc = lib().svf_wait(self.h, ticket, timeout_s, C.byref(info))
        out = {k: getattr(info, k) for k, _ in RequestInfo._fields_}
        if rc != 0:
            raise SvfError(rc, lib().svf_last_error().decode())
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(lib().svf_stats_get(self.h, C.byref(s)))
        return s.as_dict()

    @property
    def n_slots(self) -> int:
        return self.stats()["n_slots"]

    def export_graph(self):
        n = self.n_slots
        rows = np.empty((n, self.degree), np.int32)
        ed = np.empty((n, self.degree), np.float32)
        alive = np.empty(n, np.uint8)
        _check(lib().svf_export_graph(self.h, _p(rows), _p(ed), _p(alive), n))
        return rows, ed, alive

    def cache_slots(self):
        """(slot -> id table of the tiered store's cache, -1 empty; clock hand)."""
        c = int(self.stats()["cache_slots"])
        out = np.empty(max(c, 1), np.int32)
        clock = C.c_int64()
        _check(lib().svf_cache_slots(self.h, _p(out), c, C.byref(clock)))
        return out[:c], clock.value

    def cache_calibrate(self) -> dict:
        """Measure the hit, miss and transfer costs and set cache_theta from
        them (``svf_cache_calibrate``)."""
        out = np.empty(4, np.float64)
        _check(lib().svf_cache_calibrate(self.h, _p(out)))
        return dict(t_hit_ns=out[0], t_miss_ns=out[1], t_transfer_ns=out[2], theta=out[3])

    def save(self, path: str):
        """Checkpoint to a file (``svf_save``)."""
        _check(lib().svf_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path: str) -> "Index":
        """A new handle resumed from ``save``'s file (``svf_load``)."""
        h = C.c_void_p()
        _check(lib().svf_load(os.fsencode(path), C.byref(h)))
        ix = cls.__new__(cls)
        ix.h = h
        ix.dim, ix.degree, ix.metric = (int(ix.get_option(k)) for k in ("dim", "degree", "metric"))
        return ix

    def import_graph(self, vecs, rows, edge_d, alive):
        v = np.ascontiguousarray(vecs, dtype=np.float32).reshape(-1, self.dim)
        r = np.ascontiguousarray(rows, dtype=np.int32)
        e = np.ascontiguousarray(edge_d, dtype=np.float32)
        a = np.ascontiguousarray(alive, dtype=np.uint8)
        _check(lib().svf_import_graph(self.h, _p(v), v.shape[0], _p(r), _p(e), _p(a)))


def _mcheck(rc):
    if rc != 0:
        raise SvfError(rc, lib().svf_mlp_last_error().decode())


class Mlp:
    """The entry/stop predictor on its own (``svf_mlp_*``)."""

    def __init__(self, din: int, hidden: int, n_clusters: int, seed: int = 0):
        h = C.c_void_p()
        _mcheck(lib().svf_mlp_create(din, hidden, n_clusters, seed, C.byref(h)))
        self.h = h
        self.din, self.hidden, self.nc = din, hidden, n_clusters
        n = C.c_int64()
        _mcheck(lib().svf_mlp_num_params(self.h, C.byref(n)))
        self.n_params = n.value

    def __del__(self):
        if getattr(self, "h", None):
            lib().svf_mlp_destroy(self.h)
            self.h = None

    def shapes(self):
        d, h, no = self.din, self.hidden, self.nc + 1
        return [(d, h), (h,), (h, h), (h,), (h, no), (no,)]

    def split(self, flat):
        out, o = [], 0
        for s in self.shapes():
            n = int(np.prod(s))
            out.append(flat[o:o + n].reshape(s))
            o += n
        return out

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        _mcheck(lib().svf_mlp_get_params(self.h, _p(p)))
        return p

    def set_params(self, flat):
        p = np.ascontiguousarray(flat, dtype=np.float32)
        _mcheck(lib().svf_mlp_set_params(self.h, _p(p)))

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        out = np.empty((x.shape[0], self.nc + 1), np.float32)
        _mcheck(lib().svf_mlp_forward(self.h, _p(x), x.shape[0], _p(out)))
        return out

    def loss_grad(self, x, label, log_stop, lam=0.1, delta=1.0):
        x = np.ascontiguousarray(x, dtype=np.float32)
        lab = np.ascontiguousarray(label, dtype=np.int32)
        ls = np.ascontiguousarray(log_stop, dtype=np.float32)
        g = np.empty(self.n_params, np.float32)
        loss = C.c_float()
        _mcheck(lib().svf_mlp_loss_grad(self.h, _p(x), _p(lab), _p(ls), x.shape[0], lam, delta,
                                        C.byref(loss), _p(g)))
        return loss.value, g

    def train(self, x, label, log_stop, epochs=5, batch=256, lr=1e-3, lam=0.1, delta=1.0):
        x = np.ascontiguousarray(x, dtype=np.float32)
        lab = np.ascontiguousarray(label, dtype=np.int32)
        ls = np.ascontiguousarray(log_stop, dtype=np.float32)
        loss = C.c_float()
        _mcheck(lib().svf_mlp_train(self.h, _p(x), _p(lab), _p(ls), x.shape[0], epochs, batch, lr,
                                    lam, delta, C.byref(loss)))
        return loss.value
