"""ctypes front-end of the plain FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import this package.  The product library never loads it, and it
never loads the product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "svf_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

L2, IP = 0, 1
P_FP32, P_FP16, P_BF16, P_FP8 = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (plain scalar C, no SIMD intrinsics)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp,
                               "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        vp, i32, i64, f64, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_uint64
        L.orc_create.restype = vp
        L.orc_create.argtypes = [i32, i32, i32, u64]
        L.orc_destroy.argtypes = [vp]
        L.orc_set.argtypes = [vp, C.c_char_p, f64]
        L.orc_n_slots.restype = i64
        L.orc_n_slots.argtypes = [vp]
        L.orc_n_alive.restype = i64
        L.orc_n_alive.argtypes = [vp]
        L.orc_build.argtypes = [vp, vp, i64, i64]
        L.orc_insert.argtypes = [vp, vp, i64, vp]
        L.orc_delete.argtypes = [vp, vp, i64]
        L.orc_consolidate.argtypes = [vp]
        L.orc_consolidate_wait.argtypes = [vp]
        L.orc_search.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, vp, vp, vp, vp, i32]
        L.orc_bruteforce.argtypes = [vp, i64, i32, vp, i32, vp, i64, i32, vp, vp, i32]
        L.orc_export.argtypes = [vp, vp, vp, vp]
        L.orc_import.argtypes = [vp, vp, i64, vp, vp, vp]
        L.orc_dist_ids.restype = f64
        L.orc_dist_ids.argtypes = [vp, i32, i32]
        L.orc_round_fp16.restype = f64
        L.orc_round_fp16.argtypes = [f64]
        L.orc_round_bf16.restype = f64
        L.orc_round_bf16.argtypes = [f64]
        L.orc_round_e4m3.restype = f64
        L.orc_round_e4m3.argtypes = [f64]
        L.orc_fp8_vectors.argtypes = [vp, i64, i32, i32, vp, vp]
        L.orc_fnv1a64.restype = u64
        L.orc_fnv1a64.argtypes = [vp, i64]
        L.orc_splitmix64.restype = u64
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_prune_explicit.argtypes = [i32, i32, vp, vp, vp, i64, vp, vp]
        L.orc_query_dists.argtypes = [vp, vp, i64, i32, vp, vp]
        L.orc_search_expansions.argtypes = [vp, vp, i64, i32, vp, i32, vp]
        L.orc_wavp_replay.argtypes = [i64, i64, vp, vp, vp, vp, i32, f64, f64, f64, i32, i32, f64, vp,
                                      vp, vp]
        L.orc_policy_replay.argtypes = [i32, i64, i64, vp, vp, vp, vp, i32, i32, i32, vp, vp]
        L.orc_search_listed.argtypes = [vp, vp, i64, i32, i32, vp, i32, vp, vp, vp, vp]
        L.orc_search_trace.argtypes = [vp, vp, i64, i32, i32, vp, vp]
        L.orc_mlp_forward.argtypes = [i32, i32, i32] + [vp] * 6 + [vp, i64, vp]
        L.orc_model_decide.argtypes = [vp, i64, i32, f64, f64, i32, vp, vp]
        L.orc_mlp_loss_grad.restype = f64
        L.orc_mlp_loss_grad.argtypes = [i32, i32, i32] + [vp] * 6 + [vp, vp, vp, i64, f64, f64] + [vp] * 6
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle call failed with status %d" % rc)


class OracleIndex:
    """FP64 reference of search / insert / delete / consolidate."""

    def __init__(self, dim: int, degree: int, metric: int = L2, seed: int = 0, **opts):
        self.dim, self.R, self.metric = dim, degree, metric
        self.h = lib().orc_create(dim, degree, metric, seed)
        if not self.h:
            raise ValueError("invalid oracle parameters")
        for k, v in opts.items():
            self.set(k, v)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def set(self, key: str, value: float):
        _check(lib().orc_set(self.h, key.encode(), float(value)))

    @property
    def n_slots(self):
        return lib().orc_n_slots(self.h)

    @property
    def n_alive(self):
        return lib().orc_n_alive(self.h)

    def build(self, vecs: np.ndarray, batch_max: int = 10_000):
        v = np.ascontiguousarray(vecs, dtype=np.float32)
        _check(lib().orc_build(self.h, _p(v), v.shape[0], batch_max))

    def insert(self, vecs: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(vecs, dtype=np.float32)
        ids = np.empty(v.shape[0], dtype=np.int32)
        _check(lib().orc_insert(self.h, _p(v), v.shape[0], _p(ids)))
        return ids

    def delete(self, ids) -> int:
        a = np.ascontiguousarray(ids, dtype=np.int32)
        return lib().orc_delete(self.h, _p(a), a.shape[0])

    def consolidate(self):
        _check(lib().orc_consolidate(self.h))

    def consolidate_wait(self):
        """Merge a consolidation pending in the background (Sec. 5.3)."""
        _check(lib().orc_consolidate_wait(self.h))

    def search(self, q: np.ndarray, k: int, beam: int, rerank: bool = True, threads: int = 1):
        q = np.ascontiguousarray(q, dtype=np.float32)
        nq = q.shape[0]
        ids = np.empty((nq, k), dtype=np.int32)
        d = np.empty((nq, k), dtype=np.float64)
        nd = np.empty(nq, dtype=np.int64)
        ne = np.empty(nq, dtype=np.int64)
        it = np.empty(nq, dtype=np.int64)
        mg = np.empty(nq, dtype=np.float64)
        _check(lib().orc_search(self.h, _p(q), nq, k, beam, int(rerank), _p(ids), _p(d), _p(nd),
                                _p(ne), _p(it), _p(mg), threads))
        return ids, d, dict(n_dist=nd, n_exp=ne, iters=it, margin=mg)

    def search_listed(self, q, k, beam, entries, max_iters=None):
        """Search whose pools start from given entry lists (nq x ecap, -1 pad)
        with optional per-query expansion caps."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        e = np.ascontiguousarray(entries, dtype=np.int32)
        mi = None if max_iters is None else np.ascontiguousarray(max_iters, dtype=np.int32)
        nq = q.shape[0]
        ids = np.empty((nq, k), np.int32)
        d = np.empty((nq, k), np.float64)
        ne = np.empty(nq, np.int64)
        _check(lib().orc_search_listed(self.h, _p(q), nq, k, beam, _p(e), e.shape[1], _p(mi),
                                       _p(ids), _p(d), _p(ne)))
        return ids, d, ne

    def search_trace(self, q, k, beam):
        """Plain search plus the expansion count after which the top-k stopped
        changing."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        ids = np.empty((q.shape[0], k), np.int32)
        lc = np.empty(q.shape[0], np.int32)
        _check(lib().orc_search_trace(self.h, _p(q), q.shape[0], k, beam, _p(ids), _p(lc)))
        return ids, lc

    def search_expansions(self, q, beam, cap=4096):
        """Per query, the vertices expanded in order (first `cap`), and counts."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        tr = np.full((q.shape[0], cap), -1, np.int32)
        cnt = np.empty(q.shape[0], np.int32)
        _check(lib().orc_search_expansions(self.h, _p(q), q.shape[0], beam, _p(tr), cap, _p(cnt)))
        return tr, cnt

    def export(self):
        n = self.n_slots
        rows = np.empty((n, self.R), dtype=np.int32)
        ed = np.empty((n, self.R), dtype=np.float64)
        alive = np.empty(n, dtype=np.uint8)
        _check(lib().orc_export(self.h, _p(rows), _p(ed), _p(alive)))
        return rows, ed, alive

    def import_state(self, vecs, rows, edge_d, alive):
        v = np.ascontiguousarray(vecs, dtype=np.float32)
        r = np.ascontiguousarray(rows, dtype=np.int32)
        e = np.ascontiguousarray(edge_d, dtype=np.float64)
        a = np.ascontiguousarray(alive, dtype=np.uint8)
        _check(lib().orc_import(self.h, _p(v), v.shape[0], _p(r), _p(e), _p(a)))

    def dist_ids(self, a: int, b: int) -> float:
        return lib().orc_dist_ids(self.h, int(a), int(b))

    def query_dists(self, q, ids):
        """Exact FP64 distances of each query to the given stored ids."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        out = np.empty(ids.shape, dtype=np.float64)
        lib().orc_query_dists(self.h, _p(q), q.shape[0], ids.shape[1], _p(ids), _p(out))
        return out


def bruteforce(base, q, k, metric=L2, alive=None, threads=1):
    """Exact k nearest by (d, id) over the alive rows of base, FP64."""
    base = np.ascontiguousarray(base, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    a = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    ids = np.empty((q.shape[0], k), dtype=np.int32)
    d = np.empty((q.shape[0], k), dtype=np.float64)
    lib().orc_bruteforce(_p(base), base.shape[0], base.shape[1], _p(a), metric, _p(q), q.shape[0],
                         k, _p(ids), _p(d), threads)
    return ids, d


def round_fp16(x: float) -> float:
    return lib().orc_round_fp16(float(x))


def round_bf16(x: float) -> float:
    return lib().orc_round_bf16(float(x))


def round_e4m3(x: float) -> float:
    """OCP FP8 E4M3 value grid, round to nearest even, saturating at 448."""
    return lib().orc_round_e4m3(float(x))


def fp8_vectors(x, query: bool = False):
    """FP8 form of the rows of x (float32): (per-row scale, reconstructed values
    in float64).  query=True gives the query form (FP32 products)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, d = x.shape
    sc = np.empty(n, dtype=np.float32)
    out = np.empty((n, d), dtype=np.float64)
    lib().orc_fp8_vectors(_p(x), n, d, 1 if query else 0, _p(sc), _p(out))
    return sc, out


def fnv1a64(b: bytes) -> int:
    buf = np.frombuffer(b, dtype=np.uint8).copy()
    return lib().orc_fnv1a64(_p(buf), len(b))


def splitmix64(state: int, j: int) -> int:
    return lib().orc_splitmix64(state, j)


def prune_explicit(R, cand_ids, cand_d, table):
    """Rank-based reordering of an explicit (d,id)-ordered candidate list."""
    cid = np.ascontiguousarray(cand_ids, dtype=np.int32)
    cd = np.ascontiguousarray(cand_d, dtype=np.float64)
    tab = np.ascontiguousarray(table, dtype=np.int32)
    oi = np.empty(R, dtype=np.int32)
    od = np.empty(R, dtype=np.float64)
    lib().orc_prune_explicit(R, cid.shape[0], _p(cid), _p(cd), _p(tab), tab.shape[0], _p(oi), _p(od))
    return oi, od


def recall_at_k(found_ids, exact_d, gt_d, k):
    """Tie-aware recall@k.  A returned id counts when its exact distance
    (computed by the oracle, the same routine as the ground truth) does not
    exceed the exact k-th nearest distance; integer data has exact ties."""
    kth = gt_d[:, k - 1:k]
    ok = (found_ids[:, :k] >= 0) & (exact_d[:, :k] <= kth)
    return ok.sum() / (found_ids.shape[0] * k)


class MLP:
    """FP64 reference of the entry/stop predictor din -> h -> h -> nc+1 (ReLU).
    Weights are row-major (in x out) numpy float64 arrays."""

    def __init__(self, w1, b1, w2, b2, w3, b3):
        self.p = [np.ascontiguousarray(a, dtype=np.float64) for a in (w1, b1, w2, b2, w3, b3)]
        self.din, self.h = self.p[0].shape
        self.nc = self.p[4].shape[1] - 1

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.empty((x.shape[0], self.nc + 1))
        lib().orc_mlp_forward(self.din, self.h, self.nc, *[_p(a) for a in self.p], _p(x), x.shape[0],
                              _p(out))
        return out

    def loss_grad(self, x, label, log_stop, lam=0.1, delta=1.0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        lab = np.ascontiguousarray(label, dtype=np.int32)
        ls = np.ascontiguousarray(log_stop, dtype=np.float64)
        g = [np.empty_like(a) for a in self.p]
        loss = lib().orc_mlp_loss_grad(self.din, self.h, self.nc, *[_p(a) for a in self.p], _p(x),
                                       _p(lab), _p(ls), x.shape[0], lam, delta, *[_p(a) for a in g])
        return loss, g


def model_decide(z, conf, stop_scale, min_iters):
    """Gating of the learned form from outputs z (n x (nc + 1)): per query
    the entry cluster or -1 (plain search), and the expansion cap (0 for
    plain search)."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    n, nc = z.shape[0], z.shape[1] - 1
    qe = np.empty(n, np.int32)
    qm = np.empty(n, np.int32)
    lib().orc_model_decide(_p(z), n, nc, conf, stop_scale, min_iters, _p(qe), _p(qm))
    return qe, qm


def wavp_replay(n, C, e_in, alive, batches, alpha=0.6, beta=0.4, theta=1.0, promote_max=2048,
                warm=False, adapt=0.0, with_theta=False):
    """Batched workload-aware placement (Alg. 2) over per-batch access
    traces; returns (hits per batch, final slot table), plus the theta in
    force for each batch when with_theta.  warm=True starts from the
    cold-start placement (highest in-degree alive vectors first); adapt > 1
    turns on the theta adaptation by that factor."""
    e = np.ascontiguousarray(e_in, dtype=np.int32)
    a = np.ascontiguousarray(alive, dtype=np.uint8)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(b, np.int32) for b in batches])
                                if batches else np.zeros(0, np.int32), dtype=np.int32)
    off = np.zeros(len(batches) + 1, np.int64)
    off[1:] = np.cumsum([len(b) for b in batches])
    hits = np.empty(len(batches), np.int64)
    slots = np.empty(max(C, 1), np.int32)
    th = np.empty(max(len(batches), 1), np.float64)
    lib().orc_wavp_replay(n, C, _p(e), _p(a), _p(flat), _p(off), len(batches), alpha, beta, theta,
                          promote_max, int(warm), float(adapt), _p(hits), _p(slots), _p(th))
    if with_theta:
        return hits, slots[:C], th[:len(batches)]
    return hits, slots[:C]


POLICY_WAVP, POLICY_LRU, POLICY_LFU, POLICY_LRFU = 0, 1, 2, 3


def policy_replay(policy, n, C, e_in, alive, batches, promote_max=2048, warm=False):
    """The classic replacement policies (LRU, LFU, LRFU) in the batched form
    over per-batch access traces; returns (hits per batch, final slot table)."""
    e = np.ascontiguousarray(e_in, dtype=np.int32)
    a = np.ascontiguousarray(alive, dtype=np.uint8)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(b, np.int32) for b in batches])
                                if batches else np.zeros(0, np.int32), dtype=np.int32)
    off = np.zeros(len(batches) + 1, np.int64)
    off[1:] = np.cumsum([len(b) for b in batches])
    hits = np.empty(len(batches), np.int64)
    slots = np.empty(max(C, 1), np.int32)
    lib().orc_policy_replay(policy, n, C, _p(e), _p(a), _p(flat), _p(off), len(batches),
                            promote_max, int(warm), _p(hits), _p(slots))
    return hits, slots[:C]
