"""Seeded synthetic inputs shaped like the paper's workloads.

The paper evaluates on real embedding datasets (its Table 2) that are not
available here; these generators stand in for them with Gaussian mixtures of
the sizes and dimensions the workloads use.  This module holds only input
generation (random numbers, mixture sampling, normalisation of generated
points, request-stream shapes); it contains none of the search or update
arithmetic, so both the HIP path and the CPU oracle may take their inputs
from it.

Every stream is a numpy ``Philox`` counter-based generator keyed by
``1000 * workload + role`` with roles::

    0 component means   1 base vectors   2 queries   3 request stream
    4 training queries  5 clustering      6 component shapes
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ROLE_MEANS, ROLE_BASE, ROLE_QUERIES, ROLE_STREAM, ROLE_TRAIN, ROLE_CLUSTER, ROLE_SHAPE = range(7)


def rng(workload: int, role: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=1000 * workload + role))


def _chunked_mixture(g, means, n, sigma, comp_p=None, chunk=1 << 18):
    """Draw n points m_c + sigma * N(0, I); component c uniform (or comp_p)."""
    k, d = means.shape
    out = np.empty((n, d), dtype=np.float32)
    comps = np.empty(n, dtype=np.int32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        if comp_p is None:
            c = g.integers(0, k, size=e - s)
        else:
            c = g.choice(k, size=e - s, p=comp_p)
        x = means[c] + sigma * g.standard_normal((e - s, d))
        out[s:e] = x.astype(np.float32)
        comps[s:e] = c
    return out, comps


def zipf_weights(k: int, s: float, perm_rng: np.random.Generator) -> np.ndarray:
    """Zipf(s) probabilities over k components, ranked by a seeded permutation."""
    w = 1.0 / np.arange(1, k + 1, dtype=np.float64) ** s
    w /= w.sum()
    p = np.empty(k)
    p[perm_rng.permutation(k)] = w
    return p


def gmm_float_device_chunks(torch, workload: int, n_base: int, dim: int, n_comp: int,
                            first: int = 0, chunk: int = 1 << 22, mean_std: float = 2.0,
                            sigma: float = 1.0, device: str = "cuda"):
    """The base points of gmm_float's mixture (same means), drawn on the device
    for sizes that do not fit host memory.  Rows [first, first + n_base) are
    yielded as (start row, n x dim FP32 tensor) blocks of at most `chunk`
    rows; block i of the full sequence comes from a torch Philox generator
    keyed by (workload, i), so any block can be drawn again on its own.
    `first` must be a multiple of `chunk`."""
    if first % chunk:
        raise ValueError("first must be a multiple of chunk")
    means = torch.from_numpy(rng(workload, ROLE_MEANS).standard_normal((n_comp, dim)) * mean_std)
    means = means.to(device=device, dtype=torch.float32)
    for s in range(first, first + n_base, chunk):
        e = min(first + n_base, s + chunk)
        g = torch.Generator(device=device)
        g.manual_seed((1000 * workload + ROLE_BASE) * (1 << 24) + s // chunk)
        c = torch.randint(0, n_comp, (e - s,), generator=g, device=device)
        x = torch.randn((e - s, dim), generator=g, device=device, dtype=torch.float32)
        yield s, means[c].add_(x, alpha=sigma)


def lowrank_mixture(workload: int, dim: int, n_comp: int, rank: int = 16,
                    mean_std: float = 2.0):
    """Means m_c ~ N(0, mean_std^2 I) and loadings W_c (dim x rank, entries
    N(0, 1/rank)) of a mixture whose component c draws m_c + W_c z + noise e,
    z ~ N(0, I_rank), e ~ N(0, I_dim): most of each component's spread lies
    in a rank-dimensional subspace, as in learned embeddings, with about
    unit variance per coordinate."""
    means = rng(workload, ROLE_MEANS).standard_normal((n_comp, dim)) * mean_std
    w = rng(workload, ROLE_SHAPE).standard_normal((n_comp, dim, rank)) / math.sqrt(rank)
    return means, w


def lowrank_device_chunks(torch, workload: int, n_base: int, dim: int, n_comp: int,
                          rank: int = 16, noise: float = 0.1, first: int = 0,
                          chunk: int = 1 << 22, sub: int = 1 << 16, device: str = "cuda"):
    """Base points of lowrank_mixture drawn on the device, in the block scheme
    of gmm_float_device_chunks (block i keyed by (workload, i))."""
    if first % chunk:
        raise ValueError("first must be a multiple of chunk")
    means, w = lowrank_mixture(workload, dim, n_comp, rank)
    means = torch.from_numpy(means).to(device=device, dtype=torch.float32)
    w = torch.from_numpy(w).to(device=device, dtype=torch.float32)
    for s in range(first, first + n_base, chunk):
        e = min(first + n_base, s + chunk)
        g = torch.Generator(device=device)
        g.manual_seed((1000 * workload + ROLE_BASE) * (1 << 24) + s // chunk)
        c = torch.randint(0, n_comp, (e - s,), generator=g, device=device)
        z = torch.randn((e - s, rank, 1), generator=g, device=device, dtype=torch.float32)
        x = torch.randn((e - s, dim), generator=g, device=device, dtype=torch.float32).mul_(noise)
        x += means[c]
        for o in range(0, e - s, sub):
            x[o:o + sub] += torch.bmm(w[c[o:o + sub]], z[o:o + sub]).squeeze(-1)
        yield s, x


def lowrank_points(workload: int, role: int, n: int, dim: int, n_comp: int, rank: int = 16,
                   noise: float = 0.1, comp_p=None, chunk: int = 8192):
    """n points of lowrank_mixture on the host and their components (uniform,
    or comp_p), from the stream of `role`."""
    means, w = lowrank_mixture(workload, dim, n_comp, rank)
    g = rng(workload, role)
    out = np.empty((n, dim), dtype=np.float32)
    comps = np.empty(n, dtype=np.int32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        c = g.choice(n_comp, size=e - s, p=comp_p) if comp_p is not None else g.integers(0, n_comp, e - s)
        z = g.standard_normal((e - s, rank))
        x = means[c] + np.einsum("nij,nj->ni", w[c], z) + noise * g.standard_normal((e - s, dim))
        out[s:e] = x.astype(np.float32)
        comps[s:e] = c
    return out, comps


def lowrank_queries(workload: int, n_query: int, dim: int, n_comp: int, rank: int = 16,
                    noise: float = 0.1, query_zipf: float | None = 1.2, chunk: int = 8192):
    """Queries of lowrank_mixture on the host, components Zipf(query_zipf)."""
    qp = None if query_zipf is None else zipf_weights(n_comp, query_zipf, rng(workload, ROLE_CLUSTER))
    return lowrank_points(workload, ROLE_QUERIES, n_query, dim, n_comp, rank, noise, qp, chunk)[0]


# ----------------------------------------------------------------------------
# Streaming workload families (operation sequences only).  Each returns a list
# of steps (insert ids, delete ids) over rows 0..n-1 of a dataset, and the
# first step at which evaluation starts.
# ----------------------------------------------------------------------------
def sliding_window_ops(n: int, t_max: int = 200):
    """n rows in t_max equal segments; step t inserts segment t and, from
    step t_max / 2 on, deletes the segment inserted t_max / 2 steps earlier;
    evaluation starts at step t_max / 2 + 1 (counting from 1)."""
    seg = np.array_split(np.arange(n, dtype=np.int32), t_max)
    half = t_max // 2
    ops = []
    for t in range(t_max):
        dele = seg[t - half] if t >= half else np.empty(0, np.int32)
        ops.append((seg[t], dele))
    return ops, half


def expiration_time_ops(workload: int, n: int, t_max: int = 200, lifetimes=(10, 50, 100),
                        ratio=(10, 2, 1)):
    """Each step inserts the next n / t_max rows; a row lives for 10, 50 or
    100 steps (drawn 10 : 2 : 1) and is deleted at the step its lifetime
    ends; evaluation starts once the longest lifetime has passed once."""
    g = rng(workload, ROLE_STREAM)
    p = np.asarray(ratio, np.float64) / np.sum(ratio)
    life = np.asarray(lifetimes)[g.choice(len(lifetimes), size=n, p=p)]
    seg = np.array_split(np.arange(n, dtype=np.int32), t_max)
    born = np.empty(n, np.int64)
    for t, sg in enumerate(seg):
        born[sg] = t
    death = born + life
    ops = []
    for t in range(t_max):
        ops.append((seg[t], np.nonzero(death == t)[0].astype(np.int32)))
    return ops, max(lifetimes)


def clustered_ops(workload: int, comps, n_clusters: int, rounds: int = 5):
    """Spatially correlated updates over clusters of rows (comps[i] is row i's
    cluster): each round inserts a fresh 1/rounds of every cluster, one
    cluster per step in a seeded order, then deletes a random half of every
    cluster's live rows, one cluster per step; evaluation starts after the
    first round's insertions."""
    g = rng(workload, ROLE_STREAM)
    parts = []
    for c in range(n_clusters):
        rows_c = np.nonzero(comps == c)[0].astype(np.int32)
        g.shuffle(rows_c)
        parts.append(np.array_split(rows_c, rounds))
    live = [np.empty(0, np.int32) for _ in range(n_clusters)]
    ops = []
    none = np.empty(0, np.int32)
    for r in range(rounds):
        for c in g.permutation(n_clusters):
            ops.append((parts[c][r], none))
            live[c] = np.concatenate([live[c], parts[c][r]])
        for c in g.permutation(n_clusters):
            k = len(live[c]) // 2
            pick = g.permutation(len(live[c]))
            ops.append((none, np.sort(live[c][pick[:k]])))
            live[c] = np.sort(live[c][pick[k:]])
    return ops, n_clusters


# ----------------------------------------------------------------------------
# Workload 1: 16-component mixture, dim 128, float values, L2.
# ----------------------------------------------------------------------------
def gmm_float(workload: int, n_base: int, n_query: int, dim: int, n_comp: int,
              mean_std: float = 2.0, sigma: float = 1.0, normalise: bool = False,
              query_zipf: float | None = None):
    """Means ~ N(0, mean_std^2 I); points m_c + sigma N(0, I); optional unit norm."""
    means = rng(workload, ROLE_MEANS).standard_normal((n_comp, dim)) * mean_std
    base, _ = _chunked_mixture(rng(workload, ROLE_BASE), means, n_base, sigma)
    qp = None
    if query_zipf is not None:
        qp = zipf_weights(n_comp, query_zipf, rng(workload, ROLE_CLUSTER))
    queries, _ = _chunked_mixture(rng(workload, ROLE_QUERIES), means, n_query, sigma, qp)
    if normalise:
        base /= np.linalg.norm(base, axis=1, keepdims=True).astype(np.float32)
        queries /= np.linalg.norm(queries, axis=1, keepdims=True).astype(np.float32)
    return np.ascontiguousarray(base), np.ascontiguousarray(queries)


def gmm_uint8_valued(workload: int, n_base: int, n_query: int, dim: int, n_comp: int,
                     mean_mu: float = 128.0, mean_std: float = 32.0, sigma: float = 16.0):
    """Integer-valued mixture: means ~ N(128, 32^2) per dim, sigma 16, rint, clip [0,255].

    Stored as float32; every value is an integer in 0..255.
    """
    means = mean_mu + mean_std * rng(workload, ROLE_MEANS).standard_normal((n_comp, dim))
    base, _ = _chunked_mixture(rng(workload, ROLE_BASE), means, n_base, sigma)
    queries, _ = _chunked_mixture(rng(workload, ROLE_QUERIES), means, n_query, sigma)
    for a in (base, queries):
        np.rint(a, out=a)
        np.clip(a, 0, 255, out=a)
    return np.ascontiguousarray(base), np.ascontiguousarray(queries)


# Integers whose eightfold lies on the FP8 E4M3 grid: 0..16, even 18..32,
# multiples of 4 from 36 to 56.
FP8_EXACT_LEVELS = np.array(list(range(0, 17)) + list(range(18, 33, 2)) + list(range(36, 57, 4)),
                            dtype=np.float32)


def gmm_fp8_exact_valued(workload: int, n_base: int, n_query: int, dim: int, n_comp: int):
    """The integer-valued mixture mapped onto FP8_EXACT_LEVELS (each value v in
    0..255 goes to the level nearest 56 v / 255), with coordinate 0 set to 56
    in every row, so each row's largest magnitude is 56."""
    out = []
    for a in gmm_uint8_valued(workload, n_base, n_query, dim, n_comp):
        t = a * np.float32(56.0 / 255.0)
        idx = np.searchsorted(FP8_EXACT_LEVELS, t)
        idx = np.clip(idx, 1, len(FP8_EXACT_LEVELS) - 1)
        lo, hi = FP8_EXACT_LEVELS[idx - 1], FP8_EXACT_LEVELS[idx]
        v = np.where(t - lo <= hi - t, lo, hi).astype(np.float32)
        v[:, 0] = 56.0
        out.append(np.ascontiguousarray(v))
    return out[0], out[1]


def training_queries_uint8(workload: int, n: int, dim: int, n_comp: int,
                           mean_mu: float = 128.0, mean_std: float = 32.0, sigma: float = 16.0):
    means = mean_mu + mean_std * rng(workload, ROLE_MEANS).standard_normal((n_comp, dim))
    q, _ = _chunked_mixture(rng(workload, ROLE_TRAIN), means, n, sigma)
    np.rint(q, out=q)
    np.clip(q, 0, 255, out=q)
    return np.ascontiguousarray(q)


# Named workloads ----------------------------------------------------------------
def workload_small_float(n_base=10_000, n_query=100):
    """10k x 128 float mixture (16 comps), 100 queries, L2, degree 32, k 10, beam 64."""
    return gmm_float(1, n_base, n_query, 128, 16)


def workload_1m_int(n_base=1_000_000, n_query=10_000):
    """1M x 128 integer-valued mixture (256 comps), 10k queries, L2, degree 64."""
    return gmm_uint8_valued(2, n_base, n_query, 128, 256)


def workload_stream_ip(n_base, n_query, query_zipf=1.1):
    """Unit-norm 96-d mixture (1024 comps) for the inner-product streaming mix."""
    return gmm_float(3, n_base, n_query, 96, 1024, normalise=True, query_zipf=query_zipf)


@dataclass
class Request:
    kind: str          # "search" | "insert" | "delete"
    size: int
    arrival_s: float


def request_stream(n_rounds: int, insert_batch: int, delete_batch: int,
                   queries_per_round: int, max_query: int, rate_hz: float,
                   workload: int = 3):
    """Open-loop request stream: per round one insert, one delete and
    ``queries_per_round`` query batches with log-uniform sizes in [1, max_query],
    Poisson arrivals at ``rate_hz`` requests per second."""
    g = rng(workload, ROLE_STREAM)
    reqs = []
    t = 0.0
    for _ in range(n_rounds):
        kinds = ["insert", "delete"] + ["search"] * queries_per_round
        order = g.permutation(len(kinds))
        for i in order:
            t += g.exponential(1.0 / rate_hz)
            kind = kinds[i]
            if kind == "insert":
                size = insert_batch
            elif kind == "delete":
                size = delete_batch
            else:
                size = int(math.floor(math.exp(g.uniform(0.0, math.log(max_query)))))
                size = max(1, min(max_query, size))
            reqs.append(Request(kind, size, t))
    return reqs


# ----------------------------------------------------------------------------
# Large imported graphs: integer points along a folded random walk, with rows
# that mix walk neighbours and uniform long links.
# ----------------------------------------------------------------------------
def walk_graph_uint8(workload: int, n: int, dim: int, R: int, n_query: int, step: int = 3,
                     window: int | None = None):
    """Points x_i: a random walk in Z^dim with steps uniform in [-step, step],
    folded into 0..255 (reflection at 0 and 255), so ids close in order lie
    close in space.  Row i: R/2 ids at offsets +-1, +-2, ... (mod n) and R - R/2
    distinct uniform ids (no self, no repeats).  Queries: walk points of
    uniform ids plus integer noise in [-4, 4], clipped to 0..255.  Every value
    is an integer, stored FP32.  Returns base, rows (n x R int32), queries."""
    g = rng(workload, ROLE_BASE)
    walk = np.cumsum(g.integers(-step, step + 1, size=(n, dim), dtype=np.int64), axis=0)
    walk += 128
    walk %= 510
    base = np.where(walk > 255, 510 - walk, walk).astype(np.float32)
    half = R // 2
    offs = np.array([s * (j // 2 + 1) for j, s in zip(range(half), [1, -1] * half)], np.int64)
    ids = np.arange(n, dtype=np.int64)
    rows = np.empty((n, R), np.int64)
    rows[:, :half] = (ids[:, None] + offs[None, :]) % n
    gr = rng(workload, ROLE_SHAPE)
    far = gr.integers(0, n, size=(n, R - half), dtype=np.int64)
    while True:
        rows[:, half:] = far
        srt = np.sort(rows, axis=1)
        bad = (np.diff(srt, axis=1) == 0).any(axis=1) | (rows == ids[:, None]).any(axis=1)
        nb = int(bad.sum())
        if nb == 0:
            break
        far[bad] = gr.integers(0, n, size=(nb, R - half), dtype=np.int64)
    gq = rng(workload, ROLE_QUERIES)
    pick = gq.integers(0, n, size=n_query)
    q = base[pick] + gq.integers(-4, 5, size=(n_query, dim)).astype(np.float32)
    np.clip(q, 0, 255, out=q)
    return np.ascontiguousarray(base), rows.astype(np.int32), np.ascontiguousarray(q)
