#!/usr/bin/env python3
"""Throughput of batched graph search on one MI355X.

Workload (synthetic, seeded): 1,000,000 base vectors of dimension 128 with
integer values 0..255 stored as FP32 (a 256-component clipped, rounded
Gaussian mixture), squared-L2 metric, graph degree 64 built on the GPU by the
insertion rule, 10,000 queries from the same mixture, k = 10.

A step is one search of the whole 10k-query batch with the plain FP32 form
at the smallest beam reaching recall@10 >= 0.95 (tie-aware, against exact
ground truth): the sweep 32, 48, 64, 96, ... finds the first beam at the
target, then bisection on multiples of 8 between it and the beam before.  Inputs are resident in HBM before timing; HIP
events on the launch stream bracket the timed steps.  The same JSON line
reports the reduced-precision forms (BF16 or FP8-E4M3 traversal + exact FP32
re-scoring, with their distance errors against FP64), the chosen form
(reduced precision + the learned entry/stop predictor),
the insertion (build) and deletion throughput of the update path, the
roofline of the search kernel, the same search on a 5M x 96 index whose
vectors are far larger than the Infinity Cache, the serving mix and the CPU
oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "queries/sec at recall@10\u22650.95 (batch 10k), plain vs chosen form; p50/p99 mixed"
DIM, DEGREE, K = 128, 64, 10
BEAMS = [32, 48, 64, 96, 128, 192, 256, 384, 512]

# Beyond-L2 traffic of one timed search launch (FP32, beam 88, this workload), from
# two rocprofv3 counter passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean
# of the steady dispatches).  Each counter is scaled by what it reads for a 1 GiB
# device-to-device copy in the same process (FETCH_SIZE reads 524,300 KiB there,
# WRITE_SIZE 1,048,576).  The figure describes the kernel built from the sources
# whose hash is recorded; any edit to them makes it stale and it is reported as null.
COUNTED = {"sources": ("common.hpp", "wave_ops.hpp", "search.hip"),
           "sha256_16": "2edd73c46cd52efd", "beam": 88,
           "fetch_kib": 9004520.1, "fetch_scale": 1048576.0 / 524300.0,
           "write_kib": 2516.0, "write_scale": 1.0}


def counted_traffic(beam):
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2601_08528_amd", "csrc")
    h = hashlib.sha256()
    for f in COUNTED["sources"]:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != COUNTED["sha256_16"] or beam != COUNTED["beam"]:
        return None
    return round((COUNTED["fetch_kib"] * COUNTED["fetch_scale"]
                  + COUNTED["write_kib"] * COUNTED["write_scale"]) * 1024.0)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def exact_kth(torch, base_t, q_t, k, extra=64, chunk=1024):
    """Exact k-th nearest squared-L2 distance per query: FP32 GEMM screening
    of all base vectors, then FP64 re-evaluation of the best k+extra."""
    out = torch.empty(q_t.shape[0], dtype=torch.float64, device=q_t.device)
    bn = (base_t.double() ** 2).sum(1).float()
    for s in range(0, q_t.shape[0], chunk):
        q = q_t[s:s + chunk]
        d = (q * q).sum(1, keepdim=True) + bn[None, :] - 2.0 * (q @ base_t.T)
        cand = torch.topk(d, k + extra, dim=1, largest=False).indices
        ex = ((base_t[cand].double() - q[:, None, :].double()) ** 2).sum(-1)
        out[s:s + chunk] = torch.sort(ex, dim=1).values[:, k - 1]
    return out


def recall(torch, base_t, q_t, ids_t, kth):
    valid = ids_t >= 0
    safe = torch.where(valid, ids_t, torch.zeros_like(ids_t)).long()
    ex = ((base_t[safe].double() - q_t[:, None, :].double()) ** 2).sum(-1)
    hit = valid & (ex <= kth[:, None])
    return hit.double().mean().item()


def dist_errors(torch, base_t, q_t, bufs):
    """Largest absolute and relative error of the returned distances against
    FP64 distances of the same ids."""
    ids, d = bufs[0], bufs[1]
    ok = ids >= 0
    safe = torch.where(ok, ids, torch.zeros_like(ids)).long()
    ex = ((base_t[safe].double() - q_t[:, None, :].double()) ** 2).sum(-1)
    err = (d.double() - ex).abs()[ok]
    rel = err / ex[ok].clamp_min(1e-30)
    return {"max_abs": float(err.max()), "max_rel": float(rel.max())}


def run_search(torch, ix, q_t, beam, bufs):
    ids, d, nd, ne = bufs
    st = torch.cuda.current_stream()
    ix.search_dev(q_t.data_ptr(), q_t.shape[0], K, beam, ids.data_ptr(), d.data_ptr(),
                  nd.data_ptr(), ne.data_ptr(), st.cuda_stream)


def timed_steps(torch, ix, q_t, beam, bufs, steps, warmup):
    for _ in range(warmup):
        run_search(torch, ix, q_t, beam, bufs)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        run_search(torch, ix, q_t, beam, bufs)
        e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    return ms, wall


def sweep(torch, ix, q_t, base_t, kth, bufs, beams, target=0.95, refine=8):
    """Smallest beam reaching `target` recall: the first of `beams` that
    does, then bisection on multiples of `refine` between it and the beam
    before it.  Returns (beam or None, rows sorted by beam)."""
    rows = []

    def probe(beam):
        run_search(torch, ix, q_t, beam, bufs)
        torch.cuda.synchronize()
        r = recall(torch, base_t, q_t, bufs[0], kth)
        ms, _ = timed_steps(torch, ix, q_t, beam, bufs, 3, 0)
        rows.append({"beam": beam, "recall@10": round(r, 5), "ms": round(float(np.median(ms)), 3),
                     "qps": round(q_t.shape[0] / (np.median(ms) / 1e3), 1)})
        log("beam", beam, "recall", round(r, 4), "ms", round(float(np.median(ms)), 3))
        return r

    chosen, below = None, None
    for beam in beams:
        if probe(beam) >= target:
            chosen = beam
            break
        below = beam
    if chosen is not None and below is not None and refine:
        lo, hi = below, chosen
        while hi - lo > refine:
            mid = (lo + hi) // 2 // refine * refine
            if mid <= lo:
                break
            if probe(mid) >= target:
                hi = mid
            else:
                lo = mid
        chosen = hi
    rows.sort(key=lambda r: r["beam"])
    return chosen, rows


def serving_bench(torch, svf, datagen, n_build=5_000_000, rounds=(167, 167, 166),
                  rates=(60.0, 240.0, 480.0), consolidation_rate=240.0, consolidation_rounds=60,
                  consolidate_frac=0.004, recall_sample=1000, beams=(64, 96, 128, 192, 256, 320, 384)):
    """Streaming mix on the serving loop: an n_build-vector unit-norm 96-d
    mixture (1024 components, inner product, degree 48, BF16 traversal + FP32
    re-score), then, at each offered load in turn, rounds[i] rounds of [one
    10k-vector insert, one 1k-id delete of uniformly chosen live ids, four
    query batches of log-uniform size 1..10k with Zipf(1.1)-skewed
    components] as open-loop Poisson arrivals; 500 rounds take the index from
    5M to 10M vectors.  The index keeps changing from one load to the next.
    Then the recall of a query sample on the final index, and two more phases
    at one load with a consolidation threshold low enough that
    consolidations happen inside the phase: synchronous, then in the
    background on a snapshot."""
    n_extra = (sum(rounds) + 2 * consolidation_rounds) * 10_000
    base, queries = datagen.workload_stream_ip(n_build + n_extra, 20_000)
    ix = svf.Index(96, 48, svf.METRIC_IP, seed=0, precision=svf.PREC_BF16)
    ix.set_option("capacity", n_build + n_extra)
    t0 = time.perf_counter()
    ix.build(base[:n_build])
    build_s = time.perf_counter() - t0
    # the serving beam: the smallest of a sweep whose recall@10 on a query
    # sample reaches 0.95 on the built index
    kth, alive = stream_kth(torch, ix, base[:n_build], queries[:recall_sample])
    beam, beam_sweep = beams[-1], []
    for b in beams:
        ids, _ = ix.search(queries[:recall_sample], 10, b)
        r = stream_recall_of(torch, ids, base[:n_build], queries[:recall_sample], kth, alive)
        beam_sweep.append({"beam": b, "recall@10": round(r, 4)})
        log("serving: beam %d recall@10 %.4f at %d vectors" % (b, r, n_build))
        if r >= 0.95:
            beam = b
            break
    del kth, alive
    g = np.random.Generator(np.random.Philox(31))
    victims = g.permutation(n_build).astype(np.int32)
    ix.serve_start(streams=4, max_batch=16384)
    pos_ins, pos_del, pos_q = n_build, 0, 0
    loads = []
    phases = [(r, n, None) for r, n in zip(rates, rounds)] + \
             [(consolidation_rate, consolidation_rounds, 0), (consolidation_rate, consolidation_rounds, 1)]
    rec_after = None
    for rate_hz, n_rounds, async_mode in phases:
        if async_mode is not None:
            ix.serve_stop()
            ix.consolidate_wait()
            if rec_after is None:
                rec_after = stream_recall(torch, ix, base[:pos_ins], queries[:recall_sample], beam)
                log("serving: recall@10 %.4f on %d queries at %d vectors"
                    % (rec_after, recall_sample, pos_ins))
            ix.set_option("consolidate_frac", consolidate_frac)
            ix.set_option("consolidate_async", async_mode)
            ix.serve_start(streams=4, max_batch=16384)
        reqs = datagen.request_stream(n_rounds, 10_000, 1_000, 4, 10_000, rate_hz)
        cons0 = ix.stats()["consolidations"]
        tickets = []
        keep = []
        t_start = time.perf_counter()
        for r in reqs:
            now = time.perf_counter() - t_start
            if r.arrival_s > now:
                time.sleep(r.arrival_s - now)
            if r.kind == "insert":
                t, ids = ix.submit_insert(base[pos_ins:pos_ins + r.size])
                pos_ins += r.size
                keep.append(ids)
            elif r.kind == "delete":
                t = ix.submit_delete(victims[pos_del:pos_del + r.size])
                pos_del += r.size
            else:
                idx = (pos_q + np.arange(r.size)) % queries.shape[0]
                pos_q += r.size
                t, ids, d = ix.submit_search(queries[idx], 10, beam)
                keep.append((ids, d))
            tickets.append((t, r.kind, r.size))
        infos = [(kind, size, ix.wait(t, 300.0)) for t, kind, size in tickets]
        wall = time.perf_counter() - t_start
        out = {"offered_req_per_s": rate_hz, "rounds": n_rounds, "requests": len(reqs),
               "wall_s": round(wall, 3), "vectors_after": pos_ins}
        if async_mode is not None:
            out["consolidation"] = ("background on a snapshot" if async_mode else "synchronous") + \
                " (consolidate_frac %g)" % consolidate_frac
        out["consolidations_done"] = int(ix.stats()["consolidations"] - cons0)
        nq = sum(size for kind, size, _ in infos if kind == "search")
        out["qps"] = round(nq / wall, 1)
        for kind in ("search", "insert", "delete"):
            lat = np.array([inf["total_ms"] for k, _, inf in infos if k == kind])
            if lat.size:
                out[kind] = {"n": int(lat.size), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat, 99)), 3),
                             "mean_ms": round(float(lat.mean()), 3)}
        out["max_batch_queries"] = int(max(inf["batch_queries"] for _, _, inf in infos))
        log("serving load %g req/s: %d vectors, %.0f QPS, search p50 %.2f p99 %.2f ms"
            % (rate_hz, pos_ins, out["qps"], out["search"]["p50_ms"], out["search"]["p99_ms"]))
        loads.append(out)
    ix.serve_stop()
    ix.consolidate_wait()
    ix.close()
    del base
    cols = ["offered_req_per_s", "qps", "search_p50_ms", "search_p99_ms", "insert_p50_ms",
            "insert_p99_ms", "delete_p50_ms", "delete_p99_ms"]
    rows = [[L["offered_req_per_s"], L["qps"]] +
            [L[k][q] if k in L else None for k in ("search", "insert", "delete")
             for q in ("p50_ms", "p99_ms")] for L in loads[:len(rates)]]
    headline = {"build": n_build, "after": n_build + sum(rounds) * 10_000, "beam": beam,
                "recall@10_build": beam_sweep[-1]["recall@10"],
                "recall@10": None if rec_after is None else round(rec_after, 4),
                "cols": cols, "loads": rows}
    return {"workload": "%dM x 96 unit-norm GMM (1024 comps, Zipf(1.1) queries), IP, degree 48, "
                        "BF16 + FP32 re-score, k=10, beam %d (the smallest of a sweep reaching "
                        "recall@10 0.95 after the build); %d rounds of insert 10k / delete 1k / "
                        "4 query batches 1..10k over %d loads, Poisson arrivals"
                        % (n_build // 1_000_000, beam, sum(rounds), len(rates)),
            "build_s": round(build_s, 2), "beam_sweep": beam_sweep,
            "recall@10_after_stream": rec_after,
            "headline": headline, "loads": loads}


def stream_kth(torch, ix, vecs, q):
    """Exact 10th-largest inner product of each query over the live vectors
    of the index (FP64), and the alive flags."""
    _, _, alive = ix.export_graph()
    live = np.flatnonzero(alive[:vecs.shape[0]])
    q_t = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    best = torch.full((q.shape[0], 10), -float("inf"), device="cuda", dtype=torch.float64)
    chunk = 1 << 18
    for c0 in range(0, live.size, chunk):
        sel = live[c0:c0 + chunk]
        b = torch.from_numpy(np.ascontiguousarray(vecs[sel])).cuda()
        s = (q_t.double() @ b.double().T)
        top = torch.topk(s, min(10, s.shape[1]), dim=1).values
        best = torch.topk(torch.cat([best, top], dim=1), 10, dim=1).values
        del b, s
    return best[:, 9], alive


def stream_recall_of(torch, ids, vecs, q, kth, alive):
    """Tie-aware recall@10 of result ids against the exact 10th product."""
    q_t = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    got = np.where(ids >= 0, ids, 0)
    g_t = torch.from_numpy(np.ascontiguousarray(vecs[got.ravel()].reshape(got.shape + (-1,)))).cuda()
    prod = (g_t.double() * q_t.double()[:, None, :]).sum(-1)
    # kth comes from an FP64 GEMM, prod from an element-wise sum: the two may
    # round the same product apart in the last bits
    ok = (prod >= kth[:, None] - 1e-12) & torch.from_numpy(ids >= 0).cuda()
    alive_t = torch.from_numpy(alive[got.ravel()].reshape(got.shape).astype(bool)).cuda()
    ok &= alive_t
    return float(ok.double().sum().item() / (10 * q.shape[0]))


def stream_recall(torch, ix, vecs, q, beam):
    """Tie-aware recall@10 of a search (k=10) over the live vectors of the
    index, against an exact inner-product top-10."""
    kth, alive = stream_kth(torch, ix, vecs, q)
    ids, _ = ix.search(q, 10, beam)
    return stream_recall_of(torch, ids, vecs, q, kth, alive)


def small_batch_bench(torch, ix, q_t, base_t, kth, beam, reps=30):
    """Latency of small batches (1..1024 queries) of the plain FP32 search at
    one beam: one parent per iteration, four parents with one wave per query,
    and four parents with one wave per parent (the waves of a query sharing
    its pool).  Recall@10 over the batch's queries."""
    out = []
    for nb in (1, 16, 128, 1024):
        qb = q_t[:nb]
        bufs = (torch.empty((nb, K), dtype=torch.int32, device="cuda"),
                torch.empty((nb, K), dtype=torch.float32, device="cuda"),
                torch.empty(nb, dtype=torch.int32, device="cuda"),
                torch.empty(nb, dtype=torch.int32, device="cuda"))
        row = {"batch": nb}
        for name, width, coop in (("w1", 1, 0), ("w4_one_wave", 4, 0), ("w4_wave_per_parent", 4, 1 << 20)):
            ix.set_option("search_width", width)
            ix.set_option("coop_max_batch", coop)
            ms, _ = timed_steps(torch, ix, qb, beam, bufs, reps, 3)
            rec = recall(torch, base_t, qb, bufs[0], kth[:nb])
            row[name] = {"ms": round(float(np.median(ms)), 4), "recall@10": round(rec, 4),
                         "n_exp_per_query": round(float(bufs[3].double().mean()), 1)}
        out.append(row)
    ix.set_option("search_width", 1)
    ix.set_option("coop_max_batch", 1024)
    return {"workload": "1M x 128 integer-valued GMM, L2, degree 64, plain FP32, beam %d" % beam,
            "batches": out}


def exact_kth_ip(torch, base_t, q_t, k, extra=64, chunk=64):
    """Exact k-th smallest -<q,x> per query: FP32 GEMM screening of all base
    vectors, then FP64 re-evaluation of the best k+extra."""
    out = torch.empty(q_t.shape[0], dtype=torch.float64, device=q_t.device)
    for s in range(0, q_t.shape[0], chunk):
        q = q_t[s:s + chunk]
        cand = torch.topk(q @ base_t.T, k + extra, dim=1, largest=True).indices
        ex = -(base_t[cand].double() * q[:, None, :].double()).sum(-1)
        out[s:s + chunk] = torch.sort(ex, dim=1).values[:, k - 1]
    return out


def big_int_bench(torch, svf, datagen, n_base, steps, warmup, sample=1000):
    """The 1M integer-valued workload's shape at n_base vectors (128-d,
    256 components, L2, degree 64; 10k-query batch, k = 10), far larger than
    the 256 MB Infinity Cache: plain FP32 at the smallest beam reaching
    recall@10 >= 0.95 on a `sample`-query subsample."""
    dim, R = 128, 64
    base, queries = datagen.gmm_uint8_valued(2, n_base, 10_000, dim, 256)
    ix = svf.Index(dim, R, svf.METRIC_L2, seed=0)
    t0 = time.perf_counter()
    ix.build(base)
    build_s = time.perf_counter() - t0
    base_t = torch.from_numpy(base).cuda()
    q_t = torch.from_numpy(queries).cuda()
    del base
    nq = q_t.shape[0]
    kth = exact_kth(torch, base_t, q_t[:sample], K, chunk=128)
    bufs = (torch.empty((nq, K), dtype=torch.int32, device="cuda"),
            torch.empty((nq, K), dtype=torch.float32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"))
    rows, beam = [], None
    for b in BEAMS:
        run_search(torch, ix, q_t, b, bufs)
        torch.cuda.synchronize()
        r = recall(torch, base_t, q_t[:sample], bufs[0][:sample], kth)
        rows.append({"beam": b, "recall@10_sample": round(r, 5)})
        log("10M beam", b, "recall", round(r, 4))
        if r >= 0.95:
            beam = b
            break
    beam = beam or BEAMS[-1]
    ms, _ = timed_steps(torch, ix, q_t, beam, bufs, steps, warmup)
    n_exp = int(bufs[3].sum().item())
    slots = ix.get_option("visited_slots")
    ix.set_option("visited_slots", 16384)
    run_search(torch, ix, q_t, beam, bufs)
    torch.cuda.synchronize()
    n_dist = int(bufs[2].sum().item())
    ix.set_option("visited_slots", slots)
    ix.close()
    alg = n_dist * dim * 4 + n_exp * R * 4
    ms_step = float(np.mean(ms))
    achieved = alg / (ms_step / 1e3) / 1e9
    del base_t
    return {"workload": "%dM x 128 integer-valued GMM (256 comps), L2, degree 64, 10k-query batch, "
                        "k=10, plain FP32; recall on a %d-query sample" % (n_base // 1_000_000, sample),
            "vector_bytes": n_base * dim * 4, "build_s": round(build_s, 2),
            "beam": beam, "recall@10_sample": rows[-1]["recall@10_sample"], "sweep": rows,
            "ms_per_step": round(ms_step, 4), "qps": round(nq / (ms_step / 1e3), 1),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "alg_bytes_per_launch": alg,
                         "n_dist_per_query": round(n_dist / nq, 1),
                         "n_exp_per_query": round(n_exp / nq, 1)}}


def large_bench(torch, svf, datagen, n_base, steps, warmup):
    """Plain FP32 search on an index whose vectors are far larger than the
    256 MB Infinity Cache: n_base x 96 unit-norm mixture (1024 components,
    Zipf(1.1)-skewed queries), inner product, degree 48, 10k-query batch,
    k = 10, at the smallest beam reaching recall@10 >= 0.95."""
    dim, R = 96, 48
    base, queries = datagen.workload_stream_ip(n_base, 10_000)
    ix = svf.Index(dim, R, svf.METRIC_IP, seed=0)
    t0 = time.perf_counter()
    ix.build(base)
    build_s = time.perf_counter() - t0
    base_t = torch.from_numpy(base).cuda()
    q_t = torch.from_numpy(queries).cuda()
    del base
    nq = q_t.shape[0]
    kth = exact_kth_ip(torch, base_t, q_t, K)
    bufs = (torch.empty((nq, K), dtype=torch.int32, device="cuda"),
            torch.empty((nq, K), dtype=torch.float32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"))

    def rec_ip():
        ids = bufs[0]
        ok = ids >= 0
        safe = torch.where(ok, ids, torch.zeros_like(ids)).long()
        ex = -(base_t[safe].double() * q_t[:, None, :].double()).sum(-1)
        return (ok & (ex <= kth[:, None])).double().mean().item()

    rows, beam = [], None
    for b in BEAMS:
        run_search(torch, ix, q_t, b, bufs)
        torch.cuda.synchronize()
        r = rec_ip()
        rows.append({"beam": b, "recall@10": round(r, 5)})
        if r >= 0.95:
            beam = b
            break
    beam = beam or BEAMS[-1]
    ms, _ = timed_steps(torch, ix, q_t, beam, bufs, steps, warmup)
    n_exp = int(bufs[3].sum().item())
    slots = ix.get_option("visited_slots")
    ix.set_option("visited_slots", 16384)
    run_search(torch, ix, q_t, beam, bufs)
    torch.cuda.synchronize()
    n_dist = int(bufs[2].sum().item())
    ix.set_option("visited_slots", slots)
    alg = n_dist * dim * 4 + n_exp * R * 4
    ms_step = float(np.mean(ms))
    achieved = alg / (ms_step / 1e3) / 1e9
    # The same search expanding four parents per iteration: each iteration
    # then gathers four rows' unvisited neighbours at once, where one parent
    # leaves about 18 new vectors per iteration to carry its fixed costs.
    ix.set_option("search_width", 4)
    rows4, beam4 = [], None
    for b in BEAMS:
        run_search(torch, ix, q_t, b, bufs)
        torch.cuda.synchronize()
        r = rec_ip()
        rows4.append({"beam": b, "recall@10": round(r, 5)})
        if r >= 0.95:
            beam4 = b
            break
    beam4 = beam4 or BEAMS[-1]
    ms4, _ = timed_steps(torch, ix, q_t, beam4, bufs, steps, warmup)
    ms4 = float(np.mean(ms4))
    ix.set_option("search_width", 1)
    del base_t
    return {"workload": "%dM x 96 unit-norm GMM (1024 comps, Zipf(1.1) queries), IP, degree 48, "
                        "10k-query batch, k=10, plain FP32" % (n_base // 1_000_000),
            "width4": {"beam": beam4, "recall@10": rows4[-1]["recall@10"], "sweep": rows4,
                       "ms_per_step": round(ms4, 4), "qps": round(nq / (ms4 / 1e3), 1),
                       "speedup_vs_width1": round(ms_step / ms4, 3)},
            "vector_bytes": n_base * dim * 4, "build_s": round(build_s, 2),
            "beam": beam, "recall@10": rows[-1]["recall@10"], "sweep": rows,
            "ms_per_step": round(ms_step, 4), "qps": round(nq / (ms_step / 1e3), 1),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "alg_bytes_per_launch": alg,
                         "n_dist_per_query": round(n_dist / nq, 1),
                         "n_exp_per_query": round(n_exp / nq, 1)}}


def tier_bench(torch, svf, datagen, n_base, rounds=20, cache_frac=0.25):
    """Tiered store (X4) on a scaled version of the paper's largest workload:
    n_base x 128 mixture of 4096 components, L2, degree 32, batches of 10k
    queries whose components follow Zipf(1.2).  The index is built in HBM
    and searched untiered; then its FP32 vectors move to pinned host memory
    behind an HBM cache of cache_frac of them (warmed by in-degree).  Two
    phases of `rounds` fresh batches follow: FP32 traversal through the
    cache, then FP8 traversal (codes in HBM) with only the exact FP32
    re-scoring going through the cache.  After every batch the workload-aware
    placement updates the cache."""
    dim, R, nq = 128, 32, 10_000
    base, queries = datagen.gmm_float(5, n_base, (2 * rounds + 1) * nq, dim, 4096, query_zipf=1.2)
    ix = svf.Index(dim, R, svf.METRIC_L2, seed=0)
    t0 = time.perf_counter()
    ix.build(base)
    build_s = time.perf_counter() - t0
    bufs = (torch.empty((nq, K), dtype=torch.int32, device="cuda"),
            torch.empty((nq, K), dtype=torch.float32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"))
    q0 = torch.from_numpy(queries[:nq]).cuda()
    base_t = torch.from_numpy(base).cuda()
    del base

    def rec1k(qs):
        kth = exact_kth(torch, base_t, qs, K, chunk=128)
        ids = bufs[0][:qs.shape[0]].long()
        ex = ((base_t[ids].double() - qs[:, None, :].double()) ** 2).sum(-1)
        return (ex <= kth[:, None]).double().mean().item()

    def pick_beam():
        # smallest beam of the sweep reaching recall@10 >= 0.95 (1k-query sample)
        rows = []
        for b in BEAMS:
            run_search(torch, ix, q0, b, bufs)
            torch.cuda.synchronize()
            r = rec1k(q0[:1000])
            rows.append({"beam": b, "recall@10_1k": round(r, 4)})
            if r >= 0.95:
                return b, rows
        return BEAMS[-1], rows

    def run_rounds(beam, first):
        out = []
        for r in range(first, first + rounds):
            qr = torch.from_numpy(queries[r * nq:(r + 1) * nq]).cuda()
            s0 = ix.stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_search(torch, ix, qr, beam, bufs)
            torch.cuda.synchronize()
            wall_ms = (time.perf_counter() - t0) * 1e3
            s1 = ix.stats()
            h = s1["cache_gather_hits"] - s0["cache_gather_hits"]
            m = s1["cache_gather_misses"] - s0["cache_gather_misses"]
            kms = s1["last_search_ms"]
            out.append({"round": r, "kernel_ms": round(kms, 3), "call_ms": round(wall_ms, 3),
                        "gather_hit_rate": round(h / max(h + m, 1), 4),
                        "host_link_gbs": round(m * dim * 4 / (kms / 1e3) / 1e9, 1),
                        "placed": s1["cache_last_placed"]})
        steady = out[-10:]
        kms = float(np.mean([x["kernel_ms"] for x in steady]))
        cms = float(np.mean([x["call_ms"] for x in steady]))
        return {"beam": beam, "steady_kernel_ms": round(kms, 3), "steady_call_ms": round(cms, 3),
                "steady_qps_kernel": round(nq / (kms / 1e3), 1),
                "steady_qps_with_placement": round(nq / (cms / 1e3), 1),
                "steady_gather_hit_rate":
                    round(float(np.mean([x["gather_hit_rate"] for x in steady])), 4),
                "recall@10_last_batch_1k": round(rec1k(qr[:1000]), 4), "rounds": out}

    beam, sweep_rows = pick_beam()
    ms_hbm, _ = timed_steps(torch, ix, q0, beam, bufs, 5, 1)
    ref_ids = bufs[0].clone()
    cache_bytes = int(cache_frac * n_base) * dim * 4
    ix.set_option("cache_bytes", cache_bytes)
    run_search(torch, ix, q0, beam, bufs)
    torch.cuda.synchronize()
    same = bool(torch.equal(bufs[0], ref_ids))
    fp32 = run_rounds(beam, 1)
    # Alg. 1's co-processing: uncached neighbours' distances on the host
    # cores, cached ones on the GPU, round by round (results unchanged)
    ix.set_option("cache_cpu_miss", 1)
    calib = ix.cache_calibrate()
    r0 = ix.get_option("cache_cpu_rounds")
    cpu = run_rounds(beam, 1)
    cpu["rounds_per_batch"] = round((ix.get_option("cache_cpu_rounds") - r0) / rounds, 1)
    cpu["theta_from_measured_costs"] = calib
    ix.set_option("cache_cpu_miss", 0)
    # the threshold for the miss path in force from here on (GPU reads over the link)
    calib_gpu = ix.cache_calibrate()
    ix.set_option("precision", svf.PREC_FP8)
    beam8, sweep8 = pick_beam()
    fp8 = run_rounds(beam8, rounds + 1)
    fp8["beam_sweep"] = sweep8
    fp8["theta_from_measured_costs"] = calib_gpu
    del base_t
    return {"workload": "%dM x 128 GMM (4096 comps, Zipf(1.2) queries), L2, degree 32, "
                        "10k-query batches, k=10; cache of %d%% of the FP32 vectors in HBM, the "
                        "rest in pinned host memory" % (n_base // 1_000_000, round(cache_frac * 100)),
            "build_s": round(build_s, 2), "cache_bytes": cache_bytes, "beam_sweep": sweep_rows,
            "untiered_fp32": {"beam": beam, "ms_per_batch": round(float(np.mean(ms_hbm)), 4),
                              "qps": round(nq / (float(np.mean(ms_hbm)) / 1e3), 1)},
            "tiered_same_results_as_untiered": same,
            "tiered_fp32_traversal": fp32,
            "tiered_fp32_cpu_miss": cpu,
            "tiered_fp8_traversal_fp32_rescore": fp8}


def stream_exact_topk(torch, blocks, q, k, extra=64, sub=1 << 19):
    """Exact nearest (k + extra) ids and FP64 squared-L2 distances of the
    queries q over the base rows that `blocks` yields as (start row, rows)
    on the device: an FP32 GEMM screen per sub-block, then FP64
    re-evaluation of the screen's best k + extra."""
    nq = q.shape[0]
    m = k + extra
    best_d = torch.full((nq, m), float("inf"), dtype=torch.float64, device=q.device)
    best_i = torch.full((nq, m), -1, dtype=torch.int64, device=q.device)
    qn = (q * q).sum(1, keepdim=True)
    qd = q.double()
    for s0, x in blocks:
        for o in range(0, x.shape[0], sub):
            xs = x[o:o + sub]
            d = qn + (xs * xs).sum(1)[None, :] - 2.0 * (q @ xs.T)
            c = torch.topk(d, min(m, xs.shape[0]), dim=1, largest=False).indices
            ex = ((xs[c].double() - qd[:, None, :]) ** 2).sum(-1)
            dd = torch.cat([best_d, ex], 1)
            ii = torch.cat([best_i, c + (s0 + o)], 1)
            top = torch.topk(dd, m, dim=1, largest=False)
            best_d, best_i = top.values, torch.gather(ii, 1, top.indices)
    order = torch.argsort(best_d, dim=1)
    return torch.gather(best_i, 1, order), torch.gather(best_d, 1, order)


def full_tier_bench(torch, svf, datagen, n_base, cache_gb=None, steps=8, sample=1000,
                    beam_insert=256):
    """The tiered workload at its own size: n_base x 128 mixture of 4096
    components whose spread lies mostly in 16 dimensions each (a stand-in for
    learned embeddings; see datagen.lowrank_mixture), L2, degree 32,
    100k-vector insert batches, insertion beam beam_insert, built in HBM,
    then FP8-E4M3 traversal codes in HBM with the FP32 vectors moved to
    pinned host memory behind a cache of cache_gb.  Queries: 10k batches with
    Zipf(1.2) components.  Reports the build, an HBM-resident baseline, the
    tiered search (FP32 re-scoring through the cache) and a stream of
    insert-then-search steps.  The cache defaults to 32 GB per 200M vectors."""
    W, dim, R, nq, ins_b, ncomp = 5, 128, 32, 10_000, 100_000, 4096
    if cache_gb is None:
        cache_gb = 32.0 * n_base / 200e6
    chunk = 1 << 22
    ix = svf.Index(dim, R, svf.METRIC_L2, seed=0, insert_batch_max=ins_b, beam_insert=beam_insert)
    ix.set_option("capacity", n_base + steps * ins_b)
    t0 = time.perf_counter()
    for s0, x in datagen.lowrank_device_chunks(torch, W, n_base, dim, ncomp, chunk=chunk):
        ix.insert_dev(x.data_ptr(), x.shape[0], stream=torch.cuda.current_stream().cuda_stream)
        if (s0 // chunk) % 8 == 7 or s0 + x.shape[0] == n_base:
            log("full tier: built %d vectors in %.0f s" % (s0 + x.shape[0], time.perf_counter() - t0))
    build_s = time.perf_counter() - t0
    del x
    queries = datagen.lowrank_queries(W, (steps + 1) * nq, dim, ncomp, query_zipf=1.2)
    q0 = torch.from_numpy(queries[:nq]).cuda()
    t1 = time.perf_counter()
    gt_i, gt_d = stream_exact_topk(
        torch, datagen.lowrank_device_chunks(torch, W, n_base, dim, ncomp, chunk=chunk), q0[:sample], K)
    torch.cuda.synchronize()
    gt_s = time.perf_counter() - t1
    kth = gt_d[:, K - 1]
    log("full tier: exact top-%d of %d queries in %.0f s" % (K, sample, gt_s))
    bufs = (torch.empty((nq, K), dtype=torch.int32, device="cuda"),
            torch.empty((nq, K), dtype=torch.float32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"))

    def rec():
        ids = bufs[0][:sample].long()
        hit = (ids[:, :, None] == gt_i[:, None, :]) & (gt_d[:, None, :] <= kth[:, None, None])
        return hit.any(-1).double().mean().item()

    def pick(beams):
        rows = []
        for b in beams:
            run_search(torch, ix, q0, b, bufs)
            torch.cuda.synchronize()
            r = rec()
            ms, _ = timed_steps(torch, ix, q0, b, bufs, 3, 0)
            st = ix.stats()
            rows.append({"beam": b, "recall@10_sample": round(r, 4), "ms": round(float(np.median(ms)), 3),
                         "n_dist_per_query": round(st["last_n_dist"] / nq, 1),
                         "n_exp_per_query": round(st["last_n_exp"] / nq, 1)})
            log("full tier: beam %d recall %.4f %.2f ms" % (b, r, rows[-1]["ms"]))
            if r >= 0.95:
                return b, rows
        return beams[-1], rows

    beam32, sweep32 = pick((64, 96, 128, 192, 256, 384, 512, 768, 1024))
    fp32_row = sweep32[-1]
    ix.set_option("precision", svf.PREC_FP8)
    beam8, sweep8 = pick((64, 96, 128, 192, 256, 384, 512, 768, 1024))
    run_search(torch, ix, q0, beam8, bufs)
    torch.cuda.synchronize()
    ref_ids = bufs[0].clone()
    out = {"workload": "%dM x 128 mixture of 4096 rank-16 components + 0.1 noise (Zipf(1.2) "
                       "queries), L2, degree 32, insertion beam %d, 10k-query batches, k=10, "
                       "100k-vector insert batches; FP8-E4M3 traversal codes in HBM, FP32 vectors "
                       "in pinned host memory behind a %.1f GB HBM cache"
                       % (n_base // 1_000_000, beam_insert, cache_gb),
           "build_s": round(build_s, 1), "build_vectors_per_s": round(n_base / build_s, 1),
           "exact_topk_sample_s": round(gt_s, 1), "recall_sample_queries": sample,
           "hbm_fp32": {"beam": beam32, "ms_per_batch": fp32_row["ms"],
                        "qps": round(nq / (fp32_row["ms"] / 1e3), 1), "sweep": sweep32},
           "hbm_fp8_rescore": {"beam": beam8, "ms_per_batch": sweep8[-1]["ms"],
                               "qps": round(nq / (sweep8[-1]["ms"] / 1e3), 1), "sweep": sweep8}}
    t2 = time.perf_counter()
    try:
        ix.set_option("cache_bytes", cache_gb * 1e9)
    except svf.SvfError as e:
        # the FP32 store goes to pinned host segments; hosts cap pinned memory in all
        out["tiered"] = "not set up: %s" % e
        log("full tier: %s" % e)
        ix.close()
        return out
    tier_s = time.perf_counter() - t2
    log("full tier: FP32 store moved to host memory, cache warmed, in %.0f s" % tier_s)
    run_search(torch, ix, q0, beam8, bufs)
    torch.cuda.synchronize()
    same = bool(torch.equal(bufs[0], ref_ids))
    rows = []
    gen = datagen.lowrank_device_chunks(torch, W, steps * ins_b, dim, ncomp, first=n_base, chunk=ins_b)
    for r in range(steps):
        _, xb = next(gen)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ix.insert_dev(xb.data_ptr(), xb.shape[0], stream=torch.cuda.current_stream().cuda_stream)
        tb = time.perf_counter()
        qr = torch.from_numpy(queries[(r + 1) * nq:(r + 2) * nq]).cuda()
        s0 = ix.stats()
        torch.cuda.synchronize()
        tc = time.perf_counter()
        run_search(torch, ix, qr, beam8, bufs)
        torch.cuda.synchronize()
        td = time.perf_counter()
        s1 = ix.stats()
        h = s1["cache_gather_hits"] - s0["cache_gather_hits"]
        m = s1["cache_gather_misses"] - s0["cache_gather_misses"]
        kms = s1["last_search_ms"]
        rows.append({"step": r, "insert_100k_ms": round((tb - ta) * 1e3, 1),
                     "search_kernel_ms": round(kms, 3), "search_call_ms": round((td - tc) * 1e3, 2),
                     "gather_hit_rate": round(h / max(h + m, 1), 4),
                     "host_link_gbs": round(m * dim * 4 / (kms / 1e3) / 1e9, 1),
                     # the placement's phases on the host (count waits for the kernel)
                     **{k: round(s1[k], 2) for k in ("place_count_ms", "place_indeg_ms",
                                                     "place_walk_ms", "place_evict_ms",
                                                     "place_apply_ms")}})
        log("full tier: step", rows[-1])
    st = rows[steps // 2:]
    kms = float(np.mean([x["search_kernel_ms"] for x in st]))
    cms = float(np.mean([x["search_call_ms"] for x in st]))
    ims = float(np.mean([x["insert_100k_ms"] for x in st]))
    sd = ix.stats()
    out.update({
           "tier_setup_s": round(tier_s, 1), "cache_slots": sd["cache_slots"],
           "device_bytes": sd["device_bytes"],
           "tiered_same_results_as_hbm": same,
           "tiered_stream": {"steady_search_kernel_ms": round(kms, 3),
                             "steady_search_call_ms": round(cms, 2),
                             "steady_qps_kernel": round(nq / (kms / 1e3), 1),
                             "steady_qps_with_placement": round(nq / (cms / 1e3), 1),
                             "steady_insert_100k_ms": round(ims, 1),
                             "steady_gather_hit_rate":
                                 round(float(np.mean([x["gather_hit_rate"] for x in st])), 4),
                             "steps": rows}})
    ix.close()
    return out


def workloads_bench(torch, svf, datagen, n=1_000_000, beam=64, nq=2000, evals=10):
    """Streaming workload families of the paper (SlidingWindow, ExpirationTime,
    Clustered; datagen's operation sequences) over n x 128 rows of a 64-component
    low-rank mixture, L2, degree 32, under the three deletion strategies the
    paper compares: lazy deletion alone, with global consolidation at 20%, and
    with localized repair as well (the method).  Recall@10 of nq queries at
    `evals` evenly spaced steps, against the exact top-10 of the live rows;
    insert and delete times are summed over the whole sequence.  Also the
    share of alive vertices by share of deleted neighbours after a lazy 10%
    deletion."""
    W, dim, R, ncomp = 8, 128, 32, 64
    base, comps = datagen.lowrank_points(W, datagen.ROLE_BASE, n, dim, ncomp)
    queries = datagen.lowrank_queries(W, nq, dim, ncomp, query_zipf=None)
    base_t = torch.from_numpy(base).cuda()
    q_t = torch.from_numpy(queries).cuda()
    bufs = (torch.empty((nq, K), dtype=torch.int32, device="cuda"),
            torch.empty((nq, K), dtype=torch.float32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"))
    # Clustered fills empty regions one cluster at a time; insert batches do
    # not see their batch-mates, so they are kept small there (500 rows).
    fams = {"sliding_window": (datagen.sliding_window_ops(n), 10_000),
            "expiration_time": (datagen.expiration_time_ops(W, n), 10_000),
            "clustered": (datagen.clustered_ops(W, comps, ncomp), 500)}
    modes = {"lazy": dict(localized_repair=0, consolidate_frac=0.0),
             "lazy+consolidation": dict(localized_repair=0, consolidate_frac=0.2),
             "lazy+consolidation+localized_repair": dict(localized_repair=1, consolidate_frac=0.2)}
    out = {"workload": "%dk x 128 mixture of 64 rank-16 components, L2, degree 32, beam %d, "
                       "%d uniform queries per evaluation" % (n // 1000, beam, nq), "families": {}}
    for fam, ((ops, first), ibm) in fams.items():
        at = set(np.linspace(first, len(ops) - 1, evals).round().astype(int).tolist())
        res = {}
        for mname, mopts in modes.items():
            ix = svf.Index(dim, R, svf.METRIC_L2, seed=0, insert_batch_max=ibm, **mopts)
            id2row = np.full(n, -1, np.int64)
            row2id = np.full(n, -1, np.int64)
            alive = np.zeros(n, bool)
            t_ins = t_del = 0.0
            recs, sms = [], []
            for t, (ins, dele) in enumerate(ops):
                if len(ins):
                    t0 = time.perf_counter()
                    ids = ix.insert(base[ins])
                    t_ins += time.perf_counter() - t0
                    id2row[ids] = ins
                    row2id[ins] = ids
                    alive[ins] = True
                if len(dele):
                    t0 = time.perf_counter()
                    ix.delete(row2id[dele].astype(np.int32))
                    t_del += time.perf_counter() - t0
                    alive[dele] = False
                if t in at:
                    live = torch.from_numpy(np.nonzero(alive)[0]).cuda()
                    kth = exact_kth(torch, base_t[live], q_t, K, chunk=256)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    run_search(torch, ix, q_t, beam, bufs)
                    torch.cuda.synchronize()
                    sms.append((time.perf_counter() - t0) * 1e3)
                    ids = bufs[0].long()
                    rows = torch.from_numpy(id2row).cuda()[ids.clamp_min(0)]
                    ex = ((base_t[rows].double() - q_t[:, None, :].double()) ** 2).sum(-1)
                    hit = (ids >= 0) & (ex <= kth[:, None])
                    recs.append(hit.double().mean().item())
            ix.close()
            res[mname] = {"mean_recall@10": round(float(np.mean(recs)), 4),
                          "min_recall@10": round(float(np.min(recs)), 4),
                          "insert_s": round(t_ins, 3), "delete_s": round(t_del, 3),
                          "search_ms_%d_queries" % nq: round(float(np.mean(sms)), 3)}
            log("workloads %s %s: recall %.4f, delete %.2f s, insert %.2f s"
                % (fam, mname, res[mname]["mean_recall@10"], t_del, t_ins))
        out["families"][fam] = {"steps": len(ops), "insert_batch_max": ibm,
                                "evaluated_steps": sorted(at), "modes": res}
    # deleted-neighbour shares after deleting 10% of the vertices lazily
    ix = svf.Index(dim, R, svf.METRIC_L2, seed=0, localized_repair=0, consolidate_frac=0.0)
    ix.build(base)
    g = np.random.Generator(np.random.Philox(11))
    gone = g.choice(n, n // 10, replace=False).astype(np.int32)
    ix.delete(gone)
    rows, _, al = ix.export_graph()
    ix.close()
    al = al.astype(bool)
    valid = rows >= 0
    dead = valid & ~al[np.where(valid, rows, 0)]
    share = dead.sum(1) / np.maximum(valid.sum(1), 1)
    share = share[al]
    out["deleted_neighbour_share_after_10pct"] = {
        "below_10pct": round(float((share < 0.1).mean()), 4),
        "10_to_40pct": round(float(((share >= 0.1) & (share < 0.4)).mean()), 4),
        "40pct_or_more": round(float((share >= 0.4).mean()), 4),
        "above_half_(repaired_by_localized_repair)": round(float((share > 0.5).mean()), 5)}
    del base_t
    return out


def policy_bench(torch, svf, datagen, n_total=2_000_000, steps=12, measured=8, beam=64,
                 ratios=(0.2, 0.4, 0.6, 0.8, 1.0), cpu_ratios=(0.2, 0.6, 1.0)):
    """Replacement-policy ablation under a sliding window on the tiered store.
    n_total x 128 mixture of 4096 components (L2, degree 32) in 200 equal
    segments; the index starts from the first 100 (built once, then imported
    into a fresh index per setting).  Each step inserts the next segment,
    deletes the oldest live one and searches a batch of 10k queries whose
    components follow Zipf(1.2), FP32 traversal through the cache.  For each
    share of the live vectors held in HBM and each policy (workload-aware
    placement, LRU, LFU, LRFU, none) the last `measured` steps are reported."""
    dim, R, nq, nseg = 128, 32, 10_000, 200
    seg = n_total // nseg
    win = nseg // 2
    base, queries = datagen.gmm_float(6, n_total, steps * nq, dim, 4096, query_zipf=1.2)
    ix = svf.Index(dim, R, svf.METRIC_L2, seed=0)
    t0 = time.perf_counter()
    ix.build(base[:win * seg])
    build_s = time.perf_counter() - t0
    rows, ed, alive = ix.export_graph()
    ix.close()
    bufs = (torch.empty((nq, K), dtype=torch.int32, device="cuda"),
            torch.empty((nq, K), dtype=torch.float32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"))
    qs = [torch.from_numpy(queries[r * nq:(r + 1) * nq]).cuda() for r in range(steps)]
    out = []
    settings = [(r, 0) for r in ratios] + [(r, 1) for r in cpu_ratios]
    for ratio, cpu_miss in settings:
        for name, pol, pmax in (("wavp", 0, 2048), ("lru", 1, 2048), ("lfu", 2, 2048),
                                ("lrfu", 3, 2048), ("none", 0, 0)):
            g = svf.Index(dim, R, svf.METRIC_L2, seed=0)
            g.import_graph(base[:win * seg], rows, ed, alive)
            g.set_option("cache_policy", pol)
            g.set_option("cache_promote_max", pmax)
            g.set_option("cache_cpu_miss", cpu_miss)
            g.set_option("cache_bytes", int(ratio * win * seg) * dim * 4)
            res = []
            for st in range(steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.insert(base[(win + st) * seg:(win + st + 1) * seg])
                g.delete(np.arange(st * seg, (st + 1) * seg, dtype=np.int32))
                t1 = time.perf_counter()
                s0 = g.stats()
                run_search(torch, g, qs[st], beam, bufs)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                s1 = g.stats()
                h = s1["cache_gather_hits"] - s0["cache_gather_hits"]
                m = s1["cache_gather_misses"] - s0["cache_gather_misses"]
                res.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3, s1["last_search_ms"], h / max(h + m, 1)))
            g.close()
            st_ = res[steps - measured:]
            upd = float(np.mean([x[0] for x in st_]))
            srch = float(np.mean([x[1] for x in st_]))
            out.append({"cache_share": ratio, "policy": name,
                        "miss_path": "host cores (co-processing)" if cpu_miss else "GPU over the host link",
                        "gather_hit_rate": round(float(np.mean([x[3] for x in st_])), 4),
                        "update_ms": round(upd, 3), "search_call_ms": round(srch, 3),
                        "search_kernel_ms": round(float(np.mean([x[2] for x in st_])), 3),
                        "step_ms": round(upd + srch, 3),
                        "updates_per_s": round(2 * seg / (upd / 1e3), 1),
                        "queries_per_s": round(nq / (srch / 1e3), 1)})
            log("policy %s share %.1f%s: hit %.3f, update %.1f ms, search %.1f ms"
                % (name, ratio, " cpu-miss" if cpu_miss else "", out[-1]["gather_hit_rate"], upd, srch))
    return {"workload": "sliding window over %dM x 128 GMM (4096 comps) in %d segments of %d, "
                        "%d live; per step insert one segment, delete the oldest, search 10k "
                        "queries (Zipf(1.2) comps), L2, degree 32, k=10, beam %d, FP32 traversal "
                        "through the cache, misses read by the GPU over the host link or (at "
                        "shares %s) computed on the host cores; cache share of the live vectors; "
                        "%d steps, the last %d averaged"
                        % (n_total // 1_000_000, nseg, seg, win * seg, beam, list(cpu_ratios), steps,
                           measured),
            "build_s": round(build_s, 2), "settings": out}


def cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def cpu_baseline(ix, base, queries, beam, gpu_ids, n_single=500):
    """The FP64 oracle, as it stands, on the GPU-built graph of this workload
    (exported through the C ABI and imported into the oracle): all queries of
    the batch at the plain form's beam on every host core, and a sample on
    one core.  Its ids are compared with the GPU's (integer-valued data:
    every distance is exact on both sides)."""
    import oracle as O
    ncore = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    rows, ed, alive = ix.export_graph()
    oix = O.OracleIndex(DIM, DEGREE, O.L2, seed=0)
    oix.import_state(base, rows, ed.astype(np.float64), alive)
    del rows, ed
    nq = queries.shape[0]
    t0 = time.perf_counter()
    oi, _, _ = oix.search(queries, K, beam, threads=ncore)
    ts = time.perf_counter() - t0
    t0 = time.perf_counter()
    oix.search(queries[:n_single], K, beam, threads=1)
    t1 = time.perf_counter() - t0
    same = float(np.mean(np.all(oi == gpu_ids, axis=1)))
    del oix
    return {"value": round(nq / ts, 1), "unit": "queries/s", "cores": ncore, "kind": "oracle",
            "sample": "FP64 oracle, all %d queries at beam %d on the GPU-built %d-vector graph, "
                      "%d threads (%s)" % (nq, beam, base.shape[0], ncore, cpu_info() or "cpu"),
            "single_core_qps": round(n_single / t1, 1), "wall_s": round(ts, 2),
            "query_ids_equal_gpu": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-base", type=int, default=1_000_000)
    ap.add_argument("--n-query", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large-footprint (5M x 96) search leg")
    ap.add_argument("--large-n", type=int, default=5_000_000)
    ap.add_argument("--big-n", type=int, default=10_000_000,
                    help="size of the integer-valued leg beside the large-footprint one")
    ap.add_argument("--no-tier", action="store_true", help="skip the tiered-store leg")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the workload-family / deletion-strategy ablation")
    ap.add_argument("--no-policies", action="store_true",
                    help="skip the replacement-policy and memory-share ablation")
    ap.add_argument("--tier-n", type=int, default=4_000_000)
    ap.add_argument("--full-tier", type=int, default=0, metavar="N",
                    help="also run the tiered workload at N base vectors (200M is its own size; "
                         "takes minutes and about 110 GB of pinned host memory)")
    ap.add_argument("--full-tier-beam-insert", type=int, default=256,
                    help="insertion beam of the --full-tier build (256 reaches recall@10 0.95 at "
                         "200M with degree 32; 128 builds twice as fast)")
    ap.add_argument("--search-only", type=int, default=0, metavar="BEAM",
                    help="build, then only time the plain FP32 search at this beam (for "
                         "hardware counter runs); prints a short JSON line")
    ap.add_argument("--insert-only", type=int, default=0, metavar="K",
                    help="build, then only run K insert batches of 10k vectors and print their "
                         "median phase times (for kernel traces and hardware counter runs)")
    ap.add_argument("--search-precision", choices=("fp32", "bf16", "fp8"), default="fp32",
                    help="traversal precision of --search-only (re-scored in FP32)")
    ap.add_argument("--fp8-row-scales", type=int, choices=(-1, 0, 1), default=-1,
                    help="FP8 scales beside the graph rows for --search-only (-1: the library's "
                         "choice by size)")
    ap.add_argument("--detail", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file that receives every leg's figures (sweeps, ablations, serving); "
                         "stdout's last line is the headline")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device three times (a reference "
                         "kernel of known traffic for hardware counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(each GPU would hold an independent shard; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_08528_amd as svf
    from paper_2601_08528_amd import datagen

    torch.cuda.set_device(0)
    # a dedicated stream: the search kernels and the timing events share it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log("generating workload")
    base, queries = datagen.workload_1m_int(args.n_base, args.n_query)
    ix = svf.Index(DIM, DEGREE, svf.METRIC_L2, seed=0)
    log("building graph on the GPU")
    t0 = time.perf_counter()
    ix.build(base)
    build_s = time.perf_counter() - t0
    log("build %.2f s" % build_s)

    if args.insert_only:
        extra, _ = datagen.gmm_uint8_valued(2, 10_000 * args.insert_only, 1, DIM, 256)
        keys = ("ins_search_ms", "ins_prune_ms", "ins_reverse_ms", "ins_commit_ms")
        ph, wall = {k: [] for k in keys}, []
        for i in range(args.insert_only):
            t0 = time.perf_counter()
            ix.insert(extra[i * 10_000:(i + 1) * 10_000])
            wall.append((time.perf_counter() - t0) * 1e3)
            st = ix.stats()
            for k in keys:
                ph[k].append(st[k])
        print(json.dumps({"insert_batches": args.insert_only, "batch": 10_000,
                          "wall_ms": round(float(np.median(wall)), 3),
                          **{k: round(float(np.median(v)), 3) for k, v in ph.items()},
                          "long_lists_total": int(ix.stats()["long_lists"])}), flush=True)
        return
    base_t = torch.from_numpy(base).cuda()
    q_t = torch.from_numpy(queries).cuda()
    nq = q_t.shape[0]
    bufs = (torch.empty((nq, K), dtype=torch.int32, device="cuda"),
            torch.empty((nq, K), dtype=torch.float32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"),
            torch.empty(nq, dtype=torch.int32, device="cuda"))
    if args.search_only:
        prec = {"fp32": svf.PREC_FP32, "bf16": svf.PREC_BF16, "fp8": svf.PREC_FP8}[args.search_precision]
        ix.set_option("precision", prec)
        ix.set_option("fp8_row_scales", args.fp8_row_scales)
        ms, _ = timed_steps(torch, ix, q_t, args.search_only, bufs, args.steps, args.warmup)
        n_dist = int(bufs[2].sum().item())
        n_exp = int(bufs[3].sum().item())
        per = {"fp32": DIM * 4, "bf16": DIM * 2, "fp8": DIM + 4}[args.search_precision]
        rescore = 0 if prec == svf.PREC_FP32 else nq * args.search_only * DIM * 4
        print(json.dumps({"beam": args.search_only, "precision": args.search_precision,
                          "fp8_row_scales": int(ix.get_option("fp8_row_scales_on")),
                          "ms_per_step": round(float(np.mean(ms)), 4),
                          "n_dist": n_dist, "n_exp": n_exp,
                          "alg_bytes": n_dist * per + n_exp * DEGREE * 4 + rescore}), flush=True)
        return
    kth = exact_kth(torch, base_t, q_t, K)
    torch.cuda.synchronize()

    # plain FP32 form
    beam, rows = sweep(torch, ix, q_t, base_t, kth, bufs, BEAMS)
    if beam is None:
        beam = BEAMS[-1]
    ms, wall = timed_steps(torch, ix, q_t, beam, bufs, args.steps, args.warmup)
    rec = recall(torch, base_t, q_t, bufs[0], kth)
    gpu_ids = bufs[0].cpu().numpy()
    n_dist_run = int(bufs[2].sum().item())
    n_exp = int(bufs[3].sum().item())
    # algorithmic bytes: count distance evaluations with the largest visited
    # table (results are identical; it re-evaluates the fewest vectors)
    slots = ix.get_option("visited_slots")
    ix.set_option("visited_slots", 16384)
    run_search(torch, ix, q_t, beam, bufs)
    torch.cuda.synchronize()
    n_dist = int(bufs[2].sum().item())
    ix.set_option("visited_slots", slots)
    alg_bytes = n_dist * DIM * 4 + n_exp * DEGREE * 4
    ms_step = float(np.mean(ms))
    achieved = alg_bytes / (ms_step / 1e3) / 1e9
    qps = nq / (ms_step / 1e3)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": counted_traffic(beam), "traffic_unit": "bytes/launch",
            "kernel": "search_kernel<float,1>",
            "alg_bytes_per_launch": alg_bytes,
            "n_dist_per_query": round(n_dist / nq, 1),
            "n_dist_per_query_timed": round(n_dist_run / nq, 1),
            "n_exp_per_query": round(n_exp / nq, 1)}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the GPU-built graph")
        cpu = cpu_baseline(ix, base, queries[:nq], beam, gpu_ids)
        log("oracle %.0f queries/s on %d threads, ids equal to the GPU's for %.4f of queries"
            % (cpu["value"], cpu["cores"], cpu["query_ids_equal_gpu"]))
    # the same batch through svf_search with host buffers (copies included)
    q_host = queries[:nq]
    ix.search(q_host, K, beam)
    e2e = []
    for _ in range(5):
        t0 = time.perf_counter()
        ix.search(q_host, K, beam)
        e2e.append((time.perf_counter() - t0) * 1e3)
    e2e_ms = float(np.median(e2e))
    log("small batches")
    small = small_batch_bench(torch, ix, q_t, base_t, kth, beam)

    # reduced-precision forms: BF16 or FP8 traversal + exact FP32 re-score
    lowp = {}
    for name, prec in (("bf16", svf.PREC_BF16), ("fp8", svf.PREC_FP8)):
        ix.set_option("precision", prec)
        b, rws = sweep(torch, ix, q_t, base_t, kth, bufs, BEAMS)
        bb = b or BEAMS[-1]
        ms_p, _ = timed_steps(torch, ix, q_t, bb, bufs, 5, 1)
        err_post = dist_errors(torch, base_t, q_t, bufs)
        ix.set_option("rerank", 0)
        run_search(torch, ix, q_t, bb, bufs)
        torch.cuda.synchronize()
        err_pre = dist_errors(torch, base_t, q_t, bufs)
        ix.set_option("rerank", 1)
        lowp[name] = {"beam": b, "ms_per_step": round(float(np.mean(ms_p)), 4),
                      "value": round(nq / (float(np.mean(ms_p)) / 1e3), 1),
                      "dist_err_vs_fp64": {"pre_rerank": err_pre, "post_rerank": err_post},
                      "sweep": rws}
    ix.set_option("precision", svf.PREC_FP32)

    # chosen form: reduced precision + the learned entry/stop predictor,
    # trained on the GPU from traces of plain search.  The predictor's head
    # is 64 entry clusters + 1 stop output; a 256-cluster head is measured
    # beside it.  Queries whose softmax confidence is below model_conf fall
    # back to plain search; thresholds 0 and 0.3 are both tried.
    train = datagen.training_queries_uint8(2, 200_000, DIM, 256)
    slots0 = int(ix.get_option("visited_slots"))

    def chosen(n_clusters, grid, entries=1):
        ix.set_option("model_entries", entries)
        t0 = time.perf_counter()
        loss = ix.model_fit(train, K, 64, n_clusters=n_clusters, epochs=12)
        fit = time.perf_counter() - t0
        ix.set_option("use_model", 1)
        best, tried = None, []
        for pname, prec, slots, width, stop_scale, conf in grid:
            ix.set_option("precision", prec)
            ix.set_option("visited_slots", slots)
            ix.set_option("search_width", width)
            ix.set_option("model_stop_scale", stop_scale)
            ix.set_option("model_conf", conf)
            b, rws = sweep(torch, ix, q_t, base_t, kth, bufs, [32, 48, 64, 96, 128])
            tried.append({"precision": pname, "visited_slots": slots, "search_width": width,
                          "stop_scale": stop_scale, "model_conf": conf, "beam": b, "sweep": rws})
            if b is not None:
                ms_b = [r["ms"] for r in rws if r["beam"] == b][0]
                if best is None or ms_b < best[0]:
                    best = (ms_b, pname, prec, slots, width, stop_scale, conf, b)
        if best is None:
            best = (None, "bf16", svf.PREC_BF16, slots0, 1, 1e6, 0.0, BEAMS[-1])
        _, pname, prec, slots, width, stop_scale, conf, b = best
        for k_, v_ in (("precision", prec), ("visited_slots", slots), ("search_width", width),
                       ("model_stop_scale", stop_scale), ("model_conf", conf)):
            ix.set_option(k_, v_)
        ms_b, _ = timed_steps(torch, ix, q_t, b, bufs, args.steps, args.warmup)
        fallback = ix.stats()["last_model_fallback"] / nq
        rec_b = recall(torch, base_t, q_t, bufs[0], kth)
        err = dist_errors(torch, base_t, q_t, bufs)["max_abs"]
        ix.set_option("use_model", 0)
        ix.set_option("search_width", 1)
        ix.set_option("visited_slots", slots0)
        ix.set_option("model_conf", 0.5)
        ix.set_option("precision", svf.PREC_FP32)
        ms_m = float(np.mean(ms_b))
        return {"form": "%s traversal + FP32 re-score + learned entry clusters and stop cap "
                        "(MLP 128-256-256-%d, BF16, trained on the GPU; entry lists %s)"
                        % (pname.upper(), n_clusters + 1,
                           "spread over each cluster" if entries else "nearest to each centroid"),
                "model_entries": entries,
                "precision": pname, "beam": b, "search_width": width, "model_stop_scale": stop_scale,
                "model_conf": conf, "fallback_share": round(fallback, 4), "visited_slots": slots,
                "recall@10": round(rec_b, 5), "value": round(nq / (ms_m / 1e3), 1),
                "ms_per_step": round(ms_m, 4), "speedup_vs_plain": round(ms_step / ms_m, 3),
                "max_abs_dist_err_vs_fp64": err, "model_fit_s": round(fit, 2),
                "model_fit_loss": round(loss, 4), "training_queries": train.shape[0],
                "n_clusters": n_clusters, "configs_tried": tried}

    grid = [(pn, pr, 2048, w, ss, cf)
            for pn, pr in (("bf16", svf.PREC_BF16), ("fp8", svf.PREC_FP8))
            for w, ss in ((1, 1e6), (2, 1e6), (2, 1.5), (1, 2.0))
            for cf in (0.0, 0.3)]
    chosen64 = chosen(64, grid)
    c = chosen64
    grid_best = [(c["precision"], {"bf16": svf.PREC_BF16, "fp8": svf.PREC_FP8}[c["precision"]],
                  c["visited_slots"], c["search_width"], c["model_stop_scale"], cf)
                 for cf in (0.0, 0.3)]
    chosen64_nearest = chosen(64, grid_best, entries=0)
    chosen256 = chosen(256, grid_best)

    # update path: delete 1% then insert 10k fresh vectors (one batch each)
    g = np.random.Generator(np.random.Philox(77))
    victims = g.choice(args.n_base, 10_000, replace=False).astype(np.int32)
    t0 = time.perf_counter()
    ix.delete(victims)
    del_s = time.perf_counter() - t0
    extra, _ = datagen.gmm_uint8_valued(2, 10_000, 1, DIM, 256)
    t0 = time.perf_counter()
    ix.insert(extra)
    ins_s = time.perf_counter() - t0
    st = ix.stats()

    large = None
    if not args.no_large:
        log("large-footprint search leg")
        del base_t
        ix.close()
        torch.cuda.empty_cache()
        large = large_bench(torch, svf, datagen, args.large_n, args.steps, args.warmup)
        torch.cuda.empty_cache()
        log("10M integer-valued search leg")
        large["integer_10m"] = big_int_bench(torch, svf, datagen, args.big_n, args.steps, args.warmup)

    tier = None
    if not args.no_tier:
        log("tiered-store leg")
        torch.cuda.empty_cache()
        tier = tier_bench(torch, svf, datagen, args.tier_n)

    full_tier = None
    if args.full_tier > 0:
        log("full-size tiered workload")
        torch.cuda.empty_cache()
        full_tier = full_tier_bench(torch, svf, datagen, args.full_tier,
                                    beam_insert=args.full_tier_beam_insert)

    workloads = None
    if not args.no_workloads:
        log("workload families and deletion strategies")
        torch.cuda.empty_cache()
        workloads = workloads_bench(torch, svf, datagen)

    policies = None
    if not args.no_policies:
        log("replacement policies")
        torch.cuda.empty_cache()
        policies = policy_bench(torch, svf, datagen)

    serving = None
    if not args.no_serving:
        log("serving mix")
        torch.cuda.empty_cache()
        serving = serving_bench(torch, svf, datagen)

    detail = {
        "config": {"workload": "1M x 128 integer-valued GMM (256 comps), L2, degree 64, "
                               "10k-query batch, k=10",
                   "n_base": args.n_base, "n_query": nq, "dim": DIM, "degree": DEGREE, "k": K,
                   "beam": beam, "recall@10": round(rec, 5)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "chosen_form": chosen64,
        "chosen_form_64_nearest_entries": chosen64_nearest,
        "chosen_form_256_clusters": chosen256,
        "reduced_precision": lowp,
        "sweep_fp32": rows,
        "update": {"build_s": round(build_s, 3), "build_vectors_per_s": round(args.n_base / build_s, 1),
                   "delete_10k_ms": round(del_s * 1e3, 3), "insert_10k_ms": round(ins_s * 1e3, 3),
                   "phase_ms": {k: round(st[k], 3) for k in ("ins_search_ms", "ins_prune_ms",
                                                               "ins_reverse_ms", "ins_commit_ms",
                                                               "del_mark_ms", "del_repair_ms")},
                   "repaired_rows": st["last_repaired"]},
        "end_to_end_host_buffers": {"note": "svf_search with host buffers: query upload and "
                                            "result download included; not the value",
                                    "beam": beam, "ms_per_batch": round(e2e_ms, 3),
                                    "qps": round(nq / (e2e_ms / 1e3), 1)},
        "small_batches": small,
        "large_footprint": large,
        "tiered": tier,
        "cache_policies": policies,
        "workload_families": workloads,
        "tiered_full_size": full_tier,
        "serving": serving,
        "wall_s_timed": round(wall, 4),
    }
    os.makedirs(os.path.dirname(args.detail) or ".", exist_ok=True)
    with open(args.detail, "w") as f:
        json.dump(detail, f)
    c = chosen64
    head = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain FP32 search, 1M x 128 integer-valued GMM (256 comps), L2, "
                               "degree 64, 10k-query batch, k=10",
                   "beam": beam, "recall@10": round(rec, 4)},
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                          "kernel", "alg_bytes_per_launch")},
        "cpu_baseline": None if cpu is None else {
            "value": cpu["value"], "unit": cpu["unit"], "cores": cpu["cores"], "kind": "oracle",
            "sample": cpu["sample"], "ids_equal_gpu": cpu["query_ids_equal_gpu"]},
        "chosen_form": {"precision": c["precision"], "n_clusters": c["n_clusters"],
                        "beam": c["beam"], "search_width": c["search_width"],
                        "model_conf": c["model_conf"], "fallback_share": c["fallback_share"],
                        "recall@10": round(c["recall@10"], 4), "value": c["value"],
                        "speedup_vs_plain": c["speedup_vs_plain"],
                        "speedup_64_nearest_entries": chosen64_nearest["speedup_vs_plain"],
                        "speedup_256_clusters": chosen256["speedup_vs_plain"]},
        "serving": None if serving is None else serving.get("headline"),
        "detail": args.detail,
    }
    print(json.dumps(head, separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
