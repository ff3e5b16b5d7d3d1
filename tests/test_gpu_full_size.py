"""Parity at the benchmark's full size: the 1M x 128 integer-valued workload
(degree 64, 10k-query batches) built on the GPU and searched in the
launch configuration the benchmark times (the whole 10k batch through
svf_search_dev at beam 88, default visited table).  The oracle, given the
GPU-built graph, recomputes a sample of the queries one by one; on
integer-valued data every distance is exact on both sides, so ids,
distances and expansion counts must be equal.  The benchmark's update step
(a 10k-id delete, then a 10k-vector insert) is checked through invariants
that hold at any size and through exact edge distances of sampled rows, and
the search after it is sampled against the oracle again."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen

pytestmark = pytest.mark.gpu

DIM, R, K, BEAM, NQ = 128, 64, 10, 88, 10_000


def dev_search(g, q):
    import torch
    qt = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
    n = q.shape[0]
    ids = torch.empty((n, K), dtype=torch.int32, device="cuda")
    d = torch.empty((n, K), dtype=torch.float32, device="cuda")
    nd = torch.empty(n, dtype=torch.int32, device="cuda")
    ne = torch.empty(n, dtype=torch.int32, device="cuda")
    g.search_dev(qt.data_ptr(), n, K, BEAM, ids.data_ptr(), d.data_ptr(), nd.data_ptr(),
                 ne.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy(), ne.cpu().numpy()


def oracle_of(g, vecs, prec=None):
    rows, ed, alive = g.export_graph()
    o = O.OracleIndex(DIM, R, O.L2, seed=0)
    o.import_state(vecs, rows, ed.astype(np.float64), alive)
    if prec is not None:
        o.set("precision", prec)
    return o, rows, ed, alive


def sampled_equal(g, o, q, every=50):
    gi, gd, gne = dev_search(g, q)
    s = np.arange(0, q.shape[0], every)
    oi, od, ost = o.search(q[s], K, BEAM)
    np.testing.assert_array_equal(gi[s], oi)
    np.testing.assert_array_equal(gd[s].astype(np.float64), od)
    np.testing.assert_array_equal(gne[s], ost["n_exp"])


@pytest.fixture(scope="module")
def full():
    base, q = datagen.workload_1m_int(1_000_000, NQ)
    g = svf.Index(DIM, R, svf.METRIC_L2, seed=0)
    g.build(base)
    return g, base, q


def test_full_size_fp32_search_sampled_against_oracle(full):
    g, base, q = full
    o, _, _, _ = oracle_of(g, base)
    sampled_equal(g, o, q)


def test_full_size_bf16_search_sampled_against_oracle(full):
    """BF16 traversal (values 0..255 are exact on its grid) with the FP32
    re-score, the reduced-precision default table (2048 slots)."""
    g, base, q = full
    g.set_option("precision", svf.PREC_BF16)
    try:
        o, _, _, _ = oracle_of(g, base, O.P_BF16)
        sampled_equal(g, o, q)
    finally:
        g.set_option("precision", svf.PREC_FP32)


def test_full_size_update_step_invariants_and_sampled_search(full):
    """The benchmark's update step on the 1M index: every row keeps the fixed
    degree or stays short only when padded with -1 at its end, names no
    vertex twice and never itself, is sorted by (stored distance, id), and a
    sample of rows carries the exact FP64 distances (integer data).  The
    search after the step equals the oracle's on a query sample."""
    g, base, q = full
    gen = np.random.Generator(np.random.Philox(77))
    victims = gen.choice(base.shape[0], 10_000, replace=False).astype(np.int32)
    extra, _ = datagen.gmm_uint8_valued(2, 10_000, 1, DIM, 256)
    g.delete(victims)
    g.insert(extra)
    vecs = np.concatenate([base, extra])
    o, rows, ed, alive = oracle_of(g, vecs)
    n = rows.shape[0]
    assert n == vecs.shape[0] and int(alive.sum()) == n - 10_000
    valid = rows >= 0
    # padding only at the end of a row
    assert not (~valid[:, :-1] & valid[:, 1:]).any()
    assert (rows < n).all()
    assert not (rows == np.arange(n, dtype=np.int32)[:, None]).any()
    srt = np.sort(np.where(valid, rows, -1 - np.arange(R)), axis=1)
    assert not (srt[:, 1:] == srt[:, :-1]).any()              # no vertex named twice
    d = np.where(valid, ed.astype(np.float64), np.inf)
    step = (d[:, 1:] > d[:, :-1]) | ((d[:, 1:] == d[:, :-1]) & (rows[:, 1:] > rows[:, :-1]))
    assert (step | ~valid[:, 1:]).all()                         # (d, id) order
    assert valid[alive.astype(bool)].sum(1).min() > 0
    s = np.concatenate([np.arange(0, n, 997), np.arange(base.shape[0], n, 37)])
    for v in s:
        m = valid[v]
        exact = ((vecs[rows[v, m]].astype(np.float64) - vecs[v].astype(np.float64)) ** 2).sum(1)
        np.testing.assert_array_equal(ed[v, m].astype(np.float64), exact)
    sampled_equal(g, o, q, every=100)
