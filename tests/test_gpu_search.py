"""Search parity: the HIP path against the FP64 oracle on identical graphs.

Integer-valued data makes every FP32 partial sum exact (squared L2 and inner
products of 0..255 values in <= 200 dims stay below 2^24), so ids, distances
and even per-query expansion counts must be identical.  On float data the
decisions of the two differ only where the oracle saw a near tie."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen
from gpu_util import gpu_from_oracle, oracle_index, tol_close

pytestmark = pytest.mark.gpu


def dev_search(g, q, k, beam):
    import torch
    qt = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
    nq = q.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    d = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    nd = torch.empty(nq, dtype=torch.int32, device="cuda")
    ne = torch.empty(nq, dtype=torch.int32, device="cuda")
    g.search_dev(qt.data_ptr(), nq, k, beam, ids.data_ptr(), d.data_ptr(), nd.data_ptr(),
                 ne.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy(), nd.cpu().numpy(), ne.cpu().numpy()


@pytest.fixture(scope="module")
def int_l2():
    base, q = datagen.gmm_uint8_valued(201, 6000, 157, 128, 24)
    oix = oracle_index(base, 32, seed=11)
    return oix, base, q


@pytest.mark.parametrize("beam", [10, 64, 256, 1024])
def test_search_bit_exact_integer_l2(int_l2, beam):
    oix, base, q = int_l2
    g = gpu_from_oracle(oix, base, seed=11)
    oi, od, ost = oix.search(q, 10, beam)
    gi, gd, gnd, gne = dev_search(g, q, 10, beam)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gd.astype(np.float64), od)
    np.testing.assert_array_equal(gne, ost["n_exp"])          # same trajectory
    assert (gnd >= ost["n_dist"]).all()                         # forgetting only adds work
    hi, hd = g.search(q, 10, beam)                              # host-pointer entry point
    np.testing.assert_array_equal(hi, oi)


@pytest.mark.parametrize("coop", [0, 1024])
@pytest.mark.parametrize("width", [2, 4])
def test_search_width_bit_exact(int_l2, width, coop):
    """Several parents per iteration (a method option the oracle implements),
    with one wave per query (coop 0) and with one wave per parent (coop 1024:
    the 157-query batch runs the cooperative kernel)."""
    oix, base, q = int_l2
    g = gpu_from_oracle(oix, base, seed=11, search_width=width, coop_max_batch=coop)
    oix.set("search_width", width)
    try:
        oi, od, ost = oix.search(q, 10, 64)
        ol, olc = oix.search_trace(q, 10, 64)
    finally:
        oix.set("search_width", 1)
    gi, gd, gnd, gne = dev_search(g, q, 10, 64)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gd.astype(np.float64), od)
    np.testing.assert_array_equal(gne, ost["n_exp"])


@pytest.mark.parametrize("prec,width,coop", [(0, 4, 1024), (2, 1, 0), (2, 2, 1024)])
def test_largest_beam_every_form(int_l2, prec, width, coop):
    """The largest pool (beam 1024, 16 KB of keys per query in LDS): several
    parents per iteration with one wave per parent, and BF16 traversal with
    its FP32 re-score of all 1024 entries (integer data is exact on the BF16
    grid), against the oracle."""
    oix, base, q = int_l2
    g = gpu_from_oracle(oix, base, seed=11, precision=prec, search_width=width,
                        coop_max_batch=coop)
    oix.set("search_width", width)
    oix.set("precision", O.P_BF16 if prec == 2 else O.P_FP32)
    try:
        oi, od, ost = oix.search(q[:60], 10, 1024)
    finally:
        oix.set("search_width", 1)
        oix.set("precision", O.P_FP32)
    gi, gd, gnd, gne = dev_search(g, q[:60], 10, 1024)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gd.astype(np.float64), od)
    np.testing.assert_array_equal(gne, ost["n_exp"])


def test_search_ragged_shapes_inner_product():
    """dim 200 (two 128-chunks, ragged), degree 48 (partial wave), IP metric."""
    base, q = datagen.gmm_uint8_valued(202, 2500, 67, 200, 9)
    oix = oracle_index(base, 48, metric=O.IP, seed=3)
    g = gpu_from_oracle(oix, base, seed=3)
    for beam in (48, 100):
        oi, od, ost = oix.search(q, 7, beam)
        gi, gd, _, gne = dev_search(g, q, 7, beam)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(gd.astype(np.float64), od)
        np.testing.assert_array_equal(gne, ost["n_exp"])


def test_visited_table_size_does_not_change_results(int_l2):
    oix, base, q = int_l2
    ref = None
    for slots, compact in ((256, 0), (256, 1), (2048, 1), (2048, 0), (8192, 1), (16384, 1)):
        g = gpu_from_oracle(oix, base, seed=11, visited_slots=slots, visited_compact=compact)
        gi, gd, gnd, gne = dev_search(g, q, 10, 128)
        if ref is None:
            ref = (gi, gd, gne, gnd)
        else:
            np.testing.assert_array_equal(gi, ref[0])
            np.testing.assert_array_equal(gd, ref[1])
            np.testing.assert_array_equal(gne, ref[2])
    assert ref[3].sum() >= gnd.sum()          # the small table re-evaluates more


def test_batch_composition_invariance(int_l2):
    oix, base, q = int_l2
    g = gpu_from_oracle(oix, base, seed=11)
    big = np.concatenate([q] * 40)            # 6280 queries in one launch
    bi, bd = g.search(big, 10, 64)
    for i in (0, 5, 156):
        si, sd = g.search(q[i:i + 1], 10, 64)
        np.testing.assert_array_equal(si[0], bi[i])
        np.testing.assert_array_equal(si[0], bi[i + 157 * 17])


def test_deleted_ids_are_skipped_on_imported_state(int_l2):
    oix, base, q = int_l2
    rows, ed, alive = oix.export()
    alive = alive.copy()
    g0 = np.random.Generator(np.random.Philox(5))
    alive[g0.choice(len(alive), 900, replace=False)] = 0
    o2 = O.OracleIndex(128, 32, O.L2, seed=11)
    o2.import_state(base, rows, ed, alive)
    g = svf.Index(128, 32, svf.METRIC_L2, seed=11)
    g.import_graph(base, rows, ed.astype(np.float32), alive)
    oi, od, _ = o2.search(q, 10, 64)
    gi, gd = g.search(q, 10, 64)
    np.testing.assert_array_equal(gi, oi)
    assert alive[gi[gi >= 0]].all()


def test_edge_cases_padding_and_limits():
    base, q = datagen.gmm_uint8_valued(203, 5, 3, 16, 2)
    g = svf.Index(16, 4, svf.METRIC_L2)
    g.build(base)
    oix = oracle_index(base, 4)
    gi, gd = g.search(q, 8, 8)                    # fewer alive than k: padded
    oi, od, _ = oix.search(q, 8, 8)
    np.testing.assert_array_equal(gi, oi)
    assert (gi[:, 5:] == -1).all() and np.isinf(gd[:, 5:]).all()
    gi, gd = g.search(q, 1, 1)
    oi, od, _ = oix.search(q, 1, 1)
    np.testing.assert_array_equal(gi, oi)
    gi, gd = g.search(q, 10, 1024)                # maximum beam
    assert gi.shape == (3, 10)
    e, _ = g.search(np.zeros((0, 16), np.float32), 5, 5)
    assert e.shape == (0, 5)
    with pytest.raises(svf.SvfError):
        g.search(q, 5, 4)                         # beam < k
    with pytest.raises(svf.SvfError):
        g.search(q, 5, 1025)
    bad = q.copy()
    bad[0, 0] = np.nan
    with pytest.raises(svf.SvfError):
        g.search(bad, 5, 5)


def test_float_workload_matches_except_near_ties():
    base, q = datagen.workload_small_float()
    oix = oracle_index(base, 32, seed=1)
    g = gpu_from_oracle(oix, base, seed=1)
    oi, od, ost = oix.search(q, 10, 64)
    gi, gd = g.search(q, 10, 64)
    decisive = ost["margin"] > 1e-5
    same = (gi == oi).all(axis=1)
    assert same[decisive].all(), np.nonzero(decisive & ~same)
    assert decisive.mean() >= 0.6
    # every query, decisive or not: the k distances equal the oracle's
    assert tol_close(gd, od, O.L2).all()
    # every returned distance is the exact one to within the FP32 bound
    exact = oix.query_dists(q, gi)
    assert tol_close(gd, exact, O.L2).all()
    assert (np.diff(gd, axis=1) >= 0).all()
    gt_i, gt_d = O.bruteforce(base, q, 10)
    assert O.recall_at_k(gi, exact, gt_d, 10) >= 0.95


def test_stats_before_any_search_leave_no_error():
    """Reading the statistics before any timed call (events never recorded by
    work) leaves no stale HIP error behind for the next call."""
    base, q = datagen.gmm_uint8_valued(203, 800, 20, 32, 4)
    oix = oracle_index(base, 8, seed=2)
    g = gpu_from_oracle(oix, base, seed=2)
    st = g.stats()
    assert st["last_search_ms"] >= 0.0
    gi, gd = g.search(q, 5, 16)
    oi, od, _ = oix.search(q, 5, 16)
    np.testing.assert_array_equal(gi, oi)


@pytest.mark.parametrize("width", [2, 4])
def test_cooperative_search_shapes_and_forms(width):
    """One wave per parent on: the inner product at dim 200 (two chunks, ragged)
    with degree 48, deleted vertices, odd beams, and the BF16 and FP8 forms on
    data exact on their grids; every case bit-exact against the oracle."""
    base, q = datagen.gmm_uint8_valued(204, 2500, 67, 200, 9)
    oix = oracle_index(base, 48, metric=O.IP, seed=3)
    oix.delete(np.arange(5, 2500, 13, dtype=np.int32))
    oix.set("search_width", width)
    g = gpu_from_oracle(oix, base, seed=3, search_width=width, coop_max_batch=4096)
    for beam in (17, 100):
        oi, od, ost = oix.search(q, 7, beam)
        gi, gd, _, gne = dev_search(g, q, 7, beam)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(gd.astype(np.float64), od)
        np.testing.assert_array_equal(gne, ost["n_exp"])
    base8, q8 = datagen.gmm_fp8_exact_valued(205, 3000, 50, 64, 8)
    o8 = oracle_index(base8, 24, seed=4)
    o8.set("search_width", width)
    for prec, oprec in ((svf.PREC_BF16, O.P_BF16), (svf.PREC_FP8, O.P_FP8)):
        o8.set("precision", oprec)
        g8 = gpu_from_oracle(o8, base8, seed=4, search_width=width, coop_max_batch=4096,
                             precision=prec)
        for rr in (0, 1):
            g8.set_option("rerank", rr)
            oi, od, ost = o8.search(q8, 10, 48, rerank=bool(rr))
            gi, gd, _, gne = dev_search(g8, q8, 10, 48)
            np.testing.assert_array_equal(gi, oi)
            np.testing.assert_array_equal(gd.astype(np.float64), od)
            np.testing.assert_array_equal(gne, ost["n_exp"])
