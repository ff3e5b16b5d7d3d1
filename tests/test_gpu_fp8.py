"""FP8 traversal (OCP E4M3 codes, one FP32 scale per vector, FP32
accumulation, exact FP32 re-scoring) on the GPU against the FP64 oracle.

On rows whose values are levels of FP8_EXACT_LEVELS with largest magnitude 56
the scale is 1/8 and every code is exact, and all distances are integers
below 2^24: the FP8 search must then equal the oracle's bit for bit.  On float
data the two may differ only where the oracle decided by a near tie."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen
from gpu_util import gpu_from_oracle, oracle_index, tol_close

pytestmark = pytest.mark.gpu


def dev_counts(g, q, k, beam):
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
    return ids.cpu().numpy(), d.cpu().numpy(), ne.cpu().numpy()


@pytest.mark.parametrize("dim,metric,row_scales", [(128, O.L2, 0), (72, O.L2, 0), (200, O.IP, 0),
                                                    (128, O.L2, 1), (200, O.IP, 1)])
@pytest.mark.parametrize("rerank", [0, 1])
def test_fp8_search_bit_exact_on_exact_levels(dim, metric, row_scales, rerank):
    """dim 72: a 16-byte-ragged FP8 row; dim 200: two 128-element chunks with
    the inner product (a scale of 1/8 keeps s * sum exact).  row_scales: the
    scales read beside the graph rows instead of per vector."""
    base, q = datagen.gmm_fp8_exact_valued(401, 5000, 131, dim, 16)
    oix = oracle_index(base, 24, metric=metric, seed=3)
    oix.set("precision", O.P_FP8)
    g = gpu_from_oracle(oix, base, seed=3, precision=svf.PREC_FP8, rerank=rerank,
                        fp8_row_scales=row_scales)
    assert g.get_option("fp8_row_scales_on") == row_scales
    for beam in (16, 96):
        oi, od, ost = oix.search(q, 10, beam, rerank=bool(rerank))
        gi, gd, gne = dev_counts(g, q, 10, beam)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(gd.astype(np.float64), od)
        np.testing.assert_array_equal(gne, ost["n_exp"])


def test_fp8_build_bit_exact_on_exact_levels():
    """Insertion with FP8 traversal (edges take exact distances) builds the
    oracle's graph."""
    base, _ = datagen.gmm_fp8_exact_valued(402, 2500, 1, 128, 12)
    oix = O.OracleIndex(128, 16, O.L2, seed=4, insert_batch_max=300)
    oix.set("precision", O.P_FP8)
    oix.build(base, batch_max=300)
    g = svf.Index(128, 16, svf.METRIC_L2, seed=4, insert_batch_max=300, precision=svf.PREC_FP8)
    g.build(base)
    gr, ge, ga = g.export_graph()
    orows, oe, oa = oix.export()
    np.testing.assert_array_equal(ga, oa)
    np.testing.assert_array_equal(gr, orows)
    np.testing.assert_array_equal(ge.astype(np.float64), oe)


@pytest.mark.parametrize("metric,dim", [(O.L2, 128), (O.IP, 200)])
def test_fp8_float_matches_except_near_ties(metric, dim):
    """Float data: decisive queries (oracle margin above 1e-5) return the
    oracle's ids; every query's k distances equal the oracle's element by
    element within the parity tolerance.  The inner-product shape uses 256
    components: with few, tight components a unit-norm pool holds many
    products within 1e-5 of each other and few queries are decisive."""
    comps = 16 if metric == O.L2 else 256
    base, q = datagen.gmm_float(403, 8000, 120, dim, comps, normalise=(metric == O.IP))
    oix = oracle_index(base, 32, metric=metric, seed=5)
    oix.set("precision", O.P_FP8)
    g = gpu_from_oracle(oix, base, seed=5, precision=svf.PREC_FP8)
    oi, od, ost = oix.search(q, 10, 64)
    gi, gd = g.search(q, 10, 64)
    decisive = ost["margin"] > 1e-5
    same = (gi == oi).all(axis=1)
    assert same[decisive].all(), np.nonzero(decisive & ~same)
    assert decisive.mean() >= 0.5
    scale = np.linalg.norm(q, axis=1)[:, None] * np.linalg.norm(base, axis=1).max()
    assert tol_close(gd, od, metric, scale=scale).all()
    exact = oix.query_dists(q, gi)
    assert tol_close(gd, exact, metric, scale=scale).all()
    assert (np.diff(gd, axis=1) >= 0).all()
    gt_i, gt_d = O.bruteforce(base, q, 10, metric=metric)
    grec = O.recall_at_k(gi, exact, gt_d, 10)
    orec = O.recall_at_k(oi, oix.query_dists(q, oi), gt_d, 10)
    assert grec >= 0.9 and abs(grec - orec) <= 0.02


def test_fp8_switch_and_growth_keep_results():
    """Switching precision on a filled index, then growing it by insertion,
    gives the results of an index built in FP8 form from the start."""
    base, q = datagen.gmm_fp8_exact_valued(404, 3000, 60, 96, 10)
    a = svf.Index(96, 16, svf.METRIC_L2, seed=9, insert_batch_max=500)
    a.build(base[:1200])
    a.set_option("precision", svf.PREC_FP8)
    a.insert(base[1200:])
    b = svf.Index(96, 16, svf.METRIC_L2, seed=9, insert_batch_max=500)
    b.build(base[:1200])
    b.insert(base[1200:])
    b.set_option("precision", svf.PREC_FP8)
    ia, da = a.search(q, 10, 48)
    ib, db = b.search(q, 10, 48)
    # exact levels: FP8 traversal equals FP32 traversal, so both graphs agree
    np.testing.assert_array_equal(ia, ib)
    np.testing.assert_array_equal(da, db)


def test_fp8_row_scales_follow_every_row_write():
    """With the scales kept beside the graph rows, every search equals the
    per-vector-scale search bit for bit (ids, distances, expansion counts)
    after a build, an insertion, deletions with localized repair, a
    synchronous and a background consolidation (with insertions in its
    window) and an import: every kind of row write refreshes the row scales.
    Integer data gives each vector its own scale, so a stale one would show."""
    base, q = datagen.gmm_uint8_valued(405, 4200, 80, 64, 12)
    opts = dict(seed=5, insert_batch_max=300, consolidate_frac=0.0, precision=svf.PREC_FP8)
    a = svf.Index(64, 16, svf.METRIC_L2, fp8_row_scales=1, **opts)
    b = svf.Index(64, 16, svf.METRIC_L2, fp8_row_scales=0, **opts)

    def same():
        for beam in (16, 64):
            ia, da, na = dev_counts(a, q, 10, beam)
            ib, db, nb = dev_counts(b, q, 10, beam)
            np.testing.assert_array_equal(ia, ib)
            np.testing.assert_array_equal(da, db)
            np.testing.assert_array_equal(na, nb)

    g = np.random.Generator(np.random.Philox(405))
    for x in (a, b):
        x.build(base[:2500])
    assert a.get_option("fp8_row_scales_on") == 1 and b.get_option("fp8_row_scales_on") == 0
    same()
    for x in (a, b):
        x.insert(base[2500:3100])
    same()
    gone = g.choice(3100, 600, replace=False).astype(np.int32)
    for x in (a, b):
        x.delete(gone)                                    # localized repair
    same()
    for x in (a, b):
        x.consolidate()
    same()
    more = np.setdiff1d(g.choice(3100, 700, replace=False), gone).astype(np.int32)
    for x in (a, b):
        x.set_option("consolidate_async", 1)
        x.set_option("consolidate_frac", 0.05)
        x.delete(more)                                    # starts a background consolidation
        x.insert(base[3100:3700])                         # rows logged for the merge
        x.consolidate_wait()
    same()
    for x in (a, b):
        x.insert(base[3700:])                             # growth past the capacity
    same()
    rows, ed, alive = a.export_graph()
    c = svf.Index(64, 16, svf.METRIC_L2, fp8_row_scales=1, **opts)
    n = len(alive)
    c.import_graph(np.ascontiguousarray(base[:n]), rows, ed, alive)
    ia, da, na = dev_counts(a, q, 10, 48)
    ic, dc, nc = dev_counts(c, q, 10, 48)
    np.testing.assert_array_equal(ia, ic)
    np.testing.assert_array_equal(da, dc)
    assert svf.Index(64, 16, svf.METRIC_L2, **opts).get_option("fp8_row_scales") == -1
