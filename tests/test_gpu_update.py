"""Insertion, deletion, repair and consolidation on the GPU against the
FP64 oracle.  On integer-valued data every distance is exact, so the whole
graph (ids and edge distances) must be identical after every operation."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen
from gpu_util import gpu_from_oracle, oracle_index

pytestmark = pytest.mark.gpu


def assert_same_graph(g, oix, check_dist=True):
    gr, ge, ga = g.export_graph()
    orows, oe, oa = oix.export()
    np.testing.assert_array_equal(ga, oa)
    np.testing.assert_array_equal(gr, orows)
    if check_dist:
        np.testing.assert_array_equal(ge.astype(np.float64), oe)


@pytest.mark.parametrize("dim,R,metric,n", [(128, 16, O.L2, 3000), (72, 24, O.IP, 2000),
                                            (64, 48, O.L2, 2500), (48, 64, O.IP, 2000),
                                            (32, 80, O.L2, 1500)])
def test_build_bit_exact_integer(dim, R, metric, n):
    """Degrees up to 32 take the prune's lane-per-entry row walk; degrees 33-64
    read whole rows per step (48: lanes past the row re-read its last entry);
    degree 80 walks entries again, and its rows, wider than a wave, are
    merged into the reverse-edge pool key by key."""
    base, _ = datagen.gmm_uint8_valued(301, n, 1, dim, 12)
    oix = oracle_index(base, R, metric=metric, seed=7, batch_max=400)
    g = svf.Index(dim, R, metric, seed=7, insert_batch_max=400)
    g.build(base)
    assert_same_graph(g, oix)


def test_insert_and_delete_sequence_bit_exact():
    base, q = datagen.gmm_uint8_valued(302, 4200, 50, 64, 10)
    R = 20
    oix = oracle_index(base[:3000], R, seed=9, batch_max=500)
    g = gpu_from_oracle(oix, base[:3000], seed=9, insert_batch_max=500)
    rng = np.random.Generator(np.random.Philox(3))
    # interleave inserts and deletes: batches of new vectors, random live ids
    pos = 3000
    for step in range(4):
        new = base[pos:pos + 300]
        pos += 300
        assert g.insert(new).tolist() == oix.insert(new).tolist()
        assert_same_graph(g, oix)
        _, _, alive = oix.export()
        victims = rng.choice(np.nonzero(alive)[0], 120, replace=False).astype(np.int32)
        g.delete(victims)
        assert oix.delete(victims) == 0
        assert_same_graph(g, oix)
        st = g.stats()
        assert st["n_alive"] == oix.n_alive
    oi, od, _ = oix.search(q, 10, 40)
    gi, gd = g.search(q, 10, 40)
    np.testing.assert_array_equal(gi, oi)
    g.consolidate()
    oix.consolidate()
    assert_same_graph(g, oix)
    gr, ge, ga = g.export_graph()
    for v in np.nonzero(ga)[0]:
        r = gr[v][gr[v] >= 0]
        assert ga[r].all() and v not in r and len(set(r.tolist())) == len(r)


def test_insert_delete_sequence_whole_row_prune_bit_exact():
    """Degree 40, so every prune (forward rows, reverse edges, repair and
    consolidation lists) reads whole rows per step with lanes 40..63 idle:
    inserts, deletions with local repair, then consolidation, the graph equal
    to the oracle's after each step."""
    base, q = datagen.gmm_uint8_valued(305, 3300, 30, 48, 10)
    R = 40
    oix = oracle_index(base[:2400], R, seed=13, batch_max=300)
    g = gpu_from_oracle(oix, base[:2400], seed=13, insert_batch_max=300)
    rng = np.random.Generator(np.random.Philox(14))
    pos = 2400
    for step in range(3):
        new = base[pos:pos + 300]
        pos += 300
        assert g.insert(new).tolist() == oix.insert(new).tolist()
        assert_same_graph(g, oix)
        _, _, alive = oix.export()
        victims = rng.choice(np.nonzero(alive)[0], 150, replace=False).astype(np.int32)
        g.delete(victims)
        assert oix.delete(victims) == 0
        assert_same_graph(g, oix)
    g.consolidate()
    oix.consolidate()
    assert_same_graph(g, oix)
    oi, od, _ = oix.search(q, 10, 64)
    gi, gd = g.search(q, 10, 64)
    np.testing.assert_array_equal(gi, oi)


def test_repair_topup_path_bit_exact():
    """Heavy deletion: many rows fall short of R candidates and take the
    search top-up; consolidation threshold set out of reach first."""
    base, _ = datagen.gmm_uint8_valued(303, 1500, 1, 32, 6)
    R = 12
    oix = oracle_index(base, R, seed=4, batch_max=300, consolidate_frac=0.95, repair_c=2)
    g = gpu_from_oracle(oix, base, seed=4, insert_batch_max=300, consolidate_frac=0.95, repair_c=2)
    victims = np.arange(0, 1500, 3, dtype=np.int32)
    g.delete(victims)
    oix.delete(victims)
    assert_same_graph(g, oix)
    assert g.stats()["last_repaired"] > 0


def test_delete_errors_leave_index_unchanged():
    base, _ = datagen.gmm_uint8_valued(304, 600, 1, 16, 3)
    g = svf.Index(16, 8, svf.METRIC_L2)
    g.build(base)
    before = g.export_graph()
    with pytest.raises(svf.SvfError) as e:
        g.delete([3, 600])
    assert e.value.code == svf.E_NOTFOUND
    after = g.export_graph()
    for a, b in zip(before, after):
        np.testing.assert_array_equal(a, b)
    g.delete([3, 3, 4])
    g.delete([3])
    assert g.stats()["n_alive"] == 598


def test_reduced_precision_exact_on_integer_data():
    base, q = datagen.gmm_uint8_valued(305, 3000, 80, 128, 10)
    oix = oracle_index(base, 24, seed=2)
    ref_i, ref_d, _ = oix.search(q, 10, 48)
    for prec in (svf.PREC_FP16, svf.PREC_BF16):
        g = gpu_from_oracle(oix, base, seed=2, precision=prec)
        gi, gd = g.search(q, 10, 48)
        np.testing.assert_array_equal(gi, ref_i)
        np.testing.assert_array_equal(gd.astype(np.float64), ref_d)


def test_build_float_recall_and_invariants():
    base, q = datagen.workload_small_float()
    g = svf.Index(128, 32, svf.METRIC_L2, seed=1)
    g.build(base)
    rows, ed, alive = g.export_graph()
    assert ((rows >= 0).sum(1) == 32).all()
    assert (rows != np.arange(len(rows))[:, None]).all()
    srt = np.sort(rows, axis=1)
    assert (np.diff(srt, axis=1) != 0).all()
    oix = O.OracleIndex(128, 32, O.L2)
    oix.import_state(base, rows, ed.astype(np.float64), alive)
    for v in range(0, 10_000, 997):
        for r in range(32):
            ex = oix.dist_ids(v, rows[v, r])
            assert abs(ed[v, r] - ex) <= 1e-5 * ex
    gi, gd = g.search(q, 10, 64)
    gt_i, gt_d = O.bruteforce(base, q, 10)
    assert O.recall_at_k(gi, oix.query_dists(q, gi), gt_d, 10) >= 0.95


@pytest.mark.parametrize("pass_stream", [True, False])
def test_insert_dev_waits_for_the_producer(pass_stream):
    """svf_insert_dev reads device vectors only after the work queued on the
    given stream (or the default stream) has finished: vectors whose
    producer is still running insert exactly as host vectors do."""
    import torch
    base, _ = datagen.gmm_uint8_valued(705, 3000, 10, 64, 8)
    host = svf.Index(64, 16, svf.METRIC_L2, seed=4, insert_batch_max=500)
    dev = svf.Index(64, 16, svf.METRIC_L2, seed=4, insert_batch_max=500)
    for g in (host, dev):
        g.build(base[:2000])
    host.insert(base[2000:])
    src = torch.from_numpy(np.ascontiguousarray(base[2000:])).cuda()
    torch.cuda.synchronize()
    busy = torch.full((2048, 2048), 1.0 / 2048, device="cuda")
    for _ in range(30):                        # keep the stream busy ahead of the copy
        busy = busy @ busy
    zero = torch.where(torch.isfinite(busy[0, 0]), busy[0, 0] * 0, torch.zeros((), device="cuda"))
    x = src + zero
    stream = torch.cuda.current_stream().cuda_stream if pass_stream else None
    dev.insert_dev(x.data_ptr(), x.shape[0], stream=stream)
    for a, b in zip(host.export_graph(), dev.export_graph()):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("lr,cf", [(0, 0.0), (0, 0.2), (1, 0.0)])
def test_deletion_modes_bit_exact(lr, cf):
    """Lazy deletion alone, with global consolidation alone, and with
    localized repair but no consolidation: graphs equal the oracle's after
    every delete and after inserts that follow them."""
    base, _ = datagen.gmm_uint8_valued(707, 3500, 10, 64, 12)
    oix = oracle_index(base[:3000], 16, seed=9, batch_max=500, localized_repair=lr,
                       consolidate_frac=cf)
    g = gpu_from_oracle(oix, base[:3000], seed=9, insert_batch_max=500, localized_repair=lr,
                        consolidate_frac=cf)
    gen = np.random.Generator(np.random.Philox(3))
    for _ in range(3):
        victims = gen.choice(3000, 250, replace=False).astype(np.int32)
        assert oix.delete(victims) == 0
        g.delete(victims)
        assert_same_graph(g, oix)
    oix.insert(base[3000:])
    g.insert(base[3000:])
    assert_same_graph(g, oix)


def test_background_consolidation_bit_exact(tmp_path):
    """A consolidation that falls due runs in the background on a snapshot
    while insertions and deletions continue on the live graph; live graphs
    and the merged graph equal the oracle's, and saving waits for the merge."""
    base, q = datagen.gmm_uint8_valued(708, 4200, 60, 64, 12)
    oix = oracle_index(base[:3000], 16, seed=10, batch_max=400, consolidate_async=1)
    g = gpu_from_oracle(oix, base[:3000], seed=10, insert_batch_max=400, consolidate_async=1)
    gen = np.random.Generator(np.random.Philox(8))
    for cycle in range(2):
        lo = 3000 + 600 * cycle
        victims = gen.choice(lo, int(0.25 * lo), replace=False).astype(np.int32)
        assert oix.delete(victims) == 0
        g.delete(victims)
        assert g.get_option("consolidate_pending") == 1
        assert_same_graph(g, oix)
        oix.insert(base[lo:lo + 300])
        g.insert(base[lo:lo + 300])
        few = gen.choice(lo, 40, replace=False).astype(np.int32)
        assert oix.delete(few) == 0
        g.delete(few)
        assert_same_graph(g, oix)
        with pytest.raises(svf.SvfError):
            g.save(str(tmp_path / "pending.svf"))
        oix.insert(base[lo + 300:lo + 600])
        g.insert(base[lo + 300:lo + 600])
        oix.consolidate_wait()
        g.consolidate_wait()
        assert g.get_option("consolidate_pending") == 0
        assert_same_graph(g, oix)
        oi, od, _ = oix.search(q, 10, 48)
        gi, gd = g.search(q, 10, 48)
        np.testing.assert_array_equal(gi, oi)


def test_hand_worked_merge_on_the_gpu():
    """The oracle's hand-worked pin of a background consolidation merged
    after an insertion in its window, on the GPU."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "merge_example.json")))
    ix = svf.Index(g["dim"], g["R"], g["metric"], seed=g["seed"], beam_insert=g["beam_insert"],
                   consolidate_frac=g["consolidate_frac"], consolidate_async=1)
    pts = np.array(g["points"], np.float32).reshape(-1, g["dim"])
    ix.import_graph(pts, np.array(g["rows"], np.int32), np.array(g["edge_d"], np.float32),
                    np.ones(len(pts), np.uint8))
    ix.delete(np.array(g["delete"], np.int32))
    assert ix.get_option("consolidate_pending") == 1
    assert ix.insert(np.array(g["insert"], np.float32).reshape(-1, g["dim"])).tolist() == [5]
    ix.consolidate_wait()
    rows, ed, alive = ix.export_graph()
    assert rows.tolist() == g["expect_rows"]
    assert ed.astype(np.float64).tolist() == g["expect_edge_d"]
    assert alive.tolist() == g["expect_alive"]
