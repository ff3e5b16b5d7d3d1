"""Checkpoint and resume (svf_save / svf_load): a loaded index has the saved
graph, options and deletion counters, answers searches identically and keeps
evolving identically; damaged files are refused."""
import os

import numpy as np
import pytest

import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen

pytestmark = pytest.mark.gpu

OPTS = dict(seed=7, insert_batch_max=400, search_width=2, visited_slots=2048, repair_c=6,
            consolidate_frac=0.5)


def make_index():
    base, q = datagen.gmm_uint8_valued(801, 3600, 60, 48, 10)
    g = svf.Index(48, 16, svf.METRIC_L2, **OPTS)
    g.build(base[:3000])
    g.delete(np.arange(0, 3000, 9, dtype=np.int32))
    g.insert(base[3000:3300])
    g.set_option("precision", svf.PREC_BF16)
    return g, base, q


def test_round_trip_and_continued_updates(tmp_path):
    g, base, q = make_index()
    path = str(tmp_path / "index.svf")
    g.save(path)
    h = svf.Index.load(path)
    assert (h.dim, h.degree, h.metric) == (48, 16, svf.METRIC_L2)
    for a, b in zip(g.export_graph(), h.export_graph()):
        np.testing.assert_array_equal(a, b)
    for k in list(OPTS) + ["precision", "rerank", "beam_insert", "entry_samples"]:
        assert g.get_option(k) == h.get_option(k), k
    assert g.stats()["n_alive"] == h.stats()["n_alive"]
    gi, gd = g.search(q, 10, 40)
    hi, hd = h.search(q, 10, 40)
    np.testing.assert_array_equal(gi, hi)
    np.testing.assert_array_equal(gd, hd)
    # both keep evolving identically: inserts, deletes, a consolidation
    for x in (g, h):
        x.insert(base[3300:])
        x.delete(np.arange(1, 3600, 5, dtype=np.int32))
        x.consolidate()
    for a, b in zip(g.export_graph(), h.export_graph()):
        np.testing.assert_array_equal(a, b)


def test_tiered_segmented_store_round_trip(tmp_path):
    """A tiered index whose host store spans four 1024-row segments saves the
    vectors of every segment: the loaded (untiered) index has the same graph
    and answers searches identically."""
    base, q = datagen.gmm_uint8_valued(802, 3600, 60, 48, 10)
    g = svf.Index(48, 16, svf.METRIC_L2, seed=3, insert_batch_max=400)
    g.set_option("host_segment_rows", 1024)
    g.set_option("cache_bytes", 600 * 48 * 4)
    g.build(base[:3300])
    g.delete(np.arange(0, 3300, 13, dtype=np.int32))
    assert g.get_option("host_segments") == 4
    path = str(tmp_path / "tiered.svf")
    g.save(path)
    h = svf.Index.load(path)
    for a, b in zip(g.export_graph(), h.export_graph()):
        np.testing.assert_array_equal(a, b)
    gi, gd = g.search(q, 10, 40)
    hi, hd = h.search(q, 10, 40)
    np.testing.assert_array_equal(gi, hi)
    np.testing.assert_array_equal(gd, hd)


def test_damaged_files_are_refused(tmp_path):
    g, _, _ = make_index()
    path = str(tmp_path / "index.svf")
    g.save(path)
    blob = open(path, "rb").read()
    bad = bytearray(blob)
    bad[len(bad) // 2] ^= 0x40
    cases = {"flipped": bytes(bad), "truncated": blob[:len(blob) - 100],
             "magic": b"XXXXXXXX" + blob[8:], "empty": b""}
    for name, data in cases.items():
        p = str(tmp_path / (name + ".svf"))
        with open(p, "wb") as f:
            f.write(data)
        with pytest.raises(svf.SvfError) as e:
            svf.Index.load(p)
        assert e.value.code == -1, name
    with pytest.raises(svf.SvfError) as e:
        svf.Index.load(str(tmp_path / "missing.svf"))
    assert e.value.code == -4


def test_save_refused_while_serving(tmp_path):
    g, _, _ = make_index()
    g.serve_start(streams=2, max_batch=1024)
    try:
        with pytest.raises(svf.SvfError) as e:
            g.save(str(tmp_path / "x.svf"))
        assert e.value.code == -5
    finally:
        g.serve_stop()
    assert not os.path.exists(str(tmp_path / "x.svf"))
