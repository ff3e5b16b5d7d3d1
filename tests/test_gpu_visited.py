"""Visited-table forms above 2^20 ids, against the FP64 oracle.

The table packs a scrambled id into (set, tag); its tag field is 12 bits wide
while the tag needs at most 11 bits and 16 bits wide up to 15 (ids of
id_bits bits, log2(slots / 4) of them picking the set).  The 16-bit form is
what indexes of 2^20 to 2^24 ids take at 2048 slots, so these tests import a
graph of 2^20 + 50,000 integer-valued points (every distance exact in FP32)
into both sides and require ids, distances and expansion counts to be equal
for every table size from 256 slots (15-bit tags) to 16384 and for the 32-bit
form, and at 300,000 ids with 256 slots (13-bit tags)."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen

pytestmark = pytest.mark.gpu

DIM, R = 8, 16


def exact_edges(base, rows):
    b = base.astype(np.int64)
    out = np.empty(rows.shape, np.float64)
    for c0 in range(0, rows.shape[0], 1 << 18):
        c1 = min(rows.shape[0], c0 + (1 << 18))
        d = b[rows[c0:c1]] - b[c0:c1, None, :]
        out[c0:c1] = (d * d).sum(axis=2)
    return out


def counts(g, q, k, beam):
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


def imported(n, workload):
    base, rows, q = datagen.walk_graph_uint8(workload, n, DIM, R, 300)
    ed = exact_edges(base, rows)
    alive = np.ones(n, np.uint8)
    alive[7::97] = 0                         # a few deleted ids the search must skip
    oix = O.OracleIndex(DIM, R, O.L2, seed=21)
    oix.import_state(base, rows, ed, alive)
    return base, rows, ed, alive, q, oix


@pytest.fixture(scope="module")
def big():
    return imported((1 << 20) + 50_000, 31)


@pytest.mark.parametrize("prec", [svf.PREC_FP32, svf.PREC_BF16])
def test_tag_forms_above_2_20_ids_bit_exact(big, prec):
    base, rows, ed, alive, q, oix = big
    oi, od, ost = oix.search(q, 10, 64)
    g = svf.Index(DIM, R, svf.METRIC_L2, seed=21, precision=prec)
    g.import_graph(base, rows, ed.astype(np.float32), alive)
    # 0 is the default: 2048 slots (16-bit tags) for BF16, 4096 for FP32
    for slots, compact in ((0, 1), (256, 1), (512, 1), (1024, 1), (2048, 1), (4096, 1),
                           (16384, 1), (2048, 0)):
        g.set_option("visited_slots", slots)
        g.set_option("visited_compact", compact)
        gi, gd, gnd, gne = counts(g, q, 10, 64)
        np.testing.assert_array_equal(gi, oi, err_msg="slots %d compact %d" % (slots, compact))
        np.testing.assert_array_equal(gd.astype(np.float64), od)
        np.testing.assert_array_equal(gne, ost["n_exp"])
        assert (gnd >= ost["n_dist"]).all()
    assert alive[oi[oi >= 0]].all()


def test_tag_form_at_300k_ids_with_256_slots():
    base, rows, ed, alive, q, oix = imported(300_000, 32)
    oi, od, ost = oix.search(q, 10, 96)
    g = svf.Index(DIM, R, svf.METRIC_L2, seed=21, visited_slots=256)
    g.import_graph(base, rows, ed.astype(np.float32), alive)
    gi, gd, gnd, gne = counts(g, q, 10, 96)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gd.astype(np.float64), od)
    np.testing.assert_array_equal(gne, ost["n_exp"])
