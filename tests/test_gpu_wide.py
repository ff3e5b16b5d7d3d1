"""Rows wider than two 128-element chunks on the GPU against the FP64 oracle:
400 dimensions (four chunks, the last one ragged) and 768 (six chunks, run
by the eight-chunk kernels), for FP32, BF16 and FP8 traversal.

Values are FP8-exact levels of magnitude <= 56 (datagen.gmm_fp8_exact_valued),
so every stored element is exact in each precision and every distance and
inner product is an integer below 2^24 (768 * 112^2 < 2^24): ids, distances
and expansion counts must equal the oracle's bit for bit."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen
from gpu_util import gpu_from_oracle, oracle_index

pytestmark = pytest.mark.gpu

PRECS = [(O.P_FP32, svf.PREC_FP32), (O.P_BF16, svf.PREC_BF16), (O.P_FP8, svf.PREC_FP8)]


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
    return ids.cpu().numpy(), d.cpu().numpy(), ne.cpu().numpy()


@pytest.mark.parametrize("dim,metric", [(400, O.IP), (768, O.L2)])
def test_wide_rows_search_bit_exact(dim, metric):
    base, q = datagen.gmm_fp8_exact_valued(404, 2500, 53, dim, 12)
    oix = oracle_index(base, 24, metric=metric, seed=6)
    for oprec, gprec in PRECS:
        print("wide search dim %d metric %d precision %d" % (dim, metric, gprec), flush=True)
        oix.set("precision", oprec)
        g = gpu_from_oracle(oix, base, seed=6, precision=gprec)
        for beam in (24, 80):
            oi, od, ost = oix.search(q, 10, beam)
            gi, gd, gne = dev_search(g, q, 10, beam)
            np.testing.assert_array_equal(gi, oi)
            np.testing.assert_array_equal(gd.astype(np.float64), od)
            np.testing.assert_array_equal(gne, ost["n_exp"])
        g.close()
    oix.set("precision", O.P_FP32)


def test_wide_rows_build_bit_exact():
    """Insertion at 400 dimensions (FP32 traversal, several batches) builds the
    oracle's graph."""
    print("wide build dim 400", flush=True)
    base, _ = datagen.gmm_fp8_exact_valued(405, 1800, 1, 400, 10)
    oix = O.OracleIndex(400, 16, O.L2, seed=7, insert_batch_max=400)
    oix.build(base, batch_max=400)
    g = svf.Index(400, 16, svf.METRIC_L2, seed=7, insert_batch_max=400)
    g.build(base)
    gr, ge, ga = g.export_graph()
    orows, oe, oa = oix.export()
    np.testing.assert_array_equal(ga, oa)
    np.testing.assert_array_equal(gr, orows)
    np.testing.assert_array_equal(ge.astype(np.float64), oe)
