"""The allocation-free search entry point against svf_search_dev and the
oracle: two calls in a row on one index, the second with fewer queries, then
a call on a second index (the fixed workspace is shared by every index on
the GPU and keeps the last call's contents), and its refusals."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen
from gpu_util import gpu_from_oracle, oracle_index

pytestmark = pytest.mark.gpu


def run(g, q, k, beam, noalloc):
    import torch
    qt = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
    nq = q.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int32, device="cuda")
    d = torch.full((nq, k), -7.0, dtype=torch.float32, device="cuda")
    nd = torch.zeros(nq, dtype=torch.int32, device="cuda")
    ne = torch.zeros(nq, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    f = g.search_dev_noalloc if noalloc else g.search_dev
    f(qt.data_ptr(), nq, k, beam, ids.data_ptr(), d.data_ptr(), nd.data_ptr(), ne.data_ptr(), st)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy(), nd.cpu().numpy(), ne.cpu().numpy()


def test_noalloc_search_equals_search_dev_and_oracle():
    base, q = datagen.gmm_uint8_valued(611, 6000, 900, 96, 24)
    oix = oracle_index(base, 24, seed=4)
    g = gpu_from_oracle(oix, base, seed=4)
    for nq, beam in ((900, 64), (37, 32)):          # the second call is smaller
        ref = run(g, q[:nq], 10, beam, noalloc=False)
        got = run(g, q[:nq], 10, beam, noalloc=True)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        oi, od, ost = oix.search(q[:nq], 10, beam)
        np.testing.assert_array_equal(got[0], oi)
        np.testing.assert_array_equal(got[1].astype(np.float64), od)
        np.testing.assert_array_equal(got[3], ost["n_exp"])
    # another index on the same GPU, at another precision, reuses the workspace
    base2, q2 = datagen.gmm_uint8_valued(612, 3000, 300, 64, 12)
    o2 = oracle_index(base2, 16, seed=9)
    g2 = gpu_from_oracle(o2, base2, seed=9, precision=svf.PREC_BF16)
    got = run(g2, q2, 5, 40, noalloc=True)
    ref = run(g2, q2, 5, 40, noalloc=False)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    oi, od, _ = o2.search(q2, 5, 40)
    np.testing.assert_array_equal(got[0], oi)
    np.testing.assert_array_equal(got[1].astype(np.float64), od)


def test_noalloc_refusals_and_empty_index():
    import torch
    g = svf.Index(32, 8, svf.METRIC_L2)
    q = torch.zeros((3, 32), dtype=torch.float32, device="cuda")
    ids = torch.empty((3, 4), dtype=torch.int32, device="cuda")
    d = torch.empty((3, 4), dtype=torch.float32, device="cuda")
    # nothing indexed: padded results
    g.search_dev_noalloc(q.data_ptr(), 3, 4, 8, ids.data_ptr(), d.data_ptr())
    torch.cuda.synchronize()
    assert (ids.cpu().numpy() == -1).all() and np.isinf(d.cpu().numpy()).all()
    # beyond the fixed workspace: refused before any launch
    with pytest.raises(svf.SvfError):
        g.search_dev_noalloc(q.data_ptr(), (1 << 19) + 1, 4, 8, ids.data_ptr(), d.data_ptr())
    with pytest.raises(svf.SvfError):
        g.search_dev_noalloc(q.data_ptr(), 3, 4, 2, ids.data_ptr(), d.data_ptr())   # beam < k
