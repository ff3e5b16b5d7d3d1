"""Helpers for GPU parity tests: build states with the oracle, import them
into the HIP library, and compare results."""
import numpy as np

import oracle as O
import paper_2601_08528_amd as svf


def oracle_index(base, R, metric=O.L2, seed=0, batch_max=10_000, **opts):
    ix = O.OracleIndex(base.shape[1], R, metric, seed=seed, insert_batch_max=batch_max, **opts)
    ix.build(base, batch_max=batch_max)
    return ix


def gpu_from_oracle(oix, base, **opts):
    rows, ed, alive = oix.export()
    g = svf.Index(base.shape[1], oix.R, oix.metric, seed=opts.pop("seed", 0), **opts)
    g.import_graph(base, rows, ed.astype(np.float32), alive)
    return g


def tol_close(a, b, metric, scale=None, rel=1e-5):
    """Distance tolerance: L2 relative to the larger value, IP relative to
    |q| * max|x| (passed as scale)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if metric == O.L2:
        lim = rel * np.maximum(np.abs(a), np.abs(b))
    else:
        lim = rel * scale
    both_inf = np.isinf(a) & np.isinf(b)
    return both_inf | (np.abs(a - b) <= lim + 1e-30)
