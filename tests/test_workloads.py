"""The streaming workload families' operation sequences (host logic, no GPU):
each family's definition checked on the sequence it generates."""
import numpy as np

from paper_2601_08528_amd import datagen


def _replay(ops, n):
    born = np.full(n, -1)
    died = np.full(n, -1)
    for t, (ins, dele) in enumerate(ops):
        assert (born[ins] == -1).all()                     # inserted once
        born[ins] = t
        assert (born[dele] >= 0).all() and (born[dele] <= t).all()
        assert (died[dele] == -1).all()                    # deleted once, while live
        died[dele] = t
    return born, died


def test_sliding_window():
    n = 2000
    ops, first = datagen.sliding_window_ops(n, 200)
    assert len(ops) == 200 and first == 100
    born, died = _replay(ops, n)
    assert (born >= 0).all()
    gone = died >= 0
    assert (died[gone] - born[gone] == 100).all()         # deleted T_max/2 steps later
    assert gone.sum() == n // 2                           # the last 100 segments stay


def test_expiration_time():
    n = 60_000
    ops, first = datagen.expiration_time_ops(4, n)
    assert len(ops) == 200 and first == 100
    born, died = _replay(ops, n)
    assert (born >= 0).all()
    gone = died >= 0
    life = died[gone] - born[gone]
    assert set(np.unique(life).tolist()) <= {10, 50, 100}
    # rows that could expire within 200 steps: their lifetime mix is 10 : 2 : 1
    early = born < 100
    mix = np.array([(life[born[gone] < 100] == L).sum() for L in (10, 50, 100)], float)
    assert gone[early].all()
    np.testing.assert_allclose(mix / mix.sum(), np.array([10, 2, 1]) / 13, atol=0.01)


def test_clustered():
    _, comps = datagen.lowrank_points(4, datagen.ROLE_BASE, 20_000, 16, 64)
    ops, first = datagen.clustered_ops(4, comps, 64, rounds=5)
    assert len(ops) == 5 * 2 * 64 and first == 64
    born, died = _replay(ops, len(comps))
    assert (born >= 0).all()                              # every row inserted
    for ins, dele in ops:
        touched = np.concatenate([ins, dele])
        assert len(np.unique(comps[touched])) <= 1        # one cluster per step
        assert len(ins) == 0 or len(dele) == 0            # a step inserts or deletes
