"""Pins of the oracle parts used by the learned entry/stop form: the FP64
predictor network (finite differences, closed forms) and search from given
entry points with expansion caps (brute force, invariants)."""
import numpy as np
import pytest

import oracle as O
from paper_2601_08528_amd import datagen


def rand_mlp(rng, din=12, h=16, nc=5, scale=0.4):
    return O.MLP(rng.standard_normal((din, h)) * scale, rng.standard_normal(h) * 0.1,
                 rng.standard_normal((h, h)) * scale, rng.standard_normal(h) * 0.1,
                 rng.standard_normal((h, nc + 1)) * scale, rng.standard_normal(nc + 1) * 0.1)


def test_mlp_gradients_match_central_differences():
    rng = np.random.Generator(np.random.Philox(21))
    m = rand_mlp(rng)
    x = rng.standard_normal((7, m.din))
    lab = rng.integers(0, m.nc, 7)
    ls = rng.standard_normal(7)
    loss, g = m.loss_grad(x, lab, ls, lam=0.3, delta=0.5)
    eps = 1e-6
    for t in range(6):
        flat = m.p[t].reshape(-1)
        for idx in rng.choice(flat.size, min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = m.loss_grad(x, lab, ls, lam=0.3, delta=0.5)
            flat[idx] = old - eps
            lm, _ = m.loss_grad(x, lab, ls, lam=0.3, delta=0.5)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[t].reshape(-1)[idx]) <= 1e-6 + 1e-5 * abs(fd)


def test_mlp_closed_form_with_zero_weights():
    """All weights zero: outputs equal b3; the cross-entropy gradient on b3 is
    mean(softmax(b3) - onehot), and Huber in its linear range gives
    lambda * delta * sign."""
    din, h, nc = 6, 8, 4
    b3 = np.array([0.5, -1.0, 2.0, 0.0, 3.0])
    m = O.MLP(np.zeros((din, h)), np.zeros(h), np.zeros((h, h)), np.zeros(h),
              np.zeros((h, nc + 1)), b3)
    x = np.ones((3, din))
    np.testing.assert_array_equal(m.forward(x), np.tile(b3, (3, 1)))
    lab = np.array([0, 2, 2])
    ls = np.array([0.0, 10.0, 3.0])       # residuals 3, -7, 0: delta = 1
    loss, g = m.loss_grad(x, lab, ls, lam=0.5, delta=1.0)
    sm = np.exp(b3[:4]) / np.exp(b3[:4]).sum()
    want = np.zeros(5)
    for l in lab:
        want[:4] += sm - np.eye(4)[l]
    want[4] = 0.5 * (1.0 + (-1.0) + 0.0)
    np.testing.assert_allclose(g[5], want / 3, rtol=1e-12, atol=1e-15)
    ce = np.mean([np.log(np.exp(b3[:4]).sum()) - b3[l] for l in lab])
    hub = 0.5 * np.mean([(3 - 0.5), (7 - 0.5), 0.0])
    assert abs(loss - (ce + hub)) < 1e-12
    for t in range(5):
        assert not g[t].any()


@pytest.fixture(scope="module")
def idx():
    base, q = datagen.gmm_uint8_valued(401, 500, 30, 16, 5)
    ix = O.OracleIndex(16, 8, O.L2, seed=3)
    ix.build(base, batch_max=100)
    return ix, base, q


def test_listed_entries_all_ids_give_bruteforce(idx):
    ix, base, q = idx
    ent = np.tile(np.arange(500, dtype=np.int32), (q.shape[0], 1))
    ids, d, ne = ix.search_listed(q, 10, 500, ent)
    gi, gd = O.bruteforce(base, q, 10)
    np.testing.assert_array_equal(ids, gi)
    np.testing.assert_array_equal(d, gd)


def test_listed_without_usable_ids_is_plain_search(idx):
    ix, base, q = idx
    ent = -np.ones((q.shape[0], 4), np.int32)
    a = ix.search_listed(q, 10, 24, ent)
    b = ix.search(q, 10, 24)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[2], b[2]["n_exp"])


def test_expansion_caps(idx):
    ix, base, q = idx
    ent = np.tile(np.arange(0, 500, 7, dtype=np.int32), (q.shape[0], 1))
    caps = np.arange(q.shape[0], dtype=np.int32) % 5
    ids, d, ne = ix.search_listed(q, 5, 24, ent, caps)
    assert ((ne <= caps) | (caps == 0)).all()


def test_stop_step_label_is_where_topk_settles(idx):
    """Capping a search at the recorded stopping step leaves its top-k as is."""
    ix, base, q = idx
    ids, lc = ix.search_trace(q, 10, 32)
    ref = ix.search(q, 10, 32)
    np.testing.assert_array_equal(ids, ref[0])
    assert (lc <= ref[2]["iters"]).all() and (lc >= 0).all()
    for i in range(q.shape[0]):
        ix.set("max_iters", max(int(lc[i]), 1))
        capped = ix.search(q[i:i + 1], 10, 32)
        np.testing.assert_array_equal(capped[0][0], ref[0][i])
    ix.set("max_iters", 0)


def test_wavp_hand_worked():
    """Alg. 2 worked by hand: the victim is the first slot in clock order
    whose bit is clear and whose prediction is the minimum over clear bits;
    the second case separates this from "the first vector predicted below
    the candidate" and covers the sweep with every bit set."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "wavp_example.json")))
    for c in g["cases"]:
        hits, slots = O.wavp_replay(c["n"], c["C"], c["e_in"], np.ones(c["n"], np.uint8),
                                    c["batches"], c["alpha"], c["beta"], c["theta"],
                                    c["promote_max"])
        assert hits.tolist() == c["expect_hits"]
        assert slots.tolist() == c["expect_slots"]


def test_wavp_threshold_and_indegree_terms():
    """theta above every prediction keeps the cache empty; with no recency,
    in-degree alone orders the candidates (Eq. 2): ln 201 and ln 51 fill the
    two slots, then ln 8 replaces the minimum ln 51 and ln 2 replaces ln 8,
    since Alg. 2 admits every candidate above theta whatever its rank."""
    hits, slots = O.wavp_replay(4, 2, [0, 0, 0, 0], np.ones(4, np.uint8), [[0, 1, 2, 3]] * 3,
                                theta=10.0)
    assert (slots == -1).all() and (hits == 0).all()
    e_in = [1, 50, 7, 200]
    hits, slots = O.wavp_replay(4, 2, e_in, np.ones(4, np.uint8), [[0, 1, 2, 3]], alpha=0.0,
                                beta=1.0, theta=0.0)
    assert slots.tolist() == [3, 0]
    hits, slots = O.wavp_replay(4, 2, e_in, np.ones(4, np.uint8), [[0, 1, 2, 3]], alpha=0.0,
                                beta=1.0, theta=2.1)
    assert slots.tolist() == [3, 1]                      # ln 8 and ln 2 stay below theta


def test_wavp_theta_adaptation_hand_worked():
    """Sec. 4.4: theta rises when the miss rate and the mean prediction of
    the missed vectors both rise, falls back (never below its start) when
    both fall, and holds otherwise.  alpha = 1, beta = 0, one slot:
      batch 0: miss rate 1/1, mean F 1 (vector 0): no previous batch, 0.5;
      batch 1: rate 3/4 fell, mean F(1) = 3 rose: 0.5 held;
      batch 2: rate 8/8 rose, mean of F(2) = F(3) = 4 rose: theta 1.0;
      batch 3: rate 1/1 equal: 1.0 held, and vector 4 (F = 1) is not above it,
      so 3 stays; with the adaptation off, 4 replaces 3."""
    b = [[0], [0, 1, 1, 1], [2, 2, 2, 2, 3, 3, 3, 3], [4]]
    hits, slots, th = O.wavp_replay(5, 1, [0] * 5, np.ones(5, np.uint8), b, alpha=1.0, beta=0.0,
                                    theta=0.5, adapt=2.0, with_theta=True)
    assert th.tolist() == [0.5, 0.5, 1.0, 1.0]
    assert hits.tolist() == [0, 1, 0, 0] and slots.tolist() == [3]
    hits, slots, th = O.wavp_replay(5, 1, [0] * 5, np.ones(5, np.uint8), b, alpha=1.0, beta=0.0,
                                    theta=0.5, with_theta=True)
    assert th.tolist() == [0.5] * 4 and slots.tolist() == [4]
    # both fall: batch 3 of [3, 0] halves theta back to its start
    b2 = [[0], [0, 1, 1, 1], [2, 2, 2, 2, 3, 3, 3, 3], [3, 0]]
    hits, slots, th = O.wavp_replay(4, 1, [0] * 4, np.ones(4, np.uint8), b2, alpha=1.0, beta=0.0,
                                    theta=0.5, adapt=2.0, with_theta=True)
    assert th.tolist() == [0.5, 0.5, 1.0, 0.5] and hits.tolist() == [0, 1, 0, 1]
    assert slots.tolist() == [0]


def test_wavp_warm_start_hand_worked():
    """Cold-start placement: alive vectors by in-degree (ties by id) fill the
    slots in order; then one batch worked by hand with theta = 0.5:
    F(3) = 0.6*1 + 0.4*ln 2 = 0.877 is above theta; among the clear bits
    (slot 1: F(2) = 0.4*ln 10 = 0.921, slot 2: F(0) = 0.4*ln 5 = 0.644) the
    minimum is F(0); the hand clears slot 0's bit (vector 1, just hit), passes
    slot 1 and replaces 0.  With theta = 1.0 vector 3 stays on the host."""
    e_in = [4, 9, 9, 1, 7]
    alive = np.array([1, 1, 1, 1, 0], np.uint8)        # vector 4 is deleted
    hits, slots = O.wavp_replay(5, 3, e_in, alive, [], warm=True)
    assert slots.tolist() == [1, 2, 0]
    hits, slots = O.wavp_replay(5, 3, e_in, alive, [[3, 1]], theta=0.5, warm=True)
    assert hits.tolist() == [1] and slots.tolist() == [1, 2, 3]
    hits, slots = O.wavp_replay(5, 3, e_in, alive, [[3, 1]], theta=1.0, warm=True)
    assert hits.tolist() == [1] and slots.tolist() == [1, 2, 0]


def test_expansion_trace_matches_search(idx):
    ix, base, q = idx
    tr, cnt = ix.search_expansions(q, 24)
    ref = ix.search(q, 10, 24)
    np.testing.assert_array_equal(cnt, ref[2]["n_exp"])
    for i in range(q.shape[0]):
        t = tr[i, :cnt[i]]
        assert len(set(t.tolist())) == len(t)        # each vertex expanded once


def test_classic_policies_hand_worked():
    """LRU, LFU and LRFU in the batched form, worked by hand."""
    ones = lambda n: np.ones(n, np.uint8)
    # LRU, two slots: batch 0 admits 2, 1, then 0 evicts 1 (oldest of 2 and 1);
    # batch 1 admits 3 (evicts 0) and 1 (evicts 2)
    h, s = O.policy_replay(O.POLICY_LRU, 6, 2, [0] * 6, ones(6), [[0, 1, 2], [1, 3]])
    assert h.tolist() == [0, 0] and s.tolist() == [1, 3]
    # LFU: 0 (2 accesses) and 1 (1) fill the slots; in batch 1 vector 1 hits
    # once, both have 2 accesses and the larger id (1) goes for 2
    h, s = O.policy_replay(O.POLICY_LFU, 3, 2, [0] * 3, ones(3), [[0, 0, 1], [2, 2, 2, 1]])
    assert h.tolist() == [0, 1] and s.tolist() == [0, 2]
    # recency against recency-frequency on one stream: LRU admits 4 (latest)
    # before 5 and later evicts 5 (accessed earlier in batch 0); LRFU admits 5
    # (F_recent 3) before 4 and evicts 4 (F_recent 0.5 against 1.5)
    tr = [[5, 5, 5, 4], [6]]
    h, s = O.policy_replay(O.POLICY_LRU, 7, 2, [0] * 7, ones(7), tr)
    assert s.tolist() == [4, 6]
    h, s = O.policy_replay(O.POLICY_LRFU, 7, 2, [0] * 7, ones(7), tr)
    assert s.tolist() == [5, 6]
    # promote_max 0: nothing moves after the warm start
    h, s = O.policy_replay(O.POLICY_LRU, 7, 2, [3, 9, 1, 0, 0, 0, 0], ones(7), tr, promote_max=0,
                           warm=True)
    assert s.tolist() == [1, 0] and h.tolist() == [0, 0]


def test_model_gating_hand_worked():
    """The learned form's gating, worked by hand: the first largest logit
    picks the cluster; its softmax probability against the threshold picks
    listed or plain search; the cap is ceil(scale * exp(z_stop)) with z_stop
    taken at most 20, at least min_iters, and held at 2^30."""
    z = np.array([
        [2.0, 0.0, 0.0, 2.0],      # p = 1/(1 + 2e^-2) = 0.787 >= 0.5; cap ceil(1.5 e^2 = 11.08) = 12
        [0.0, 0.0, 0.0, 3.0],      # p = 1/3 < 0.5: plain search
        [1.0, 3.0, 3.0, 0.0],      # tie: cluster 1; p = 1/(2 + e^-2) = 0.468 < 0.5
        [0.0, -50.0, -50.0, 0.0],  # p ~ 1; cap ceil(1.5) = 2, raised to min_iters 8
        [5.0, 0.0, 0.0, 30.0],     # z_stop taken at 20: ceil(1.5 e^20) = 727,747,794
    ])
    qe, qm = O.model_decide(z, 0.5, 1.5, 8)
    assert qe.tolist() == [0, -1, -1, 0, 0]
    assert qm.tolist() == [12, 0, 0, 8, int(np.ceil(1.5 * np.exp(20.0)))]
    assert qm[4] == 727747794
    qe, qm = O.model_decide(z[2:3], 0.4, 1.5, 8)           # now confident: the tie's first index
    assert qe.tolist() == [1] and qm.tolist() == [8]
    qe, qm = O.model_decide(z[4:5], 0.0, 1e6, 8)            # 1e6 e^20 = 4.85e14: held at 2^30
    assert qm.tolist() == [1 << 30]
    qe, qm = O.model_decide(np.array([[0.0, 0.0, 0.0]]), 0.5, 1.0, 1)   # p = conf exactly
    assert qe.tolist() == [0]
