"""The learned entry/stop form: the predictor's forward pass and gradients
against the FP64 oracle, its training, the listed-entry search step against
the oracle bit for bit, and what the trained predictor gains over plain
search."""
import numpy as np
import pytest

import oracle as O
import paper_2601_08528_amd as svf
from paper_2601_08528_amd import datagen
from gpu_util import gpu_from_oracle, oracle_index

pytestmark = pytest.mark.gpu

# BF16 keeps 8 significant bits: unit roundoff u = 2^-8.  Activations are
# rounded once per layer (two hidden layers, then the gradients on the way
# back), so relative errors of a few u are expected; 8u bounds them.
BF16_REL = 8 * 2.0 ** -8


def random_params(m, rng):
    p = m.get_params()
    parts = m.split(p.copy())
    for i in (1, 3, 5):
        parts[i][:] = rng.standard_normal(parts[i].shape) * 0.05
    p = np.concatenate([a.reshape(-1) for a in parts]).astype(np.float32)
    m.set_params(p)
    return m.get_params()           # weights now on the BF16 grid


def test_mlp_forward_matches_oracle():
    rng = np.random.Generator(np.random.Philox(31))
    m = svf.Mlp(128, 256, 64, seed=3)
    p = random_params(m, rng)
    x, _ = datagen.gmm_uint8_valued(501, 300, 1, 128, 8)
    x = x / 64.0                    # exact in BF16 (integers / power of two)
    ref = O.MLP(*m.split(p.astype(np.float64))).forward(x.astype(np.float64))
    got = m.forward(x.astype(np.float32))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= BF16_REL, rel
    assert (np.argmax(got[:, :64], 1) == np.argmax(ref[:, :64], 1)).mean() > 0.9


def test_mlp_gradients_match_oracle():
    rng = np.random.Generator(np.random.Philox(32))
    m = svf.Mlp(128, 256, 64, seed=4)
    p = random_params(m, rng)
    x, _ = datagen.gmm_uint8_valued(502, 512, 1, 128, 8)
    x = x / 64.0
    lab = rng.integers(0, 64, 512)
    ls = rng.uniform(0, 5, 512)
    gl, gg = m.loss_grad(x.astype(np.float32), lab, ls.astype(np.float32), lam=0.1, delta=1.0)
    ol, og = O.MLP(*m.split(p.astype(np.float64))).loss_grad(x, lab, ls, lam=0.1, delta=1.0)
    assert abs(gl - ol) <= BF16_REL * abs(ol)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), m.split(gg), og):
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        assert rel <= 2 * BF16_REL, (name, rel)


def test_mlp_training_learns_a_separable_task():
    means = 128 + 32 * datagen.rng(503, 0).standard_normal((8, 32))
    g = np.random.Generator(np.random.Philox(9))
    lab = g.integers(0, 8, 6144)
    x = np.clip(np.rint(means[lab] + 16 * g.standard_normal((6144, 32))), 0, 255) / 64.0
    ls = (lab % 3).astype(np.float32)
    m = svf.Mlp(32, 64, 8, seed=5)
    z0 = m.forward(x[5120:].astype(np.float32))
    l0, _ = m.loss_grad(x[:1024].astype(np.float32), lab[:1024], ls[:1024])
    last = m.train(x[:5120].astype(np.float32), lab[:5120], ls[:5120], epochs=15, batch=256, lr=3e-3)
    z = m.forward(x[5120:].astype(np.float32))
    acc = (np.argmax(z[:, :8], 1) == lab[5120:]).mean()
    assert last < 0.5 * l0
    assert acc > 0.9, acc
    assert np.abs(z[:, 8] - ls[5120:]).mean() < np.abs(z0[:, 8] - ls[5120:]).mean()


def test_listed_entry_search_bit_exact():
    base, q = datagen.gmm_uint8_valued(504, 5000, 120, 64, 16)
    oix = oracle_index(base, 24, seed=2)
    g = gpu_from_oracle(oix, base, seed=2)
    rng = np.random.Generator(np.random.Philox(10))
    ent = rng.integers(-1, 5000, (120, 40)).astype(np.int32)
    ent[:7] = -1                                  # no usable id: random entries
    caps = rng.integers(0, 40, 120).astype(np.int32)
    for beam in (16, 48):
        oi, od, _ = oix.search_listed(q, 10, beam, ent, caps)
        gi, gd = g.search_listed(q, 10, beam, ent, caps)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(gd.astype(np.float64), od)


def test_learned_form_gain_over_plain():
    """200k x 128 integer mixture with 256 components: random entry points
    rarely land in the query's component, so at a small beam the search often
    ends in the wrong one; entry points from the predicted cluster raise
    recall@10 at the same beam."""
    base, q = datagen.gmm_uint8_valued(505, 200_000, 1000, 128, 256)
    train = datagen.training_queries_uint8(505, 50_000, 128, 256)
    g = svf.Index(128, 32, svf.METRIC_L2, seed=1)
    g.build(base)
    loss = g.model_fit(train, 10, 64, n_clusters=256, epochs=8)
    assert np.isfinite(loss)
    gt_i, gt_d = O.bruteforce(base, q, 10, threads=16)
    n = base.shape[0]
    ref = O.OracleIndex(128, 32, O.L2)           # vectors only: exact distances
    ref.import_state(base, -np.ones((n, 32), np.int32), np.full((n, 32), np.inf),
                     np.ones(n, np.uint8))

    def rec(ids):
        return O.recall_at_k(ids, ref.query_dists(q, ids), gt_d, 10)

    beam = 32
    plain = rec(g.search(q, 10, beam)[0])
    g.set_option("use_model", 1)
    g.set_option("model_conf", 0.0)
    g.set_option("model_stop_scale", 1e6)        # entry points only
    learned = rec(g.search(q, 10, beam)[0])
    g.set_option("use_model", 0)
    print("recall@10 at beam", beam, "plain", plain, "learned entries", learned)
    assert learned >= plain + 0.02


@pytest.mark.parametrize("width", [1, 2])
def test_search_trace_labels_match_oracle(width):
    """The stop labels the predictor trains on: per query, the iteration
    after which the top-k ids last changed, from the GPU's plain search and
    from the oracle's, on integer-valued data (every distance exact)."""
    base, q = datagen.gmm_uint8_valued(507, 6000, 150, 128, 24)
    oix = oracle_index(base, 32, seed=7)
    oix.set("search_width", width)
    g = gpu_from_oracle(oix, base, seed=7, search_width=width)
    for k, beam in ((10, 16), (10, 64), (1, 32)):
        oi, olc = oix.search_trace(q, k, beam)
        gi, gd, glc = g.search_trace(q, k, beam)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(glc, olc)
    assert (olc > 0).mean() > 0.5


def _near_integer(x, rel):
    return np.abs(x - np.rint(x)) <= rel * np.maximum(1.0, np.abs(x))


def test_learned_search_replays_through_the_oracle():
    """use_model = 1 end to end: the GPU-trained predictor is exported, its
    outputs z (computed by the same kernels) go through the oracle's gating
    rule (argmax cluster, softmax confidence against the threshold, cap
    max(min_iters, ceil(scale * exp(z_stop)))), and the oracle's listed-entry
    search with those entries and caps must return the GPU's ids and
    distances bit for bit.  Queries whose gating sits within 1e-5 (relative)
    of a decision boundary, where FP32 and FP64 may round the rule's own
    arithmetic apart, are set aside; they must be few."""
    base, q = datagen.gmm_uint8_valued(506, 12_000, 600, 64, 32)
    train = datagen.training_queries_uint8(506, 4096, 64, 32)
    oix = oracle_index(base, 24, seed=6)
    g = gpu_from_oracle(oix, base, seed=6)
    g.model_fit(train, 10, 32, n_clusters=16, epochs=4)
    params, lists = g.model_get()
    assert lists.shape[0] == 16 and (lists >= -1).all() and (lists < 12_000).all()
    m = svf.Mlp(64, 256, 16)
    m.set_params(params)
    z = m.forward(q).astype(np.float64)
    nc = 16
    zc = z[:, :nc]
    zs = np.sort(zc, axis=1)
    p = 1.0 / np.exp(zc - zs[:, -1:]).sum(axis=1)
    # the threshold: the middle of the widest gap between consecutive
    # confidences among the middle 60% of queries, so that between 20% and
    # 80% of them fall back and none sits next to the threshold
    ps = np.sort(p)
    lo, hi = int(0.2 * len(ps)), int(0.8 * len(ps))
    j = lo + int(np.argmax(np.diff(ps[lo:hi + 1])))
    conf = float(0.5 * (ps[j] + ps[j + 1]))
    scale, min_iters = 1.0, 4
    qe, qm = O.model_decide(z, conf, scale, min_iters)
    assert 0.2 <= (qe < 0).mean() <= 0.8
    capv = scale * np.exp(np.minimum(z[:, nc], 20.0))
    c1 = (zs[:, -1] - zs[:, -2]) > 1e-5 * np.maximum(1.0, np.abs(zs[:, -1]))
    c2 = np.abs(p - conf) > 1e-5 * conf
    # the ceiling decides the cap only above min_iters, and a cap above the
    # number of alive vectors never binds (each expansion takes a new vertex)
    c3 = ~_near_integer(capv, 1e-5) | (capv < min_iters - 0.5) | (capv > 12_001)
    safe = c1 & c2 & c3
    assert safe.mean() > 0.9, (c1.mean(), c2.mean(), c3.mean(), ps[::60], conf)
    qs = q[safe]
    ent = np.where(qe[safe, None] >= 0, lists[np.maximum(qe[safe], 0)], -1).astype(np.int32)
    g.set_option("use_model", 1)
    g.set_option("model_conf", conf)
    g.set_option("model_stop_scale", scale)
    g.set_option("model_min_iters", min_iters)
    for beam in (16, 48):
        oi, od, _ = oix.search_listed(qs, 10, beam, ent, qm[safe])
        gi, gd = g.search(qs, 10, beam)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(gd.astype(np.float64), od)
        assert g.stats()["last_model_fallback"] == int((qe[safe] < 0).sum())
    gated = safe & (qe >= 0)
    assert (qm[gated] > 0).all()                       # gated queries run with a cap
    print("gated %d, of which capped below 12000 expansions: %d; fallback %d"
          % (gated.sum(), (qm[gated] <= 12_000).sum(), (safe & (qe < 0)).sum()))
    g.set_option("use_model", 0)
