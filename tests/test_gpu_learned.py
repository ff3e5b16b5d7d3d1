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
