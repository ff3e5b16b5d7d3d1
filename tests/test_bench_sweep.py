"""The benchmark's beam selection (host logic, no GPU): the first sweep beam
that reaches the recall target, then bisection on multiples of 8 against
the beam before it.  Search, recall and timing are replaced by a recall
table, so the test checks only which beams are probed and chosen."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    state = {"beam": None, "probed": []}

    def run_search(torch, ix, q_t, beam, bufs):
        state["beam"] = beam
        state["probed"].append(beam)

    monkeypatch.setattr(mod, "run_search", run_search)
    monkeypatch.setattr(mod, "timed_steps", lambda *a, **k: ([1.0, 1.0, 1.0], 0.0))
    monkeypatch.setattr(mod, "log", lambda *a: None)
    return mod, state


class _Torch:
    class cuda:
        @staticmethod
        def synchronize():
            pass


class _Q:
    shape = (10_000, 128)


def _run(bench, recall_of, beams, **kw):
    mod, state = bench
    mod.recall = lambda torch, base_t, q_t, ids, kth: recall_of(state["beam"])
    state["probed"].clear()
    chosen, rows = mod.sweep(_Torch, None, _Q, None, None, (None,), beams, **kw)
    return chosen, rows, list(state["probed"])


def test_bisects_between_the_last_miss_and_the_first_hit(bench):
    # recall rises with the beam and first reaches 0.95 at 84
    rec = lambda b: 0.95 if b >= 84 else 0.90
    chosen, rows, probed = _run(bench, rec, [32, 48, 64, 96, 128])
    assert probed == [32, 48, 64, 96, 80, 88]
    assert chosen == 88                       # smallest multiple of 8 at the target
    assert [r["beam"] for r in rows] == sorted(probed)
    assert all(r["recall@10"] >= 0.95 for r in rows if r["beam"] >= 88)


def test_first_beam_hit_needs_no_bisection(bench):
    chosen, rows, probed = _run(bench, lambda b: 0.99, [32, 48, 64])
    assert (chosen, probed) == (32, [32])


def test_target_never_reached(bench):
    chosen, rows, probed = _run(bench, lambda b: 0.5, [32, 48, 64])
    assert chosen is None and probed == [32, 48, 64]


def test_refine_off_keeps_the_sweep_point(bench):
    rec = lambda b: 0.95 if b >= 84 else 0.90
    chosen, _, probed = _run(bench, rec, [32, 48, 64, 96], refine=0)
    assert (chosen, probed) == (96, [32, 48, 64, 96])


def test_gap_of_one_step_is_not_split(bench):
    rec = lambda b: 0.95 if b >= 40 else 0.90
    chosen, _, probed = _run(bench, rec, [32, 40, 48])
    assert (chosen, probed) == (40, [32, 40])
