"""Warm-start plumbing on the oracle evaluator (CPU only): feature/target
layout, the rule that turns a prediction into an IPM start, rejection of
non-finite predictions, and the cold fallback in the comparison."""
import numpy as np

from paper_2509_22462_amd import datagen, ipm, warmstart
from test_ipm import OracleEval

DIMS = (64, 32, 32, 5)
ACTS = ["tanh", "tanh", "identity"]


def setup():
    Ws, bs = datagen.mlp_weights(DIMS, seed=5)
    ev = OracleEval(Ws, bs, ACTS)
    probs = warmstart.make_problems(ev.nn, 8, seed=3, m=5, side=8)
    return ev, probs


def test_problem_generation_and_layouts():
    ev, probs = setup()
    for p in probs:
        assert p.t != p.c
        assert p.c == int(np.argmax(ev.nn(p.x0[None])[0]))
        assert p.x0.shape == (64,) and np.all((p.x0 >= 0) & (p.x0 <= 1))
    F = warmstart.features(probs, 5)
    assert F.shape == (8, 69)
    assert np.all(F[:, 64:].sum(axis=1) == 0) and np.all(np.abs(F[:, 64:]).sum(axis=1) == 2)
    res = ipm.solve_batch(probs, ev)
    Y = warmstart.targets(res)
    assert Y.shape == (8, 64 + 10)
    np.testing.assert_array_equal(Y[0, :64], res[0].x)


def test_good_prediction_cuts_iterations_and_keeps_the_optimum():
    ev, probs = setup()
    cold = ipm.solve_batch(probs, ev)
    starts = [warmstart.start_from_prediction(p, np.concatenate([r.x, r.y, r.lam]), 64, 5, 1e-2)
              for p, r in zip(probs, cold)]
    cmp_ = warmstart.compare(probs, starts, ev)
    assert cmp_.fallbacks == 0 and cmp_.rejected == 0
    assert cmp_.warm_iters.mean() < 0.7 * cmp_.cold_iters.mean()
    assert np.max(np.abs(cmp_.warm_obj - cmp_.cold_obj)) < 1e-4


def test_nonfinite_prediction_is_rejected_and_failures_fall_back():
    ev, probs = setup()
    row = np.full(74, np.nan)
    assert warmstart.start_from_prediction(probs[0], row, 64, 5, 1e-2) is None
    # a start whose multipliers are absurd: the warm solve may fail; the
    # comparison must still return converged (cold) results
    bad = ipm.Start(x=np.ones(64), lam=np.full(5, 1e6), nu=-1e6, mu0=1e-8)
    cmp_ = warmstart.compare(probs[:2], [None, bad], ev, opts=ipm.Options(max_iter=5))
    assert cmp_.rejected == 1
    assert all(s in ("converged", "max_iter") for s in cmp_.warm_status)


def test_dataset_checkpoint_resume_matches_one_pass(tmp_path):
    """Cold solves stopped by the time budget and resumed from the checkpoint
    give the same dataset as one uninterrupted pass."""
    import argparse

    from paper_2509_22462_amd import warmstart_run as wr

    ev, _ = setup()
    train = warmstart.make_problems(ev.nn, 6, seed=11, m=5, side=8)
    cfg = np.array([6, 0, 2], dtype=np.float64)
    opts = ipm.Options()
    whole = argparse.Namespace(out=str(tmp_path / "whole.npz"), chunk=2, max_seconds=0.0)
    d1, done1 = wr.build_dataset(train, ev, opts, whole, 5, cfg)
    assert done1 and int(d1["done"]) == 6
    part = argparse.Namespace(out=str(tmp_path / "part.npz"), chunk=2, max_seconds=1e-9)
    d2, done2 = wr.build_dataset(train, ev, opts, part, 5, cfg)
    assert not done2 and int(d2["done"]) == 2  # the budget is checked between chunks
    part.max_seconds = 0.0
    d3, done3 = wr.build_dataset(train, ev, opts, part, 5, cfg)
    assert done3
    for k in ("F", "Y", "iters", "ok"):
        np.testing.assert_array_equal(d3[k], d1[k])
    # a checkpoint of another configuration is not reused
    assert wr.load_checkpoint(part.out, np.array([7, 0, 2.0])) is None
