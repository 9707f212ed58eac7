"""GPU tests of batched FastFCA-AS (many mixtures of uneven N, I, J advanced
together, one launch per (I, J) group per batch step, recorded as a HIP
graph), against the FP64 oracle and against single-mixture contexts."""

import numpy as np
import pytest

from paper_1805_09498_amd import synth
from tests.gpu_common import (TOL_PARAM, check_as_params, oracle_as_bounded, params, problem, rel, run_as,
                              sub_problem, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available()
    from paper_1805_09498_amd import fastfca
    return fastfca


def uneven_batch(n_mix, F, seed, n_range=(40, 700)):
    """Mixtures with N ~ U[n_range], I in {2,3,4,6}, J ~ U[2, I+1] (the uneven
    batch recipe at a reduced size), rounded to single precision."""
    return [p.rounded_c64() for p in synth.make_batch(n_mix=n_mix, F=F, seed=seed, n_range=n_range)]


def batch_of(ff, probs, graph=1):
    tens = [to_dev(p) for p in probs]
    b = ff.fca_batch_init([(t["x"], t["v0"], t["lam0"], t["P0"]) for t in tens])
    ff.fca_batch_set_option(b, "graph", graph)
    return b, tens


def test_batch_matches_oracle_per_mixture(ff):
    probs = uneven_batch(8, 9, seed=7)
    b, _ = batch_of(ff, probs)
    ff.fca_batch_iterate(b, 1)
    for m, p in enumerate(probs):
        check_as_params(params(ff, ff.fca_batch_context(b, m)), oracle_as_bounded(p, 1),
                        tag=f" batch mixture {m} {p.shape}")


def test_batch_equals_single_contexts_at_the_same_shape(ff):
    """Each mixture of the batch is advanced by the same workgroup body as a
    single context with the group's wave count and one bin per workgroup."""
    probs = uneven_batch(6, 5, seed=8)
    b, _ = batch_of(ff, probs)
    ff.fca_batch_iterate(b, 4)
    ngroups = ff.fca_batch_get_option(b, "groups")
    waves = {}
    for g in range(ngroups):
        waves[(ff.fca_batch_get_option(b, "group_I", g), ff.fca_batch_get_option(b, "group_J", g))] = \
            ff.fca_batch_get_option(b, "group_waves", g)
    for m, p in enumerate(probs):
        F, N, I, J = p.shape
        w = waves[(I, J)]
        if w == 0:
            continue
        single = run_as(ff, p, 4, path=1, waves=w, bpw=1)
        a = params(ff, ff.fca_batch_context(b, m))
        s = params(ff, single)
        for x, y in zip(a, s):
            assert rel(x, y) <= 1e-6, (m, p.shape, w)


def test_graph_and_direct_launches_agree_bitwise(ff):
    probs = uneven_batch(5, 4, seed=9)
    out = []
    for graph in (1, 0):
        b, _ = batch_of(ff, probs, graph=graph)
        ff.fca_batch_set_option(b, "autotune", 0)
        ff.fca_batch_iterate(b, 3)
        out.append([params(ff, ff.fca_batch_context(b, m)) for m in range(len(probs))])
    for ma, mb in zip(*out):
        for x, y in zip(ma, mb):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("graph", [1, 0])
def test_work_queue_equals_one_workgroup_per_tile_bitwise(ff, graph):
    """The persistent work-queue launch (option "queue") gives the bits of
    the one-workgroup-per-tile launch: same tiles, same workgroup body; the
    device counter is reset before every launch (4 + 2 iterations in two
    calls, replayed graphs included)."""
    probs = uneven_batch(7, 6, seed=12)
    out = []
    for queue in (0, 1):
        b, _ = batch_of(ff, probs, graph=graph)
        ff.fca_batch_set_option(b, "autotune", 0)
        ff.fca_batch_set_option(b, "queue", queue)
        assert ff.fca_batch_get_option(b, "queue") == queue
        ff.fca_batch_iterate(b, 4)
        ff.fca_batch_iterate(b, 2)
        queued = [ff.fca_batch_get_option(b, "group_queued", g) for g in range(ff.fca_batch_get_option(b, "groups"))]
        # groups whose queue kernel would need scratch memory keep the first form
        assert (max(queued) == 1) if queue else (max(queued) == 0), queued
        out.append([params(ff, ff.fca_batch_context(b, m)) for m in range(len(probs))])
    for ma, mb in zip(*out):
        for x, y in zip(ma, mb):
            np.testing.assert_array_equal(x, y)


def test_split_iterations_equal_one_call_bitwise(ff):
    """3 + 3 batch iterations (two graph replays) equal 6 in one call: the
    state written back between launches is the state kept in registers."""
    probs = uneven_batch(4, 4, seed=10)
    b1, _ = batch_of(ff, probs)
    ff.fca_batch_set_option(b1, "autotune", 0)
    ff.fca_batch_iterate(b1, 3)
    ff.fca_batch_iterate(b1, 3)
    b2, _ = batch_of(ff, probs)
    ff.fca_batch_set_option(b2, "autotune", 0)
    ff.fca_batch_iterate(b2, 6)
    for m in range(len(probs)):
        for x, y in zip(params(ff, ff.fca_batch_context(b1, m)), params(ff, ff.fca_batch_context(b2, m))):
            np.testing.assert_array_equal(x, y)


def test_full_size_uneven_batch_sampled(ff):
    """The uneven-batch workload at full size (64 mixtures, F = 513,
    N ~ U[200, 2000]), one batch step of 2 iterations, sampled mixtures and
    bins against the oracle."""
    probs = [p.rounded_c64() for p in synth.make_batch(n_mix=64, F=513, seed=4000)]
    b, _ = batch_of(ff, probs)
    ff.fca_batch_iterate(b, 2)
    rng = np.random.default_rng(0)
    for m in (0, 17, 42, 63):
        p = probs[m]
        bins = np.sort(rng.choice(p.shape[0], size=3, replace=False))
        v, lam, P = params(ff, ff.fca_batch_context(b, m))
        check_as_params((v[bins], lam[bins], P[bins]), oracle_as_bounded(sub_problem(p, bins), 2),
                        tag=f" full batch mixture {m} {p.shape}")


def test_batch_options_and_errors(ff):
    probs = uneven_batch(2, 3, seed=11)
    b, _ = batch_of(ff, probs)
    for key, val in [("graph", 2), ("queue", 2), ("waves", 3), ("K", 0), ("nope", 1)]:
        with pytest.raises(ff.FcaError):
            ff.fca_batch_set_option(b, key, val)
    with pytest.raises(ff.FcaError):
        ff.fca_batch_context(b, 2)
    ctx = ff.fca_batch_context(b, 0)
    with pytest.raises(ValueError):
        ff.fca_destroy(ctx)          # owned by the batch
