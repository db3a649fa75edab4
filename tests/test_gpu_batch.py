"""Batched persistent apply (mwns_apply_batch) and the hipGraph plan (mwns_plan_*) against the
single applies: the per-brick arithmetic is the same, so results must agree bit for bit."""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_0706_0747_amd as M
    return M


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0)


# uneven members: Poisson, Yukawa and fractional kernels, k = 5, 6, 8, different depths
MEMBERS = [
    dict(seed=21, k=6, eps=1e-4, jmax=5),
    dict(seed=22, k=8, eps=1e-5, jmax=5, mu=3.0),
    dict(seed=23, k=6, eps=1e-3, jmax=4, alpha=0.6),
    dict(seed=24, k=8, eps=1e-6, jmax=4, n=5),
    dict(seed=25, k=5, eps=1e-4, jmax=5, mu=8.0),
    dict(seed=26, k=6, eps=1e-4, jmax=6, n=1),
]


def _member(M, ctx, spec):
    w = workloads.small_adaptive(**spec)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth)
    return w, f, op


@pytest.fixture(scope="module")
def batch(M, ctx):
    return [_member(M, ctx, s) for s in MEMBERS]


def test_batch_equals_single_applies(M, ctx, batch):
    singles, count = [], 0
    for w, f, op in batch:
        g, st = M.mwns_apply(ctx, op, f)
        singles.append(M.mwns_tree_export(ctx, g)[2])
        count += st["contractions"]
    gs, st = M.mwns_apply_batch(ctx, [op for _, _, op in batch], [f for _, f, _ in batch])
    assert st["contractions"] == count
    for i, g in enumerate(gs):
        assert np.array_equal(M.mwns_tree_export(ctx, g)[2], singles[i]), "member %d" % i


def test_routed_batch_equals_routed_singles(M, ctx, batch):
    tols = []
    for w, f, op in batch:
        _, st = M.mwns_apply(ctx, op, f)
        tols.append(w.eps * st["g_norm"])
    singles = [M.mwns_tree_export(ctx, M.mwns_apply_mixed(ctx, op, f, tol)[0])[2]
               for (w, f, op), tol in zip(batch, tols)]
    gs, st = M.mwns_apply_batch(ctx, [op for _, _, op in batch], [f for _, f, _ in batch], mixed=tols)
    assert 0.0 < st["err_bound"] <= max(tols)
    for i, g in enumerate(gs):
        assert np.array_equal(M.mwns_tree_export(ctx, g)[2], singles[i]), "member %d" % i


def test_set_leaves_round_trip(M, ctx):
    w, f, op = _member(M, ctx, MEMBERS[0])
    keys, leaf, coef = M.mwns_tree_export(ctx, f)
    M.mwns_tree_set_leaves(ctx, f, 2.0 * coef[leaf == 1])
    _, _, coef2 = M.mwns_tree_export(ctx, f)
    assert np.array_equal(coef2, 2.0 * coef)       # decomposition is linear; scaling by 2 is exact


@pytest.mark.parametrize("routed", [False, True])
def test_plan_replays_match_applies(M, ctx, routed):
    """Three replays of the captured graph, the inputs changed in place before the second, eager
    applies and synchronisations between replays: every replay equals the direct apply."""
    import torch
    members = [_member(M, ctx, s) for s in MEMBERS[:4]]
    ops = [op for _, _, op in members]
    fs = [f for _, f, _ in members]
    tols = None
    if routed:
        tols = [w.eps * M.mwns_apply(ctx, op, f)[1]["g_norm"] for w, f, op in members]
    plan = M.mwns_plan_create(ctx, ops, fs, mixed=tols)
    rng = np.random.Generator(np.random.PCG64(41))
    for rep in range(3):
        if rep == 1:
            for f in fs:
                _, leaf, coef = M.mwns_tree_export(ctx, f)
                # a new input of the same structure, within the norms the routing was made for
                M.mwns_tree_set_leaves(ctx, f, coef[leaf == 1] * rng.uniform(0.5, 1.0, (int(leaf.sum()), 1, 1, 1)))
        plan.execute()
        torch.cuda.synchronize()
        outs = [M.mwns_tree_export(ctx, plan.output(i))[2] for i in range(len(members))]
        if routed:
            # the plan keeps its creation-time routing; a fresh routed batch at the same tols routes
            # the new inputs by their own (smaller) norms, so compare against FP64 within the bound
            for i, (w, f, op) in enumerate(members):
                ref = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])
                err = math.sqrt(float(np.sum((outs[i] - ref[2])[ref[1] == 1] ** 2)))
                assert err <= tols[i], (i, err, tols[i])
        else:
            refs = [M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])[2] for _, f, op in members]
            for i in range(len(members)):
                assert np.array_equal(outs[i], refs[i]), "replay %d member %d" % (rep, i)
    st = plan.stats()
    assert st["contractions"] > 0
    plan.close()


def test_autotuner_picks_a_variant_and_caches_it(M, tmp_path):
    """mwns_tune_apply times every tile variant and sets the fastest; the apply after tuning is
    bit-identical to the default one; autotune() reuses the cached choice."""
    c = M.Context(0)
    w, f, op = _member(M, c, MEMBERS[1])
    ref = M.mwns_tree_export(c, M.mwns_apply(c, op, f)[0])[2]
    best, times = M.mwns_tune_apply(c, op, f, reps=2)
    assert 0 <= best < M.mwns_num_variants() and np.all(times > 0.0)
    assert best == int(np.argmin(times)) and M.mwns_ctx_get_variant(c, w.k) == best
    assert np.array_equal(M.mwns_tree_export(c, M.mwns_apply(c, op, f)[0])[2], ref)
    path = str(tmp_path / "tiles.json")
    v1 = M.autotune(c, op, f, cache_path=path, reps=1)
    M.mwns_ctx_set_variant(c, w.k, (v1 + 1) % M.mwns_num_variants())
    assert M.autotune(c, op, f, cache_path=path) == v1 and M.mwns_ctx_get_variant(c, w.k) == v1


def test_device_block_cache_reuse(M):
    """Freed device blocks stay with the context and serve the next apply (results unchanged);
    release_cache hands them back."""
    c = M.Context(0)
    w, f, op = _member(M, c, MEMBERS[1])
    g, _ = M.mwns_apply(c, op, f)
    ref = M.mwns_tree_export(c, g)[2]
    g.close()
    cached = c.bytes_cached()
    assert cached > 0
    live = c.bytes_in_use()
    g2, _ = M.mwns_apply(c, op, f)
    assert np.array_equal(M.mwns_tree_export(c, g2)[2], ref)
    assert c.bytes_cached() <= cached and c.bytes_in_use() >= live
    c.release_cache()
    assert c.bytes_cached() == 0
