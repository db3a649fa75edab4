"""Alg. 3 in two dimensions on the GPU against the d = 2 oracle: the fit, the plan, the adaptive
projection (bit-exact trees), the applied output node by node (the screened plan and random plans on
random trees), evaluation, and the error paths."""
import itertools
import math

import numpy as np
import pytest

from parity_util import per_node_ok

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


def _case(seed, k, eps, n=3, jmax=7, lo=1.5, hi=3.0):
    rng = np.random.default_rng(seed)
    xy = rng.uniform(0.3, 0.7, (n, 2))
    a = 10 ** rng.uniform(lo, hi, n)
    c = rng.normal(size=n)
    return k, eps, xy, a, c, jmax


@pytest.mark.parametrize("mu,alpha,eps", [(5.0, 1.0, 1e-6), (1.0, 1.0, 1e-8), (0.0, 0.5, 1e-6), (3.0, 0.7, 1e-5)])
def test_fit_matches_oracle(M, mu, alpha, eps):
    from oracle import ns2d as N
    delta, R = math.sqrt(eps) * 2.0 ** -8, math.sqrt(2.0)
    tau, w = M.mwns_fit_kernel2d(mu, alpha, eps, delta, R)
    ot, ow = N.fit_kernel2d(mu, alpha, eps, delta, R)
    assert tau.size == ot.size
    assert np.abs(tau / ot - 1).max() < 1e-13 and np.abs(w / ow - 1).max() < 1e-13


@pytest.mark.parametrize("k,eps,mu", [(6, 1e-5, 5.0), (8, 1e-6, 2.0), (4, 1e-3, 8.0)])
def test_plan_matches_oracle(M, ctx, k, eps, mu):
    from oracle import mra
    from oracle import ns2d as N
    nlev = 6
    tau, w = N.fit_kernel2d(mu, 1.0, eps, math.sqrt(eps) * 2.0 ** -nlev, math.sqrt(2.0))
    F = mra.F_table(k, tau, nlev)
    H0, H1 = mra.two_scale_filters(k)
    R, _ = N.make_plan2d(F, H0, H1, w, eps, nlev, allow_overflow=True)
    op = M.mwns_op2d_create(ctx, k, tau, w, eps, nlev, allow_band_overflow=True)
    assert np.array_equal(M.mwns_op2d_plan_export(op), R)


def _keys(tr):
    return tr.keys


@pytest.mark.parametrize("seed,k,eps", [(4, 6, 1e-5), (5, 8, 1e-6), (6, 4, 1e-4), (7, 10, 1e-7)])
def test_projection_and_apply_match_oracle(M, ctx, seed, k, eps):
    """Tree bit-exact; the operator with the oracle's fit and its own plan (equal to the oracle's); g on
    every node within 1e-12 (global and node by node); evaluation at random points."""
    from oracle import mra
    from oracle import ns2d as N
    k, eps, xy, a, c, jmax = _case(seed, k, eps, jmax=6 if k >= 8 else 7)
    tr = N.project2d(k, eps, 2, jmax, xy, a, c)
    f = M.mwns_project2d(ctx, k, eps, 2, jmax, xy, a, c)
    keys, leaf, coef = M.mwns_tree2d_export(ctx, f)
    assert np.array_equal(keys, tr.keys) and np.array_equal(leaf, tr.leaf)
    assert np.abs(coef - tr.coef).max() <= 1e-13 * np.abs(tr.coef).max()
    tau, w = N.fit_kernel2d(5.0, 1.0, eps, math.sqrt(eps) * 2.0 ** -tr.depth, math.sqrt(2.0))
    F = mra.F_table(k, tau, tr.depth)
    H0, H1 = mra.two_scale_filters(k)
    R, _ = N.make_plan2d(F, H0, H1, w, eps, tr.depth, allow_overflow=True)
    g_ref = N.assemble2d(tr, N.apply_modified2d(tr, F, w, R))
    op = M.mwns_op2d_create(ctx, k, tau, w, eps, tr.depth, allow_band_overflow=True)
    assert np.array_equal(M.mwns_op2d_plan_export(op), R)
    g, ms, fl = M.mwns_apply2d(ctx, op, f)
    gk, gl, gc = M.mwns_tree2d_export(ctx, g)
    assert np.array_equal(gk, tr.keys)
    assert np.linalg.norm(gc - g_ref) <= 1e-12 * np.linalg.norm(g_ref)
    assert per_node_ok(gc, g_ref)
    print("k=%d: %d nodes, depth %d, %d terms, contraction %.3f ms, %.3g flops" % (k, tr.keys.size, tr.depth, tau.size, ms, fl),
          flush=True)
    pts = np.random.default_rng(seed).uniform(0.0, 1.0, (300, 2))
    got = M.mwns_tree2d_eval(ctx, g, pts)
    want = N.evaluate2d(tr, g_ref, pts)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def _random_tree(rng, k, depth):
    from oracle import ns2d as N
    leaves, todo = {}, [(1, x, y) for x in range(2) for y in range(2)]
    while todo:
        j, x, y = todo.pop()
        if j < depth and rng.random() < 0.4:
            todo += [(j + 1, 2 * x + sx, 2 * y + sy) for sx in (0, 1) for sy in (0, 1)]
        else:
            leaves[(j, x, y)] = rng.normal(size=(k, k))
    return N.redundant_tree2(k, leaves)


@pytest.mark.parametrize("seed,k", [(1, 3), (2, 5), (3, 8), (4, 1)])
def test_apply_random_trees_random_plans(M, ctx, seed, k):
    from oracle import mra
    from oracle import ns2d as N
    rng = np.random.default_rng(seed)
    tr = _random_tree(rng, k, 5)
    tau, w = N.fit_kernel2d(3.0, 1.0, 1e-4, 1e-4, math.sqrt(2.0))
    tau, w = tau[:40], w[:40]
    F = mra.F_table(k, tau, tr.depth)
    R = np.zeros((tr.depth + 1, 7, 7, 2), dtype=np.int32)
    R[..., 1] = -1
    R[0, 3, 3] = (0, tau.size - 1)
    for j in range(1, tr.depth + 1):
        for L in itertools.product(range(7), repeat=2):
            if rng.random() < 0.8:
                m1 = int(rng.integers(0, tau.size))
                R[j, L[0], L[1]] = (m1, min(tau.size - 1, m1 + int(rng.integers(0, 15))))
    g_ref = N.assemble2d(tr, N.apply_modified2d(tr, F, w, R))
    lf = tr.leaf == 1
    f = M.mwns_tree2d_from_leaves(ctx, k, tr.keys[lf], tr.coef[lf])
    keys, leaf, coef = M.mwns_tree2d_export(ctx, f)
    assert np.array_equal(keys, tr.keys) and np.abs(coef - tr.coef).max() <= 1e-13 * np.abs(tr.coef).max()
    op = M.mwns_op2d_create(ctx, k, tau, w, 1e-4, tr.depth, allow_band_overflow=True)
    M.mwns_op2d_plan_import(op, R)
    g, _, _ = M.mwns_apply2d(ctx, op, f)
    _, _, gc = M.mwns_tree2d_export(ctx, g)
    assert np.linalg.norm(gc - g_ref) <= 1e-12 * np.linalg.norm(g_ref)
    assert per_node_ok(gc, g_ref)


def test_apply_against_the_fitted_kernel_in_closed_form(M, ctx):
    """The library's own fit, plan, projection and apply: the potential on a grid within eps ||f||_2
    of the fitted kernel applied in closed form to the square-truncated source."""
    from oracle import ns2d as N
    k, eps, xy, a, c, jmax = _case(9, 8, 1e-6, n=5, jmax=10, lo=1.0, hi=3.5)
    f = M.mwns_project2d(ctx, k, eps, 2, jmax, xy, a, c)
    keys, leaf, _ = M.mwns_tree2d_export(ctx, f)
    depth = int((keys >> np.uint64(57)).max())
    tau, w = M.mwns_fit_kernel2d(5.0, 1.0, eps, math.sqrt(eps) * 2.0 ** -depth, math.sqrt(2.0))
    op = M.mwns_op2d_create(ctx, k, tau, w, eps, depth)
    g, ms, fl = M.mwns_apply2d(ctx, op, f)
    gx, gy = np.linspace(0.03, 0.97, 25), np.linspace(0.02, 0.98, 23)
    ref = N.fitted_truncated2d(tau, w, xy, a, c, gx, gy)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    val = M.mwns_tree2d_eval(ctx, g, np.stack([X.ravel(), Y.ravel()], 1)).reshape(ref.shape)
    bound = eps * N.source_norm2d(xy, a, c)
    print("%d leaves, depth %d: max error %.3e against eps ||f|| = %.3e" % (int(leaf.sum()), depth, np.abs(val - ref).max(), bound))
    assert np.abs(val - ref).max() <= bound


def test_error_paths(M, ctx):
    from paper_0706_0747_amd import _lib
    with pytest.raises(M.MwnsError) as e:
        M.mwns_fit_kernel2d(0.0, 1.0, 1e-6, 1e-4, 1.0)          # the plane's Poisson kernel diverges
    assert e.value.status == _lib.MWNS_EINVAL
    tau, w = M.mwns_fit_kernel2d(5.0, 1.0, 1e-4, 1e-4, 1.5)
    with pytest.raises(M.MwnsError) as e:
        M.mwns_op2d_create(ctx, 11, tau, w, 1e-4, 4)
    assert e.value.status == _lib.MWNS_EINVAL
    f = M.mwns_project2d(ctx, 6, 1e-4, 2, 6, [[0.5, 0.5]], [300.0], [1.0])
    op5 = M.mwns_op2d_create(ctx, 5, tau, w, 1e-4, 6, allow_band_overflow=True)
    with pytest.raises(M.MwnsError) as e:
        M.mwns_apply2d(ctx, op5, f)
    assert e.value.status == _lib.MWNS_EINVAL
    with pytest.raises(M.MwnsError) as e:
        M.mwns_tree2d_eval(ctx, f, [[0.5, 1.5]])
    assert e.value.status == _lib.MWNS_EINVAL
    with pytest.raises(M.MwnsError) as e:
        M.mwns_op2d_plan_import(op5, np.zeros(3, dtype=np.int32))
    assert e.value.status == _lib.MWNS_EINVAL
