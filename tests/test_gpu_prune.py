"""Detail norms and l2 pruning of the library (App. A.2-A.3, Sec. 2.2, Alg. 3 Step 4) against the
oracle: the norms node by node, the pruned trees' structure bit-exact, their coefficients those of
the kept nodes, the removed norm within the budget; and Step 4's discard on an applied output."""
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


CASES = {
    "k4": lambda: workloads.small_adaptive(3, k=4, eps=1e-4, jmax=5),
    "k6": lambda: workloads.small_adaptive(11, k=6, eps=1e-4, jmax=5),
    "k10": lambda: workloads.small_adaptive(31, k=10, eps=1e-7, jmax=4),
}


def _both(M, ctx, w):
    from oracle import tree as T
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    ot = T.redundant_tree(w.k, keys, coef)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    k2, leaf, _ = M.mwns_tree_export(ctx, f)
    assert np.array_equal(k2, ot.keys) and np.array_equal(leaf, ot.leaf)
    return ot, f


@pytest.mark.parametrize("case", list(CASES))
def test_detail_norms_match_oracle(M, ctx, case):
    from oracle import tree as T
    ot, f = _both(M, ctx, CASES[case]())
    ref = T.detail_norms(ot)
    got = M.mwns_tree_detail_norms(ctx, f)
    assert np.all(got[ot.leaf == 1] == 0.0)
    internal = np.nonzero(ot.leaf == 0)[0]
    assert np.all(np.abs(got[internal] - ref[internal]) <= _tol(ot, internal, ref))


def _tol(tree, nodes, ref):
    """Rounding bound of a squared detail norm: each detail entry is a sum over the children's
    entries, so it carries an absolute error of a few units of roundoff times the children's norm
    x; the squared norm ||d||^2 then errs by about 2 ||d|| times that."""
    from oracle import tree as T
    ch = tree.index(T.children_keys(tree.keys[nodes])).reshape(-1, 8)
    x = np.sqrt(np.sum(tree.coef[ch].reshape(nodes.size, -1) ** 2, axis=1))
    return 1e-13 * (2.0 * np.sqrt(ref[nodes]) * x + x * x * 1e-3)


@pytest.mark.parametrize("case", list(CASES))
def test_prune_matches_oracle(M, ctx, case):
    """For budgets from none to everything: the same kept nodes and leaves as the oracle, the kept
    nodes' coefficients unchanged (bit for bit), the removed norm within eta^2 and equal to the
    oracle's; the pruned tree evaluates and applies like any other."""
    from oracle import tree as T
    ot, f = _both(M, ctx, CASES[case]())
    keys, leaf, coef = M.mwns_tree_export(ctx, f)
    fn = math.sqrt(float(np.sum(ot.coef[ot.leaf == 1] ** 2)))
    for rel in (0.0, 1e-7, 1e-5, 1e-3, 1e-1, 10.0):
        eta = rel * fn
        pr, removed = T.prune_l2(ot, eta)
        g, used = M.mwns_tree_prune(ctx, f, eta)
        k2, l2, c2 = M.mwns_tree_export(ctx, g)
        assert np.array_equal(k2, pr.keys) and np.array_equal(l2, pr.leaf), rel
        assert used <= eta * eta
        # the removed norm sums detail norms that each carry rounding of order u ||d|| ||x||
        assert abs(used - removed) <= 1e-9 * removed + 1e-26 * fn * fn
        assert np.array_equal(c2, coef[np.searchsorted(keys, k2)])
        info = M.mwns_tree_get_info(g)
        assert info["nnodes"] == k2.size and info["nleaves"] == int(l2.sum())
        print("%s eta = %g ||f||: %d -> %d nodes" % (case, rel, ot.keys.size, k2.size), flush=True)
    assert M.mwns_tree_get_info(M.mwns_tree_prune(ctx, f, 10.0 * fn)[0])["nnodes"] == 1
    from paper_0706_0747_amd import _lib
    with pytest.raises(M.MwnsError) as e:
        M.mwns_tree_prune(ctx, f, -1.0)
    assert e.value.status == _lib.MWNS_EINVAL


def test_discard_after_apply_matches_oracle(M, ctx):
    """Alg. 3 Step 4 on an applied output.  The oracle's g goes into the library as leaves (its
    internal nodes recomputed there) and both discard it at eps: the same kept nodes and leaves.
    (The library's own g differs from the oracle's by ~1e-12 relative, which at eps = 1e-6 is the
    size of the budget eps^2 itself, so decisions at the budget's edge may differ there; on its
    own g the library's discard is checked against its budget and by evaluation.)"""
    from oracle import apply as A
    from oracle import fit
    from oracle import tree as T
    w = CASES["k6"]()
    ot, f = _both(M, ctx, w)
    tau, wt = fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -ot.depth, math.sqrt(3))
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    g = A.assemble(ot, A.apply_modified(oo, ot))
    og = T.Tree(w.k, ot.keys, ot.leaf, g)
    gl = M.mwns_tree_from_leaves(ctx, w.k, ot.keys[ot.leaf == 1], g[ot.leaf == 1])
    gt, _ = M.mwns_apply(ctx, op, f)
    gn2 = float(np.sum(g[ot.leaf == 1] ** 2))
    for eps in (1e-6, 1e-4, 1e-2):
        pr, removed = T.discard(og, eps)
        gp, used = M.mwns_tree_discard(ctx, gl, eps)
        k2, l2, _ = M.mwns_tree_export(ctx, gp)
        assert np.array_equal(k2, pr.keys) and np.array_equal(l2, pr.leaf), eps
        assert used <= (eps * eps) * gn2 * (1 + 1e-12)
        assert k2.size < ot.keys.size
        gp, used = M.mwns_tree_discard(ctx, gt, eps)
        assert used <= (eps * eps) * gn2 * (1 + 1e-9)
        print("discard at eps %g: %d -> %d nodes" % (eps, ot.keys.size, k2.size), flush=True)
    # the pruned potential still evaluates within the removed norm of the full one (L2 over the cube)
    pts = workloads.points(20000, seed=9)
    gp, used = M.mwns_tree_discard(ctx, gt, 1e-4)
    a = M.mwns_tree_eval(ctx, gt, pts)
    b = M.mwns_tree_eval(ctx, gp, pts)
    assert math.sqrt(float(np.mean((a - b) ** 2))) <= 5.0 * math.sqrt(used) + 1e-14


def test_prune_c2_size(M, ctx):
    """The C2 tree (about 3e4 nodes, k = 8): detail norms against the oracle on sampled internal
    nodes, and a prune at eps ||f|| whose removed norm stays within the budget."""
    from oracle import tree as T
    w = workloads.c2()
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    keys, leaf, coef = M.mwns_tree_export(ctx, f)
    dn = M.mwns_tree_detail_norms(ctx, f)
    internal = np.nonzero(leaf == 0)[0]
    rng = np.random.Generator(np.random.PCG64(44))
    pick = rng.choice(internal, 64, replace=False)
    pos = np.searchsorted(keys, T.children_keys(keys[pick])).reshape(-1, 8)
    _, d = T.details(w.k, coef[pos])
    ref = np.sum(d.reshape(pick.size, -1) ** 2, axis=1)
    x = np.sqrt(np.sum(coef[pos].reshape(pick.size, -1) ** 2, axis=1))
    assert np.all(np.abs(dn[pick] - ref) <= 1e-13 * (2.0 * np.sqrt(ref) * x + x * x * 1e-3))
    fn = math.sqrt(float(np.sum(coef[leaf == 1] ** 2)))
    g, used = M.mwns_tree_prune(ctx, f, w.eps * fn)
    assert used <= (w.eps * fn) ** 2
    print("C2 prune at eps ||f||: %d -> %d nodes" % (keys.size, M.mwns_tree_get_info(g)["nnodes"]))
