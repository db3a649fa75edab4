"""GPU path (libmwns through the C ABI) against the CPU oracle on the same seeded inputs."""
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


def _oracle_tree(w):
    from oracle import tree as T
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    return T.redundant_tree(w.k, keys, coef)


def _fit(w, depth):
    from oracle import fit
    return fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))


CASES = {
    "c1": lambda: workloads.c1(),
    "adaptive_k6": lambda: workloads.small_adaptive(11, k=6, eps=1e-3, jmax=5),
    "adaptive_k8": lambda: workloads.small_adaptive(8, k=8, eps=1e-5, jmax=5),
}


@pytest.mark.parametrize("case", list(CASES))
def test_tree_bit_exact(M, ctx, case):
    w = CASES[case]()
    ot = _oracle_tree(w)
    g = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    keys, leaf, coef = M.mwns_tree_export(ctx, g)
    assert keys.size == ot.keys.size and np.array_equal(keys, ot.keys)
    assert np.array_equal(leaf, ot.leaf)
    err = np.abs(coef - ot.coef).max() / np.abs(ot.coef).max()
    assert err < 1e-13, err


@pytest.mark.parametrize("case", ["c1", "adaptive_k8"])
def test_operator_tables_and_plan(M, ctx, case):
    from oracle import apply as A
    w = CASES[case]()
    depth = 3 if case == "c1" else 5
    tau, wt = _fit(w, depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth)
    F = M.mwns_op_tables_export(ctx, op)
    oo = A.Operator(w.k, tau, wt, w.eps, depth)
    scale = np.abs(oo.F[:, :, 7]).max(axis=(2, 3))          # largest block of each (j, m)
    err = (np.abs(F - oo.F).max(axis=(2, 3, 4)) / scale).max()
    assert err < 1e-13, err
    plan = M.mwns_op_plan_export(op)
    assert np.array_equal(plan, oo.R)
    assert abs(op.threshold - oo.theta) <= 1e-14 * oo.theta


@pytest.mark.parametrize("case", list(CASES))
def test_apply_matches_oracle(M, ctx, case):
    """FP64 apply with the oracle's plan imported: relative L2 <= 1e-12 on every node, both before
    (ghat) and after assembly (g)."""
    from oracle import apply as A
    w = CASES[case]()
    ot = _oracle_tree(w)
    tau, wt = _fit(w, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    gh = A.apply_modified(oo, ot)
    g = A.assemble(ot, gh)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    gt, st = M.mwns_apply(ctx, op, f, M.MWNS_NO_ASSEMBLY)
    _, _, ghat = M.mwns_tree_export(ctx, gt)
    assert np.linalg.norm(ghat - gh) <= 1e-12 * np.linalg.norm(gh)
    gt2, st2 = M.mwns_apply(ctx, op, f)
    _, _, gg = M.mwns_tree_export(ctx, gt2)
    assert np.linalg.norm(gg - g) <= 1e-12 * np.linalg.norm(g)
    assert st2["contractions"] > 0 and st2["useful_flops"] > 0


def test_apply_is_deterministic(M, ctx):
    w = CASES["adaptive_k8"]()
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth)
    a = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])[2]
    b = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])[2]
    assert np.array_equal(a, b)


def test_eval_matches_oracle(M, ctx):
    from oracle import tree as T
    w = CASES["adaptive_k6"]()
    ot = _oracle_tree(w)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    P = workloads.points(5000, seed=12)
    P[:10] = [[0, 0, 0], [1, 1, 1], [0.5, 0.5, 0.5], [0.25, 0.75, 1.0], [1, 0, 0.5], [0.125, 0.125, 0.125],
              [0.999999, 0.5, 0.5], [0.5, 0.0, 1.0], [0.75, 0.75, 0.75], [0.0625, 1.0, 0.3]]
    v = M.mwns_tree_eval(ctx, f, P)
    ref = T.evaluate(ot, P)
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()
