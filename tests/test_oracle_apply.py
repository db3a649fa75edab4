"""Pins of the oracle's modified ns-form apply (eq. apply_algo, Alg. 3, eq. g_assemble) against
the plain definition, the difference form and closed forms."""
import math

import numpy as np
import pytest

import workloads
from oracle import apply as A
from oracle import closed_forms, fit
from oracle import tree as T


def _tree_of(w):
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    return T.redundant_tree(w.k, keys, coef)


def _operator(w, depth, R=None, group=True):
    tau, wt = fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    return A.Operator(w.k, tau, wt, w.eps, depth, group=group, R=R)


def _apply(op, tr, form="modified"):
    gh = A.apply_modified(op, tr) if form == "modified" else A.apply_difference(op, tr)
    return A.assemble(tr, gh)


def _uniform_random_tree(k, n, seed):
    keys = T.uniform_leaves(k, n)
    coef = np.random.default_rng(seed).normal(size=(keys.size, k, k, k))
    return T.redundant_tree(k, keys, coef)


@pytest.mark.parametrize("k,n", [(4, 2), (6, 2)])
def test_full_plan_equals_dense_definition(k, n):
    """P-A1: with screening off, the modified ns-form on a uniform tree equals P_n T P_n f."""
    tr = _uniform_random_tree(k, n, 1)
    w = workloads.Workload(k=k, eps=1e-4, mu=0.0, alpha=1.0)
    op = _operator(w, n)
    opf = A.Operator(k, op.tau, op.w, op.eps, n, R=A.full_plan(op.M, n))
    g = _apply(opf, tr)
    gd = A.dense_uniform(opf, tr)
    sel = tr.level == n
    assert np.linalg.norm(g[sel] - gd) <= 1e-13 * np.linalg.norm(gd)


def test_full_plan_is_self_adjoint():
    k, n = 4, 2
    t1, t2 = _uniform_random_tree(k, n, 2), _uniform_random_tree(k, n, 3)
    w = workloads.Workload(k=k, eps=1e-4, mu=0.0, alpha=1.0)
    op = _operator(w, n)
    opf = A.Operator(k, op.tau, op.w, op.eps, n, R=A.full_plan(op.M, n))
    sel = t1.level == n
    g1, g2 = _apply(opf, t1), _apply(opf, t2)
    lhs, rhs = np.sum(t1.coef[sel] * g2[sel]), np.sum(g1[sel] * t2.coef[sel])
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("screened", [False, True])
def test_linearity_and_translation_equivariance(screened):
    """Linearity; translation equivariance of interior outputs, exact without screening and to
    O(eps) with it (the band structure depends on the parity of boxes within their parents)."""
    k, n = 4, 3
    w = workloads.Workload(k=k, eps=1e-4, mu=0.0, alpha=1.0)
    op = _operator(w, n)
    if not screened:
        op = A.Operator(k, op.tau, op.w, op.eps, n, R=A.full_plan(op.M, n))
    t1, t2 = _uniform_random_tree(k, n, 4), _uniform_random_tree(k, n, 5)
    t3 = T.Tree(k, t1.keys, t1.leaf, 2.0 * t1.coef - 3.0 * t2.coef)
    g1, g2, g3 = _apply(op, t1), _apply(op, t2), _apply(op, t3)
    assert np.abs(g3 - (2 * g1 - 3 * g2)).max() <= 1e-13 * np.abs(g3).max()
    # a single nonzero input block at (2,3,3) and at (3,3,3): outputs shift by one box in x
    sel = np.nonzero(t1.level == n)[0]
    L = t1.l[sel]
    blk = np.random.default_rng(6).normal(size=(k, k, k))
    outs = []
    for src in ((2, 3, 3), (3, 3, 3)):
        leaves = np.zeros((sel.size, k, k, k))
        leaves[np.all(L == src, axis=1)] = blk
        tr = T.redundant_tree(k, t1.keys[sel], leaves)
        outs.append(_apply(op, tr)[tr.level == n])
    for dst in [(3, 3, 3), (3, 4, 2), (4, 2, 3)]:
        a = outs[0][np.all(L == dst, axis=1)][0]
        b = outs[1][np.all(L == (dst[0] + 1, dst[1], dst[2]), axis=1)][0]
        tol = 10 * w.eps if screened else 1e-13
        assert np.abs(a - b).max() <= tol * np.abs(a).max()


def _random_plan(op, seed):
    rng = np.random.default_rng(seed)
    R = op.R.copy()
    for j in range(1, R.shape[0]):
        for idx in np.ndindex(7, 7, 7):
            if rng.random() < 0.3:
                R[j][idx] = (0, -1)
            else:
                a, b = sorted(rng.integers(0, op.M, 2))
                R[j][idx] = (a, b)
    return R


@pytest.mark.parametrize("case", ["c1", "adaptive", "adaptive_random_plan"])
def test_modified_form_equals_difference_form(case):
    """P-A2: eq. apply_algo and eq. g_scales_band agree after assembly for any tree and plan
    (down-up identity, eq. down_up)."""
    if case == "c1":
        w = workloads.c1()
    else:
        w = workloads.small_adaptive(11, k=6, eps=1e-3, jmax=5)
    tr = _tree_of(w)
    op = _operator(w, tr.depth)
    if case == "adaptive_random_plan":
        op = A.Operator(w.k, op.tau, op.w, op.eps, tr.depth, R=_random_plan(op, 3))
    g, gD = _apply(op, tr), _apply(op, tr, "difference")
    lf = tr.leaf == 1
    assert np.linalg.norm(g[lf] - gD[lf]) <= 1e-13 * np.linalg.norm(gD[lf])


def test_screened_apply_within_eps_of_unscreened():
    """Screening drops blocks whose estimated contribution is below eps (Sec. 4); the result stays
    within a few eps of the full modified form (Table 2 shows E2 up to ~5 eps)."""
    w = workloads.small_adaptive(3, k=6, eps=1e-4, jmax=4)
    tr = _tree_of(w)
    op = _operator(w, tr.depth)
    opf = A.Operator(w.k, op.tau, op.w, op.eps, tr.depth, R=A.full_plan(op.M, tr.depth))
    lf = tr.leaf == 1
    g, gf = _apply(op, tr), _apply(opf, tr)
    assert np.linalg.norm(g[lf] - gf[lf]) <= 5 * w.eps * np.linalg.norm(gf[lf])


def test_c1_against_closed_form():
    """Config C1 against the erf potential of the unit-mass Gaussian (1/(4 pi r) kernel)."""
    w = workloads.c1()
    tr = _tree_of(w)
    op = _operator(w, tr.depth)
    g = _apply(op, tr)
    P = workloads.points(4000)
    v = T.evaluate(T.Tree(w.k, tr.keys, tr.leaf, g), P)
    ex = closed_forms.poisson_gaussian(100.0, np.linalg.norm(P - 0.5, axis=1))
    assert np.abs(v - ex).max() <= 5e-4 * np.abs(ex).max()
    assert np.linalg.norm(v - ex) <= 1.5e-4 * np.linalg.norm(ex)
    # the fitted kernel applied to the cube-truncated source agrees with the free-space form here
    ft = closed_forms.fitted_truncated(op.tau, op.w, w.xyz, w.a, w.c, P[:200])
    assert np.abs(ft - ex[:200]).max() <= 1e-5 * np.abs(ex).max()


def test_adaptive_against_semi_closed_form():
    w = workloads.small_adaptive(8, k=8, eps=1e-5, jmax=5)
    tr = _tree_of(w)
    op = _operator(w, tr.depth)
    g = _apply(op, tr)
    P = workloads.points(300, seed=10)
    v = T.evaluate(T.Tree(w.k, tr.keys, tr.leaf, g), P)
    ref = closed_forms.fitted_truncated(op.tau, op.w, w.xyz, w.a, w.c, P)
    assert np.abs(v - ref).max() <= 50 * w.eps * np.abs(ref).max()


def test_assemble_chain_equals_whole_tree_assembly():
    """assemble_chain (g at one node from the ghat of its ancestor chain, used by the full-size
    parity tests) equals the whole-tree assembly of eq. g_assemble at sampled nodes of adaptive
    trees, with an arbitrary ghat so that a dropped transpose, parity bit or ancestor shows."""
    for seed, k in ((11, 6), (8, 5)):
        w = workloads.small_adaptive(seed, k=k, eps=1e-3, jmax=5)
        tr = _tree_of(w)
        ghat = np.random.default_rng(seed).normal(size=tr.coef.shape)
        g = A.assemble(tr, ghat)
        deep = np.nonzero(tr.level == tr.depth)[0]
        pick = np.concatenate([deep[:3], np.random.default_rng(seed + 1).choice(tr.keys.size, 12, replace=False)])
        for i in pick:
            gc = A.assemble_chain(tr, int(i), lambda n: ghat[n])
            assert np.abs(gc - g[i]).max() <= 1e-13 * np.abs(g[i]).max(), (seed, i)
        # the root has no ancestors: its g is its own ghat
        assert np.array_equal(A.assemble_chain(tr, 0, lambda n: ghat[n]), ghat[0])
