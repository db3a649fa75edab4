"""Precision-routed apply (mwns_apply_mixed) against the FP64 apply and the CPU oracle.

The routing promises ||g - g_F64||_2 <= err_bound <= tol, where err_bound is the a-priori bound
sum over routed jobs of gamma_class * beta_job.  These tests check that promise on small and full
workloads, that every reduced class alone stays within it and at its own precision (a wrong
operand layout in any class would give O(1) errors), and that tol = 0 reproduces the FP64 apply
bit for bit."""
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
    "adaptive_k6": lambda: workloads.small_adaptive(11, k=6, eps=1e-3, jmax=5),
    "adaptive_k8": lambda: workloads.small_adaptive(8, k=8, eps=1e-5, jmax=5),
}


def _setup(M, ctx, w):
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth)
    return f, op, tau, wt, depth


def _leaf_norm(leaf, coef):
    return math.sqrt(float(np.sum(coef[leaf == 1] ** 2)))


@pytest.mark.parametrize("case", list(CASES))
def test_tol_zero_is_the_fp64_apply(M, ctx, case):
    f, op, *_ = _setup(M, ctx, CASES[case]())
    _, leaf, a = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])
    gm, st = M.mwns_apply_mixed(ctx, op, f, 0.0)
    _, _, b = M.mwns_tree_export(ctx, gm)
    assert np.array_equal(a, b)
    assert st["err_bound"] == 0.0 and st["class_flops"][1:] == [0.0, 0.0, 0.0]
    assert abs(st["g_norm"] - _leaf_norm(leaf, a)) <= 1e-12 * st["g_norm"]


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("cls,idx,rel", [("MWNS_CLASS_F32", 1, 1e-5), ("MWNS_CLASS_BF16C", 2, 1e-3),
                                         ("MWNS_CLASS_BF16", 3, 5e-2)])
def test_each_class_alone_within_bound(M, ctx, case, cls, idx, rel):
    """Every job forced into one reduced class (unbounded tol, an operator without narrow terms):
    the error against the FP64 apply is within the a-priori bound and at the class's precision."""
    w = CASES[case]()
    f, _, tau, wt, depth = _setup(M, ctx, w)
    keep = tau < 4.0 * w.k ** 2      # never a narrow near-diagonal term (tau_m < 4 k^2 4^j at every level)
    assert keep.sum() >= 3
    op = M.mwns_op_create(ctx, w.k, tau[keep], wt[keep], w.eps, depth)
    g64, st64 = M.mwns_apply(ctx, op, f)
    _, leaf, a = M.mwns_tree_export(ctx, g64)
    gm, st = M.mwns_apply_mixed(ctx, op, f, 1e300, classes=getattr(M, cls))
    _, _, b = M.mwns_tree_export(ctx, gm)
    assert st["class_flops"][0] == 0.0 and st["class_flops"][idx] == pytest.approx(st64["useful_flops"])
    err = _leaf_norm(leaf, b - a)
    assert err <= st["err_bound"]
    assert err <= rel * st64["g_norm"], (err / st64["g_norm"])


def test_near_diagonal_narrow_terms_stay_fp64(M, ctx):
    """The routing rule that keeps narrow Gaussians at the zero displacement in FP64: with an
    unbounded budget, an operator whose exponents are all below 4 k^2 (never narrower than 1/(2k)
    of a box, at any level) runs entirely in the reduced class; adding one exponent above
    4 k^2 4^depth pins that term's jobs whose box holds L = 0 to FP64 at every level, and the result
    stays within the bound.  BF16 classes are refused for k > 8."""
    from paper_0706_0747_amd import _lib
    w = CASES["adaptive_k6"]()
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    wide = M.mwns_op_create(ctx, w.k, np.array([0.3, 0.7]), np.array([1.0, 0.5]), w.eps, depth)
    _, st = M.mwns_apply_mixed(ctx, wide, f, 1e300, classes=M.MWNS_CLASS_F32)
    assert st["class_flops"][0] == 0.0 and st["class_flops"][1] > 0.0
    narrow = M.mwns_op_create(ctx, w.k, np.array([0.3, 4.0 * w.k ** 2 * 4.0 ** (depth + 1)]), np.array([1.0, 0.5]), w.eps, depth)
    g64, st64 = M.mwns_apply(ctx, narrow, f)
    gm, st = M.mwns_apply_mixed(ctx, narrow, f, 1e300, classes=M.MWNS_CLASS_F32)
    assert st["class_flops"][0] > 0.0 and st["class_flops"][1] > 0.0
    assert st["class_flops"][0] + st["class_flops"][1] == pytest.approx(st64["useful_flops"])
    _, leaf, a = M.mwns_tree_export(ctx, g64)
    _, _, b = M.mwns_tree_export(ctx, gm)
    assert _leaf_norm(leaf, b - a) <= st["err_bound"]
    w10 = workloads.small_adaptive(31, k=10, eps=1e-6, jmax=3)
    f10 = M.mwns_project_gaussians(ctx, w10.k, w10.eps, w10.j0, w10.jmax, w10.xyz, w10.a, w10.c)
    op10 = M.mwns_op_create(ctx, 10, np.array([0.3, 0.7]), np.array([1.0, 0.5]), w10.eps, M.mwns_tree_get_info(f10)["depth"])
    for cls in (M.MWNS_CLASS_BF16C, M.MWNS_CLASS_BF16, M.MWNS_CLASS_F32 | M.MWNS_CLASS_BF16):
        with pytest.raises(M.MwnsError) as e:
            M.mwns_apply_mixed(ctx, op10, f10, 1.0, classes=cls)
        assert e.value.status == _lib.MWNS_EINVAL
    _, st = M.mwns_apply_mixed(ctx, op10, f10, 1e300)      # the binding's default for k = 10: FP32
    assert st["class_flops"][2] == st["class_flops"][3] == 0.0 and st["class_flops"][1] > 0.0


@pytest.mark.parametrize("case", list(CASES))
def test_mixed_at_eps_against_oracle(M, ctx, case):
    """tol = eps ||g||: the routed result is within err_bound <= tol of the oracle's FP64 apply (up to
    FP64 round-off), on every node after assembly."""
    from oracle import apply as A
    from oracle import tree as T
    w = CASES[case]()
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    ot = T.redundant_tree(w.k, keys, coef)
    f, op, tau, _, depth = _setup(M, ctx, w)
    # the oracle's operator comes from the oracle's own fit; the library applies the oracle's plan
    from oracle import fit
    to, wo = fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -ot.depth, math.sqrt(3))
    assert to.size == tau.size
    oo = A.Operator(w.k, to, wo, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    g = A.assemble(ot, A.apply_modified(oo, ot))
    gnorm = _leaf_norm(ot.leaf, g)
    tol = w.eps * gnorm
    gm, st = M.mwns_apply_mixed(ctx, op, f, tol)
    _, _, b = M.mwns_tree_export(ctx, gm)
    assert st["err_bound"] <= tol
    assert _leaf_norm(ot.leaf, b - g) <= st["err_bound"] + 1e-12 * gnorm


def test_c2_mixed_at_eps(M, ctx):
    """The benchmark workload (Poisson, k=8, eps=1e-6): relative L2 error against the FP64 apply
    <= eps, and a real share of the work in reduced classes."""
    w = workloads.c2()
    f, op, *_ = _setup(M, ctx, w)
    g64, st64 = M.mwns_apply(ctx, op, f)
    _, leaf, a = M.mwns_tree_export(ctx, g64)
    tol = w.eps * st64["g_norm"]
    gm, st = M.mwns_apply_mixed(ctx, op, f, tol)
    _, _, b = M.mwns_tree_export(ctx, gm)
    err = _leaf_norm(leaf, b - a)
    print("C2 mixed: rel err %.3e, bound %.3e, class flop shares %s, contract %.3f ms vs %.3f ms FP64"
          % (err / st64["g_norm"], st["err_bound"] / st64["g_norm"],
             [round(x / st["useful_flops"], 3) for x in st["class_flops"]], st["ms_contract"], st64["ms_contract"]))
    assert err <= st["err_bound"] <= tol
    assert sum(st["class_flops"][1:]) >= 0.25 * st["useful_flops"]
