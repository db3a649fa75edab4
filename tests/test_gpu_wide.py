"""Orders 9 and 10 (2k = 18, 20: the two-tile contraction kernel) against the CPU oracle, and in
the batched, planned and routed entry points."""
import math

import numpy as np
import pytest

import workloads
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


def _fit(w, depth):
    from oracle import fit
    return fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))


CASES = {
    "k10_poisson": lambda: workloads.small_adaptive(31, k=10, eps=1e-6, jmax=4),
    "k9_yukawa": lambda: workloads.small_adaptive(32, k=9, eps=1e-5, jmax=4, mu=4.0),
    "k10_fractional": lambda: workloads.small_adaptive(33, k=10, eps=1e-7, jmax=3, n=2, alpha=0.7),
}


@pytest.mark.parametrize("case", list(CASES))
def test_wide_orders_match_oracle(M, ctx, case):
    """Tree bit-exact, operator tables and plan, and the FP64 apply (ghat and g) within 1e-12."""
    from oracle import apply as A
    from oracle import tree as T
    w = CASES[case]()
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    ot = T.redundant_tree(w.k, keys, coef)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    k2, leaf, c2 = M.mwns_tree_export(ctx, f)
    assert np.array_equal(k2, ot.keys) and np.array_equal(leaf, ot.leaf)
    assert np.abs(c2 - ot.coef).max() <= 1e-13 * np.abs(ot.coef).max()
    tau, wt = _fit(w, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    F = M.mwns_op_tables_export(ctx, op)
    scale = np.abs(oo.F).max(axis=(2, 3, 4), keepdims=True)
    assert np.all(np.abs(F - oo.F) <= 1e-13 * scale + 1e-300)
    assert np.array_equal(M.mwns_op_plan_export(op), oo.R)
    gh = A.apply_modified(oo, ot)
    g = A.assemble(ot, gh)
    _, _, ghat = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f, M.MWNS_NO_ASSEMBLY)[0])
    assert np.linalg.norm(ghat - gh) <= 1e-12 * np.linalg.norm(gh)
    assert per_node_ok(ghat, gh)
    gt, st = M.mwns_apply(ctx, op, f)
    _, _, gg = M.mwns_tree_export(ctx, gt)
    assert np.linalg.norm(gg - g) <= 1e-12 * np.linalg.norm(g)
    assert per_node_ok(gg, g)
    import bench
    assert st["contractions"] == bench._count_contractions(oo.R, ot, np.arange(ot.keys.size))


def test_wide_full_plan_random_coefficients(M, ctx):
    """Screening off (every term at every |L_d| <= 3) on random leaf coefficients of an uneven tree:
    every super-block quadrant, mask and boundary case of the two-tile kernel is exercised."""
    from oracle import apply as A
    from oracle import tree as T
    w = CASES["k10_poisson"]()
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, 3, w.xyz, w.a, w.c)
    rng = np.random.Generator(np.random.PCG64(51))
    coef = rng.standard_normal(coef.shape)
    ot = T.redundant_tree(w.k, keys, coef)
    tau, wt = _fit(w, ot.depth)
    tau, wt = tau[::8].copy(), wt[::8].copy()          # a handful of terms keeps the oracle quick
    R = A.full_plan(tau.size, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth, R=R)
    g = A.assemble(ot, A.apply_modified(oo, ot))
    f = M.mwns_tree_from_leaves(ctx, w.k, keys, coef)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, R)
    _, _, gg = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])
    assert np.linalg.norm(gg - g) <= 1e-12 * np.linalg.norm(g)


@pytest.mark.parametrize("case", ["k10_poisson", "k9_yukawa"])
def test_wide_variants_match_oracle(M, ctx, case):
    """Every tile variant of the k = 9, 10 kernel (one term group with and without the slice
    prefetch, two term groups, one term group with one exchange buffer) under the full plan on random leaf coefficients, so that every mask,
    the down band at bricks with leaf children (two-pass mode 1) and odd term counts (the second
    group idle for the last term) are exercised: each against the oracle within 1e-12; the
    one-group variants bit for bit equal."""
    from oracle import apply as A
    from oracle import tree as T
    w = CASES[case]()
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, 3, w.xyz, w.a, w.c)
    rng = np.random.Generator(np.random.PCG64(52))
    coef = rng.standard_normal(coef.shape)
    ot = T.redundant_tree(w.k, keys, coef)
    tau, wt = _fit(w, ot.depth)
    tau, wt = tau[::9].copy(), wt[::9].copy()
    R = A.full_plan(tau.size, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth, R=R)
    gh = A.apply_modified(oo, ot)
    f = M.mwns_tree_from_leaves(ctx, w.k, keys, coef)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, R)
    assert M.mwns_num_variants_for(w.k) == 4
    out = []
    try:
        for v in range(4):
            M.mwns_ctx_set_variant(ctx, w.k, v)
            _, _, ghat = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f, M.MWNS_NO_ASSEMBLY)[0])
            assert np.linalg.norm(ghat - gh) <= 1e-12 * np.linalg.norm(gh), "variant %d" % v
            assert per_node_ok(ghat, gh), "variant %d" % v
            out.append(ghat)
    finally:
        M.mwns_ctx_set_variant(ctx, w.k, -1)
    assert np.array_equal(out[0], out[2]) and np.array_equal(out[0], out[3])


def test_wide_in_batch_plan_and_routing(M, ctx):
    """k = 10 and k = 8 trees in one batch equal their single applies; the plan replays them; the
    BF16 classes are refused at k = 10 and tol = 0 keeps every job in FP64 (bound 0, result
    identical); a routed batch equals the routed single applies."""
    import torch
    specs = [CASES["k10_poisson"](), workloads.small_adaptive(34, k=8, eps=1e-5, jmax=4), CASES["k9_yukawa"]()]
    ops, fs = [], []
    for w in specs:
        f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
        depth = M.mwns_tree_get_info(f)["depth"]
        tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
        ops.append(M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth))
        fs.append(f)
    singles = [M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])[2] for op, f in zip(ops, fs)]
    gs, _ = M.mwns_apply_batch(ctx, ops, fs)
    for i, g in enumerate(gs):
        assert np.array_equal(M.mwns_tree_export(ctx, g)[2], singles[i]), "member %d" % i
    plan = M.mwns_plan_create(ctx, ops, fs)
    for _ in range(2):
        plan.execute()
        torch.cuda.synchronize()
        for i in range(len(specs)):
            assert np.array_equal(M.mwns_tree_export(ctx, plan.output(i))[2], singles[i])
    plan.close()
    from paper_0706_0747_amd import _lib
    with pytest.raises(M.MwnsError) as e:
        M.mwns_apply_mixed(ctx, ops[0], fs[0], 1e300, classes=M.MWNS_CLASS_BF16C | M.MWNS_CLASS_BF16)
    assert e.value.status == _lib.MWNS_EINVAL
    gm, st = M.mwns_apply_mixed(ctx, ops[0], fs[0], 0.0)
    assert st["err_bound"] == 0.0 and st["class_flops"][1:] == [0.0, 0.0, 0.0]
    assert np.array_equal(M.mwns_tree_export(ctx, gm)[2], singles[0])
    tols = [w.eps * M.mwns_apply(ctx, op, f)[1]["g_norm"] for w, op, f in zip(specs, ops, fs)]
    routed = [M.mwns_tree_export(ctx, M.mwns_apply_mixed(ctx, op, f, tol)[0])[2] for op, f, tol in zip(ops, fs, tols)]
    gs, st = M.mwns_apply_batch(ctx, ops, fs, mixed=tols)
    assert 0.0 < st["err_bound"] <= max(tols)
    for i, g in enumerate(gs):
        assert np.array_equal(M.mwns_tree_export(ctx, g)[2], routed[i]), "routed member %d" % i


def _lib_setup(M, ctx, w):
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    return f, M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth), tau, wt


def _leaf_norm(leaf, coef):
    return math.sqrt(float(np.sum(coef[leaf == 1] ** 2)))


@pytest.mark.parametrize("case", list(CASES))
def test_wide_fp32_class_alone_within_bound(M, ctx, case):
    """Every job of the whole-brick kernel forced into the FP32 class (unbounded tol, an operator
    without narrow terms): the error against the FP64 apply is within the a-priori bound and at
    FP32 precision (a wrong operand layout or K-slot permutation would give O(1) errors)."""
    w = CASES[case]()
    f, _, tau, wt = _lib_setup(M, ctx, w)
    # the fit's terms wider than 1/(2k) of the root box (tau < 4 k^2): none of them is a narrow
    # near-diagonal term at any level, so every job can go to the FP32 class
    keep = tau < 4.0 * w.k ** 2
    assert keep.sum() >= 3
    op = M.mwns_op_create(ctx, w.k, tau[keep], wt[keep], w.eps, M.mwns_tree_get_info(f)["depth"])
    g64, st64 = M.mwns_apply(ctx, op, f)
    _, leaf, a = M.mwns_tree_export(ctx, g64)
    gm, st = M.mwns_apply_mixed(ctx, op, f, 1e300, classes=M.MWNS_CLASS_F32)
    _, _, b = M.mwns_tree_export(ctx, gm)
    assert st["class_flops"][0] == 0.0 and st["class_flops"][1] == pytest.approx(st64["useful_flops"])
    err = _leaf_norm(leaf, b - a)
    assert 0.0 < err <= st["err_bound"]
    assert err <= 1e-5 * st64["g_norm"], err / st64["g_norm"]


def test_wide_mixed_at_eps_against_oracle(M, ctx):
    """tol = eps ||g|| at k = 10: the routed result is within err_bound <= tol of the oracle's FP64
    apply (up to FP64 round-off)."""
    from oracle import apply as A
    from oracle import tree as T
    w = CASES["k10_poisson"]()
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    ot = T.redundant_tree(w.k, keys, coef)
    f, op, tau, _ = _lib_setup(M, ctx, w)
    # the oracle's operator comes from the oracle's own fit; the library applies the oracle's plan
    to, wo = _fit(w, ot.depth)
    assert to.size == tau.size
    oo = A.Operator(w.k, to, wo, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    g = A.assemble(ot, A.apply_modified(oo, ot))
    gnorm = _leaf_norm(ot.leaf, g)
    tol = w.eps * gnorm
    gm, st = M.mwns_apply_mixed(ctx, op, f, tol)
    _, _, b = M.mwns_tree_export(ctx, gm)
    assert st["class_flops"][1] > 0.0 and st["class_flops"][2:] == [0.0, 0.0]
    assert st["err_bound"] <= tol
    assert _leaf_norm(ot.leaf, b - g) <= st["err_bound"] + 1e-12 * gnorm


def test_c3_mixed_at_eps(M, ctx):
    """The bound-state Helmholtz workload (k = 10, eps = 1e-8) routed at tol = eps ||g||: relative
    L2 error against the FP64 apply <= eps, with a share of the work in the FP32 class."""
    w = workloads.c3()
    f, op, *_ = _lib_setup(M, ctx, w)
    g64, st64 = M.mwns_apply(ctx, op, f)
    _, leaf, a = M.mwns_tree_export(ctx, g64)
    tol = w.eps * st64["g_norm"]
    gm, st = M.mwns_apply_mixed(ctx, op, f, tol)
    _, _, b = M.mwns_tree_export(ctx, gm)
    err = _leaf_norm(leaf, b - a)
    print("C3 mixed: rel err %.3e, bound %.3e, class flop shares %s, contract %.3f ms vs %.3f ms FP64"
          % (err / st64["g_norm"], st["err_bound"] / st64["g_norm"],
             [round(x / st["useful_flops"], 3) for x in st["class_flops"]], st["ms_contract"], st64["ms_contract"]))
    assert err <= st["err_bound"] <= tol
    # the narrow near-diagonal terms stay FP64 (at k = 10 most of the work); a class that would
    # carry less than a tenth of it is not launched
    assert st["class_flops"][1] == 0.0 or st["class_flops"][1] >= 0.1 * st["useful_flops"]


def test_c3_yukawa_full_size_sampled(M, ctx):
    """The bound-state Helmholtz workload (e^{-mu r}/(4 pi r), k=10, eps=1e-8, 20 Gaussians) at full
    size: tree bit-exact, and g at sampled leaves and their ancestor chains within 1e-12 of the
    oracle (which applies only the nodes on those chains)."""
    from oracle import apply as A
    from oracle import tree as T
    from oracle.tree import make_keys
    w = workloads.c3()
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    ot = T.redundant_tree(w.k, keys, coef)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    k2, leaf, c2 = M.mwns_tree_export(ctx, f)
    assert np.array_equal(k2, ot.keys) and np.array_equal(leaf, ot.leaf)
    assert np.abs(c2 - ot.coef).max() <= 1e-13 * np.abs(ot.coef).max()
    tau, wt = _fit(w, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    assert np.array_equal(M.mwns_op_plan_export(op), oo.R)
    _, _, gg = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])
    rng = np.random.Generator(np.random.PCG64(33))
    leaves = np.nonzero(ot.leaf)[0]
    sample = list(rng.choice(leaves, 12, replace=False))
    deepest = np.nonzero(ot.level == ot.depth)[0]
    sample += [leaves[0], leaves[-1], deepest[0], deepest[-1]]
    chain = set()
    for i in sample:
        j, l = int(ot.level[i]), ot.l[i]
        for lev in range(j + 1):
            chain.add(int(ot.index(make_keys(np.array([lev]), *(l[None, :] >> (j - lev)).T))[0]))
    chain = np.array(sorted(chain))
    gh = dict(zip(chain, A.apply_modified(oo, ot, chain)))
    ref = np.stack([A.assemble_chain(ot, i, lambda n: gh[n]) for i in sample])
    assert np.linalg.norm(gg[sample] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert per_node_ok(gg[sample], ref)
