"""GPU path (libmwns through the C ABI) against the CPU oracle on the same seeded inputs."""
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


def test_operator_plan_many_terms(M, ctx):
    """157 Gaussian terms (Poisson, eps = 1e-8): the plan kernel sums the terms' estimates in
    chunks of 64, so the prefix and suffix scans cross chunk boundaries.  At k = 6 this eps keeps
    terms at the edge of the band; built with the overflow allowed on both sides, the edge ranges
    are compared too."""
    from oracle import apply as A, fit
    eps, depth = 1e-8, 4
    tau, wt = fit.fit_kernel(0.0, 1.0, eps, math.sqrt(eps) * 2.0 ** -depth, math.sqrt(3))
    assert len(tau) > 128
    op = M.mwns_op_create(ctx, 6, tau, wt, eps, depth, allow_band_overflow=1)
    oo = A.Operator(6, tau, wt, eps, depth, allow_overflow=True)
    assert np.any(oo.R[1:, 0, :, :, 1] >= oo.R[1:, 0, :, :, 0])
    F = M.mwns_op_tables_export(ctx, op)
    scale = np.abs(oo.F[:, :, 7]).max(axis=(2, 3))
    assert (np.abs(F - oo.F).max(axis=(2, 3, 4)) / scale).max() < 1e-13
    assert np.array_equal(M.mwns_op_plan_export(op), oo.R)
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
    assert per_node_ok(ghat, gh)
    gt2, st2 = M.mwns_apply(ctx, op, f)
    _, _, gg = M.mwns_tree_export(ctx, gt2)
    assert np.linalg.norm(gg - g) <= 1e-12 * np.linalg.norm(g)
    assert per_node_ok(gg, g)
    assert st2["useful_flops"] > 0
    # the device's contraction count equals the count of non-zero coefficients from the plan
    import bench
    assert st2["contractions"] == bench._count_contractions(oo.R, ot, np.arange(ot.keys.size))


def test_apply_is_deterministic(M, ctx):
    w = CASES["adaptive_k8"]()
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth)
    a = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])[2]
    b = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])[2]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("case", ["adaptive_k6", "adaptive_k8"])
def test_tile_variants_bit_identical(M, case):
    """Every contraction-kernel tile variant with one term per pass computes the same g bit for bit
    (they change only the wave count, prefetch depth and occupancy, not the order of the
    arithmetic); variants with several terms per pass add the plane results of consecutive terms
    in another order and agree to rounding."""
    w = CASES[case]()
    c = M.Context(0)
    f = M.mwns_project_gaussians(c, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = M.mwns_op_create(c, w.k, tau, wt, w.eps, depth)
    outs = []
    for v in range(M.mwns_num_variants()):
        M.mwns_ctx_set_variant(c, w.k, v)
        assert M.mwns_ctx_get_variant(c, w.k) == v
        outs.append(M.mwns_tree_export(c, M.mwns_apply(c, op, f)[0])[2])
    for v, o in enumerate(outs[1:], 1):
        if M.mwns_variant_shape(v)[3] == 1:
            assert np.array_equal(o, outs[0]), "variant %d differs from variant 0" % v
        else:
            assert np.linalg.norm(o - outs[0]) <= 1e-14 * np.linalg.norm(outs[0]), "variant %d" % v
    with pytest.raises(M.MwnsError):
        M.mwns_ctx_set_variant(c, w.k, M.mwns_num_variants())


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


@pytest.mark.parametrize("k", list(range(1, 11)))
def test_every_order_tables_plan_tree_eval(M, ctx, k):
    """Every order has its own instantiation of the projection, moment and evaluation kernels: the
    projected tree (keys and leaves exact), the operator's 1-D blocks, plan and threshold, and
    point values against the oracle."""
    from oracle import apply as A, tree as T
    w = workloads.small_adaptive(5, k=k, eps=1e-3 if k > 2 else (1e-2 if k == 2 else 5e-2), jmax=3)
    ot = _oracle_tree(w)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    keys, leaf, coef = M.mwns_tree_export(ctx, f)
    assert np.array_equal(keys, ot.keys) and np.array_equal(leaf, ot.leaf)
    assert np.abs(coef - ot.coef).max() <= 1e-13 * np.abs(ot.coef).max()
    tau, wt = _fit(w, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    F = M.mwns_op_tables_export(ctx, op)
    scale = np.abs(oo.F[:, :, 7]).max(axis=(2, 3))
    assert (np.abs(F - oo.F).max(axis=(2, 3, 4)) / scale).max() < 1e-13
    assert np.array_equal(M.mwns_op_plan_export(op), oo.R)
    assert abs(op.threshold - oo.theta) <= 1e-14 * oo.theta
    P = workloads.points(500, seed=30 + k)
    v = M.mwns_tree_eval(ctx, f, P)
    ref = T.evaluate(ot, P)
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()


def test_c2_full_size_sampled(M, ctx):
    """The benchmark workload (Poisson, k=8, eps=1e-6, 50 Gaussians) at full size: tree bit-exact,
    and g at sampled leaves (and their ancestor chains) within 1e-12 of the oracle."""
    from oracle import apply as A
    w = workloads.c2()
    ot = _oracle_tree(w)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    keys, leaf, coef = M.mwns_tree_export(ctx, f)
    assert np.array_equal(keys, ot.keys) and np.array_equal(leaf, ot.leaf)
    assert np.abs(coef - ot.coef).max() <= 1e-13 * np.abs(ot.coef).max()
    tau, wt = _fit(w, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    g, st = M.mwns_apply(ctx, op, f)
    _, _, gg = M.mwns_tree_export(ctx, g)
    rng = np.random.Generator(np.random.PCG64(31))
    leaves = np.nonzero(ot.leaf)[0]
    sample = list(rng.choice(leaves, 48, replace=False))
    deepest = np.nonzero(ot.level == ot.depth)[0]
    sample += [leaves[0], leaves[-1], deepest[0], deepest[-1]]          # cube corners and deepest boxes
    from oracle.tree import make_keys
    chain = set()
    for i in sample:
        j, l = int(ot.level[i]), ot.l[i]
        for lev in range(j + 1):
            chain.add(int(ot.index(make_keys(np.array([lev]), *(l[None, :] >> (j - lev)).T))[0]))
    chain = np.array(sorted(chain))
    gh = dict(zip(chain, A.apply_modified(oo, ot, chain)))
    ref = np.stack([A.assemble_chain(ot, i, lambda n: gh[n]) for i in sample])
    got = gg[sample]
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    assert per_node_ok(got, ref)


@pytest.mark.parametrize("k", [1, 3, 5, 7])
def test_odd_and_small_orders(M, ctx, k):
    """Orders whose 2k is not a multiple of 4 take the element-wise load path of the kernel."""
    from oracle import apply as A
    w = workloads.small_adaptive(4, k=k, eps=1e-3 if k > 2 else (1e-2 if k == 2 else 5e-2), jmax=4)
    ot = _oracle_tree(w)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    keys, leaf, _ = M.mwns_tree_export(ctx, f)
    assert np.array_equal(keys, ot.keys)
    tau, wt = _fit(w, ot.depth)
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    ref = A.assemble(ot, A.apply_modified(oo, ot))
    _, _, gg = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])
    assert np.linalg.norm(gg - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("j0,jmax", [(0, 0), (0, 3), (2, 2)])
def test_coarse_start_and_uniform_trees(M, ctx, j0, jmax):
    """Root-only tree, refinement from the root, and a uniform tree (no refinement test)."""
    from oracle import apply as A
    w = workloads.small_adaptive(6, k=4, eps=1e-3, jmax=jmax)
    w["j0"] = j0
    ot = _oracle_tree(w)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, j0, jmax, w.xyz, w.a, w.c)
    keys, leaf, coef = M.mwns_tree_export(ctx, f)
    assert np.array_equal(keys, ot.keys) and np.array_equal(leaf, ot.leaf)
    tau, wt = _fit(w, max(ot.depth, 1))
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    ref = A.assemble(ot, A.apply_modified(oo, ot))
    _, _, gg = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])
    assert np.linalg.norm(gg - ref) <= 1e-12 * np.linalg.norm(ref)


def test_projection_source_screening_edges(M, ctx):
    """The projection skips, per box, the sources whose values there stay below 2^-64 of the threshold:
    with 130 narrow Gaussians at k = 10 (two windows of 64 sources, chunks filled across windows) and
    every fifth weight zero (never kept), the tree is the oracle's bit for bit and the coefficients agree
    to 1e-13; with every weight zero (threshold 0: every source kept, nothing refined) the tree is the
    level-j0 grid of zero blocks."""
    from oracle import tree as T
    rng = np.random.default_rng(21)
    n = 130
    xyz = rng.uniform(0.2, 0.8, (n, 3))
    a = 10 ** rng.uniform(2.5, 4.5, n)
    c = rng.normal(size=n)
    c[::5] = 0.0
    keys, coef = T.project_gaussians(10, 1e-6, 2, 5, xyz, a, c)
    ot = T.redundant_tree(10, keys, coef)
    g = M.mwns_project_gaussians(ctx, 10, 1e-6, 2, 5, xyz, a, c)
    gk, gl, gc = M.mwns_tree_export(ctx, g)
    assert np.array_equal(gk, ot.keys) and np.array_equal(gl, ot.leaf)
    assert np.abs(gc - ot.coef).max() <= 1e-13 * np.abs(ot.coef).max()
    z = M.mwns_project_gaussians(ctx, 6, 1e-6, 2, 6, xyz[:3], a[:3], np.zeros(3))
    zk, zl, zc = M.mwns_tree_export(ctx, z)
    assert int(zl.sum()) == 64 and np.all((zk >> np.uint64(57))[zl == 1] == 2) and not np.any(zc)


def test_tree_from_leaves_full_plan_random_coefficients(M, ctx):
    """Imported leaves (random blocks on an adaptive structure) with screening off: every term on
    every coarse displacement, against the oracle."""
    from oracle import apply as A
    from oracle import tree as T
    w = workloads.small_adaptive(9, k=4, eps=1e-3, jmax=4)
    ot0 = _oracle_tree(w)
    lf = np.nonzero(ot0.leaf)[0]
    rng = np.random.Generator(np.random.PCG64(5))
    coef = rng.normal(size=(lf.size, 4, 4, 4))
    perm = rng.permutation(lf.size)                       # any leaf order is accepted
    ot = T.redundant_tree(4, ot0.keys[lf], coef)
    f = M.mwns_tree_from_leaves(ctx, 4, ot0.keys[lf][perm], coef[perm])
    keys, leaf, fc = M.mwns_tree_export(ctx, f)
    assert np.array_equal(keys, ot.keys) and np.abs(fc - ot.coef).max() <= 1e-13 * np.abs(ot.coef).max()
    tau, wt = _fit(w, ot.depth)
    R = A.full_plan(tau.size, ot.depth)
    oo = A.Operator(4, tau, wt, w.eps, ot.depth, R=R)
    op = M.mwns_op_create(ctx, 4, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, R)
    ref = A.assemble(ot, A.apply_modified(oo, ot))
    _, _, gg = M.mwns_tree_export(ctx, M.mwns_apply(ctx, op, f)[0])
    assert np.linalg.norm(gg - ref) <= 1e-12 * np.linalg.norm(ref)


def test_error_paths(M, ctx):
    from paper_0706_0747_amd import _lib
    w = workloads.small_adaptive(4, k=4, eps=1e-3, jmax=3)
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(0.0, 1.0, 1e-3, 1e-3, 1.8)
    cases = [
        lambda: M.mwns_op_create(ctx, 11, tau, wt, 1e-3, 3),                     # k beyond the kernels
        lambda: M.mwns_op_create(ctx, 4, -tau, wt, 1e-3, 3),                     # tau <= 0
        lambda: M.mwns_apply(ctx, M.mwns_op_create(ctx, 4, tau, wt, 1e-3, depth - 1), f),   # max_level < depth
        lambda: M.mwns_apply(ctx, M.mwns_op_create(ctx, 5, tau, wt, 1e-3, depth), f),       # k mismatch
        lambda: M.mwns_tree_eval(ctx, f, [[0.5, 0.5, 1.5]]),                      # outside the cube
        lambda: M.mwns_project_gaussians(ctx, 4, 1e-3, 3, 2, w.xyz, w.a, w.c),  # jmax < j0
        lambda: M.mwns_project_gaussians(ctx, 4, 1e-3, 0, 3, w.xyz, -w.a, w.c), # a <= 0
        lambda: M.mwns_tree_from_leaves(ctx, 4, np.array([0], dtype=np.uint64) | np.uint64(1 << 57),
                                        np.zeros((1, 4, 4, 4))),                 # one child only: no tiling
    ]
    for c in cases:
        with pytest.raises(M.MwnsError) as e:
            c()
        assert e.value.status == _lib.MWNS_EINVAL, str(e.value)
    op = M.mwns_op_create(ctx, 4, tau, wt, 1e-3, depth)
    bad = M.mwns_op_plan_export(op).copy()
    bad[1, 3, 3, 3] = (0, tau.size + 5)
    with pytest.raises(M.MwnsError):
        M.mwns_op_plan_import(op, bad)


def test_times_only_statistics(M, ctx):
    """MWNS_TIMES_ONLY fills the device times and the host-known figures, skips the contraction
    count and ||g|| (-1 and 0), and leaves g unchanged."""
    w = CASES["adaptive_k6"]()
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth)
    g1, s1 = M.mwns_apply(ctx, op, f)
    g2, s2 = M.mwns_apply(ctx, op, f, M.MWNS_TIMES_ONLY)
    assert s2["contractions"] == -1 and s2["g_norm"] == 0.0 and s1["contractions"] > 0
    assert s2["ms_contract"] > 0.0 and s2["useful_flops"] == s1["useful_flops"]
    assert np.array_equal(M.mwns_tree_export(ctx, g1)[2], M.mwns_tree_export(ctx, g2)[2])


def test_band_overflow_is_erange(M, ctx):
    """An operator whose screening keeps terms at the edge of the band fails with ERANGE (the oracle
    raises BandOverflow on the same inputs); allowed explicitly, it carries the oracle's plan."""
    from oracle import apply as A
    from oracle import plan as Pl
    from paper_0706_0747_amd import _lib
    from oracle import fit
    tau, wt = fit.fit_kernel(0.0, 1.0, 1e-4, 1e-2 * 2.0 ** -4, math.sqrt(3))
    with pytest.raises(Pl.BandOverflow):
        A.Operator(2, tau, wt, 1e-4, 4)
    with pytest.raises(M.MwnsError) as e:
        M.mwns_op_create(ctx, 2, tau, wt, 1e-4, 4)
    assert e.value.status == _lib.MWNS_ERANGE and "band" in str(e.value)
    op = M.mwns_op_create(ctx, 2, tau, wt, 1e-4, 4, allow_band_overflow=1)
    assert np.array_equal(M.mwns_op_plan_export(op), A.Operator(2, tau, wt, 1e-4, 4, allow_overflow=True).R)


def test_byte_budget_enomem_without_leaks(M):
    """A context whose byte budget is too small for a call fails with ENOMEM, creates no handle and
    holds no more device memory afterwards than before the call: for the projection, and for an
    apply whose tree and operator fit but whose working set does not."""
    from paper_0706_0747_amd import _lib
    w = CASES["adaptive_k6"]()
    small = M.Context(0, byte_budget=1 << 16)
    with pytest.raises(M.MwnsError) as e:
        M.mwns_project_gaussians(small, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    assert e.value.status == _lib.MWNS_ENOMEM
    small.release_cache()
    assert small.bytes_in_use() == 0
    probe = M.Context(0)
    f = M.mwns_project_gaussians(probe, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = _fit(w, depth)
    op = M.mwns_op_create(probe, w.k, tau, wt, w.eps, depth)
    probe.release_cache()
    held = probe.bytes_in_use()
    # budgets between what the tree and operator hold and what the apply needs on top (the
    # projection's own transient arrays may need more than the first ones)
    failed_apply = 0
    for factor in (1.15, 1.3, 1.5, 1.75, 2.0):
        tight = M.Context(0, byte_budget=int(held * factor))
        try:
            f2 = M.mwns_project_gaussians(tight, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
            op2 = M.mwns_op_create(tight, w.k, tau, wt, w.eps, depth)
        except M.MwnsError as e:
            assert e.status == _lib.MWNS_ENOMEM
            continue
        tight.release_cache()
        held2 = tight.bytes_in_use()
        try:
            M.mwns_apply(tight, op2, f2)
        except M.MwnsError as e:
            assert e.status == _lib.MWNS_ENOMEM
            tight.release_cache()
            assert tight.bytes_in_use() == held2
            failed_apply += 1
    assert failed_apply >= 1
