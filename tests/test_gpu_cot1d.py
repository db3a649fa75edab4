"""The 1-D cotangent path of the library (Sec. 2.4, Alg. 2; Sec. 2.4.2) against the oracle: blocks,
bands, the adaptive projection (bit-exact trees), the applied output on Table 1's inputs and on
random trees with arbitrary bands (the same output tree, coefficients within 1e-12), evaluation,
and the error paths."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

A300 = 300.0
TABLE1 = [(5, 1e-3), (8, 1e-6), (11, 1e-9), (14, 1e-12)]


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_0706_0747_amd as M
    return M


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0)


def _keys(tr):
    return (tr.level.astype(np.uint64) << np.uint64(57)) | tr.trans.astype(np.uint64)


@pytest.mark.parametrize("k", [1, 5, 8, 14])
def test_blocks_match_oracle(M, ctx, k):
    from oracle import cot1d as C
    op = M.mwns_cot1d_op_create(ctx, k, 1e-6, 8)
    R = M.mwns_cot1d_op_blocks(ctx, op)
    ls = list(range(-65, 66))
    for j in range(9):
        ref = C.cot_blocks(k, j, ls)
        assert np.abs(R[j] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max()), j


@pytest.mark.parametrize("k,eps,nlev", [(5, 1e-3, 9), (8, 1e-6, 9), (11, 1e-9, 8), (14, 1e-12, 8), (3, 1e-2, 10)])
def test_bands_match_oracle(M, ctx, k, eps, nlev):
    from oracle import cot1d as C
    op = M.mwns_cot1d_op_create(ctx, k, eps, nlev)
    got = M.mwns_cot1d_op_bands(op)
    R = C.cot_table(k, nlev, lmax=C.DMAX * 2 + 1)
    want = C.choose_bands(k, R, eps)
    assert list(got) == list(want)


@pytest.mark.parametrize("k,eps", TABLE1)
def test_projection_matches_oracle_and_table1(M, ctx, k, eps):
    from oracle import cot1d as C
    tr = C.project_periodic(k, eps, 2, 20, [0.5], [A300], [1.0])
    f = M.mwns_cot1d_project(ctx, k, eps, 2, 20, [0.5], [A300], [1.0])
    keys, leaf, coef = M.mwns_cot1d_export(ctx, f)
    assert np.array_equal(keys, _keys(tr)) and np.array_equal(leaf, tr.leaf)
    assert np.abs(coef - tr.coef).max() <= 1e-14 * np.abs(tr.coef).max()


def _l2_error(C, mra, k, keys, leaf, g):
    x, w = mra.gauss_legendre01(48)
    err = 0.0
    for kk, lf, gi in zip(keys, leaf, g):
        if not lf:
            continue
        j, l = int(kk >> np.uint64(57)), int(kk & np.uint64((1 << 57) - 1))
        val = 2.0 ** (j / 2.0) * mra.phi(k, x) @ gi
        err += np.sum(w / 2.0 ** j * (val - C.exact_fourier((l + x) / 2.0 ** j, A300)) ** 2)
    return math.sqrt(err)


@pytest.mark.parametrize("k,eps", TABLE1)
def test_apply_matches_oracle_on_table1(M, ctx, k, eps):
    """The whole path on the paper's example: projection, operator, apply and evaluation, node by
    node against the oracle; the l2 error against the exact C f next to Table 1's."""
    from oracle import cot1d as C
    from oracle import mra
    tr = C.project_periodic(k, eps, 2, 20, [0.5], [A300], [1.0])
    R = C.cot_table(k, tr.depth)
    B = C.choose_bands(k, R, eps)
    sk = C.skeleton(tr, B)
    g_ref = C.assemble(sk, C.apply_modified(tr, R, B, sk))
    f = M.mwns_cot1d_project(ctx, k, eps, 2, 20, [0.5], [A300], [1.0])
    op = M.mwns_cot1d_op_create(ctx, k, eps, tr.depth)
    assert list(M.mwns_cot1d_op_bands(op)) == list(B)
    g, ms = M.mwns_cot1d_apply(ctx, op, f)
    keys, leaf, coef = M.mwns_cot1d_export(ctx, g)
    assert np.array_equal(keys, _keys(sk)) and np.array_equal(leaf, sk.leaf)
    assert np.abs(coef - g_ref).max() <= 1e-12 * np.abs(g_ref).max()
    e2 = _l2_error(C, mra, k, keys, leaf, coef)
    print("k=%d eps=%g: %d -> %d leaves, E2 %.3e, contraction %.3f ms" % (k, eps, int(tr.leaf.sum()), int(leaf.sum()), e2, ms),
          flush=True)
    assert e2 <= {5: 1.7e-4, 8: 1.5e-7, 11: 1.3e-10, 14: 4.4e-13}[k]
    y = np.random.default_rng(3).uniform(0.0, 1.0, 500)
    got = M.mwns_cot1d_eval(ctx, g, y)
    want = C.evaluate(sk, g_ref, y)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def _random_tree(rng, k, depth):
    from oracle import cot1d as C
    leaves, todo = [], [(1, 0), (1, 1)]
    while todo:
        j, l = todo.pop()
        if j < depth and rng.random() < 0.55:
            todo += [(j + 1, 2 * l), (j + 1, 2 * l + 1)]
        else:
            leaves.append((j, l, rng.normal(size=k)))
    return C.redundant_tree(k, leaves)


@pytest.mark.parametrize("seed,k", [(1, 3), (2, 6), (3, 10), (4, 16), (5, 1)])
def test_apply_random_trees_any_bands(M, ctx, seed, k):
    """Random adaptive trees (leaves imported) and random bands set on the operator: the same
    output tree and the same coefficients as the oracle's modified form on its skeleton."""
    from oracle import cot1d as C
    rng = np.random.default_rng(seed)
    tr = _random_tree(rng, k, 7)
    B = [0] + [int(rng.integers(0, 4)) for _ in range(tr.depth)] + [0]
    R = C.cot_table(k, tr.depth)
    sk = C.skeleton(tr, B)
    g_ref = C.assemble(sk, C.apply_modified(tr, R, B, sk))
    lf = tr.leaf == 1
    f = M.mwns_cot1d_from_leaves(ctx, k, _keys(tr)[lf], tr.coef[lf])
    keys, leaf, coef = M.mwns_cot1d_export(ctx, f)
    assert np.array_equal(keys, _keys(tr)) and np.abs(coef - tr.coef).max() <= 1e-13 * np.abs(tr.coef).max()
    op = M.mwns_cot1d_op_create(ctx, k, 1e-6, tr.depth)
    M.mwns_cot1d_op_set_bands(op, B)
    g, _ = M.mwns_cot1d_apply(ctx, op, f)
    keys, leaf, coef = M.mwns_cot1d_export(ctx, g)
    assert np.array_equal(keys, _keys(sk)) and np.array_equal(leaf, sk.leaf)
    assert np.abs(coef - g_ref).max() <= 1e-12 * np.abs(g_ref).max()


def test_root_only_tree(M, ctx):
    """A function resolved on the root: the output is the root leaf T_0 f_0."""
    from oracle import cot1d as C
    k = 6
    tr = C.project_periodic(k, 1e-1, 0, 10, [0.3], [2.0], [1.0])
    assert tr.coef.shape[0] == 1
    R = C.cot_table(k, 1)
    g_ref = C.apply_modified(tr, R, [0, 0, 0])
    f = M.mwns_cot1d_project(ctx, k, 1e-1, 0, 10, [0.3], [2.0], [1.0])
    op = M.mwns_cot1d_op_create(ctx, k, 1e-6, 1)
    g, _ = M.mwns_cot1d_apply(ctx, op, f)
    keys, leaf, coef = M.mwns_cot1d_export(ctx, g)
    assert keys.tolist() == [0] and leaf.tolist() == [1]
    # C nearly annihilates this wide Gaussian (|g| ~ 1e-2 of |f|): rounding scales with |r| |f|
    assert np.abs(coef[0] - g_ref[0]).max() <= 1e-13 * np.abs(tr.coef).max()


def test_error_paths(M, ctx):
    from paper_0706_0747_amd import _lib
    with pytest.raises(M.MwnsError) as e:
        M.mwns_cot1d_op_create(ctx, 0, 1e-6, 4)
    assert e.value.status == _lib.MWNS_EINVAL
    with pytest.raises(M.MwnsError) as e:
        M.mwns_cot1d_op_create(ctx, 6, -1.0, 4)
    assert e.value.status == _lib.MWNS_EINVAL
    f = M.mwns_cot1d_project(ctx, 6, 1e-6, 2, 20, [0.5], [A300], [1.0])
    op5 = M.mwns_cot1d_op_create(ctx, 5, 1e-6, 8)
    with pytest.raises(M.MwnsError) as e:
        M.mwns_cot1d_apply(ctx, op5, f)                 # orders differ
    assert e.value.status == _lib.MWNS_EINVAL
    shallow = M.mwns_cot1d_op_create(ctx, 6, 1e-6, 2)
    with pytest.raises(M.MwnsError) as e:
        M.mwns_cot1d_apply(ctx, shallow, f)             # tree deeper than the operator
    assert e.value.status == _lib.MWNS_EINVAL
    with pytest.raises(M.MwnsError) as e:
        M.mwns_cot1d_op_set_bands(shallow, [0, 0, 40, 0])
    assert e.value.status == _lib.MWNS_EINVAL
    with pytest.raises(M.MwnsError) as e:
        M.mwns_cot1d_eval(ctx, f, [0.5, 1.5])
    assert e.value.status == _lib.MWNS_EINVAL
    with pytest.raises(M.MwnsError) as e:                 # leaves that do not tile [0,1)
        M.mwns_cot1d_from_leaves(ctx, 6, np.array([(1 << 57) | 0], dtype=np.uint64), np.zeros((1, 6)))
    assert e.value.status == _lib.MWNS_EINVAL
