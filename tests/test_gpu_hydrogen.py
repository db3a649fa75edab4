"""The hydrogen iteration of Sec. 6.2 on the GPU against the oracle: the Coulomb product (the same
output tree, blocks node by node), the tree inner product, the whole iteration (mu, E and the trees'
sizes per step, against values the oracle wrote), and the error paths."""
import json
import math
import os

import numpy as np
import pytest

from parity_util import per_node_ok

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hydrogen_kalos.json")


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_0706_0747_amd as M
    return M


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0)


def _source(k, eps, jmax, s, centres, exps, seed):
    """Leaves of an adaptive projection (oracle) of a few Gaussians around the nucleus."""
    from oracle import tree as T
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 1.5, len(exps))
    keys, coef = T.project_gaussians(k, eps, 2, jmax, centres, [a * s * s for a in exps], c)
    return keys, coef


def _random_leaves(k, depth, seed):
    """A random tiling: every box split with probability 0.6 down to `depth`, random blocks."""
    from oracle import tree as T
    rng = np.random.default_rng(seed)
    leaves, todo = [], [(0, 0, 0, 0)]
    while todo:
        j, x, y, z = todo.pop()
        if j == 0 or (j < depth and rng.random() < 0.6):
            todo += [(j + 1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)) for c in range(8)]
        else:
            leaves.append((j, x, y, z))
    j, x, y, z = (np.array(v) for v in zip(*leaves))
    keys = T.make_keys(j, x, y, z)
    order = np.argsort(keys)
    return keys[order], rng.normal(size=(len(leaves), k, k, k))


@pytest.mark.parametrize("kind,k,eps,jmax,pjmax,seed", [("proj", 5, 1e-3, 6, 8, 1), ("proj", 3, 1e-4, 6, 9, 2),
                                                        ("proj", 6, 1e-3, 5, 7, 6), ("proj", 1, 1e-4, 4, 6, 5),
                                                        ("rand", 8, None, 2, 5, 3), ("rand", 9, None, 2, 2, 7),
                                                        ("rand", 10, None, 1, 4, 4)])
def test_product_matches_oracle(M, ctx, kind, k, eps, jmax, pjmax, seed):
    """The product of the library and of the oracle on the same leaves (an adaptive projection of
    Gaussians at the nucleus, or a random tiling with random blocks): the same output tree (every leaf
    split once, the nucleus' boxes down to pjmax, above or below f's depth) and the same blocks at
    every node."""
    from oracle import hydrogen as H
    from oracle import tree as T
    s = 20.0
    if kind == "proj":
        keys, coef = _source(k, eps, jmax, s, [[0.5, 0.5, 0.5], [0.52, 0.47, 0.5]], [1.0, 3.0], seed)
    else:
        keys, coef = _random_leaves(k, jmax, seed)
    f_ref = T.redundant_tree(k, keys, coef)
    ref = H.coulomb_product(f_ref, 1.7, pjmax, s)
    f = M.mwns_tree_from_leaves(ctx, k, keys, coef)
    g = M.mwns_tree_coulomb_product(ctx, f, 1.7, s, pjmax)
    gk, gl, gc = M.mwns_tree_export(ctx, g)
    assert np.array_equal(gk, ref.keys) and np.array_equal(gl, ref.leaf)
    print("k=%d: %d -> %d leaves" % (k, int(f_ref.leaf.sum()), int(gl.sum())), flush=True)
    assert per_node_ok(gc, ref.coef, rel=1e-12, floor=1e-14)
    # f is unchanged
    fk, _, fc = M.mwns_tree_export(ctx, f)
    assert np.array_equal(fk, f_ref.keys) and np.abs(fc - f_ref.coef).max() <= 1e-13 * np.abs(f_ref.coef).max()


@pytest.mark.parametrize("k", [4, 7])
def test_dot_matches_oracle(M, ctx, k):
    """<u, v> over u's leaves: u against itself and against a product on its refinement."""
    from oracle import hydrogen as H
    from oracle import tree as T
    s = 20.0
    keys, coef = _source(k, 1e-4, 7, s, [[0.5, 0.5, 0.5]], [1.0], 7)
    u_ref = T.redundant_tree(k, keys, coef)
    v_ref = H.coulomb_product(u_ref, 0.9, 7, s)
    u = M.mwns_tree_from_leaves(ctx, k, keys, coef)
    v = M.mwns_tree_coulomb_product(ctx, u, 0.9, s, 7)
    lf = u_ref.leaf == 1
    want_uu = float(np.sum(u_ref.coef[lf] ** 2))
    want_uv = float(np.sum(u_ref.coef[lf] * v_ref.coef[v_ref.index(u_ref.keys[lf])]))
    assert abs(M.mwns_tree_dot(ctx, u, u) - want_uu) <= 1e-13 * want_uu
    assert abs(M.mwns_tree_dot(ctx, u, v) - want_uv) <= 1e-12 * abs(want_uv)


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.mark.parametrize("case", range(2))
def test_kalos_matches_oracle(M, ctx, case):
    """Sec. 6.2's iteration in the library: mu and E at every step within 1e-10 of the oracle's (both
    compute in FP64; the fit, the plan, the trees and the discard are the same), and the trees the
    applies run on have the oracle's leaf counts."""
    c = _golden()[case]
    hist, leaves, ms = M.mwns_hydrogen_kalos(ctx, c["k"], c["eps"], c["L"], c["jmax"], mu0=c["mu0"], iters=c["iters"])
    print("k=%d eps=%g: E %s, leaves %s, apply ms %s" % (c["k"], c["eps"], ["%.8f" % E for _, E in hist], leaves,
                                                         ["%.2f" % t for t in ms]), flush=True)
    assert leaves == c["rho_leaves"]
    for (mu, E), mu_ref, E_ref in zip(hist, c["mu"], c["E"]):
        assert abs(mu - mu_ref) <= 1e-10 and abs(E - E_ref) <= 1e-10
    # each step closer to the ground state's -1/2
    err = [abs(E + 0.5) for _, E in hist]
    assert all(b < a for a, b in zip(err, err[1:]))


def test_error_paths(M, ctx):
    from paper_0706_0747_amd import _lib
    from oracle import tree as T
    keys, coef = _source(4, 1e-3, 5, 20.0, [[0.5, 0.5, 0.5]], [1.0], 1)
    f = M.mwns_tree_from_leaves(ctx, 4, keys, coef)
    for bad in [dict(c=1.0, s=0.0, jmax=5), dict(c=1.0, s=20.0, jmax=0), dict(c=1.0, s=20.0, jmax=20),
                dict(c=math.inf, s=20.0, jmax=5)]:
        with pytest.raises(M.MwnsError) as e:
            M.mwns_tree_coulomb_product(ctx, f, bad["c"], bad["s"], bad["jmax"])
        assert e.value.status == _lib.MWNS_EINVAL
    # dot: orders differ; a leaf of u missing from v (v coarser than u)
    k2, c2 = _source(5, 1e-3, 5, 20.0, [[0.5, 0.5, 0.5]], [1.0], 1)
    f5 = M.mwns_tree_from_leaves(ctx, 5, k2, c2)
    with pytest.raises(M.MwnsError) as e:
        M.mwns_tree_dot(ctx, f, f5)
    assert e.value.status == _lib.MWNS_EINVAL
    root = M.mwns_tree_from_leaves(ctx, 4, T.make_keys(np.array([0]), np.array([0]), np.array([0]), np.array([0])),
                                   np.ones((1, 4, 4, 4)))
    with pytest.raises(M.MwnsError) as e:
        M.mwns_tree_dot(ctx, f, root)
    assert e.value.status == _lib.MWNS_EINVAL
    r0 = T.redundant_tree(4, keys, coef).coef[0]
    assert abs(M.mwns_tree_dot(ctx, root, f) - float(np.sum(r0))) <= 1e-13 * float(np.abs(r0).sum())
    for kw in [dict(k=0), dict(eps=0.0), dict(L=-1.0), dict(jmax=19), dict(mu0=0.0), dict(iters=0)]:
        args = dict(k=4, eps=1e-3, L=10.0, jmax=6, mu0=1.0, iters=1)
        args.update(kw)
        with pytest.raises(M.MwnsError) as e:
            M.mwns_hydrogen_kalos(ctx, args["k"], args["eps"], args["L"], args["jmax"], mu0=args["mu0"],
                                  iters=args["iters"])
        assert e.value.status == _lib.MWNS_EINVAL
