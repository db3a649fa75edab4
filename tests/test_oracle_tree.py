"""Pins of the oracle's trees (Alg. 1, Sec. 2.2.1, App. A.1/A.3)."""
import math

import numpy as np
import pytest

import workloads
from oracle import closed_forms, mra
from oracle import tree as T


def test_keys_roundtrip_and_order():
    rng = np.random.default_rng(0)
    j = rng.integers(0, 20, 500)
    l = (rng.random((500, 3)) * (2.0 ** j)[:, None]).astype(np.int64)
    keys = T.make_keys(j, l[:, 0], l[:, 1], l[:, 2])
    j2, l2 = T.decode_keys(keys)
    assert np.all(j2 == j) and np.all(l2 == l)
    # x in bit 0: (1,0,0) -> 1, (0,1,0) -> 2, (0,0,1) -> 4 at the same level
    k = T.make_keys(np.array([1, 1, 1]), np.array([1, 0, 0]), np.array([0, 1, 0]), np.array([0, 0, 1]))
    assert list(k & np.uint64(7)) == [1, 2, 4]
    ch = T.children_keys(T.make_keys(np.array([3]), np.array([5]), np.array([2]), np.array([7])))
    assert np.all(ch[1:] > ch[:-1])


def test_uniform_c1_tree_sizes():
    w = workloads.c1()
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    tr = T.redundant_tree(w.k, keys, coef)
    assert keys.size == 512 and tr.keys.size == 585 and tr.leaf.sum() == 512


def test_nearly_polynomial_source_is_not_refined():
    # a very wide Gaussian is a polynomial of degree < k to within rounding: one box, no refinement
    keys, coef = T.project_gaussians(6, 1e-6, 0, 6, [[0.5, 0.5, 0.5]], [1e-7], [1.0])
    assert keys.size == 1


def _direct_test(k, key, coef, xyz, a, c, thr):
    """max |f - f~| over the 8 children's GL nodes, computed independently with numpy."""
    j, l = T.decode_keys(np.array([key]))
    j, l = int(j[0]), l[0]
    x, _ = mra.gauss_legendre01(k)
    emax = 0.0
    for s in range(8):
        sig = np.array([s & 1, (s >> 1) & 1, s >> 2 & 1])
        u = [(sig[d] + x) / 2.0 for d in range(3)]
        pts = np.stack(np.meshgrid(*[2.0 ** -j * (l[d] + u[d]) for d in range(3)], indexing="ij"), -1).reshape(-1, 3)
        f = closed_forms.gauss_sum(xyz, a, c, pts)
        ft = 2 ** (1.5 * j) * np.einsum("abc,ia,jb,kc->ijk", coef, mra.phi(k, u[0]), mra.phi(k, u[1]),
                                         mra.phi(k, u[2])).ravel()
        emax = max(emax, np.abs(f - ft).max())
    return emax


def test_refinement_criterion_holds_at_every_leaf_and_fails_at_every_internal_node():
    w = workloads.small_adaptive(11, k=6, eps=1e-4, jmax=6)
    keys, coef, (err, thr) = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c, with_margins=True)
    tr = T.redundant_tree(w.k, keys, coef)
    assert tr.depth < w.jmax and keys.size > 8
    rng = np.random.default_rng(0)
    for i in rng.choice(np.nonzero(tr.leaf)[0], 12, replace=False):
        assert _direct_test(w.k, tr.keys[i], tr.coef[i], w.xyz, w.a, w.c, thr) <= thr
    internal = np.nonzero((tr.leaf == 0) & (tr.level >= w.j0))[0]
    # internal blocks are compressed from children; the test uses the box's own projection
    for i in rng.choice(internal, min(6, internal.size), replace=False):
        j, l = int(tr.level[i]), tr.l[i]
        x, wq = mra.gauss_legendre01(w.k)
        pts = np.stack(np.meshgrid(*[2.0 ** -j * (l[d] + x) for d in range(3)], indexing="ij"), -1).reshape(-1, 3)
        f = closed_forms.gauss_sum(w.xyz, w.a, w.c, pts).reshape(w.k, w.k, w.k)
        P = mra.phi(w.k, x) * wq[:, None]
        own = 2 ** (-1.5 * j) * np.einsum("ijk,ia,jb,kc->abc", f, P, P, P)
        assert _direct_test(w.k, tr.keys[i], own, w.xyz, w.a, w.c, thr) > thr


def test_compress_upsample_identities():
    rng = np.random.default_rng(3)
    k = 6
    x = rng.normal(size=(5, 8, k, k, k))
    p = T.compress(k, x)
    # compress(upsample(p)) = p ; upsample(compress(.)) is a projection; Parseval
    assert np.abs(T.compress(k, T.upsample(k, p)) - p).max() < 1e-13
    u = T.upsample(k, p)
    assert np.abs(T.upsample(k, T.compress(k, u)) - u).max() < 1e-13
    assert np.all(np.sum(x ** 2, axis=(1, 2, 3, 4)) >= np.sum(p ** 2, axis=(1, 2, 3)) - 1e-12)
    assert np.allclose(np.sum(u ** 2, axis=(1, 2, 3, 4)), np.sum(p ** 2, axis=(1, 2, 3)))


def test_evaluation_at_gauss_nodes_inverts_the_projection():
    """Evaluating a leaf at its own GL nodes returns the sampled values (the k-point transform of
    eq. fvals2coefs is invertible), for every leaf of an adaptive tree."""
    w = workloads.small_adaptive(5, k=6, eps=1e-4, jmax=5)
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    tr = T.redundant_tree(w.k, keys, coef)
    x, _ = mra.gauss_legendre01(w.k)
    rng = np.random.default_rng(1)
    for i in rng.choice(np.nonzero(tr.leaf)[0], 10, replace=False):
        j, l = int(tr.level[i]), tr.l[i]
        pts = np.stack(np.meshgrid(*[2.0 ** -j * (l[d] + x) for d in range(3)], indexing="ij"), -1).reshape(-1, 3)
        assert np.allclose(T.evaluate(tr, pts), closed_forms.gauss_sum(w.xyz, w.a, w.c, pts), rtol=1e-12, atol=1e-12)


def test_projection_accuracy_against_source():
    w = workloads.small_adaptive(7, k=8, eps=1e-6, jmax=6)
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    tr = T.redundant_tree(w.k, keys, coef)
    P = workloads.points(3000, seed=9)
    thr = w.eps * T.source_norm(w.xyz, w.a, w.c)
    assert np.abs(T.evaluate(tr, P) - closed_forms.gauss_sum(w.xyz, w.a, w.c, P)).max() < 10 * thr


def test_project_boxes_reproduces_the_tree():
    """The per-box step on the leaves of a built tree says 'keep' (below jmax) and returns the
    same coefficients; on their parents it says 'refine'."""
    w = workloads.small_adaptive(8, k=6, eps=1e-4, jmax=5)
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    rng = np.random.Generator(np.random.PCG64(3))
    pick = rng.choice(keys.size, 20, replace=False)
    s, ref, _ = T.project_boxes(w.k, w.eps, w.jmax, w.xyz, w.a, w.c, keys[pick])
    lev, l = T.decode_keys(keys[pick])
    assert np.array_equal(s, coef[pick])
    assert np.all(ref[lev < w.jmax] == 0)
    deeper = lev > w.j0
    parents = T.make_keys(lev[deeper] - 1, *(l[deeper] >> 1).T)
    _, pref, _ = T.project_boxes(w.k, w.eps, w.jmax, w.xyz, w.a, w.c, parents)
    assert np.all(pref == 1)


def test_project_function_matches_gaussian_projection():
    """Alg. 1 for a source given as a callable (numpy) makes the same decisions and coefficients
    as the plain-C projection of the same Gaussian sum."""
    from oracle import closed_forms
    for seed, k in ((11, 6), (3, 8)):
        w = workloads.small_adaptive(seed, k=k, eps=1e-4, jmax=5)
        kg, cg = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)

        def f(x, y, z):
            out = 0.0
            for (cx, cy, cz), a, c in zip(w.xyz, w.a, w.c):
                out = out + c * (a / np.pi) ** 1.5 * np.exp(-a * ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2))
            return out
        kf, cf = T.project_function(w.k, w.eps, w.j0, w.jmax, f, T.source_norm(w.xyz, w.a, w.c))
        assert np.array_equal(kg, kf)
        assert np.abs(cg - cf).max() <= 1e-12 * np.abs(cg).max()
        pts = workloads.points(500, seed=seed)
        v = T.evaluate(T.redundant_tree(w.k, kf, cf), pts)
        ref = closed_forms.gauss_sum(w.xyz, w.a, w.c, pts)
        assert np.abs(v - ref).max() <= 50 * w.eps * T.source_norm(w.xyz, w.a, w.c)


def test_project_function_low_degree_polynomial_is_one_level():
    """A polynomial of degree < k is reproduced exactly by every box: no box is refined."""
    k = 5
    keys, coef = T.project_function(k, 1e-12, 1, 6, lambda x, y, z: 1.0 + x * y - 2 * z ** 3 + x ** 4, 1.0)
    lev, _ = T.decode_keys(keys)
    assert keys.size == 8 and np.all(lev == 1)
