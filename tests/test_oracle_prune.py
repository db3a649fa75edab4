"""Pins of the oracle's wavelet filters, detail coefficients and l2 pruning (App. A.2-A.3,
Sec. 2.2, Alg. 3 Step 4)."""
import numpy as np
import pytest

import workloads
from oracle import mra
from oracle import tree as T


@pytest.mark.parametrize("k", range(1, 11))
def test_wavelet_filters_complete_an_orthogonal_two_scale_matrix(k):
    H0, H1 = mra.two_scale_filters(k)
    G0, G1 = mra.wavelet_filters(k)
    W = np.block([[H0, H1], [G0, G1]])
    assert np.abs(W @ W.T - np.eye(2 * k)).max() < 1e-14
    assert np.abs(W.T @ W - np.eye(2 * k)).max() < 1e-14


def _half_coefficients(k, p):
    """Scaling coefficients of p (vectorised, on [0,1]) on the two halves at level 1 and on [0,1]
    at level 0, by a Gauss-Legendre rule of 2k points per interval (exact for polynomial pieces of
    degree < 3k): s^1_{a,sigma} = int p(x) sqrt2 phi_a(2x - sigma) dx, s^0_a = int p phi_a."""
    x, w = np.polynomial.legendre.leggauss(2 * k)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    s0 = np.einsum("i,i,ia->a", w, p(x), mra.phi(k, x))
    s1 = []
    for sig in (0, 1):
        y = 0.5 * (x + sig)
        s1.append(0.5 * np.einsum("i,i,ia->a", w, p(y), np.sqrt(2.0) * mra.phi(k, x)))
    return s0, s1


@pytest.mark.parametrize("k", [1, 3, 6, 10])
def test_vanishing_moments_and_scaling_part(k):
    """A polynomial of degree < k has no detail (the first k moments of the wavelets vanish), and
    the H part of its two halves is its level-0 block; a function with a kink at 1/2 has detail."""
    rng = np.random.default_rng(k)
    p = np.poly1d(rng.normal(size=k))                     # degree k - 1
    s0, (a, b) = _half_coefficients(k, p)
    H0, H1 = mra.two_scale_filters(k)
    G0, G1 = mra.wavelet_filters(k)
    assert np.abs(G0 @ a + G1 @ b).max() < 1e-13 * np.abs(s0).max()
    assert np.abs(H0 @ a + H1 @ b - s0).max() < 1e-13 * np.abs(s0).max()
    # |x - 1/2| is linear on each half (exact in V_1 for k >= 2) but not a polynomial on [0,1]
    if k >= 2:
        _, (a, b) = _half_coefficients(k, lambda x: np.abs(x - 0.5))
        assert np.linalg.norm(G0 @ a + G1 @ b) > 1e-2 * np.linalg.norm(np.concatenate([a, b]))


@pytest.mark.parametrize("k", [2, 5])
def test_details_reconstruct_and_parseval(k):
    rng = np.random.default_rng(10 + k)
    kids = rng.normal(size=(3, 8, k, k, k))
    s, d = T.details(k, kids)
    assert np.allclose(s, T.compress(k, kids), rtol=0, atol=1e-13)
    back = T.reconstruct(k, s, d)
    assert np.abs(back - kids).max() < 1e-13
    # Parseval: the children's squared norm is the parent's plus the details'
    lhs = np.sum(kids.reshape(3, -1) ** 2, axis=1)
    rhs = np.sum(s.reshape(3, -1) ** 2, axis=1) + np.sum(d.reshape(3, -1) ** 2, axis=1)
    assert np.allclose(lhs, rhs, rtol=1e-13)
    # the detail part is what zero-detail reconstruction of the parent misses
    miss = np.sum((kids - T.upsample(k, s)).reshape(3, -1) ** 2, axis=1)
    assert np.allclose(miss, np.sum(d.reshape(3, -1) ** 2, axis=1), rtol=1e-12)


def _tree(seed=3, k=4, eps=1e-4):
    w = workloads.small_adaptive(seed, k=k, eps=eps, jmax=5)
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    return T.redundant_tree(w.k, keys, coef)


def _l2_gap(full, pruned):
    """||f - f_pruned||_2^2 from the blocks: each leaf of the full tree against the pruned leaf that
    covers it, brought down to the full leaf's level by zero-detail reconstruction."""
    tot = 0.0
    pos = {int(kk): i for i, kk in enumerate(pruned.keys)}
    for i in np.nonzero(full.leaf)[0]:
        j, l = int(full.level[i]), full.l[i]
        for up in range(j + 1):
            key = int(T.make_keys(np.array([j - up]), *(l[None, :] >> up).T)[0])
            if key in pos and pruned.leaf[pos[key]]:
                block = pruned.coef[pos[key]]
                for step in range(up, 0, -1):
                    s = ((l >> (step - 1)) & 1)
                    block = T.upsample(full.k, block)[s[0] + 2 * s[1] + 4 * s[2]]
                tot += float(np.sum((full.coef[i] - block) ** 2))
                break
        else:
            raise AssertionError("leaf not covered")
    return tot


def test_detail_norms_match_the_zero_detail_residual():
    tr = _tree()
    dn = T.detail_norms(tr)
    assert np.all(dn[tr.leaf == 1] == 0.0) and np.all(dn[tr.leaf == 0] > 0.0)
    internal = np.nonzero(tr.leaf == 0)[0]
    ch = tr.index(T.children_keys(tr.keys[internal])).reshape(-1, 8)
    miss = np.sum((tr.coef[ch] - T.upsample(tr.k, tr.coef[internal])).reshape(internal.size, -1) ** 2, axis=1)
    assert np.allclose(dn[internal], miss, rtol=1e-10, atol=1e-30)


def test_prune_l2_error_equals_the_removed_details():
    tr = _tree()
    fn2 = float(np.sum(tr.coef[tr.leaf == 1] ** 2))
    for rel in (0.0, 1e-6, 1e-4, 1e-2, 1.0):
        eta = rel * np.sqrt(fn2)
        pr, used = T.prune_l2(tr, eta)
        assert used <= eta ** 2
        assert abs(_l2_gap(tr, pr) - used) <= 1e-10 * fn2
        # a valid redundant tree: the kept nodes keep their blocks, every internal node has its children
        idx = tr.index(pr.keys)
        assert np.all(idx >= 0) and np.array_equal(pr.coef, tr.coef[idx])
        internal = pr.keys[pr.leaf == 0]
        assert np.all(pr.index(T.children_keys(internal)) >= 0)
    assert T.prune_l2(tr, 0.0)[0].keys.size == tr.keys.size
    assert T.prune_l2(tr, 10.0 * np.sqrt(fn2))[0].keys.size == 1      # everything collapses to the root


def test_discard_uses_eps_times_the_norm():
    tr = _tree(seed=5)
    fn = float(np.sqrt(np.sum(tr.coef[tr.leaf == 1] ** 2)))
    a, ua = T.discard(tr, 1e-3)
    b, ub = T.prune_l2(tr, 1e-3 * fn)
    assert np.array_equal(a.keys, b.keys) and ua == ub
    assert a.keys.size < tr.keys.size
