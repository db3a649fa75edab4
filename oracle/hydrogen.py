"""The ground state of the hydrogen atom by the iteration of Sec. 6.2 (test infrastructure only).

phi = -2 G_mu V phi with G_mu = (-Delta + mu^2)^(-1) (kernel e^{-mu r} / (4 pi r)) and V = -Z / r; the
iteration applies G_mu with the modified ns-form and moves mu to sqrt(-2 E) until mu settles.

Readings of the paper taken here:
  * Domain: the physical cube [-L, L]^3 with the nucleus at its centre, mapped to the unit cube by
    x_u = (x + L) / s, s = 2 L; a tree on the unit cube holds the physical function's values.
    Physical integrals are s^3 times unit-cube ones, and the physical kernel becomes the unit-cube
    kernel s^2 e^{-(mu s) r_u} / (4 pi r_u) (the fit's scale s^2, its mu scaled by s).
  * Step 2's product: the paper refers to another paper for products of adaptively represented
    functions.  Here rho = c / r * f lives on f's tree with every leaf split once and the boxes whose
    closure holds the nucleus split further down to jmax; a leaf's block is the k-point rule (eq.
    fvals2coefs) of c / r times f's polynomial at the leaf's nodes (the nucleus is a corner of
    boxes on every scale, so no node falls on it).
  * Step 4's energy: the paper writes E = (1/2 <grad phi, grad phi> + <V phi, phi>) / <phi, phi> and
    refers elsewhere for weak derivatives.  With phi_new = -2 G_mu V phi_hat (phi_hat = phi / ||phi||),
    (-Delta + mu^2) phi_new = -2 V phi_hat, so 1/2 <grad phi_new, grad phi_new> = -<phi_new, V phi_hat>
    - mu^2 ||phi_new||^2 / 2 exactly; with rho = -2 V phi_hat:
        E = (<phi_new, rho> / 2 - mu^2 ||phi_new||^2 / 2 + <V phi_new, phi_new>) / ||phi_new||^2.
  * phi_new is discarded to eps ||phi_new|| (Alg. 3 Step 4) before its product, which would otherwise
    split every leaf once per iteration.
  * Inner products between a function and a product built on a refinement of its tree: the product's
    redundant tree holds the projections onto every coarser box, so <u, v> is the sum over u's leaves
    of the dot products with v's blocks at the same boxes (times s^3).
  * Start: phi_0 = (2/pi)^{3/4} e^{-r^2} (normalised), mu_0 given.
"""
import math

import numpy as np

from . import apply as A
from . import fit
from . import mra
from . import tree as T

__all__ = ["coulomb_product", "kalos", "nucleus_boxes"]


def nucleus_boxes(j):
    """Keys of the 8 boxes of scale j >= 1 whose closure holds the cube's centre."""
    h = 1 << (j - 1)
    out = []
    for s in range(8):
        out.append(int(T.make_keys(np.array([j]), np.array([h - 1 + (s & 1)]), np.array([h - 1 + ((s >> 1) & 1)]),
                                   np.array([h - 1 + ((s >> 2) & 1)]))[0]))
    return out


def coulomb_product(tree, c, jmax, s):
    """rho = c / r * f (r = s |x_u - 1/2|, the physical distance to the nucleus) on f's tree with every
    leaf split once and the boxes touching the nucleus split down to jmax; returns the redundant tree."""
    k = tree.k
    lk = tree.keys[tree.leaf == 1]
    kids = T.children_keys(lk)
    leaves = set(int(q) for q in kids)
    j, _ = T.decode_keys(np.array(sorted(leaves), dtype=np.uint64))
    top = int(j.max())
    for lev in range(1, max(jmax, top) + 1):
        for key in nucleus_boxes(lev):
            if key in leaves and lev < jmax:
                leaves.discard(key)
                leaves.update(int(q) for q in T.children_keys(np.array([key], dtype=np.uint64)))
    lk = np.array(sorted(leaves), dtype=np.uint64)
    lj, ll = T.decode_keys(lk)
    x, w = mra.gauss_legendre01(k)
    ph = mra.phi(k, x)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    unit = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)                  # k^3 nodes in a box
    pts = ((ll[:, None, :] + unit[None, :, :]) / (2.0 ** lj)[:, None, None]).reshape(-1, 3)
    vals = T.evaluate(tree, pts) * c / (s * np.linalg.norm(pts - 0.5, axis=1))
    vals = vals.reshape(lk.size, k, k, k) * (w[:, None, None] * w[None, :, None] * w[None, None, :])
    coef = np.einsum("nqrt,qa,rb,tc->nabc", vals, ph, ph, ph) * (2.0 ** (-1.5 * lj))[:, None, None, None]
    return T.redundant_tree(k, lk, coef)


def _leaf_dot(u, v):
    """sum over u's leaves of <u_leaf, v at the same box> (v's tree holds every box of u's leaves)."""
    idx = v.index(u.keys[u.leaf == 1])
    assert np.all(idx >= 0)
    return float(np.sum(u.coef[u.leaf == 1] * v.coef[idx]))


def kalos(k, eps, L, jmax, mu0=1.0, iters=6, Z=1.0, j0=2, leaves=None):
    """The iteration of Sec. 6.2; returns the list of (mu, E) after each step (and appends the leaf
    count of the rho each step applies to onto `leaves` when given a list)."""
    s = 2.0 * L
    a = s * s
    keys, coef = T.project_gaussians(k, eps, j0, jmax, [[0.5, 0.5, 0.5]], [a], [(2.0 / math.pi) ** 0.75 * (math.pi / a) ** 1.5])
    phi = T.redundant_tree(k, keys, coef)
    nphi = math.sqrt(s ** 3 * float(np.sum(phi.coef[phi.leaf == 1] ** 2)))
    rho = coulomb_product(phi, 2.0 * Z / nphi, jmax, s)                       # -2 V phi_hat
    mu = mu0
    hist = []
    for _ in range(iters):
        tau, w = fit.fit_kernel(mu * s, 1.0, eps, math.sqrt(eps) * 2.0 ** -rho.depth, math.sqrt(3.0), scale=s * s)
        op = A.Operator(k, tau, w, eps, rho.depth)
        if leaves is not None:
            leaves.append(int(np.sum(rho.leaf)))
        g = A.assemble(rho, A.apply_modified(op, rho))                          # phi_new on rho's tree
        lf = rho.leaf == 1
        n2 = s ** 3 * float(np.sum(g[lf] ** 2))
        ip1 = s ** 3 * float(np.sum(g[lf] * rho.coef[lf]))                     # <phi_new, rho>
        phin = T.redundant_tree(k, rho.keys[lf], g[lf])
        phin, _ = T.discard(phin, eps)
        rho_new = coulomb_product(phin, 2.0 * Z / math.sqrt(n2), jmax, s)       # -2 V phi_new / ||phi_new||
        ip2 = s ** 3 * _leaf_dot(phin, rho_new)                                 # <phi_new, rho_new>
        E = (0.5 * ip1 - 0.5 * mu * mu * n2 - 0.5 * math.sqrt(n2) * ip2) / n2
        hist.append((mu, E))
        mu = math.sqrt(-2.0 * E)
        rho = rho_new
    return hist
