"""Function trees of the oracle (test infrastructure only).

  * keys: level << 57 | morton(lx, ly, lz) with x in bit 0 of each bit triple; trees are arrays
    of nodes sorted by key (level-major, then Morton order).
  * project_gaussians: Alg. 1 (adaptive function decomposition) for a Gaussian-sum source,
    level by level from the coarse scale j0; a box is refined when, for any of its 8 children,
    the values interpolated from the box's coefficients differ from direct values at the child's
    Gauss-Legendre nodes by more than the threshold in the max norm; boxes at jmax are leaves.
    A leaf keeps its own coefficients (eq. fvals2coefs in 3-D).
  * redundant tree (Sec. 2.2.1): every ancestor of a leaf is stored too, with coefficients
    obtained bottom-up by the decomposition s^j_l = H0 s^{j+1}_{2l} + H1 s^{j+1}_{2l+1} applied
    along each of the three dimensions (App. A.3, eq. decomp_scaling).
  * evaluate: f(x) = 2^{3j/2} sum s_abc phi_a(2^j x - l1) phi_b(.) phi_c(.) on the leaf holding x
    (App. A.1, eqs. func_interp_1d/2d in 3-D); a point on a face belongs to the box with
    floor(2^j x) clamped to 2^j - 1.
  * details / detail_norms: the seven detail blocks of a sibling group, eq. decomp_wavelet along
    each dimension with G in at least one of them (App. A.2-A.3), and their squared norm.
  * prune_l2 (Sec. 2.2): on the redundant tree rebuilt from the leaves, starting on the finest
    scale, sibling groups are removed while the cumulative squared norm of the removed details
    stays within eta^2; by orthonormality that sum is exactly ||f - f_pruned||_2^2.  discard: the
    same at eta = eps ||f||_2 (Alg. 3 Step 4).
Readings: the refinement threshold is eps * ||f||_2 with the closed-form L2 norm of the
Gaussian sum over R^3 (the paper's absolute eps on a function scaled to unit norm); sources are
unit-mass Gaussians c_i (a_i/pi)^{3/2} exp(-a_i |x - x_i|^2).  Pruning: the cumulative
contribution of the removed blocks is their squared l2 norm, compared with eta^2; within a scale
the candidates (internal nodes whose eight children are leaves) are taken in ascending order of
that norm (ties by key), and a scale's first candidate that would exceed the budget ends that
scale; the remaining budget carries to the next coarser scale.
"""
import ctypes
import numpy as np

from . import mra
from ._native import lib

__all__ = ["make_keys", "decode_keys", "children_keys", "source_norm", "project_gaussians",
           "project_function", "redundant_tree", "compress", "upsample", "evaluate", "uniform_leaves", "Tree",
           "details", "reconstruct", "detail_norms", "prune_l2", "discard"]


def _spread3(v):
    v = np.asarray(v, dtype=np.uint64)
    r = np.zeros_like(v)
    for i in range(19):
        r |= ((v >> np.uint64(i)) & np.uint64(1)) << np.uint64(3 * i)
    return r


def _compact3(v):
    v = np.asarray(v, dtype=np.uint64)
    r = np.zeros_like(v)
    for i in range(19):
        r |= ((v >> np.uint64(3 * i)) & np.uint64(1)) << np.uint64(i)
    return r


def make_keys(j, lx, ly, lz):
    j = np.asarray(j, dtype=np.uint64)
    return (j << np.uint64(57)) | _spread3(lx) | (_spread3(ly) << np.uint64(1)) | (_spread3(lz) << np.uint64(2))


def decode_keys(keys):
    keys = np.asarray(keys, dtype=np.uint64)
    m = keys & np.uint64((1 << 57) - 1)
    j = (keys >> np.uint64(57)).astype(np.int64)
    l = np.stack([_compact3(m), _compact3(m >> np.uint64(1)), _compact3(m >> np.uint64(2))], axis=-1).astype(np.int64)
    return j, l


def children_keys(keys):
    """The 8 children of each key, child s = sx + 2 sy + 4 sz in Morton order."""
    j, l = decode_keys(keys)
    out = []
    for s in range(8):
        sx, sy, sz = s & 1, (s >> 1) & 1, (s >> 2) & 1
        out.append(make_keys(j + 1, 2 * l[:, 0] + sx, 2 * l[:, 1] + sy, 2 * l[:, 2] + sz))
    return np.stack(out, axis=1).ravel()


def source_norm(xyz, a, c):
    """||f||_2 over R^3 of f = sum_i c_i (a_i/pi)^{3/2} exp(-a_i |x - x_i|^2) (closed form)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    a = np.asarray(a, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    tot = 0.0
    for i in range(a.size):
        for q in range(a.size):
            s = a[i] + a[q]
            d2 = np.sum((xyz[i] - xyz[q]) ** 2)
            tot += c[i] * c[q] * (a[i] * a[q] / np.pi ** 2) ** 1.5 * (np.pi / s) ** 1.5 * np.exp(-a[i] * a[q] * d2 / s)
    return float(np.sqrt(tot))


class Tree:
    """Redundant tree: keys (sorted), leaf flags and coefficient blocks [N, k, k, k]."""

    def __init__(self, k, keys, leaf, coef):
        self.k = k
        self.keys = np.ascontiguousarray(keys, dtype=np.uint64)
        self.leaf = np.ascontiguousarray(leaf, dtype=np.uint8)
        self.coef = np.ascontiguousarray(coef, dtype=np.float64)
        self.level, self.l = decode_keys(self.keys)

    @property
    def depth(self):
        return int(self.level.max())

    def index(self, keys):
        keys = np.asarray(keys, dtype=np.uint64)
        pos = np.searchsorted(self.keys, keys)
        pos = np.minimum(pos, self.keys.size - 1)
        return np.where(self.keys[pos] == keys, pos, -1)


def project_gaussians(k, eps, j0, jmax, xyz, a, c, with_margins=False):
    """Alg. 1 for f = sum_i c_i (a_i/pi)^{3/2} exp(-a_i |x-x_i|^2).  Returns (leaf_keys, leaf_coef)
    sorted by key, and optionally the list of (err, thr) of every test made."""
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    a = np.ascontiguousarray(a, dtype=np.float64)
    cf = np.ascontiguousarray(np.asarray(c, dtype=np.float64) * (a / np.pi) ** 1.5)
    thr = eps * source_norm(xyz, a, c)
    gx, gw = mra.gauss_legendre01(k)
    n0 = 1 << j0
    lz, ly, lx = np.meshgrid(np.arange(n0), np.arange(n0), np.arange(n0), indexing="ij")
    cand = np.sort(make_keys(np.full(lx.size, j0), lx.ravel(), ly.ravel(), lz.ravel()))
    leaf_keys, leaf_coef, margins = [], [], []
    L = lib()
    j = j0
    while cand.size:
        n = cand.size
        s = np.zeros((n, k, k, k))
        ref = np.zeros(n, dtype=np.uint8)
        err = np.zeros(n)
        st = L.orc_project_level(k, j, jmax, n, cand.ctypes.data, a.size, xyz.ctypes.data, a.ctypes.data,
                                 cf.ctypes.data, thr, gx.ctypes.data, gw.ctypes.data, s.ctypes.data,
                                 ref.ctypes.data, err.ctypes.data)
        assert st == 0
        if j < jmax:
            margins.append(err)
        keep = ref == 0
        leaf_keys.append(cand[keep])
        leaf_coef.append(s[keep])
        cand = children_keys(cand[ref == 1])          # parents sorted -> children sorted
        j += 1
    keys = np.concatenate(leaf_keys)
    coef = np.concatenate(leaf_coef)
    order = np.argsort(keys, kind="stable")
    out = (keys[order], coef[order])
    if with_margins:
        return out + ((np.concatenate(margins) if margins else np.zeros(0), thr),)
    return out


def _modes(x, A1, A2, A3):
    """out[n, a, b, c] = sum_{ijk} x[n, i, j, k] A1[i, a] A2[j, b] A3[k, c], one mode at a time."""
    x = np.einsum("nijk,kc->nijc", x, A3)
    x = np.einsum("nijc,jb->nibc", x, A2)
    return np.einsum("nibc,ia->nabc", x, A1)


def project_function(k, eps, j0, jmax, f, fnorm, chunk=4096):
    """Alg. 1 for any source given as a vectorised callable f(x, y, z) -> values (numpy arrays of
    equal shape), with the refinement threshold eps * fnorm (fnorm: the caller's ||f||_2, the same
    reading as project_gaussians).  Level by level from j0: every candidate box gets its
    coefficients from the values at its own k^3 Gauss-Legendre nodes (eq. fvals2coefs in 3-D);
    the polynomial they define is evaluated at the k^3 nodes of each of the 8 children and
    compared with f there; the box is refined (all 8 children become candidates) when the
    largest difference exceeds the threshold, and boxes at jmax are leaves.
    Returns (leaf_keys, leaf_coef) sorted by key."""
    thr = eps * fnorm
    gx, gw = mra.gauss_legendre01(k)
    P = mra.phi(k, gx) * gw[:, None]                               # [node i, degree a]: phi_a(x_i) w_i
    Q = [mra.phi(k, 0.5 * (s + gx)) for s in (0, 1)]                # [node i, degree a]: phi_a((s + x_i)/2)
    n0 = 1 << j0
    lz, ly, lx = np.meshgrid(np.arange(n0), np.arange(n0), np.arange(n0), indexing="ij")
    cand = np.sort(make_keys(np.full(lx.size, j0), lx.ravel(), ly.ravel(), lz.ravel()))
    leaf_keys, leaf_coef = [], []
    j = j0
    while cand.size:
        h = 2.0 ** -j
        refine = np.zeros(cand.size, dtype=bool)
        coef = np.zeros((cand.size, k, k, k))
        for b0 in range(0, cand.size, chunk):
            _, l = decode_keys(cand[b0:b0 + chunk])
            X = h * (l[:, 0, None] + gx[None, :])                    # [box, node] per dimension
            Y = h * (l[:, 1, None] + gx[None, :])
            Z = h * (l[:, 2, None] + gx[None, :])
            fv = f(X[:, :, None, None], Y[:, None, :, None], Z[:, None, None, :])
            s = 2.0 ** (-1.5 * j) * _modes(fv, P, P, P)
            coef[b0:b0 + chunk] = s
            if j >= jmax:
                continue
            err = np.zeros(s.shape[0])
            for sg in range(8):
                sx, sy, sz = sg & 1, (sg >> 1) & 1, (sg >> 2) & 1
                ft = 2.0 ** (1.5 * j) * _modes(s, Q[sx].T, Q[sy].T, Q[sz].T)
                hc = 0.5 * h
                Xc = hc * (2 * l[:, 0, None] + sx + gx[None, :])
                Yc = hc * (2 * l[:, 1, None] + sy + gx[None, :])
                Zc = hc * (2 * l[:, 2, None] + sz + gx[None, :])
                fc = f(Xc[:, :, None, None], Yc[:, None, :, None], Zc[:, None, None, :])
                err = np.maximum(err, np.abs(fc - ft).reshape(s.shape[0], -1).max(axis=1))
            refine[b0:b0 + chunk] = err > thr
        leaf_keys.append(cand[~refine])
        leaf_coef.append(coef[~refine])
        cand = children_keys(cand[refine])
        j += 1
    keys = np.concatenate(leaf_keys)
    coef = np.concatenate(leaf_coef)
    order = np.argsort(keys, kind="stable")
    return keys[order], coef[order]


def project_boxes(k, eps, jmax, xyz, a, c, keys):
    """Alg. 1's step for arbitrary boxes: the projected coefficients, the refinement decision and
    the l-infinity test error of every box in keys (any levels, any order), made exactly as
    project_gaussians makes them; for checking sampled boxes of a tree too large to build here.
    Returns (coef [n, k, k, k], refine [n], err [n]) in the order of keys."""
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    a = np.ascontiguousarray(a, dtype=np.float64)
    cf = np.ascontiguousarray(np.asarray(c, dtype=np.float64) * (a / np.pi) ** 1.5)
    thr = eps * source_norm(xyz, a, c)
    gx, gw = mra.gauss_legendre01(k)
    keys = np.asarray(keys, dtype=np.uint64)
    lev, _ = decode_keys(keys)
    coef = np.zeros((keys.size, k, k, k))
    refine = np.zeros(keys.size, dtype=np.uint8)
    err = np.zeros(keys.size)
    L = lib()
    for j in np.unique(lev):
        sel = np.nonzero(lev == j)[0]
        cand = np.ascontiguousarray(keys[sel])
        n = cand.size
        s = np.zeros((n, k, k, k))
        ref = np.zeros(n, dtype=np.uint8)
        e = np.zeros(n)
        st = L.orc_project_level(k, int(j), jmax, n, cand.ctypes.data, a.size, xyz.ctypes.data, a.ctypes.data,
                                 cf.ctypes.data, thr, gx.ctypes.data, gw.ctypes.data, s.ctypes.data,
                                 ref.ctypes.data, e.ctypes.data)
        assert st == 0
        coef[sel], refine[sel], err[sel] = s, ref, e
    return coef, refine, err


def uniform_leaves(k, n, func_coef=None):
    """Keys of the uniform tree at level n (all 8^n boxes, sorted)."""
    m = 1 << n
    lz, ly, lx = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    return np.sort(make_keys(np.full(lx.size, n), lx.ravel(), ly.ravel(), lz.ravel()))


def _apply_sep(A1, A2, A3, x):
    """(A1 (x) A2 (x) A3) applied to blocks x[..., a, b, c]."""
    return np.einsum("ia,jb,kc,...abc->...ijk", A1, A2, A3, x)


def compress(k, child_coef):
    """Parent block from its 8 children (child s = sx + 2 sy + 4 sz): eq. decomp_scaling per dim."""
    H = mra.two_scale_filters(k)
    out = 0.0
    for s in range(8):
        out = out + _apply_sep(H[s & 1], H[(s >> 1) & 1], H[(s >> 2) & 1], child_coef[..., s, :, :, :])
    return out


def upsample(k, parent_coef):
    """The 8 children of a block with zero details: child_s = (H^{sx}T (x) H^{sy}T (x) H^{sz}T) parent."""
    H = mra.two_scale_filters(k)
    return np.stack([_apply_sep(H[s & 1].T, H[(s >> 1) & 1].T, H[(s >> 2) & 1].T, parent_coef)
                     for s in range(8)], axis=-4)


def redundant_tree(k, leaf_keys, leaf_coef):
    """Redundant tree from the leaves (Sec. 2.2.1): all ancestors are added and their blocks are
    computed bottom-up with compress()."""
    leaf_keys = np.asarray(leaf_keys, dtype=np.uint64)
    j, l = decode_keys(leaf_keys)
    allk = [leaf_keys]
    for lev in range(int(j.max()), 0, -1):
        sel = j >= lev
        anc_j = np.minimum(j[sel], lev) - 1
        sh = (j[sel] - anc_j)[:, None]
        anc = make_keys(anc_j, *(l[sel] >> sh).T)
        allk.append(anc)
    keys = np.unique(np.concatenate(allk))
    N = keys.size
    leaf = np.zeros(N, dtype=np.uint8)
    coef = np.zeros((N, k, k, k))
    pos = np.searchsorted(keys, leaf_keys)
    leaf[pos] = 1
    coef[pos] = leaf_coef
    lev, _ = decode_keys(keys)
    for lv in range(int(lev.max()) - 1, -1, -1):
        internal = np.nonzero((lev == lv) & (leaf == 0))[0]
        if internal.size == 0:
            continue
        ch = np.searchsorted(keys, children_keys(keys[internal])).reshape(-1, 8)
        coef[internal] = compress(k, coef[ch])
    return Tree(k, keys, leaf, coef)


def evaluate(tree, pts):
    """f at points (P, 3) in [0,1]^3 from the leaf blocks (App. A.1, eq. func_interp in 3-D)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    k = tree.k
    out = np.full(pts.shape[0], np.nan)
    todo = np.arange(pts.shape[0])
    for j in range(tree.depth + 1):
        if todo.size == 0:
            break
        side = 1 << j
        l = np.minimum(np.floor(pts[todo] * side).astype(np.int64), side - 1)
        idx = tree.index(make_keys(np.full(todo.size, j), l[:, 0], l[:, 1], l[:, 2]))
        hit = (idx >= 0)
        hit[hit] = tree.leaf[idx[hit]] == 1
        if hit.any():
            p = todo[hit]
            u = pts[p] * side - l[hit]
            px, py, pz = mra.phi(k, u[:, 0]), mra.phi(k, u[:, 1]), mra.phi(k, u[:, 2])
            out[p] = 2.0 ** (1.5 * j) * np.einsum("pabc,pa,pb,pc->p", tree.coef[idx[hit]], px, py, pz)
        todo = todo[~hit]
    return out


def _modes3(A1, A2, A3, x):
    """(A1 (x) A2 (x) A3) applied to blocks x[..., a, b, c], one dimension at a time."""
    y = np.einsum("ia,...abc->...ibc", A1, x)
    y = np.einsum("jb,...ibc->...ijc", A2, y)
    return np.einsum("kc,...ijc->...ijk", A3, y)


def details(k, child_coef):
    """(s, d) of sibling groups child_coef[..., 8, k, k, k] (child s = sx + 2 sy + 4 sz): s the
    parent block (eq. decomp_scaling per dimension) and d[..., 7, k, k, k] the detail blocks
    (eq. decomp_wavelet), block t = tx + 2 ty + 4 tz (t = 1..7) with G along the dimensions whose
    bit is set and H along the others."""
    H = mra.two_scale_filters(k)
    G = mra.wavelet_filters(k)
    out = []
    for t in range(8):
        F = [G if (t >> d) & 1 else H for d in range(3)]
        acc = 0.0
        for s in range(8):
            acc = acc + _modes3(F[0][s & 1], F[1][(s >> 1) & 1], F[2][(s >> 2) & 1], child_coef[..., s, :, :, :])
        out.append(acc)
    return out[0], np.stack(out[1:], axis=-4)


def reconstruct(k, parent_coef, detail):
    """The eight children from the parent block and its seven detail blocks (eqs. recon_even/odd
    per dimension, with the transposed filters)."""
    H = mra.two_scale_filters(k)
    G = mra.wavelet_filters(k)
    blocks = [parent_coef] + [detail[..., t - 1, :, :, :] for t in range(1, 8)]
    kids = []
    for s in range(8):
        acc = 0.0
        for t in range(8):
            F = [G if (t >> d) & 1 else H for d in range(3)]
            acc = acc + _modes3(F[0][s & 1].T, F[1][(s >> 1) & 1].T, F[2][(s >> 2) & 1].T, blocks[t])
        kids.append(acc)
    return np.stack(kids, axis=-4)


def detail_norms(tree):
    """||d||_2^2 of every internal node's sibling group (0 at leaves), in node order."""
    out = np.zeros(tree.keys.size)
    internal = np.nonzero(tree.leaf == 0)[0]
    if internal.size:
        ch = tree.index(children_keys(tree.keys[internal])).reshape(-1, 8)
        _, d = details(tree.k, tree.coef[ch])
        out[internal] = np.sum(d.reshape(internal.size, -1) ** 2, axis=1)
    return out


def prune_l2(tree, eta):
    """Sec. 2.2's l2 pruning, within eta (absolute), of the function that the tree's leaves
    represent: returns (pruned Tree, the removed squared norm <= eta^2).  The internal nodes are
    first rebuilt from the leaves by the two-scale decomposition (a tree from an apply holds the
    assembled partial sums there, which are not the leaves' coarse projections); the kept nodes
    then keep those blocks."""
    tree = redundant_tree(tree.k, tree.keys[tree.leaf == 1], tree.coef[tree.leaf == 1])
    dn = detail_norms(tree)
    leaf = tree.leaf.copy()
    alive = np.ones(tree.keys.size, dtype=bool)
    budget = float(eta) ** 2
    used = 0.0
    for j in range(tree.depth - 1, -1, -1):
        nodes = np.nonzero((tree.level == j) & (leaf == 0) & alive)[0]
        if nodes.size == 0:
            continue
        ch = tree.index(children_keys(tree.keys[nodes])).reshape(-1, 8)
        cand = nodes[np.all(leaf[ch] == 1, axis=1)]
        order = np.lexsort((tree.keys[cand], dn[cand]))
        for i in cand[order]:
            if used + dn[i] > budget:
                break
            used += dn[i]
            leaf[i] = 1
            alive[tree.index(children_keys(tree.keys[i:i + 1]))] = False
    # descendants of removed children go too (they are leaves by construction: only groups whose
    # children are all leaves are removed)
    keep = np.nonzero(alive)[0]
    return Tree(tree.k, tree.keys[keep], leaf[keep], tree.coef[keep]), used


def discard(tree, eps):
    """Alg. 3 Step 4 at the requested accuracy: prune_l2 within eps ||f||_2, where ||f||_2^2 is the
    sum of the squared leaf blocks (orthonormal basis)."""
    fn = float(np.sqrt(np.sum(tree.coef[tree.leaf == 1] ** 2)))
    return prune_l2(tree, eps * fn)
