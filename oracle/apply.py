"""Operator apply of the oracle (test infrastructure only).

  * Operator: F tables for scales 0..nlev (eq. KernelFactor) and the screening plan (plan.py).
  * apply_modified: ghat on requested nodes by the modified ns-form (eq. apply_algo, Alg. 3
    Steps 1-3); see ns_core.c for the per-term coefficient rule.
  * apply_difference: ghat by the banded difference form (eq. g_scales_band) -- after assembly it
    must agree with apply_modified for any tree and plan (down-up identity, eq. down_up).
  * assemble: g_child = ghat_child + up(g_parent), top-down from the root (eq. g_assemble,
    Alg. 3 Step 4); leaves hold g.
  * dense_uniform: the plain definition P_n T P_n f on a uniform tree at level n: every pair of
    level-n boxes and every Gaussian term, g_b = sum_{b'} sum_m w_m (F^{n;m,l1} (x) F^{n;m,l2}
    (x) F^{n;m,l3}) f_{b'} with l = b - b' (eqs. KernelApproxByGaussians1/2), no screening.
"""
import numpy as np

from . import mra
from . import plan as _plan
from ._native import lib
from .tree import Tree, children_keys, upsample

__all__ = ["Operator", "apply_modified", "apply_difference", "assemble", "dense_uniform", "full_plan"]


class Operator:
    """F tables for scales 0..nlev and the plan R[j, L] (j = 0..nlev)."""

    def __init__(self, k, tau, w, eps, nlev, group=True, R=None, allow_overflow=False):
        self.k, self.eps, self.nlev = k, eps, nlev
        self.tau = np.ascontiguousarray(tau, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.M = self.tau.size
        self.F = np.ascontiguousarray(mra.F_table(k, self.tau, nlev))
        self.H0, self.H1 = (np.ascontiguousarray(h) for h in mra.two_scale_filters(k))
        if R is None:
            R, self.theta = _plan.make_plan(self.F, self.H0, self.H1, self.w, eps, nlev, group=group,
                                            allow_overflow=allow_overflow)
        self.R = np.ascontiguousarray(R, dtype=np.int32)


def full_plan(M, nlev):
    """Screening off: every term at every |L_d| <= 3 on every scale."""
    n7 = 2 * _plan.LMAX + 1
    R = np.empty((nlev + 1, n7, n7, n7, 2), dtype=np.int32)
    R[..., 0] = 0
    R[..., 1] = M - 1
    R[0] = _plan.EMPTY
    R[0, 3, 3, 3] = (0, M - 1)
    return R


def _run(name, op, tree, out_idx):
    if out_idx is None:
        out_idx = np.arange(tree.keys.size)
    out_idx = np.ascontiguousarray(out_idx, dtype=np.int64)
    k = tree.k
    ghat = np.zeros((out_idx.size, k, k, k))
    fn = getattr(lib(), name)
    st = fn(k, tree.keys.size, tree.keys.ctypes.data, tree.leaf.ctypes.data, tree.coef.ctypes.data,
            op.M, op.w.ctypes.data, op.F.shape[0], op.F.ctypes.data, op.R.shape[0], op.R.ctypes.data,
            op.H0.ctypes.data, op.H1.ctypes.data, out_idx.size, out_idx.ctypes.data, ghat.ctypes.data)
    if st != 0:
        raise RuntimeError("%s failed with status %d" % (name, st))
    return ghat


def apply_modified(op, tree, out_idx=None):
    """ghat on the nodes out_idx (default: all) by the modified ns-form."""
    return _run("orc_apply_modified", op, tree, out_idx)


def apply_difference(op, tree, out_idx=None):
    """ghat on the nodes out_idx (default: all) by the banded difference form."""
    return _run("orc_apply_difference", op, tree, out_idx)


def assemble(tree, ghat):
    """g on every node: g_root = ghat_root, g_child = ghat_child + up(g_parent) (eq. g_assemble)."""
    k = tree.k
    g = np.array(ghat, dtype=np.float64, copy=True)
    for lv in range(tree.depth):
        internal = np.nonzero((tree.level == lv) & (tree.leaf == 0))[0]
        if internal.size == 0:
            continue
        ch = np.searchsorted(tree.keys, children_keys(tree.keys[internal])).reshape(-1, 8)
        g[ch] += upsample(k, g[internal])
    return g


def assemble_chain(tree, idx, ghat_of):
    """g at node idx from ghat on the node and its ancestors (a callable index -> ghat block)."""
    j = int(tree.level[idx])
    l = tree.l[idx]
    chain = []
    for lev in range(j + 1):
        from .tree import make_keys
        key = make_keys(np.array([lev]), *(l[None, :] >> (j - lev)).T)
        chain.append(int(tree.index(key)[0]))
    H = mra.two_scale_filters(tree.k)
    g = ghat_of(chain[0]).copy()
    for lev in range(1, j + 1):
        s = tree.l[chain[lev]] & 1
        g = np.einsum("ia,jb,kc,abc->ijk", H[s[0]].T, H[s[1]].T, H[s[2]].T, g) + ghat_of(chain[lev])
    return g


def dense_uniform(op, tree):
    """P_n T P_n f on a uniform tree at level n <= 3 (the plain definition; blocks ordered by key).
    Per term m the operator is G^m (x) G^m (x) G^m with the 1-D matrix
    G^m[(x, a), (x', b)] = F^{n;m, x-x'}_ab over all level-n positions (eq. KernelApproxByGaussians2),
    applied to f laid out on the full level-n grid.  Returns g on the level-n boxes in tree order."""
    n = tree.depth
    assert n <= 3, "the F tables span |l| <= 7"
    k, side = tree.k, 1 << n
    sel = np.nonzero(tree.level == n)[0]
    L = tree.l[sel]
    grid = np.zeros((side, k, side, k, side, k))
    for i, (x, y, z) in enumerate(L):
        grid[x, :, y, :, z, :] = tree.coef[sel[i]]
    out = np.zeros_like(grid)
    pos = np.arange(side)
    for m in range(op.M):
        d = pos[:, None] - pos[None, :] + 7
        G = op.F[n, m][d]                                 # [x, x', a, b]
        out += op.w[m] * np.einsum("xuap,yvbq,zwcr,upvqwr->xaybzc", G, G, G, grid, optimize=True)
    return np.stack([out[x, :, y, :, z, :] for (x, y, z) in L])
