"""The apply's flop accounting against an independent replay of its job rules.

The roofline of the contraction kernels divides the method's own flops by the kernel time, so the
counts the library reports are checked here from the plan and the tree alone: jobs are boxes of
coarse displacements L on which a plan row is constant (split to extents of at most 4), whole-band
jobs at every sibling group, down-band jobs (the finer plan row, fine displacements l = 2L + s - s')
at groups with internal children; a job over n1 x n2 x n3 in-cube displacements costs
2 (2k)^4 (n1 n2 n3 + n1 n2 + n1) flops per term (Sec. 5's factorisation).  Own work drops the
down-band jobs nested in the whole band and, of each whole-band job, the share of its (child, L,
input child, term) pairs with net coefficient 0 under eq. apply_algo: an internal child s and a term
in R_{j+1}(2L + s - s')."""
import itertools
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

LP, LF, NMAX = 3, 7, 4


def _segments(row, d):
    def sl(t):
        idx = [slice(None)] * 3
        idx[d] = t + LP
        return row[tuple(idx)]
    seg, start = [], -LP
    for t in range(-LP, LP):
        a, b = sl(t), sl(t + 1)
        ea, eb = a[..., 1] < a[..., 0], b[..., 1] < b[..., 0]
        if not (np.array_equal(ea, eb) and np.all((a == b)[~ea])):
            seg.append((start, t))
            start = t + 1
    seg.append((start, LP))
    return seg


def _jobs(row, down):
    s = [_segments(row, d) for d in range(3)]
    out = []
    for cell in itertools.product(*s):
        r = row[cell[0][0] + LP, cell[1][0] + LP, cell[2][0] + LP]
        if r[1] < r[0]:
            continue
        if down:
            lo = [math.ceil((c[0] - 1) / 2) for c in cell]
            hi = [math.floor((c[1] + 1) / 2) for c in cell]
        else:
            lo, hi = [c[0] for c in cell], [c[1] for c in cell]
        cuts = [[(x, min(hi[d], x + NMAX - 1)) for x in range(lo[d], hi[d] + 1, NMAX)] for d in range(3)]
        for bx in itertools.product(*cuts):
            out.append((down, [b[0] for b in bx], [b[1] for b in bx], int(r[0]), int(r[1])))
    return out


def _nested(row, lo, hi, m1, m2):
    """Every term of a down-band job lies in the whole band's range at every L of its box."""
    for L in itertools.product(*[range(lo[d], hi[d] + 1) for d in range(3)]):
        if max(abs(x) for x in L) > LP:
            return False
        r = row[L[0] + LP, L[1] + LP, L[2] + LP]
        if not (r[0] <= m1 and m2 <= r[1]):
            return False
    return True


def replay(tree, R, k):
    """(executed flops, own flops) of one apply of plan R to the redundant tree."""
    lev = tree.level
    depth = int(lev.max())
    unit = 2.0 * (2 * k) ** 4
    sig = np.array([[(s >> d) & 1 for d in range(3)] for s in range(8)])
    deltas = list(itertools.product((-1, 0, 1), repeat=3))
    executed = own = 0.0
    for j in range(0, depth + 1):
        idx = np.nonzero(lev == j)[0]
        if j == 0:
            # the root is a group of one node: L = 0 only; the down band when the root is internal
            r = R[0, LP, LP, LP]
            nt = r[1] - r[0] + 1 if r[1] >= r[0] else 0
            executed += nt * 3 * unit
            own += nt * 3 * unit
            for (_, lo, hi, m1, m2) in (_jobs(R[1], True) if depth >= 1 else []):
                if tree.leaf[0] or any(lo[d] > 0 or hi[d] < 0 for d in range(3)):
                    continue
                fl = (m2 - m1 + 1) * 3 * unit
                executed += fl
                if not _nested(R[0], lo, hi, m1, m2):
                    own += fl
            continue
        nb = idx.size // 8
        ch = idx.reshape(nb, 8)
        internal = 1 - tree.leaf[ch].astype(np.int64)
        anyint = internal.any(1)
        p = tree.l[ch[:, 0]] >> 1
        side = 1 << (j - 1)
        cnt = np.zeros((nb, 27))
        for di, dl in enumerate(deltas):
            ok = np.ones(8, bool)
            for d in range(3):
                sp = sig[:, d] - dl[d]
                ok &= (sp >= 0) & (sp <= 1)
            cnt[:, di] = (internal * ok[None, :]).sum(1)
        has_down = j < depth and j + 1 < R.shape[0]
        jobs = _jobs(R[j], False) + (_jobs(R[j + 1], True) if has_down else [])
        for (down, lo, hi, m1, m2) in jobs:
            nin = [np.maximum(0, np.minimum(hi[d], p[:, d]) - np.maximum(lo[d], p[:, d] - side + 1) + 1) for d in range(3)]
            cells = nin[0] * nin[1] * nin[2]
            steps = np.where(cells == 0, 0, cells + nin[0] * nin[1] + nin[0])
            nt = m2 - m1 + 1
            fl = nt * steps * unit * (anyint if down else 1)
            executed += fl.sum()
            if down:
                if not _nested(R[j], lo, hi, m1, m2):
                    own += fl.sum()
                continue
            canc = np.zeros(nb)
            if has_down:
                for L in itertools.product(*[range(lo[d], hi[d] + 1) for d in range(3)]):
                    ind = np.ones(nb, bool)
                    for d in range(3):
                        ind &= (p[:, d] - L[d] >= 0) & (p[:, d] - L[d] < side)
                    for di, dl in enumerate(deltas):
                        ll = [2 * L[d] + dl[d] for d in range(3)]
                        if max(abs(x) for x in ll) > LP:
                            continue
                        r = R[j + 1][ll[0] + LP, ll[1] + LP, ll[2] + LP]
                        o = max(0, min(r[1], m2) - max(r[0], m1) + 1)
                        if o:
                            canc += ind * cnt[:, di] * o
            share = np.where(cells > 0, canc / np.maximum(64.0 * nt * cells, 1.0), 0.0)
            own += (fl * (1.0 - share)).sum()
    return executed, own


@pytest.mark.parametrize("case", ["k6", "c2"])
def test_flop_accounting_matches_replay(case):
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_0706_0747_amd as M
    from oracle import apply as A
    from oracle import fit
    from oracle import tree as T
    w = workloads.small_adaptive(11, k=6, eps=1e-4, jmax=5) if case == "k6" else workloads.c2()
    ctx = M.Context(0)
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    ot = T.redundant_tree(w.k, keys, coef)
    tau, wt = fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -ot.depth, math.sqrt(3))
    oo = A.Operator(w.k, tau, wt, w.eps, ot.depth)
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, ot.depth)
    M.mwns_op_plan_import(op, oo.R)
    f = M.mwns_tree_from_leaves(ctx, w.k, ot.keys[ot.leaf == 1], ot.coef[ot.leaf == 1])
    _, st = M.mwns_apply(ctx, op, f)
    ex, own = replay(ot, oo.R, w.k)
    print("%s: executed %.6e (library %.6e), own %.6e (library %.6e), own/executed %.4f"
          % (case, ex, st["useful_flops"], own, st["own_flops"], own / ex), flush=True)
    assert abs(st["useful_flops"] - ex) <= 1e-12 * ex
    assert abs(st["own_flops"] - own) <= 1e-9 * ex
    assert own < ex
