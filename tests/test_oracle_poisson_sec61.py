"""The paper's own end-to-end accuracy test (Sec. 6.1, Table 2) on the oracle: the Poisson
equation with the source rho = -Laplacian(phi) of three Gaussians (alpha = 300), whose exact
potential under 1/(4 pi r) is phi itself.  The whole chain -- Alg. 1 on rho, the Gaussian-sum fit
of the kernel, the operator blocks and screening plan, the modified ns-form apply and the
assembly -- runs as the library's readings take it, and its errors are held against the values
the paper prints (tests/golden/table2_poisson.txt).

E2 is read as the relative L2 error over the unit cube (integrated on every leaf with a
(k+6)-point Gauss-Legendre rule), Einf as max |g - phi| / max |phi| over 1e4 seeded points."""
import math
import os

import numpy as np
import pytest

import workloads
from oracle import apply as A
from oracle import closed_forms as C
from oracle import fit, mra
from oracle import tree as T


def _table2():
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "table2_poisson.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                eps, p, e2, einf = line.split()
                rows.append((float(eps), int(p), float(e2), float(einf)))
    return rows


def sec61_potential(k, eps):
    """(tree of rho, g on every node) for the Sec. 6.1 test at order k and accuracy eps."""
    keys, coef = T.project_function(k, eps, 2, 12, C.three_gaussians_laplacian, C.three_gaussians_laplacian_l2norm())
    tr = T.redundant_tree(k, keys, coef)
    tau, wt = fit.fit_kernel(0.0, 1.0, eps, math.sqrt(eps) * 2.0 ** -tr.depth, math.sqrt(3))
    op = A.Operator(k, tau, wt, eps, tr.depth)
    return tr, A.assemble(tr, A.apply_modified(op, tr))


def relative_l2_error(tr, g):
    """||g - phi||_2 / ||phi||_2 over the cube, leaf by leaf with (k+6)-point Gauss-Legendre."""
    k = tr.k
    q, qw = mra.gauss_legendre01(k + 6)
    ph = mra.phi(k, q)
    W = qw[:, None, None] * qw[None, :, None] * qw[None, None, :]
    num = den = 0.0
    for j in np.unique(tr.level[tr.leaf == 1]):
        sel = np.nonzero((tr.leaf == 1) & (tr.level == j))[0]
        h = 2.0 ** -int(j)
        l = tr.l[sel]
        X, Y, Z = (h * (l[:, d, None] + q[None, :]) for d in range(3))
        ex = C.three_gaussians(X[:, :, None, None], Y[:, None, :, None], Z[:, None, None, :])
        gv = 2.0 ** (1.5 * int(j)) * np.einsum("nabc,ia,jb,kc->nijk", g[sel], ph, ph, ph, optimize=True)
        num += h ** 3 * np.sum(W * (gv - ex) ** 2)
        den += h ** 3 * np.sum(W * ex ** 2)
    return math.sqrt(num / den)


@pytest.mark.parametrize("eps,p,e2_paper,einf_paper", _table2())
def test_sec61_poisson_against_table2(eps, p, e2_paper, einf_paper):
    tr, g = sec61_potential(p, eps)
    e2 = relative_l2_error(tr, g)
    P = workloads.points(10000)
    v = T.evaluate(T.Tree(p, tr.keys, tr.leaf, g), P)
    ex = C.three_gaussians(P[:, 0], P[:, 1], P[:, 2])
    einf = np.abs(v - ex).max() / np.abs(ex).max()
    # the paper's trees and term counts are not printed, so E2 is held to the paper's value within a
    # factor of 4 either way (measured 0.6x-2.8x); Einf at or below the paper's
    assert e2_paper / 4 <= e2 <= 4 * e2_paper, (e2, e2_paper)
    assert einf <= einf_paper, (einf, einf_paper)
