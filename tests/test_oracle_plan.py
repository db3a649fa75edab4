"""Pins of the oracle's screening plan (Sec. 4, eqs. norm_estimate_ndim, BlockNorms,
NormEstimateUsing1DBlocks)."""
import itertools
import math

import numpy as np
import pytest

from oracle import fit, mra
from oracle import plan as P


@pytest.fixture(scope="module")
def op_tables():
    k, eps, n = 6, 1e-4, 3
    tau, w = fit.fit_kernel(0.0, 1.0, eps, math.sqrt(eps) * 2 ** -n, math.sqrt(3))
    F = mra.F_table(k, tau, n + 1)
    H0, H1 = mra.two_scale_filters(k)
    return k, eps, n, tau, w, F, H0, H1


def test_term_range_is_the_maximal_discard():
    """Brute force: the kept range [m1, m2] removes the longest prefix and the longest suffix whose
    sums stay <= theta/2, and is empty iff the total is <= theta."""
    rng = np.random.default_rng(0)
    for _ in range(300):
        e = rng.exponential(size=rng.integers(1, 12)) * (rng.random() < 0.9)
        theta = rng.uniform(0, 1.5) * e.sum() + 1e-12
        m1, m2 = P.term_range(e, theta)
        if e.sum() <= theta:
            assert (m1, m2) == P.EMPTY
            continue
        best_pre = max(i for i in range(len(e) + 1) if e[:i].sum() <= theta / 2)
        best_suf = max(i for i in range(len(e) + 1) if e[len(e) - i:].sum() <= theta / 2)
        assert m1 == best_pre and m2 == len(e) - 1 - best_suf and m1 <= m2


def test_estimate_bounds_the_true_difference_norm(op_tables):
    """||S1 (x) S2 (x) S3 - U1 (x) U2 (x) U3||_F <= est (triangle inequality on the telescoped
    difference, each of the 6 orderings being a bound), checked on explicit Kronecker products."""
    k, eps, n, tau, w, F, H0, H1 = op_tables
    H = np.concatenate([H0, H1], axis=1)
    for j in (1, 3):
        NF, NU, ND = P.block_norms(F, H0, H1, j)
        for m in (5, 25, 40):
            S = {L: np.block([[F[j, m, 2 * L + 7], F[j, m, 2 * L - 1 + 7]], [F[j, m, 2 * L + 1 + 7], F[j, m, 2 * L + 7]]])
                 for L in range(3)}
            U = {L: H.T @ F[j - 1, m, L + 7] @ H for L in range(3)}
            for Lc in [(0, 0, 0), (0, 1, 2), (1, 1, 0), (2, 2, 1)]:
                A = np.kron(np.kron(S[Lc[0]], S[Lc[1]]), S[Lc[2]])
                B = np.kron(np.kron(U[Lc[0]], U[Lc[1]]), U[Lc[2]])
                true = np.linalg.norm(A - B)
                est = P.estimate(NF, NU, ND, tuple(sorted(Lc)))[m]
                assert true <= est * (1 + 1e-12) + 1e-300
                assert np.isclose(NF[m, Lc[0]], np.linalg.norm(S[Lc[0]]))


def test_plan_symmetry_monotonicity_and_grouping(op_tables):
    k, eps, n, tau, w, F, H0, H1 = op_tables
    R, th = P.make_plan(F, H0, H1, w, eps, n + 1, group=False)
    Rg, _ = P.make_plan(F, H0, H1, w, eps, n + 1, group=True)
    R2, _ = P.make_plan(F, H0, H1, w, eps / 10, n + 1, group=False)
    for j in range(1, n + 2):
        for L in itertools.product(range(-3, 4), repeat=3):
            i = tuple(x + 3 for x in L)
            for perm in itertools.permutations(range(3)):
                for sg in itertools.product((-1, 1), repeat=3):
                    Lq = tuple(sg[d] * L[perm[d]] + 3 for d in range(3))
                    assert tuple(R[j][Lq]) == tuple(R[j][i])
            a, b = R[j][i]
            if b >= a:
                ag, bg = Rg[j][i]
                a2, b2 = R2[j][i]
                assert ag <= a and bg >= b          # grouping keeps a superset
                assert a2 <= a and b2 >= b          # smaller eps keeps a superset
    # root row: every term at L = 0 only
    assert tuple(R[0][3, 3, 3]) == (0, len(w) - 1)
    assert (R[0][..., 1] < R[0][..., 0]).sum() == 7 ** 3 - 1


def test_band_overflow_is_reported():
    """A term kept at the edge of the band (max |L_d| = 3) means displacements beyond the band
    would still matter: few vanishing moments (k = 2) at a small eps do that, the configurations
    of the workloads do not."""
    from oracle import apply as A
    tau, wt = fit.fit_kernel(0.0, 1.0, 1e-4, 1e-2 * 2.0 ** -4, math.sqrt(3))
    with pytest.raises(P.BandOverflow):
        A.Operator(2, tau, wt, 1e-4, 4)
    op = A.Operator(2, tau, wt, 1e-4, 4, allow_overflow=True)
    edge = op.R[1:, [0, 6]]     # L_1 = -3 or 3
    assert np.any(edge[..., 1] >= edge[..., 0])
    A.Operator(6, tau, wt, 1e-4, 4)     # within the band: no error
