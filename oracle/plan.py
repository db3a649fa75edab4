"""Screening plan of the modified ns-form (test infrastructure only).

For every scale j >= 1, Gaussian term m and coarse displacement L (a displacement between the
parents of the fine output and input boxes) the oracle follows Sec. 4:
  1-D blocks (eq. BlockNorms), read on coarse-indexed 2k x 2k super-blocks:
      S^{j;m,L} = [[F^{j;m,2L}, F^{j;m,2L-1}], [F^{j;m,2L+1}, F^{j;m,2L}]]   rows = output parity
      U^{j;m,L} = [H0 H1]^T F^{j-1;m,L} [H0 H1]                            (the upsampled coarse block)
      N_F = ||S||_F,  N_upF = ||U||_F,  N_dif = ||S - U||_F
  3-D estimate (eq. NormEstimateUsing1DBlocks) of ||T_j^L - up(T_{j-1}^L)|| for term m:
      est_m(L) = 1/6 sum over the 6 orderings (p,q,r) of (L1,L2,L3) of
                 N_dif(p) N_F(q) N_F(r) + N_upF(p) N_dif(q) N_F(r) + N_upF(p) N_upF(q) N_dif(r)
  term range: e_m = w_m est_m(L); the longest prefix and the longest suffix of m whose
      cumulative sums stay <= theta/2 are discarded, leaving [m1, m2]; the range is empty when
      sum_m e_m <= theta (Sec. 4's term screening: terms whose summed contribution is small
      against eps are dropped).
  theta = eps * sum_m w_m ||F^{0;m,0}||_F^3 (a scale-independent operator norm; reading).
  The kernel is radial, so norms are taken at |L| and the 3-D estimate at the sorted |L_d|;
  every sign/permutation variant of L gets the range of its canonical representative.
  Grouping (Sec. 4, the Core and Boundary-1/2/3 sets): with group=True every L gets the union
  (hull) of the ranges of the set it belongs to, where a coordinate is in the core when
  |L_d| <= 1.
The plan is returned as an int32 array R[j, L1+Lmax, L2+Lmax, L3+Lmax, 2] of inclusive 0-based
(m1, m2); an empty range is (0, -1).  Row j = 0 holds the root: all terms at L = 0.
"""
import itertools
import numpy as np

__all__ = ["block_norms", "estimate", "term_range", "make_plan", "BandOverflow", "LMAX", "EMPTY"]

LMAX = 3
EMPTY = (0, -1)


def block_norms(Ftab, H0, H1, j, lmax_f=7):
    """(N_F, N_upF, N_dif) arrays of shape (M, LMAX+1) for scale j >= 1 at L = 0..LMAX
    (eq. BlockNorms with the super-block reading).  Ftab[j, m, l+lmax_f] holds F^{j;m,l}."""
    M, k = Ftab.shape[1], Ftab.shape[3]
    H = np.concatenate([H0, H1], axis=1)                 # k x 2k
    NF = np.zeros((M, LMAX + 1))
    NU = np.zeros((M, LMAX + 1))
    ND = np.zeros((M, LMAX + 1))
    for m in range(M):
        for L in range(LMAX + 1):
            f = lambda l: Ftab[j, m, l + lmax_f]
            S = np.block([[f(2 * L), f(2 * L - 1)], [f(2 * L + 1), f(2 * L)]])
            U = H.T @ Ftab[j - 1, m, L + lmax_f] @ H
            NF[m, L] = np.linalg.norm(S)
            NU[m, L] = np.linalg.norm(U)
            ND[m, L] = np.linalg.norm(S - U)
    return NF, NU, ND


def estimate(NF, NU, ND, Lc):
    """est_m(L) for all m at canonical |L| = Lc (eq. NormEstimateUsing1DBlocks)."""
    tot = np.zeros(NF.shape[0])
    for (p, q, r) in itertools.permutations(Lc):
        tot += ND[:, p] * NF[:, q] * NF[:, r] + NU[:, p] * ND[:, q] * NF[:, r] + NU[:, p] * NU[:, q] * ND[:, r]
    return tot / 6.0


def term_range(e, theta):
    """[m1, m2] kept after discarding prefix and suffix with cumulative contribution <= theta/2;
    EMPTY when the whole sum is <= theta (Sec. 4)."""
    c = np.cumsum(e)                                      # sequential cumulative contributions
    if c[-1] <= theta:
        return EMPTY
    m1 = int(np.argmax(c > 0.5 * theta))
    cs = np.cumsum(e[::-1])
    m2 = len(e) - 1 - int(np.argmax(cs > 0.5 * theta))
    return (m1, m2)


def _canon(L):
    return tuple(sorted(abs(x) for x in L))


def _region(Lc):
    """Number of boundary (|L_d| > 1) coordinates: 0 = Core, 1..3 = Boundary-1..3 (Sec. 4)."""
    return sum(1 for x in Lc if x > 1)


class BandOverflow(RuntimeError):
    """The screening keeps a term at a displacement on the edge of the band (max |L_d| = LMAX):
    displacements beyond it, which the plan does not cover, would still matter (the remark of
    Sec. 4 that a narrow band suffices in practice does not hold for this operator and eps)."""


def make_plan(Ftab, H0, H1, w, eps, nlev, group=True, allow_overflow=False):
    """Plan R[j, L, 2] for j = 0..nlev (Ftab must hold scales 0..nlev).  Also returns theta.
    Raises BandOverflow when a per-L range on the band's edge is not empty (unless allowed)."""
    M = Ftab.shape[1]
    w = np.asarray(w, dtype=np.float64)
    theta = 0.0
    for m in range(M):                                    # sequential sum over m
        theta += w[m] * np.linalg.norm(Ftab[0, m, 7]) ** 3
    theta *= eps
    n7 = 2 * LMAX + 1
    R = np.empty((nlev + 1, n7, n7, n7, 2), dtype=np.int32)
    R[...] = EMPTY
    R[0, LMAX, LMAX, LMAX] = (0, M - 1)
    canon = sorted(set(_canon(L) for L in itertools.product(range(LMAX + 1), repeat=3)))
    for j in range(1, nlev + 1):
        NF, NU, ND = block_norms(Ftab, H0, H1, j)
        rng = {Lc: term_range(w * estimate(NF, NU, ND, Lc), theta) for Lc in canon}
        for Lc, (a, b) in rng.items():
            if max(Lc) == LMAX and b >= a and not allow_overflow:
                raise BandOverflow("scale %d keeps terms %d..%d at |L| = %s, the edge of the band" % (j, a, b, Lc))
        if group:
            hull = {}
            for Lc, (a, b) in rng.items():
                g = _region(Lc)
                if b >= a:
                    h = hull.get(g, (a, b))
                    hull[g] = (min(h[0], a), max(h[1], b))
            rng = {Lc: hull.get(_region(Lc), EMPTY) for Lc in canon}
        for L in itertools.product(range(-LMAX, LMAX + 1), repeat=3):
            R[j, L[0] + LMAX, L[1] + LMAX, L[2] + LMAX] = rng[_canon(L)]
    return R, theta
