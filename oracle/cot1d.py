"""1-D modified ns-form of the periodic cotangent operator (test infrastructure only).

Sec. 2.4 (the modified ns-form in 1-D, Alg. 2) and its numerical example (Sec. 2.4.2):
    (C f)(y) = p.v. int_0^1 cot(pi (y - x)) f(x) dx                          (eq. CotangetKernel)
on the periodic unit interval, applied to the periodized Gaussian f(x) = sum_n exp(-a (x + n - 1/2)^2).

  * cot_blocks: r^{j;l}_ab = 2^-j p.v. int_{-1}^{1} cot(pi 2^-j (x + l)) Phi_ab(x) dx  (eq. cot.01), the
    k x k block <phi^j_{a,l_out}, C phi^j_{b,l_in}> for l = l_out - l_in (mod 2^j), row = output degree.
    Phi is split at 0 into its polynomial pieces (App. A.4): with t in [0,1],
        r = 2^-j int_0^1 [cot(pi 2^-j (l + t)) Phi^+(t) + cot(pi 2^-j (l - t)) Phi^-(-t)] dt,
    whose integrand is analytic on [0,1]: where a cotangent has a pole at an end point, Phi^+ and
    Phi^- agree there (t = 0) or vanish (t = 1).  Gauss-Legendre rule of `ngl` points.
  * difference super-blocks and bands (Sec. 2.4, eqs. fine_scale_band, down_band; reading below).
  * project_periodic: Alg. 1 in d = 1 for periodized Gaussian sums.
  * apply_modified: eq. apply_algo / Alg. 2 on the redundant tree of f; apply_difference: eq.
    g_scales_band (a self-check: after assembly the two agree for any tree and bands, eq. down_up).
  * assemble (eq. g_assemble), evaluate, and the exact C f in two closed forms.

Readings of the paper taken here:
  * Bands are sets of coarse displacements: at scale j >= 1 the whole band holds the fine pairs
    (l_out, l_in) whose parents are at periodic distance |L| <= B_j on scale j-1; in the paper's
    parity-dependent rule (eq. fine_scale_band) this is the band b_j = 2 B_j + 1, whose
    down-sampled band (eq. down_band) is |L| <= B_j.  The part removed at internal nodes of scale j
    is the fine band |l| <= B_{j+1} of scale j (the down-sampled band of scale j+1).  Distances
    are periodic (the band's corners are filled in, Sec. 2.3).
  * B_j is the smallest B with sum over coarse distances d > B (up to DMAX) of
    ||S^{j;L} - U^{j;L}||_F <= eps, where S^{j;L} is the 2k x 2k super-block of T_j between sibling
    pairs at coarse displacement L and U^{j;L} that of the up-sampled T_{j-1} (the difference
    operator's blocks decay away from the diagonal, Sec. 2.3); B_j = 2^(j-2) (the whole row) when
    nothing can be dropped.  ||C|| = 1, so eps is relative to the operator's norm.
  * Alg. 1 in d = 1 with the paper's absolute threshold on the maximum difference between the
    parent's polynomial and f at both children's Gauss-Legendre nodes (strict >), from level j0,
    leaves at jmax without a test.  With threshold eps this gives Table 1's scales and block counts
    for all four rows.
  * The output tree (Alg. 2 copies the redundant tree of f and assumes it suffices for g): for the
    cotangent kernel a coarse leaf next to refined input would take P_j C P_j f, which misses the
    finer scales' difference terms at its (absent) children; the output tree here is the redundant
    tree with every leaf refined whose whole band holds an internal node of f of its scale, and so
    on for the added children (`skeleton`).  On Table 1's inputs this reproduces the printed E_2
    (absolute l2 error) to two digits for p = 5, 8, 11 and stays below it for p = 14; without it the
    coarse leaves carry errors 100-1000 times larger.
  * The closed form: near x = y, cot(pi (y - x)) behaves as 1 / (pi (y - x)), so C acts on
    exp(-a x^2) as the Hilbert transform with that kernel, which gives + exp(-a y^2) Erfi(sqrt(a) y);
    eq. cot_gauss prints the opposite sign.  Its Fourier form also omits the factor (-1)^n that the
    centre 1/2 brings.  From C e^{2 pi i n x} = -i sign(n) e^{2 pi i n y} (the Fourier coefficients
    of cot(pi t) are -i sign(n)):  C f(y) = 2 sqrt(pi/a) sum_{n>=1} exp(-pi^2 n^2 / a) sin(2 pi n (y - x0))
    for f centred at x0; `exact_dawson` sums the Dawson form over images as a second check.
"""
import math

import numpy as np
from scipy import special

from . import mra

__all__ = ["cot_blocks", "cot_table", "super_blocks", "difference_norms", "choose_bands", "project_periodic",
           "Tree1", "skeleton", "apply_modified", "apply_difference", "assemble", "evaluate", "exact_fourier", "exact_dawson",
           "periodic_gauss", "pv_direct"]


def cot_blocks(k, j, ls, ngl=64):
    """r^{j;l} for the displacements ls (any integers; the blocks depend on l mod 2^j): shape
    (len(ls), k, k), row = output degree (eq. cot.01)."""
    t, w = mra.gauss_legendre01(ngl)
    pp = mra.crosscorr(k, t)                     # Phi^+(t), (ngl, k, k)
    pm = mra.crosscorr(k, -t)                    # Phi^-(-t)
    s = 2.0 ** -j
    l = np.asarray(ls, dtype=np.float64)[:, None]
    cp = 1.0 / np.tan(math.pi * s * (l + t))     # (len, ngl)
    cm = 1.0 / np.tan(math.pi * s * (l - t))
    return s * (np.einsum("q,iq,qab->iab", w, cp, pp) + np.einsum("q,iq,qab->iab", w, cm, pm))


def cot_table(k, nmax, ngl=64, lmax=None):
    """r^{j;l} for j = 0..nmax, indexed by l mod 2^j: per scale an array (2^j, k, k) of every l, or,
    with lmax, a dict of the residues of l = -lmax..lmax (enough for bands up to (lmax - 1) / 2 and
    difference norms up to distance (lmax - 1) / 2)."""
    out = []
    for j in range(nmax + 1):
        n = 2 ** j
        if lmax is None or n <= 2 * lmax + 1:
            out.append(cot_blocks(k, j, list(range(n)), ngl))
        else:
            ls = list(range(-lmax, lmax + 1))
            out.append({l % n: b for l, b in zip(ls, cot_blocks(k, j, ls, ngl))})
    return out


def super_blocks(k, R, j, L):
    """S^{j;L} and U^{j;L} (2k x 2k, rows = output child sigma, columns = input child sigma'): the
    blocks of T_j between the children of two scale-(j-1) boxes at displacement L, and those of the
    up-sampled T_{j-1}, [H0 H1]^T r^{j-1;L} [H0 H1] (zero-detail reconstruction of both sides)."""
    n = 2 ** j
    H0, H1 = mra.two_scale_filters(k)
    S = np.zeros((2 * k, 2 * k))
    for so in (0, 1):
        for si in (0, 1):
            S[so * k:(so + 1) * k, si * k:(si + 1) * k] = R[j][(2 * L + so - si) % n]
    Hc = np.hstack([H0, H1])                      # k x 2k
    U = Hc.T @ R[j - 1][L % (n // 2)] @ Hc
    return S, U


def periodic_distance(l, n):
    l = l % n
    return min(l, n - l)


DMAX = 32    # largest coarse distance whose difference super-blocks enter the band choice


def difference_norms(k, R, j):
    """||S^{j;L} - U^{j;L}||_F summed over the displacements L at each coarse periodic distance
    d = 0..min(DMAX, 2^(j-2)) (a dict d -> sum)."""
    nc = 2 ** (j - 1)
    out = {}
    for L in range(nc):
        d = periodic_distance(L, nc)
        if d > DMAX:
            continue
        S, U = super_blocks(k, R, j, L)
        out[d] = out.get(d, 0.0) + float(np.linalg.norm(S - U))
    return out


def choose_bands(k, R, eps):
    """B_j for j = 1..len(R)-1 (B[0] unused, B[len(R)] = 0): the smallest B whose neglected difference
    super-blocks, at coarse periodic distances B < d <= min(DMAX, 2^(j-2)), have Frobenius norms
    summing to at most eps; 2^(j-2) (the whole periodic row) when none can be dropped.  (The blocks
    of the difference operator decay away from the diagonal like the k-th derivative of the kernel;
    beyond DMAX they are far below any eps used here, down to rounding.)"""
    nmax = len(R) - 1
    B = [0] * (nmax + 2)
    for j in range(1, nmax + 1):
        full = 2 ** (j - 1) // 2
        norms = difference_norms(k, R, j)
        b = full
        while b > 0 and sum(v for d, v in norms.items() if d > b - 1) <= eps:
            b -= 1
        B[j] = b
    return B


def periodic_gauss(x, centers, exps, weights):
    """f(x) = sum_i w_i sum_n exp(-a_i (x + n - c_i)^2) (unnormalized, as in Sec. 2.4.2)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for c, a, w in zip(centers, exps, weights):
        nimg = int(math.ceil(math.sqrt(45.0 / a))) + 1
        for n in range(-nimg, nimg + 1):
            out += w * np.exp(-a * (x + n - c) ** 2)
    return out


def periodic_gauss_norm(centers, exps, weights):
    """||f||_2 on [0,1]: int_0^1 f^2 = sum_{i,i'} w w' int_R g_i(x) sum_n g_i'(x + n) dx in closed form."""
    s = 0.0
    for c, a, w in zip(centers, exps, weights):
        for c2, a2, w2 in zip(centers, exps, weights):
            nimg = int(math.ceil(math.sqrt(45.0 / min(a, a2)))) + 2
            for n in range(-nimg, nimg + 1):
                d = c - c2 + n
                s += w * w2 * math.sqrt(math.pi / (a + a2)) * math.exp(-a * a2 / (a + a2) * d * d)
    return math.sqrt(s)


class Tree1:
    """Redundant 1-D tree: levels, translations, leaf flags, coefficient blocks (k,), sorted by
    (level, translation)."""

    def __init__(self, k, level, trans, leaf, coef):
        order = np.lexsort((trans, level))
        self.k = k
        self.level = np.asarray(level, dtype=np.int64)[order]
        self.trans = np.asarray(trans, dtype=np.int64)[order]
        self.leaf = np.asarray(leaf, dtype=np.uint8)[order]
        self.coef = np.asarray(coef, dtype=np.float64)[order]
        self.pos = {(int(j), int(l)): i for i, (j, l) in enumerate(zip(self.level, self.trans))}
        self.depth = int(self.level.max())


def _box_coeffs(k, j, l, f):
    """Eq. fvals2coefs in d = 1: s_a = 2^{-j/2} sum_q w_q f(2^-j (l + x_q)) phi_a(x_q)."""
    x, w = mra.gauss_legendre01(k)
    vals = f(2.0 ** -j * (l + x))
    return 2.0 ** (-j / 2.0) * (w * vals) @ mra.phi(k, x)


def project_periodic(k, thr, j0, jmax, centers, exps, weights):
    """Alg. 1 in d = 1: leaves (level, translation, coefficients) of the adaptive projection of the
    periodized Gaussian sum with the absolute threshold thr on the interpolation error, as a
    redundant tree (internal nodes by the two-scale relation)."""
    f = lambda x: periodic_gauss(x, centers, exps, weights)
    x, _ = mra.gauss_legendre01(k)
    leaves = []
    todo = [(j0, l) for l in range(2 ** j0)]
    while todo:
        nxt = []
        for (j, l) in todo:
            s = _box_coeffs(k, j, l, f)
            if j >= jmax:
                leaves.append((j, l, s))
                continue
            # parent's polynomial at the children's nodes against f there
            err = 0.0
            for sig in (0, 1):
                y = 0.5 * (x + sig)                     # child's nodes in the parent's coordinate
                approx = 2.0 ** (j / 2.0) * mra.phi(k, y) @ s
                direct = f(2.0 ** -(j + 1) * (2 * l + sig + x))
                err = max(err, float(np.max(np.abs(approx - direct))))
            if err > thr:
                nxt += [(j + 1, 2 * l), (j + 1, 2 * l + 1)]
            else:
                leaves.append((j, l, s))
        todo = nxt
    return redundant_tree(k, leaves)


def redundant_tree(k, leaves):
    """Leaves plus every ancestor; parents from s^j_l = H0 s^{j+1}_{2l} + H1 s^{j+1}_{2l+1}
    (App. A.3, eq. decomp_scaling)."""
    H0, H1 = mra.two_scale_filters(k)
    nodes = {(j, l): np.array(s, dtype=np.float64) for (j, l, s) in leaves}
    isleaf = {key: 1 for key in nodes}
    depth = max(j for (j, _, _) in leaves)
    for j in range(depth, 0, -1):
        for (jj, l) in [key for key in list(nodes) if key[0] == j]:
            p = (j - 1, l >> 1)
            if p in nodes:
                continue
            a, b = nodes.get((j, 2 * (l >> 1))), nodes.get((j, 2 * (l >> 1) + 1))
            if a is None or b is None:
                raise ValueError("leaves do not tile the interval")
            nodes[p] = H0 @ a + H1 @ b
            isleaf[p] = 0
    keys = sorted(nodes)
    return Tree1(k, [q[0] for q in keys], [q[1] for q in keys], [isleaf[q] for q in keys],
                 np.array([nodes[q] for q in keys]))


def _input_block(tree, j, l):
    """f^j_l from the tree, or by zero-detail reconstruction from the nearest existing ancestor
    (Alg. 2, Step 2)."""
    key = (j, l)
    if key in tree.pos:
        return tree.coef[tree.pos[key]]
    H0, H1 = mra.two_scale_filters(tree.k)
    up = 1
    while (j - up, l >> up) not in tree.pos:
        up += 1
    s = tree.coef[tree.pos[(j - up, l >> up)]]
    for step in range(up, 0, -1):
        sig = (l >> (step - 1)) & 1
        s = (H1 if sig else H0).T @ s
    return s


def skeleton(tree, B):
    """The output tree: the redundant tree of f where a leaf b of scale j is refined when an internal
    node of f of scale j lies in its whole band (parents at periodic distance <= B_j), and so on for
    the children this adds (each checked against f's internal nodes of its own scale).  The blocks
    of f at added nodes come from their nearest ancestor (Alg. 2, Step 2).  f has finer details in
    that band, and the difference operators of the finer scales carry them to b's (absent) children;
    with f's tree alone b would take P_j C P_j f, whose error next to refined input is not bounded by
    eps for this singular kernel.  Where f has no details within the band those terms project to
    zero on b."""
    finternal = {}
    for j, l, lf in zip(tree.level, tree.trans, tree.leaf):
        if not lf:
            finternal.setdefault(int(j), []).append(int(l) >> 1)
    nodes = {(int(j), int(l)): bool(lf) for j, l, lf in zip(tree.level, tree.trans, tree.leaf)}
    todo = sorted(key for key, lf in nodes.items() if lf)
    while todo:
        nxt = []
        for (j, l) in todo:
            if j == 0 or j not in finternal:
                continue
            nc = 2 ** (j - 1)
            if any(periodic_distance((l >> 1) - cp, nc) <= B[j] for cp in finternal[j]):
                nodes[(j, l)] = False
                nodes[(j + 1, 2 * l)] = True
                nodes[(j + 1, 2 * l + 1)] = True
                nxt += [(j + 1, 2 * l), (j + 1, 2 * l + 1)]
        todo = nxt
    keys = sorted(nodes)
    coef = np.array([_input_block(tree, j, l) for (j, l) in keys])
    return Tree1(tree.k, [q[0] for q in keys], [q[1] for q in keys], [1 if nodes[q] else 0 for q in keys], coef)


def apply_modified(tree, R, B, out=None):
    """ghat on every node of the output tree `out` (default: the redundant tree of f itself) for the
    input tree `tree` (eq. apply_algo, Alg. 2 Steps 1-3): at scale j >= 1, node b takes the pairs
    (b, b - l) with coarse periodic distance |L| <= B_j; an internal node drops those with fine
    periodic distance |l| <= B_{j+1}.  The root takes T_0 f_0 when it is a leaf and
    (T_0 - T_0^{B_1}) f_0 = 0 otherwise."""
    out = tree if out is None else out
    k = tree.k
    ghat = np.zeros((out.coef.shape[0], k))
    for i in range(out.coef.shape[0]):
        j, b, lf = int(out.level[i]), int(out.trans[i]), bool(out.leaf[i])
        if j == 0:
            if lf:
                ghat[i] = R[0][0] @ _input_block(tree, 0, 0)
            continue
        n = 2 ** j
        acc = np.zeros(k)
        # the coefficient is 0 unless the fine distance is <= 2 B_j + 1 (coarse distance <= B_j) or
        # <= B_{j+1} (internal nodes); each residue l mod 2^j once
        reach = max(2 * B[j] + 1, 0 if lf else B[j + 1])
        seen = set()
        for l in range(-reach, reach + 1):
            if l % n in seen:
                continue
            seen.add(l % n)
            bp = (b - l) % n
            L = periodic_distance((b >> 1) - (bp >> 1), n // 2)
            c = (1 if L <= B[j] else 0) - (0 if lf else (1 if periodic_distance(l, n) <= B[j + 1] else 0))
            if c:
                acc += c * (R[j][l % n] @ _input_block(tree, j, bp))
        ghat[i] = acc
    return ghat


def apply_difference(tree, R, B):
    """ghat by the banded difference form (eq. g_scales_band): at scale j >= 1 every node b gets
    [T_j^{B_j} - up(T_{j-1})^{B_j}] f_j over the pairs with coarse distance |L| <= B_j; scale 0
    gets T_0 f_0."""
    k = tree.k
    H0, H1 = mra.two_scale_filters(k)
    Hs = (H0, H1)
    ghat = np.zeros_like(tree.coef)
    for i in range(tree.coef.shape[0]):
        j, b = int(tree.level[i]), int(tree.trans[i])
        if j == 0:
            ghat[i] = R[0][0] @ tree.coef[i]
            continue
        n = 2 ** j
        acc = np.zeros(k)
        for l in range(n):
            bp = (b - l) % n
            Lc = ((b >> 1) - (bp >> 1)) % (n // 2)
            if periodic_distance(Lc, n // 2) > B[j]:
                continue
            blk = R[j][l] - Hs[b & 1].T @ R[j - 1][Lc] @ Hs[bp & 1]
            acc += blk @ _input_block(tree, j, bp)
        ghat[i] = acc
    return ghat


def assemble(tree, ghat):
    """g_child = ghat_child + H^(sigma)^T g_parent from the root down (eq. g_assemble)."""
    H0, H1 = mra.two_scale_filters(tree.k)
    g = np.array(ghat, copy=True)
    for i in range(g.shape[0]):
        j, l = int(tree.level[i]), int(tree.trans[i])
        if j == 0:
            continue
        p = tree.pos[(j - 1, l >> 1)]
        g[i] += (H1 if l & 1 else H0).T @ g[p]
    return g


def evaluate(tree, g, x):
    """Value of the leaves' expansion at points x in [0,1): the leaf containing x, then
    2^{j/2} sum_a g_a phi_a(2^j x - l) (App. A.1)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    for i, xv in enumerate(x):
        j = 0
        while True:
            l = min(int(math.floor(xv * 2 ** j)), 2 ** j - 1)
            p = tree.pos[(j, l)]
            if tree.leaf[p]:
                out[i] = 2.0 ** (j / 2.0) * mra.phi(tree.k, np.array([xv * 2 ** j - l]))[0] @ g[p]
                break
            j += 1
    return out


def exact_fourier(y, a, x0=0.5, weight=1.0):
    """C f for f = weight sum_n exp(-a (x + n - x0)^2):
    2 sqrt(pi/a) sum_{n>=1} exp(-pi^2 n^2 / a) sin(2 pi n (y - x0))."""
    y = np.asarray(y, dtype=np.float64)
    nmax = int(math.ceil(math.sqrt(40.0 * math.log(10.0) * a) / math.pi)) + 2
    out = np.zeros_like(y)
    for n in range(nmax, 0, -1):
        out += math.exp(-math.pi ** 2 * n * n / a) * np.sin(2.0 * math.pi * n * (y - x0))
    return weight * 2.0 * math.sqrt(math.pi / a) * out


def exact_dawson(y, a, x0=0.5, weight=1.0, nimg=200000):
    """The same by images: sum_n exp(-a t^2) Erfi(sqrt(a) t) at t = y + n - x0, symmetric partial
    sums over |n| <= nimg with the tail's leading term 1/(2 sqrt(a) t) summed by the cotangent
    lattice identity (the Hilbert transform of exp(-a x^2) is (2/sqrt(pi)) D(sqrt(a) y), D Dawson's
    integral)."""
    y = np.asarray(y, dtype=np.float64)
    t = y - x0
    n = np.arange(-nimg, nimg + 1)
    z = math.sqrt(a) * (t[..., None] + n)
    # D(z) - 1/(2z) decays like 1/(4 z^3): sum it over images, add the lattice sum of 1/(2 z)
    # (sum_n 1/(t+n) = pi cot(pi t)) in closed form
    near = 2.0 / math.sqrt(math.pi) * (special.dawsn(z) - 0.5 / z)
    return weight * (np.sum(near, axis=-1) + math.pi * (1.0 / np.tan(math.pi * t)) / (math.sqrt(math.pi * a)))


def pv_direct(y, f, m=4000):
    """C f at one point y by brute force: p.v. int_0^1 cot(pi (y - x)) f(x) dx = int_0^{1/2}
    cot(pi s) (f(y - s) - f(y + s)) ds (the kernel is odd and 1-periodic), with the regular
    integrand by composite Gauss-Legendre on m panels."""
    t, w = mra.gauss_legendre01(16)
    edges = np.linspace(0.0, 0.5, m + 1)
    s = (edges[:-1, None] + (edges[1:] - edges[:-1])[:, None] * t).ravel()
    ws = ((edges[1:] - edges[:-1])[:, None] * w).ravel()
    return float(np.sum(ws * (f(y - s) - f(y + s)) / np.tan(math.pi * s)))
