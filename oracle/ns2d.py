"""The d = 2 version of the method (test infrastructure only): Alg. 3 written for d = 2.

Sec. 5 states Alg. 3 for d = 2 and Sec. 6.1 notes that the apply is implemented for d = 2 as well;
the paper gives no 2-D kernel or example.  Here, everything follows the 3-D path with two factors:
  * kernel (-Delta + mu^2)^(-alpha) in the plane: K(r) = C2 int exp(-r^2 e^{2s} - mu^2 e^{-2s}/4
    + (2 - 2 alpha) s) ds, C2 = 2 * 2^{-2 alpha} / (pi Gamma(alpha)) (Sec. 3's representation with the
    dimension 2 in place of 3; for alpha = 1 it is K_0(mu r) / (2 pi), the bound-state Helmholtz
    Green's function of the plane); trapezoidal rule as in eq. KernelApproxByGaussians;
  * the 1-D blocks F^{j;m,l} (eq. KernelFactor) do not depend on the dimension (mra.F_table);
  * screening (Sec. 4): theta = eps sum_m w_m ||F^{0;m,0}||_F^2; the estimate of eq.
    NormEstimateUsing1DBlocks with two factors, 1/2 sum over the orderings (p, q) of (|L_1|, |L_2|)
    of N_dif(p) N_F(q) + N_upF(p) N_dif(q); term ranges, grouping (Core, Boundary-1, -2: the number of
    |L_d| > 1) and the band edge as in 3-D;
  * Alg. 1 with 2^2 children and k^2 nodes per box, threshold eps ||f||_2 (the 3-D reading), sources
    c (a/pi) exp(-a |x - x_i|^2) of unit mass;
  * apply (eq. apply_algo, Alg. 3): leaf terms R_j(L), internal terms R_j(L) minus R_{j+1}(l), root
    all terms minus R_1(0); inputs missing from the tree by zero-detail reconstruction from the
    nearest ancestor; assembly (eq. g_assemble); evaluation.
Keys: level << 57 | morton(x, y), x in bit 0; child s of a box has parities (s & 1, s >> 1).
"""
import itertools
import math

import numpy as np
from scipy import special

from . import mra

__all__ = ["c2_alpha", "kernel2d", "fit_kernel2d", "make_plan2d", "project2d", "Tree2", "apply_modified2d",
           "apply_difference2d", "dense_uniform2d", "assemble2d", "evaluate2d", "source_norm2d",
           "fitted_truncated2d", "full_plan2d", "BandOverflow2d", "LMAX", "EMPTY"]

LMAX = 3
EMPTY = (0, -1)


# ---- kernel and fit (Sec. 3 in the plane) ----------------------------------------------------

def c2_alpha(alpha):
    return 2.0 * 2.0 ** (-2.0 * alpha) / (math.pi * math.gamma(alpha))


def kernel2d(mu, alpha, r):
    """K(r) = (2 pi)^-1 2^{1-alpha} / Gamma(alpha) (mu / r)^{1-alpha} K_{1-alpha}(mu r) for mu > 0
    (the plane's Green's function of (-Delta + mu^2)^(-alpha)); for mu = 0 and alpha < 1,
    Gamma(1 - alpha) / (4^alpha pi Gamma(alpha)) r^{2 alpha - 2}."""
    r = np.asarray(r, dtype=np.float64)
    if mu > 0.0:
        nu = 1.0 - alpha
        return (2.0 ** (1.0 - alpha) / (2.0 * math.pi * math.gamma(alpha))) * (mu / r) ** nu * special.kv(nu, mu * r)
    return math.gamma(1.0 - alpha) / (4.0 ** alpha * math.pi * math.gamma(alpha)) * r ** (2.0 * alpha - 2.0)


def _terms(mu, alpha, A, B, M):
    h = (B - A) / M
    s = A + h * np.arange(1, M + 1)
    tau = np.exp(2.0 * s)
    w = h * c2_alpha(alpha) * np.exp(-mu * mu * np.exp(-2.0 * s) / 4.0 + (2.0 - 2.0 * alpha) * s)
    return tau, w


def fit_kernel2d(mu, alpha, eps, delta, R, max_iter=40):
    """(tau, w) with |K(r) - sum_m w_m exp(-tau_m r^2)| <= eps K(r) on [delta, R], relative to the
    kernel itself (for alpha = 1 the plane's kernels have no power-law reference), checked on 64
    points per decade and re-checked on 256.  Step h from the strip of analyticity as in 3-D; right
    end B where the Gaussian at r = delta has decayed (as in 3-D); left end A where the integrand's
    left tail is below eps K(R): for mu > 0, mu^2 e^{-2A} / 4 = log(1e30 / eps); for alpha < 1,
    e^{(2 - 2 alpha) A} / (2 - 2 alpha) = eps K(R) C2^{-1} / e (the smaller A of the two).  h shrinks
    by 0.9 and [A, B] widens by 1 until the checks pass.  Terms whose weight underflows to zero
    (far into the left tail for mu > 0) are dropped."""
    if not (0.0 < alpha <= 1.0) or mu < 0.0 or (mu == 0.0 and alpha >= 1.0) or not (0.0 < eps < 1.0) \
            or not (0.0 < delta < R):
        raise ValueError("need 0 < alpha <= 1, mu >= 0 (mu > 0 when alpha = 1), 0 < eps < 1, 0 < delta < R")
    h = math.pi ** 2 / (2.0 * (math.log(1.0 / eps) + math.log(8.0)))
    cands = []
    if mu > 0.0:
        cands.append(math.log(mu) - 0.5 * math.log(4.0 * math.log(1e30 / eps)))
    if alpha < 1.0:
        g = 2.0 - 2.0 * alpha
        cands.append(math.log(eps * float(kernel2d(mu, alpha, R)) * g / (c2_alpha(alpha) * math.e)) / g)
    A = min(cands)
    B = 0.5 * math.log(math.log(4.0 / eps) / delta ** 2) + 1.0
    ndec = max(1, int(math.ceil(math.log10(R / delta))))

    def max_err(tau, w, npd):
        r = np.exp(np.linspace(math.log(delta), math.log(R), npd * ndec + 1))
        ref = kernel2d(mu, alpha, r)
        got = (w[None, :] * np.exp(-tau[None, :] * r[:, None] ** 2)).sum(1)
        return float(np.max(np.abs(ref - got) / ref))

    for _ in range(max_iter):
        M = max(1, int(math.ceil((B - A) / h)))
        tau, w = _terms(mu, alpha, A, A + M * h, M)
        keep = w > 0.0                       # weights that underflow to zero contribute nothing
        tau, w = tau[keep], w[keep]
        if max_err(tau, w, 64) <= eps and max_err(tau, w, 256) <= eps:
            return tau, w
        h *= 0.9
        A -= 1.0
        B += 1.0
    raise RuntimeError("fit did not converge")


# ---- plan (Sec. 4 in the plane) --------------------------------------------------------------

class BandOverflow2d(RuntimeError):
    """A term kept at a displacement on the edge of the band (max |L_d| = LMAX)."""


def full_plan2d(M, nlev):
    """Screening off: every term at every |L_d| <= 3 on every scale."""
    n7 = 2 * LMAX + 1
    R = np.empty((nlev + 1, n7, n7, 2), dtype=np.int32)
    R[..., 0] = 0
    R[..., 1] = M - 1
    R[0] = EMPTY
    R[0, LMAX, LMAX] = (0, M - 1)
    return R


def make_plan2d(Ftab, H0, H1, w, eps, nlev, group=True, allow_overflow=False):
    """R[j, L1+3, L2+3, 2] for j = 0..nlev and theta; the blocks' norms as in the 3-D plan, the
    estimate with two factors."""
    from . import plan as P3
    M = Ftab.shape[1]
    w = np.asarray(w, dtype=np.float64)
    theta = 0.0
    for m in range(M):
        theta += w[m] * np.linalg.norm(Ftab[0, m, 7]) ** 2
    theta *= eps
    n7 = 2 * LMAX + 1
    R = np.empty((nlev + 1, n7, n7, 2), dtype=np.int32)
    R[...] = EMPTY
    R[0, LMAX, LMAX] = (0, M - 1)
    canon = sorted(set(tuple(sorted(L)) for L in itertools.product(range(LMAX + 1), repeat=2)))
    for j in range(1, nlev + 1):
        NF, NU, ND = P3.block_norms(Ftab, H0, H1, j)
        rng = {}
        for Lc in canon:
            est = np.zeros(M)
            for (p, q) in itertools.permutations(Lc):
                est += ND[:, p] * NF[:, q] + NU[:, p] * ND[:, q]
            rng[Lc] = P3.term_range(w * est / 2.0, theta)
        for Lc, (a, b) in rng.items():
            if max(Lc) == LMAX and b >= a and not allow_overflow:
                raise BandOverflow2d("scale %d keeps terms %d..%d at |L| = %s" % (j, a, b, Lc))
        if group:
            hull = {}
            for Lc, (a, b) in rng.items():
                g = sum(1 for x in Lc if x > 1)
                if b >= a:
                    hh = hull.get(g, (a, b))
                    hull[g] = (min(hh[0], a), max(hh[1], b))
            rng = {Lc: hull.get(sum(1 for x in Lc if x > 1), EMPTY) for Lc in canon}
        for L in itertools.product(range(-LMAX, LMAX + 1), repeat=2):
            R[j, L[0] + LMAX, L[1] + LMAX] = rng[tuple(sorted(abs(x) for x in L))]
    return R, theta


# ---- tree (Alg. 1 in the plane) --------------------------------------------------------------

def _spread2(v):
    out = 0
    for b in range(28):
        out |= ((v >> b) & 1) << (2 * b)
    return out


def make_key2(j, x, y):
    return (j << 57) | _spread2(x) | (_spread2(y) << 1)


class Tree2:
    """Redundant tree: keys (sorted), level, coordinates l (n, 2), leaf flags, coefficients (n, k, k)
    with coef[a][b] the degrees in x and y."""

    def __init__(self, k, nodes):
        keys = sorted(nodes, key=lambda q: make_key2(*q))
        self.k = k
        self.keys = np.array([make_key2(*q) for q in keys], dtype=np.uint64)
        self.level = np.array([q[0] for q in keys], dtype=np.int64)
        self.l = np.array([[q[1], q[2]] for q in keys], dtype=np.int64)
        self.leaf = np.array([nodes[q][0] for q in keys], dtype=np.uint8)
        self.coef = np.array([nodes[q][1] for q in keys], dtype=np.float64)
        self.pos = {q: i for i, q in enumerate(keys)}
        self.depth = int(self.level.max())


def gauss2d(x, y, xy, a, c):
    """sum_i c_i (a_i/pi) exp(-a_i ((x - x_i)^2 + (y - y_i)^2))."""
    out = np.zeros(np.broadcast(x, y).shape)
    for (cx, cy), ai, ci in zip(xy, a, c):
        out += ci * (ai / math.pi) * np.exp(-ai * ((x - cx) ** 2 + (y - cy) ** 2))
    return out


def source_norm2d(xy, a, c):
    s = 0.0
    for (x1, y1), a1, c1 in zip(xy, a, c):
        for (x2, y2), a2, c2 in zip(xy, a, c):
            d2 = (x1 - x2) ** 2 + (y1 - y2) ** 2
            s += c1 * c2 * (a1 * a2 / math.pi ** 2) * (math.pi / (a1 + a2)) * math.exp(-a1 * a2 / (a1 + a2) * d2)
    return math.sqrt(s)


def _box_coeffs(k, j, lx, ly, f):
    """s_ab = 2^-j sum_{q,r} w_q w_r f(2^-j (lx + x_q), 2^-j (ly + x_r)) phi_a(x_q) phi_b(x_r)
    (eq. fvals2coefs in two dimensions)."""
    x, w = mra.gauss_legendre01(k)
    ph = mra.phi(k, x)
    X, Y = np.meshgrid(2.0 ** -j * (lx + x), 2.0 ** -j * (ly + x), indexing="ij")
    vals = f(X, Y) * w[:, None] * w[None, :]
    return 2.0 ** -j * ph.T @ vals @ ph


def project2d(k, eps, j0, jmax, xy, a, c):
    """Alg. 1 in the plane: a box is refined when, at some child's k x k nodes, f and the box's
    polynomial differ by more than eps ||f||_2 (strict >); all four children are then refined; boxes
    at jmax are leaves.  Returns the redundant tree (internal nodes by the two-scale relation)."""
    f = lambda X, Y: gauss2d(X, Y, xy, a, c)
    thr = eps * source_norm2d(xy, a, c)
    x, _ = mra.gauss_legendre01(k)
    leaves = {}
    todo = [(j0, lx, ly) for lx in range(2 ** j0) for ly in range(2 ** j0)]
    while todo:
        nxt = []
        for (j, lx, ly) in todo:
            s = _box_coeffs(k, j, lx, ly, f)
            if j >= jmax:
                leaves[(j, lx, ly)] = s
                continue
            err = 0.0
            for sx in (0, 1):
                for sy in (0, 1):
                    px = mra.phi(k, 0.5 * (x + sx))
                    py = mra.phi(k, 0.5 * (x + sy))
                    approx = 2.0 ** j * px @ s @ py.T
                    X, Y = np.meshgrid(2.0 ** -(j + 1) * (2 * lx + sx + x), 2.0 ** -(j + 1) * (2 * ly + sy + x), indexing="ij")
                    err = max(err, float(np.abs(approx - f(X, Y)).max()))
            if err > thr:
                nxt += [(j + 1, 2 * lx + sx, 2 * ly + sy) for sy in (0, 1) for sx in (0, 1)]
            else:
                leaves[(j, lx, ly)] = s
        todo = nxt
    return redundant_tree2(k, leaves)


def redundant_tree2(k, leaves):
    """Leaves plus all ancestors, parents from s^j = sum_{sx,sy} H^(sx) s^{j+1} H^(sy)^T (eq.
    decomp_scaling in each dimension)."""
    H = mra.two_scale_filters(k)
    nodes = {q: (1, np.array(s, dtype=np.float64)) for q, s in leaves.items()}
    depth = max(q[0] for q in leaves)
    for j in range(depth, 0, -1):
        for (jj, lx, ly) in [q for q in list(nodes) if q[0] == j]:
            p = (j - 1, lx >> 1, ly >> 1)
            if p in nodes:
                continue
            acc = np.zeros((k, k))
            for sx in (0, 1):
                for sy in (0, 1):
                    ch = nodes.get((j, 2 * p[1] + sx, 2 * p[2] + sy))
                    if ch is None:
                        raise ValueError("leaves do not tile the square")
                    acc += H[sx] @ ch[1] @ H[sy].T
            nodes[p] = (0, acc)
    return Tree2(k, nodes)


# ---- apply -----------------------------------------------------------------------------------

def _input_block(tree, j, lx, ly):
    """f^j at (lx, ly): from the tree, else zero-detail reconstruction from the nearest ancestor."""
    if (j, lx, ly) in tree.pos:
        return tree.coef[tree.pos[(j, lx, ly)]]
    H = mra.two_scale_filters(tree.k)
    up = 1
    while (j - up, lx >> up, ly >> up) not in tree.pos:
        up += 1
    s = tree.coef[tree.pos[(j - up, lx >> up, ly >> up)]]
    for step in range(up, 0, -1):
        sx, sy = (lx >> (step - 1)) & 1, (ly >> (step - 1)) & 1
        s = H[sx].T @ s @ H[sy]
    return s


def _terms_of(R, j, L):
    if max(abs(L[0]), abs(L[1])) > LMAX:
        return set()
    a, b = R[j, L[0] + LMAX, L[1] + LMAX]
    return set(range(a, b + 1))


def apply_modified2d(tree, F, w, R):
    """ghat on every node (eq. apply_algo, Alg. 3 Steps 1-3): for node b at scale j >= 1 and fine
    displacement l in [-7, 7]^2 with b - l in the square, L = floor(b/2) - floor((b - l)/2), term m
    enters with c_m = [m in R_j(L)] - [b internal][m in R_{j+1}(l)] as w_m F^{j;m,l1} X F^{j;m,l2}^T;
    the root takes all terms of R_0 minus those of R_1(0) when internal.  F[j, m, l+7] (k x k, row =
    output degree)."""
    k = tree.k
    nlev = R.shape[0]
    ghat = np.zeros_like(tree.coef)
    for i in range(tree.coef.shape[0]):
        j, lf = int(tree.level[i]), bool(tree.leaf[i])
        bx, by = int(tree.l[i, 0]), int(tree.l[i, 1])
        acc = np.zeros((k, k))
        if j == 0:
            ms = _terms_of(R, 0, (0, 0))
            if not lf and nlev > 1:
                ms -= _terms_of(R, 1, (0, 0))
            X = tree.coef[i]
            for m in sorted(ms):
                acc += w[m] * F[0, m, 7] @ X @ F[0, m, 7].T
            ghat[i] = acc
            continue
        n = 2 ** j
        for l1 in range(-7, 8):
            for l2 in range(-7, 8):
                px, py = bx - l1, by - l2
                if not (0 <= px < n and 0 <= py < n):
                    continue
                L = ((bx >> 1) - (px >> 1), (by >> 1) - (py >> 1))
                plus = _terms_of(R, j, L)
                minus = _terms_of(R, j + 1, (l1, l2)) if (not lf and j + 1 < nlev) else set()
                ms = sorted(plus ^ minus)
                if not ms:
                    continue
                X = _input_block(tree, j, px, py)
                for m in ms:
                    cm = (1 if m in plus else 0) - (1 if m in minus else 0)
                    acc += cm * w[m] * F[j, m, l1 + 7] @ X @ F[j, m, l2 + 7].T
        ghat[i] = acc
    return ghat


def apply_difference2d(tree, F, w, R, H0, H1):
    """ghat by the banded difference form (eq. g_scales_band): scale 0 gets T_0 f_0 over R_0; at
    scale j >= 1 every node gets sum over fine l with coarse L in the band of
    sum_{m in R_j(L)} w_m [F1 X F2^T - (H^(s1)^T F^{j-1;m,L1} H^(s1')) X (H^(s2)^T F^{j-1;m,L2} H^(s2'))^T]."""
    k = tree.k
    H = (H0, H1)
    ghat = np.zeros_like(tree.coef)
    for i in range(tree.coef.shape[0]):
        j = int(tree.level[i])
        bx, by = int(tree.l[i, 0]), int(tree.l[i, 1])
        acc = np.zeros((k, k))
        if j == 0:
            for m in sorted(_terms_of(R, 0, (0, 0))):
                acc += w[m] * F[0, m, 7] @ tree.coef[i] @ F[0, m, 7].T
            ghat[i] = acc
            continue
        n = 2 ** j
        for l1 in range(-7, 8):
            for l2 in range(-7, 8):
                px, py = bx - l1, by - l2
                if not (0 <= px < n and 0 <= py < n):
                    continue
                L = ((bx >> 1) - (px >> 1), (by >> 1) - (py >> 1))
                ms = sorted(_terms_of(R, j, L))
                if not ms:
                    continue
                X = _input_block(tree, j, px, py)
                for m in ms:
                    U1 = H[bx & 1].T @ F[j - 1, m, L[0] + 7] @ H[px & 1]
                    U2 = H[by & 1].T @ F[j - 1, m, L[1] + 7] @ H[py & 1]
                    acc += w[m] * (F[j, m, l1 + 7] @ X @ F[j, m, l2 + 7].T - U1 @ X @ U2.T)
        ghat[i] = acc
    return ghat


def assemble2d(tree, ghat):
    """g_child = ghat_child + H^(sx)^T g_parent H^(sy) from the root down (eq. g_assemble)."""
    H = mra.two_scale_filters(tree.k)
    g = np.array(ghat, copy=True)
    for i in range(g.shape[0]):
        j = int(tree.level[i])
        if j == 0:
            continue
        lx, ly = int(tree.l[i, 0]), int(tree.l[i, 1])
        p = tree.pos[(j - 1, lx >> 1, ly >> 1)]
        g[i] += H[lx & 1].T @ g[p] @ H[ly & 1]
    return g


def dense_uniform2d(tree, F, w):
    """The plain definition on a uniform tree of level n: g_b = sum over every b' and every term of
    w_m F^{n;m,b1-b1'} f_b' F^{n;m,b2-b2'}^T (no screening; needs |b - b'| <= 7, i.e. n <= 3)."""
    n = tree.depth
    idx = np.nonzero(tree.level == n)[0]
    out = {}
    for i in idx:
        bx, by = tree.l[i]
        acc = np.zeros((tree.k, tree.k))
        for i2 in idx:
            px, py = tree.l[i2]
            for m in range(F.shape[1]):
                acc += w[m] * F[n, m, bx - px + 7] @ tree.coef[i2] @ F[n, m, by - py + 7].T
        out[int(i)] = acc
    return out


def evaluate2d(tree, g, pts):
    """Value of the leaves' expansions at points (n, 2) in [0,1]^2."""
    out = np.empty(len(pts))
    for i, (x, y) in enumerate(pts):
        j = 0
        while True:
            n = 2 ** j
            lx, ly = min(int(math.floor(x * n)), n - 1), min(int(math.floor(y * n)), n - 1)
            p = tree.pos[(j, lx, ly)]
            if tree.leaf[p]:
                px = mra.phi(tree.k, np.array([x * n - lx]))[0]
                py = mra.phi(tree.k, np.array([y * n - ly]))[0]
                out[i] = n * px @ g[p] @ py
                break
            j += 1
    return out


def fitted_truncated2d(tau, w, xy, a, c, gx, gy):
    """The fitted kernel sum_m w_m exp(-tau_m r^2) applied exactly to the square-truncated source
    f 1_[0,1]^2 on the grid gx x gy: per term and source the integral separates into two 1-D
    integrals int_0^1 exp(-tau (x - t)^2 - a (t - c)^2) dt in closed form (erf)."""
    def G(t, ai, ci, x):
        s = t + ai
        mu = (t * x + ai * ci) / s
        pre = np.exp(-t * ai * (x - ci) ** 2 / s) * math.sqrt(math.pi) / (2.0 * np.sqrt(s))
        return pre * (special.erf(np.sqrt(s) * (1.0 - mu)) + special.erf(np.sqrt(s) * mu))
    out = np.zeros((len(gx), len(gy)))
    for (cx, cy), ai, ci in zip(xy, a, c):
        for t, wm in zip(tau, w):
            out += ci * (ai / math.pi) * wm * np.outer(G(t, ai, cx, np.asarray(gx)), G(t, ai, cy, np.asarray(gy)))
    return out
