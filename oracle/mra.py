"""1-D multiresolution tables of the oracle (test infrastructure only).

Everything here follows the paper's appendix:
  * Legendre scaling functions phi_a(x) = sqrt(2a+1) P_a(2x-1) on [0,1]    (App. A.1, eq. scalingFNC)
  * Gauss-Legendre rule on [0,1] (roots of P_k(2x-1))                       (App. A.1, eq. fvals2coefs)
  * two-scale filters H^(0), H^(1)                                           (App. A.3, two-scale relations)
  * wavelet filters G^(0), G^(1): any orthonormal complement of [H0 H1]     (App. A.2-A.3)
  * cross-correlations Phi_ab(x) = int phi_a(x+y) phi_b(y) dy              (App. A.4, eqs. CrossCor, crosscor.01)
  * operator blocks F^{j;m,l}_ab = 2^-j int_{-1}^{1} exp(-tau (x+l)^2/4^j) Phi_ab(x) dx
                                                                            (Sec. 3, eq. KernelFactor)
Readings of the paper taken here:
  * H^(s)_ab = <phi_a, sqrt2 phi_b(2x-s)> = 2^-1/2 int_0^1 phi_a((u+s)/2) phi_b(u) du, i.e. the
    coefficients of the two-scale relation for phi_a.  Decomposition s^j = H0 s^{j+1}_{2l} + H1 s^{j+1}_{2l+1};
    zero-detail reconstruction s^{j+1}_{2l+s} = H^(s)^T s^j.
  * In F^{j;m,l} the displacement is l = l_out - l_in and the row index a is the output degree.
  * G^(0), G^(1) are defined only through a reference the paper does not reproduce.  The wavelets
    psi_0..psi_{k-1} span the orthogonal complement of V_0 in V_1, so [[H0, H1], [G0, G1]] is an
    orthogonal 2k x 2k matrix; any orthonormal basis of that complement serves, since only the
    norm of the detail coefficients is used.  Here: Gram-Schmidt (twice) of the columns of the
    projector I - [H0 H1]^T [H0 H1], in column order.
"""
import functools

import numpy as np

__all__ = ["gauss_legendre01", "phi", "two_scale_filters", "wavelet_filters", "crosscorr",
           "crosscorr_coeffs", "F_block", "F_blocks", "F_table"]


def gauss_legendre01(n):
    """n-point Gauss-Legendre rule on [0,1]: nodes are the roots of P_n(2x-1), weights sum to 1
    (App. A.1, below eq. fvals2coefs)."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def phi(k, x):
    """phi_a(x) for a = 0..k-1 at points x (any shape); result has shape x.shape + (k,).
    phi_a(x) = sqrt(2a+1) P_a(2x-1) for 0 <= x <= 1 and 0 outside (App. A.1, eq. scalingFNC).
    P_a by the three-term recurrence (a+1) P_{a+1} = (2a+1) t P_a - a P_{a-1}."""
    x = np.asarray(x, dtype=np.float64)
    t = 2.0 * x - 1.0
    P = np.empty(x.shape + (k,), dtype=np.float64)
    P[..., 0] = 1.0
    if k > 1:
        P[..., 1] = t
    for a in range(1, k - 1):
        P[..., a + 1] = ((2 * a + 1) * t * P[..., a] - a * P[..., a - 1]) / (a + 1)
    P *= np.sqrt(2.0 * np.arange(k) + 1.0)
    inside = (x >= 0.0) & (x <= 1.0)
    return np.where(inside[..., None], P, 0.0)


def two_scale_filters(k):
    """H^(0), H^(1) (k x k) with phi_a(x) = sqrt2 sum_b (h0_ab phi_b(2x) + h1_ab phi_b(2x-1))
    (App. A.3).  Projecting that relation on sqrt2 phi_b(2x-s) gives
    h^(s)_ab = 2^-1/2 int_0^1 phi_a((u+s)/2) phi_b(u) du; the integrand is a polynomial of
    degree <= 2k-2, so the k-point Gauss-Legendre rule is exact."""
    u, w = gauss_legendre01(k)
    H = []
    for s in (0, 1):
        pa = phi(k, 0.5 * (u + s))          # (k nodes, k) -> phi_a((u+s)/2)
        pb = phi(k, u)                      # phi_b(u)
        H.append(np.einsum("i,ia,ib->ab", w, pa, pb) / np.sqrt(2.0))
    return H[0], H[1]


def wavelet_filters(k):
    """G^(0), G^(1) (k x k) such that W = [[H0, H1], [G0, G1]] is orthogonal (App. A.3): the
    decomposition d^j = G0 s^{j+1}_{2l} + G1 s^{j+1}_{2l+1} (eq. decomp_wavelet) and the
    reconstruction s^{j+1}_{2l+s} = H^(s)^T s^j + G^(s)^T d^j."""
    H0, H1 = two_scale_filters(k)
    Hr = np.hstack([H0, H1])                     # k x 2k, orthonormal rows
    P = np.eye(2 * k) - Hr.T @ Hr                # projector onto the complement (rank k)
    basis = []
    for c in range(2 * k):
        v = P[:, c].copy()
        for _ in range(2):
            for b in basis:
                v -= (b @ v) * b
            for h in Hr:
                v -= (h @ v) * h
        n = np.linalg.norm(v)
        if n > 1e-8:
            basis.append(v / n)
        if len(basis) == k:
            break
    G = np.array(basis)                          # k x 2k
    return G[:, :k].copy(), G[:, k:].copy()


def crosscorr(k, x):
    """Phi_ab(x) = int phi_a(x+y) phi_b(y) dy for x in [-1,1] (App. A.4, eqs. CrossCor, crosscor.01):
        0 <= x <= 1 :  Phi^+_ab(x) = int_0^{1-x} phi_a(x+y) phi_b(y) dy
       -1 <= x <  0 :  Phi^-_ab(x) = int_{-x}^{1} phi_a(x+y) phi_b(y) dy
    and 0 for |x| > 1.  The integrand is a polynomial of degree a+b <= 2k-2 in y, so the
    k-point Gauss-Legendre rule on the integration interval is exact.
    Returns shape x.shape + (k, k)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t, w = gauss_legendre01(k)
    lo = np.where(x >= 0.0, 0.0, -x)
    hi = np.where(x >= 0.0, 1.0 - x, 1.0)
    lo = np.clip(lo, 0.0, 1.0)
    hi = np.clip(hi, 0.0, 1.0)
    length = np.maximum(hi - lo, 0.0)
    y = lo[..., None] + length[..., None] * t            # (..., k nodes)
    wy = length[..., None] * w
    pa = phi(k, x[..., None] + y)                         # (..., nodes, k)
    pb = phi(k, y)
    out = np.einsum("...i,...ia,...ib->...ab", wy, pa, pb)
    out[np.abs(x) > 1.0] = 0.0
    return out


def _shifted_legendre(n):
    """Integer coefficients (ascending powers of x) of P_n(2x - 1) = sum_i (-1)^(n+i) C(n,i) C(n+i,i) x^i."""
    from math import comb
    return [(-1) ** (n + i) * comb(n, i) * comb(n + i, i) for i in range(n + 1)]


def _poly_mul(p, q):
    out = [0] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _poly_shift(p, c):
    """Coefficients of p(x + c) for rational c."""
    from math import comb
    out = [0] * len(p)
    for i, a in enumerate(p):
        for j in range(i + 1):
            out[j] += a * comb(i, j) * c ** (i - j)
    return out


def _cross_rational(a, b, plus):
    """Rational coefficients (ascending powers of x) of Q_ab with Phi_ab = sqrt((2a+1)(2b+1)) Q_ab:
        plus : Q(x) = int_0^{1-x} P~_a(x+y) P~_b(y) dy            (x in [0,1])
        minus: Q(x) = int_{-x}^{1} P~_a(x+y) P~_b(y) dy           (x in [-1,0])
    with P~_n(t) = P_n(2t-1) (App. A.4, eqs. CrossCor, crosscor.01).  The integrand is expanded as
    a polynomial in (x, y), integrated in y exactly and the bounds substituted."""
    from fractions import Fraction
    pa, pb = _shifted_legendre(a), _shifted_legendre(b)
    # P~_a(x + y) = sum_i pa_i (x+y)^i = sum_{r,s} c_rs x^r y^s
    from math import comb
    terms = {}
    for i, ca in enumerate(pa):
        for r in range(i + 1):
            for sy, cb in enumerate(pb):
                key = (r, i - r + sy)
                terms[key] = terms.get(key, 0) + ca * comb(i, r) * cb
    # int y^s dy = y^(s+1)/(s+1) between the bounds; bounds are polynomials in x
    lo = [Fraction(0)] if plus else [Fraction(0), Fraction(-1)]          # 0  or  -x
    hi = [Fraction(1), Fraction(-1)] if plus else [Fraction(1)]          # 1-x or 1
    out = [Fraction(0)] * (a + b + 2)
    for (r, sy), c in terms.items():
        ph = [Fraction(1)]
        pl = [Fraction(1)]
        for _ in range(sy + 1):
            ph = _poly_mul(ph, hi)
            pl = _poly_mul(pl, lo)
        diff = [(ph[i] if i < len(ph) else 0) - (pl[i] if i < len(pl) else 0) for i in range(max(len(ph), len(pl)))]
        for i, d in enumerate(diff):
            if d:
                out[r + i] += Fraction(c) * d / (sy + 1)
    return out


@functools.lru_cache(maxsize=None)
def _crosscorr_coeffs_cached(k):
    return _crosscorr_coeffs_exact(k)


def crosscorr_coeffs(k):
    """Cp, Cm of _crosscorr_coeffs_exact (cached per k; fresh copies)."""
    Cp, Cm = _crosscorr_coeffs_cached(k)
    return Cp.copy(), Cm.copy()


def _crosscorr_coeffs_exact(k):
    """Expansion of Phi^+ and Phi^- in Legendre scaling functions of degree < 2k (App. A.4: they
    are polynomials of degree a+b+1 <= 2k-1 on each half):
        Phi^+_ab(x)  = sum_n Cp[a,b,n] phi_n(x)     on [0,1]
        Phi^-_ab(x)  = sum_n Cm[a,b,n] phi_n(x+1)   on [-1,0]
    computed in exact rational arithmetic (Phi_ab = sqrt((2a+1)(2b+1)) Q_ab, phi_n =
    sqrt(2n+1) P~_n, int_0^1 x^i dx = 1/(i+1)); only the final square-root factor is rounded, so
    coefficients of degree above a+b+1 are exactly zero and the others carry no quadrature noise
    (narrow Gaussian terms weight every coefficient with moments far larger than the block)."""
    from fractions import Fraction
    Cp = np.zeros((k, k, 2 * k))
    Cm = np.zeros((k, k, 2 * k))
    pl = [_shifted_legendre(n) for n in range(2 * k)]
    for a in range(k):
        for b in range(k):
            qp = _cross_rational(a, b, True)
            qm = _poly_shift(_cross_rational(a, b, False), Fraction(-1))   # as a polynomial in z = x + 1
            for n in range(min(a + b + 2, 2 * k)):
                prod_p = _poly_mul(qp, pl[n])
                prod_m = _poly_mul(qm, pl[n])
                ip = sum(Fraction(c) / (i + 1) for i, c in enumerate(prod_p))
                im = sum(Fraction(c) / (i + 1) for i, c in enumerate(prod_m))
                sc = np.sqrt(float((2 * a + 1) * (2 * b + 1) * (2 * n + 1)))
                Cp[a, b, n] = float(ip) * sc
                Cm[a, b, n] = float(im) * sc
    return Cp, Cm


def _panel_breaks(u0, u1, c, s):
    """Panel end points on [u0,u1] for the Gaussian exp(-((x-c)/s)^2): the centre and
    c +- s*2^q, q=-2..6, that fall inside the interval."""
    pts = [u0, u1]
    cand = [c] + [c + sg * s * 2.0 ** q for q in range(-2, 7) for sg in (-1.0, 1.0)]
    pts += [p for p in cand if u0 < p < u1]
    return np.unique(np.array(pts, dtype=np.float64))


def _moments(nbasis, beta, l, shift, breaks, ngl):
    """For every block i: mu[i, n] = int exp(-beta_i (x+l_i)^2) phi_n(x+shift) dx over
    [breaks_i[0], breaks_i[-1]] by composite Gauss-Legendre with ngl points per panel.  The
    breaks are given in the offset u = x + l_i from the Gaussian's centre, so that the exponent
    beta u^2 keeps its relative accuracy for narrow Gaussians centred at an end of the interval
    (x near 1 would lose the low digits of x + l_i = x - 1)."""
    t, w = gauss_legendre01(ngl)
    xs, ws, starts, pos = [], [], [], 0
    for br in breaks:
        a = br[:-1, None]
        b = br[1:, None]
        xs.append((a + (b - a) * t).ravel())
        ws.append(((b - a) * w).ravel())
        starts.append(pos)
        pos += xs[-1].size
    x = np.concatenate(xs)
    wx = np.concatenate(ws)
    sizes = np.diff(np.append(starts, pos))
    bb = np.repeat(beta, sizes)
    ll = np.repeat(l, sizes)
    g = wx * np.exp(-bb * x ** 2)
    return np.add.reduceat(g[:, None] * phi(nbasis, x - ll + shift), np.array(starts), axis=0)


def _half_moments(nbasis, beta, l, u0, u1, shift, ngl, rtol):
    """Gaussian moments on one half [u0,u1] for a batch of (beta, l); panels graded around
    x = -l are halved until every block's moments change by less than rtol * max|mu|."""
    breaks = [_panel_breaks(u0 + float(li), u1 + float(li), 0.0, 1.0 / np.sqrt(bi)) for bi, li in zip(beta, l)]
    mu = _moments(nbasis, beta, l, shift, breaks, ngl)
    # exp(-A) with A = beta (x+l)^2 is only good to about A*1e-16 relative: the attainable
    # tolerance grows with the smallest exponent on the interval
    dist = np.maximum(0.0, np.maximum(u0 - (-l), (-l) - u1))
    tol = rtol * (1.0 + beta * dist * dist)
    todo = np.arange(len(beta))
    for _ in range(12):
        breaks = [np.sort(np.concatenate([br, 0.5 * (br[:-1] + br[1:])])) for br in breaks]
        mu2 = _moments(nbasis, beta[todo], l[todo], shift, breaks, ngl)
        scale = np.maximum(np.max(np.abs(mu2), axis=1), 1e-300)
        ok = np.max(np.abs(mu2 - mu[todo]), axis=1) <= tol[todo] * scale
        mu[todo] = mu2
        todo = todo[~ok]
        breaks = [br for br, o in zip(breaks, ok) if not o]
        if todo.size == 0:
            return mu
    raise RuntimeError("operator-block quadrature did not converge")


def F_blocks(k, j, tau, l, coeffs=None, ngl=32, rtol=1e-14):
    """Operator blocks F^{j;m,l} (k x k; row = output degree a, column = input degree b) for a
    batch of (tau, l) pairs at scale j:
        F_ab = 2^-j int_{-1}^{1} exp(-tau (x+l)^2 / 4^j) Phi_ab(x) dx          (Sec. 3, eq. KernelFactor)
    Phi is split at x=0 into its two polynomial pieces (App. A.4, eq. crosscor.00); on each
    half, Phi_ab = sum_n C_abn phi_n, so the integral is sum_n C_abn mu_n with Gaussian moments
    mu_n computed by composite Gauss-Legendre quadrature whose panels are graded around the
    Gaussian centre x=-l; panels are halved until the moments change by less than rtol*max|mu|
    (the halved result is kept)."""
    if coeffs is None:
        coeffs = crosscorr_coeffs(k)
    Cp, Cm = coeffs
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    l = np.atleast_1d(np.asarray(l, dtype=np.float64))
    beta = tau / 4.0 ** j
    mup = _half_moments(2 * k, beta, l, 0.0, 1.0, 0.0, ngl, rtol)
    mum = _half_moments(2 * k, beta, l, -1.0, 0.0, 1.0, ngl, rtol)
    F = np.einsum("abn,in->iab", Cp, mup) + np.einsum("abn,in->iab", Cm, mum)
    return F / 2.0 ** j


def F_block(k, j, tau, l, coeffs=None):
    """Single block F^{j;m,l} (eq. KernelFactor); see F_blocks."""
    return F_blocks(k, j, [tau], [l], coeffs)[0]


def F_table(k, tau, max_level, lmax=7):
    """F[j, m, l+lmax] for j = 0..max_level, every term m, l = -lmax..lmax (eq. KernelFactor)."""
    coeffs = crosscorr_coeffs(k)
    tau = np.asarray(tau, dtype=np.float64)
    M, nl = tau.size, 2 * lmax + 1
    tt = np.repeat(tau, nl)
    ll = np.tile(np.arange(-lmax, lmax + 1, dtype=np.float64), M)
    out = np.zeros((max_level + 1, M, nl, k, k))
    for j in range(max_level + 1):
        out[j] = F_blocks(k, j, tt, ll, coeffs).reshape(M, nl, k, k)
    return out
