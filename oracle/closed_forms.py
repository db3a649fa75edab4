"""Analytic references for the operator apply (test infrastructure only).

  * poisson_gaussian: potential of a unit-mass Gaussian (a/pi)^{3/2} e^{-a r^2} under the
    Poisson kernel 1/(4 pi r) in free space: erf(sqrt(a) r) / (4 pi r).
  * yukawa_gaussian: the same source under e^{-mu r}/(4 pi r):
      e^{mu^2/(4a)} / (8 pi r) [e^{-mu r} erfc(mu/(2 sqrt a) - sqrt(a) r) - e^{mu r} erfc(mu/(2 sqrt a) + sqrt(a) r)],
    evaluated through erfcx to avoid overflow.
  * fitted_truncated: the Gaussian-sum kernel sum_m w_m e^{-tau_m r^2} applied to a sum of
    Gaussians restricted to the unit cube (f = 0 outside [0,1]^3, the paper's free-space setting):
    separability gives, per source term and kernel term, a product over the three dimensions of
      G(tau, a, c, x) = int_0^1 e^{-tau (x-y)^2} e^{-a (y-c)^2} dy
                      = e^{-tau a (x-c)^2/(tau+a)} sqrt(pi)/(2 sqrt(tau+a)) [erf(s (1-q)) + erf(s q)],
      s = sqrt(tau+a), q = (tau x + a c)/(tau+a).
  * three_gaussians / three_gaussians_laplacian / ..._l2norm: the Poisson test of Sec. 6.1:
    phi = sum_{i=1..3} e^{-alpha |r - r_i|^2} with alpha = 300 and the three printed centres, the
    source rho = -Laplacian(phi), so that phi is the exact potential of rho under 1/(4 pi r).
These are references for the exact operator; the method approximates them to about eps.
"""
import numpy as np
from scipy import special

__all__ = ["poisson_gaussian", "yukawa_gaussian", "fitted_truncated", "gauss_sum", "SEC61_ALPHA", "SEC61_CENTRES",
           "three_gaussians", "three_gaussians_laplacian", "three_gaussians_laplacian_l2norm"]

# Sec. 6.1: exponent and centres of the three Gaussians of the Poisson test
SEC61_ALPHA = 300.0
SEC61_CENTRES = np.array([[0.5, 0.5, 0.5], [0.6, 0.6, 0.5], [0.35, 0.6, 0.5]])


def three_gaussians(x, y, z, alpha=SEC61_ALPHA, centres=SEC61_CENTRES):
    """phi(r) = sum_i exp(-alpha |r - r_i|^2) (Sec. 6.1), at broadcastable coordinate arrays."""
    out = 0.0
    for cx, cy, cz in centres:
        out = out + np.exp(-alpha * ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2))
    return out


def three_gaussians_laplacian(x, y, z, alpha=SEC61_ALPHA, centres=SEC61_CENTRES):
    """rho = -Laplacian(phi) = sum_i (6 alpha - 4 alpha^2 |r - r_i|^2) exp(-alpha |r - r_i|^2):
    each term of phi is a product of three 1-D Gaussians g(t) = exp(-alpha t^2) with
    g'' = (4 alpha^2 t^2 - 2 alpha) g."""
    out = 0.0
    for cx, cy, cz in centres:
        r2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
        out = out + (6.0 * alpha - 4.0 * alpha * alpha * r2) * np.exp(-alpha * r2)
    return out


def three_gaussians_laplacian_l2norm(alpha=SEC61_ALPHA, centres=SEC61_CENTRES):
    """||rho||_2 over R^3, exact: rho_i = sum_t c_t prod_d p_td(x_d - r_id) e^{-alpha (x_d - r_id)^2}
    with the separable terms (t = 0: 6 alpha; t = d: -4 alpha^2 (x_d - r_id)^2), so <rho_i, rho_q>
    is a sum of products of 1-D integrals of polynomials (degree <= 4) times
    e^{-alpha (x-a)^2 - alpha (x-b)^2} = e^{-alpha (a-b)^2 / 2} e^{-2 alpha (x - (a+b)/2)^2},
    which 8-point Gauss-Hermite quadrature integrates exactly."""
    t, wh = np.polynomial.hermite.hermgauss(8)

    def one_d(pa, pb, a, b):
        # int (x-a)^pa (x-b)^pb e^{-alpha (x-a)^2 - alpha (x-b)^2} dx, substituting x = m + t / sqrt(2 alpha)
        m = 0.5 * (a + b)
        x = m + t / np.sqrt(2.0 * alpha)
        return np.exp(-0.5 * alpha * (a - b) ** 2) * np.sum(wh * (x - a) ** pa * (x - b) ** pb) / np.sqrt(2.0 * alpha)

    terms = [(6.0 * alpha, (0, 0, 0))] + [(-4.0 * alpha * alpha, tuple(2 if e == d else 0 for e in range(3)))
                                          for d in range(3)]
    tot = 0.0
    for ri in centres:
        for rq in centres:
            for ct, pt in terms:
                for cu, pu in terms:
                    v = ct * cu
                    for d in range(3):
                        v *= one_d(pt[d], pu[d], ri[d], rq[d])
                    tot += v
    return float(np.sqrt(tot))


def gauss_sum(xyz, a, c, pts):
    """f(x) = sum_i c_i (a_i/pi)^{3/2} exp(-a_i |x - x_i|^2)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    for xi, ai, ci in zip(np.asarray(xyz).reshape(-1, 3), a, c):
        out += ci * (ai / np.pi) ** 1.5 * np.exp(-ai * np.sum((pts - xi) ** 2, axis=1))
    return out


def poisson_gaussian(a, r):
    """erf(sqrt(a) r)/(4 pi r), with the r -> 0 limit sqrt(a/pi)/(2 pi)."""
    r = np.asarray(r, dtype=np.float64)
    sa = np.sqrt(a)
    small = r < 1e-8
    rr = np.where(small, 1.0, r)
    return np.where(small, sa / (2.0 * np.pi ** 1.5), special.erf(sa * rr) / (4.0 * np.pi * rr))


def yukawa_gaussian(mu, a, r):
    """Potential of a unit-mass Gaussian under e^{-mu r}/(4 pi r) (closed form through erfcx)."""
    r = np.asarray(r, dtype=np.float64)
    sa = np.sqrt(a)
    b = mu / (2.0 * sa)
    x1 = b - sa * r
    x2 = b + sa * r
    # e^{b^2} e^{-mu r} erfc(x1) = e^{-a r^2} erfcx(x1) when x1 >= 0 (b^2 - mu r - x1^2 = -a r^2)
    t1 = np.where(x1 >= 0, np.exp(-a * r * r) * special.erfcx(np.maximum(x1, 0.0)),
                  np.exp(b * b - mu * r) * special.erfc(x1))
    t2 = np.exp(-a * r * r) * special.erfcx(x2)
    return (t1 - t2) / (8.0 * np.pi * np.maximum(r, 1e-300))


def _G(tau, a, c, x):
    s2 = tau + a
    s = np.sqrt(s2)
    q = (tau * x + a * c) / s2
    pre = np.exp(-tau * a * (x - c) ** 2 / s2) * np.sqrt(np.pi) / (2.0 * s)
    inner = np.where(q > 1.0, special.erfc(s * (q - 1.0)) - special.erfc(s * q),
                     np.where(q < 0.0, special.erfc(-s * q) - special.erfc(s * (1.0 - q)),
                              special.erf(s * (1.0 - q)) + special.erf(s * q)))
    return pre * inner


def fitted_truncated(tau, w, xyz, a, c, pts):
    """(sum_m w_m e^{-tau_m r^2}) * (f restricted to [0,1]^3) at the points."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    for xi, ai, ci in zip(np.asarray(xyz).reshape(-1, 3), a, c):
        cn = ci * (ai / np.pi) ** 1.5
        for tm, wm in zip(tau, w):
            out += cn * wm * _G(tm, ai, xi[0], pts[:, 0]) * _G(tm, ai, xi[1], pts[:, 1]) * _G(tm, ai, xi[2], pts[:, 2])
    return out


def fitted_truncated_grid(tau, w, xyz, a, c, gx, gy, gz, chunk=8192):
    """fitted_truncated on the tensor grid gx x gy x gz, [len(gx), len(gy), len(gz)]: the factors
    G of every (source, term) pair are separable, so the sum over the pairs is one contraction of
    three per-dimension tables (rows: pairs; columns: grid coordinates)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    gx, gy, gz = (np.asarray(v, dtype=np.float64) for v in (gx, gy, gz))
    tau = np.asarray(tau, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    rows = [(i, m) for i in range(xyz.shape[0]) for m in range(tau.size)]
    out = np.zeros((gx.size, gy.size, gz.size))
    for r0 in range(0, len(rows), chunk):
        part = rows[r0:r0 + chunk]
        ii = np.array([i for i, _ in part])
        mm = np.array([m for _, m in part])
        ai = np.asarray(a, dtype=np.float64)[ii][:, None]
        cn = (np.asarray(c, dtype=np.float64)[ii] * (np.asarray(a, dtype=np.float64)[ii] / np.pi) ** 1.5 * w[mm])[:, None]
        tm = tau[mm][:, None]
        G1 = cn * _G(tm, ai, xyz[ii, 0][:, None], gx[None, :])
        G2 = _G(tm, ai, xyz[ii, 1][:, None], gy[None, :])
        G3 = _G(tm, ai, xyz[ii, 2][:, None], gz[None, :])
        A = (G1[:, :, None] * G2[:, None, :]).reshape(len(part), -1)
        out += (A.T @ G3).reshape(gx.size, gy.size, gz.size)
    return out
