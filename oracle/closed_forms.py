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
These are references for the exact operator; the method approximates them to about eps.
"""
import numpy as np
from scipy import special

__all__ = ["poisson_gaussian", "yukawa_gaussian", "fitted_truncated", "gauss_sum"]


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
