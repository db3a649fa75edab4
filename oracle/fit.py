"""Gaussian-sum fit of radial kernels (test infrastructure only).

Kernel family (-Delta + mu^2)^(-alpha), 0 < alpha < 3/2 (Sec. 3):
    K_{mu,alpha}(r) = 2^(alpha-3/2) C_alpha (mu/r)^(3/2-alpha) K_{3/2-alpha}(mu r),
    C_alpha = 2 * 2^(-2 alpha) pi^(-3/2) / Gamma(alpha),
    K_{0,alpha}(r) = Gamma(3/2-alpha) C_alpha / (2 r^(3-2alpha)),
with the integral representation (eq. IntegralRepr)
    K_{mu,alpha}(r) = C_alpha int exp(-r^2 e^{2s}) exp(-mu^2 e^{-2s}/4 + (3-2alpha) s) ds.
The trapezoidal rule with s_m = A + m h, m = 1..M, h = (B-A)/M gives (eq. KernelApproxByGaussians)
    tau_m = e^{2 s_m},   w_m = h C_alpha exp(-mu^2 e^{-2 s_m}/4 + (3-2alpha) s_m),
with |K_{mu,alpha}(r) - sum_m w_m exp(-tau_m r^2)| <= eps K_{0,alpha}(r) on [delta, R].

The paper takes A, B, h from a reference it does not reproduce.  The reading taken here,
with nu = 3/2 - alpha:
    h0 = pi^2 / (2 (ln(1/eps) + ln 8))                     strip |Im s| < pi/4 of analyticity
    A  = ln(eps Gamma(nu+1)/4) / (2 nu) - ln R              lower tail <= eps/4 * K_0 on [delta,R]
    B  = ln(t_B / delta^2) / 2, with Q(nu, t_B) <= eps/4   upper tail <= eps/4 * K_0
and then h = h0 * 0.9^i (i = 0, 1, ...) until the relative error measured on 64 points per
decade over [delta, R] is at most eps/2.
"""
import math
import numpy as np
from scipy import special

__all__ = ["c_alpha", "kernel", "kernel0", "fit_params", "fit_kernel", "max_rel_error", "check_grid"]


def c_alpha(alpha):
    """C_alpha = 2 * 2^(-2 alpha) * pi^(-3/2) / Gamma(alpha) (Sec. 3)."""
    return 2.0 * 2.0 ** (-2.0 * alpha) * math.pi ** -1.5 / math.gamma(alpha)


def kernel0(alpha, r):
    """K_{0,alpha}(r) = Gamma(3/2-alpha) C_alpha / (2 r^(3-2 alpha)) (Sec. 3, eq. KernelApproxByGaussians)."""
    r = np.asarray(r, dtype=np.float64)
    return math.gamma(1.5 - alpha) * c_alpha(alpha) / (2.0 * r ** (3.0 - 2.0 * alpha))


def kernel(mu, alpha, r):
    """K_{mu,alpha}(r) in Bessel form (Sec. 3); mu = 0 gives the power law."""
    r = np.asarray(r, dtype=np.float64)
    if mu == 0.0:
        return kernel0(alpha, r)
    nu = 1.5 - alpha
    return 2.0 ** (alpha - 1.5) * c_alpha(alpha) * (mu / r) ** nu * special.kv(nu, mu * r)


def _upper_t(nu, eps):
    """t_B with Gamma(nu, t_B)/Gamma(nu) <= eps/4 (upper tail of the s-integral)."""
    if nu <= 1.0:
        # Gamma(nu, t) <= t^(nu-1) e^-t <= e^-t for t >= 1
        return max(1.0, math.log(4.0 / (eps * math.gamma(nu))))
    # Gamma(nu, t) <= 2 t^(nu-1) e^-t for t >= 2(nu-1)
    t = math.log(8.0 / (eps * math.gamma(nu)))
    for _ in range(8):
        t = math.log(8.0 / (eps * math.gamma(nu))) + (nu - 1.0) * math.log(t)
    return max(t, 2.0 * (nu - 1.0))


def fit_params(alpha, eps, delta, R):
    """(A, B, h0) of the trapezoidal discretisation (reading in the module docstring)."""
    nu = 1.5 - alpha
    h0 = math.pi ** 2 / (2.0 * (math.log(1.0 / eps) + math.log(8.0)))
    A = math.log(eps * math.gamma(nu + 1.0) / 4.0) / (2.0 * nu) - math.log(R)
    B = 0.5 * math.log(_upper_t(nu, eps) / delta ** 2)
    return A, B, h0


def _terms(mu, alpha, A, B, M, scale):
    h = (B - A) / M
    s = A + h * np.arange(1, M + 1)                       # s_m = A + m h, m = 1..M
    tau = np.exp(2.0 * s)
    w = scale * h * c_alpha(alpha) * np.exp(-mu * mu * np.exp(-2.0 * s) / 4.0 + (3.0 - 2.0 * alpha) * s)
    return tau, w


def check_grid(delta, R):
    """64 points per decade on [delta, R], end points included."""
    n = int(math.ceil(64.0 * math.log10(R / delta)))
    r = delta * 10.0 ** (np.arange(n + 1) / 64.0)
    r[-1] = R
    return r


def max_rel_error(mu, alpha, tau, w, delta, R, scale=1.0, r=None):
    """max_r |K_{mu,alpha}(r)*scale - sum_m w_m e^{-tau_m r^2}| / (scale*K_{0,alpha}(r)) on [delta, R]."""
    if r is None:
        r = check_grid(delta, R)
    approx = np.zeros_like(r)
    for m in range(len(tau)):                              # ascending m
        approx += w[m] * np.exp(-tau[m] * r * r)
    return float(np.max(np.abs(scale * kernel(mu, alpha, r) - approx) / (scale * kernel0(alpha, r))))


def fit_kernel(mu, alpha, eps, delta, R, scale=1.0, max_iter=40):
    """Exponents tau_m and weights w_m (scaled by `scale`) of the Gaussian sum for K_{mu,alpha}
    at accuracy eps on [delta, R] (eq. KernelApproxByGaussians).  Returns (tau, w)."""
    if not (0.0 < alpha < 1.5) or mu < 0.0 or not (0.0 < eps < 1.0) or not (0.0 < delta < R):
        raise ValueError("invalid fit parameters")
    A, B, h0 = fit_params(alpha, eps, delta, R)
    for i in range(max_iter):
        M = int(math.ceil((B - A) / (h0 * 0.9 ** i)))
        tau, w = _terms(mu, alpha, A, B, M, scale)
        if max_rel_error(mu, alpha, tau, w, delta, R, scale) <= 0.5 * eps:
            return tau, w
    raise RuntimeError("Gaussian-sum fit did not reach the requested accuracy")
