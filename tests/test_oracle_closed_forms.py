"""Pins of the analytic references against direct radial quadrature and limits."""
import math

import numpy as np
from scipy import integrate

from oracle import closed_forms as cf


def _radial_potential(K_times_t, a, r):
    """Potential of the unit-mass Gaussian at distance r for a radial kernel K, by the shell
    theorem: (2 pi / r) int_0^inf s f(s) [int_{|r-s|}^{r+s} K(t) t dt] ds."""
    f = lambda s: (a / math.pi) ** 1.5 * math.exp(-a * s * s)
    inner = lambda s: integrate.quad(K_times_t, abs(r - s), r + s, epsabs=0, epsrel=1e-13)[0]
    return 2 * math.pi / r * integrate.quad(lambda s: s * f(s) * inner(s), 0, 7 / math.sqrt(a), points=[r],
                                            epsabs=0, epsrel=1e-12, limit=400)[0]


def test_poisson_gaussian():
    a = 40.0
    for r in (0.02, 0.2, 0.7):
        ref = _radial_potential(lambda t: 1 / (4 * math.pi), a, r)
        assert abs(cf.poisson_gaussian(a, r) - ref) < 1e-9 * ref
    assert np.isclose(cf.poisson_gaussian(a, 5.0), 1 / (4 * math.pi * 5.0), rtol=1e-14)
    assert np.isclose(cf.poisson_gaussian(a, 0.0), math.sqrt(a / math.pi) / (2 * math.pi), rtol=1e-14)


def test_yukawa_gaussian():
    mu, a = 3.0, 50.0
    for r in (0.01, 0.1, 0.3, 1.0):
        ref = _radial_potential(lambda t: math.exp(-mu * t) / (4 * math.pi), a, r)
        assert abs(cf.yukawa_gaussian(mu, a, r) - ref) < 1e-8 * ref
    # mu -> 0 gives the Poisson potential
    assert np.isclose(cf.yukawa_gaussian(1e-9, a, 0.3), cf.poisson_gaussian(a, 0.3), rtol=1e-8)


def test_fitted_truncated_1d_factor():
    """G(tau, a, c, x) = int_0^1 exp(-tau (x-y)^2 - a (y-c)^2) dy against direct quadrature, also
    where the completed-square centre lies outside [0,1]."""
    for tau, a, c, x in [(3.0, 20.0, 0.4, 0.9), (1e4, 50.0, 0.3, 0.95), (500.0, 10.0, 0.9, -0.2),
                         (800.0, 30.0, 0.1, 1.3)]:
        ref = integrate.quad(lambda y: math.exp(-tau * (x - y) ** 2 - a * (y - c) ** 2), 0, 1,
                             points=[min(max(x, 0), 1)], epsabs=0, epsrel=1e-13, limit=200)[0]
        assert abs(cf._G(tau, a, c, np.array([x]))[0] - ref) <= 1e-11 * ref + 1e-300
