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


def test_fitted_truncated_grid_matches_points():
    """The tensor-grid evaluation (one contraction over (source, term) pairs) equals the pointwise
    sum at every grid point, chunks smaller than the pair count included."""
    rng = np.random.Generator(np.random.PCG64(12))
    xyz = rng.uniform(0.2, 0.8, (4, 3))
    a = 10.0 ** rng.uniform(1.0, 3.0, 4)
    c = rng.normal(0.0, 1.0, 4)
    tau = 10.0 ** rng.uniform(-1.0, 3.0, 5)
    w = rng.uniform(0.1, 1.0, 5)
    gx, gy, gz = rng.uniform(0.0, 1.0, 3), rng.uniform(0.0, 1.0, 4), rng.uniform(0.0, 1.0, 5)
    G = cf.fitted_truncated_grid(tau, w, xyz, a, c, gx, gy, gz, chunk=7)
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    ref = cf.fitted_truncated(tau, w, xyz, a, c, np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)).reshape(G.shape)
    assert np.abs(G - ref).max() <= 1e-14 * np.abs(ref).max()
