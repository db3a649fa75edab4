"""Pins of the hydrogen iteration's oracle (Sec. 6.2): the Coulomb product against a closed-form
integral and pointwise values, and the iteration's energy approaching the exact ground state E = -1/2."""
import math

import numpy as np

from oracle import hydrogen as Hy
from oracle import tree as T


def _gaussian_tree(k, jmax, s, a=1.0):
    # the physical unit-mass Gaussian (a/pi)^{3/2} e^{-a r^2} at the nucleus, on the unit cube
    keys, coef = T.project_gaussians(k, 1e-6, 2, jmax, [[0.5, 0.5, 0.5]], [a * s * s], [s ** -3])
    return T.redundant_tree(k, keys, coef)


def test_coulomb_product_integral_and_values():
    """int (1/r) (a/pi)^{3/2} e^{-a r^2} d^3x = 2 sqrt(a/pi); the product's blocks integrate to it (the
    degree-0 coefficient of every leaf, physical volume s^3) within 2e-7, and its values away from
    the nucleus are c f / r within 2e-6 of the largest (f is projected at 1e-6)."""
    k, jmax, L, a = 8, 9, 10.0, 0.25
    s = 2.0 * L
    f = _gaussian_tree(k, jmax, s, a)
    rho = Hy.coulomb_product(f, 1.0, jmax, s)
    lf = rho.leaf == 1
    integral = s ** 3 * float(np.sum(rho.coef[lf, 0, 0, 0] * 2.0 ** (-1.5 * rho.level[lf])))
    assert abs(integral / (2.0 * math.sqrt(a / math.pi)) - 1.0) < 2e-7
    rng = np.random.default_rng(3)
    pts = 0.5 + rng.uniform(-0.08, 0.08, (400, 3))
    r = s * np.linalg.norm(pts - 0.5, axis=1)
    keep = r > 0.3
    want = (a / math.pi) ** 1.5 * np.exp(-a * r[keep] ** 2) / r[keep]
    got = T.evaluate(rho, pts[keep])
    assert np.abs(got - want).max() < 2e-6 * np.abs(want).max()
    # every leaf of f's tree is split once, and the nucleus' boxes reach jmax
    assert set(T.children_keys(f.keys[f.leaf == 1]).tolist()) <= set(rho.keys.tolist())
    assert all(key in set(rho.keys[lf].tolist()) for key in Hy.nucleus_boxes(jmax))


def test_kalos_iteration_approaches_the_ground_state():
    """Sec. 6.2: the iteration from mu_0 = 0.8 moves E towards -1/2 (the exact eigenvalue of the
    ground state, psi = e^{-r}), each step closer, within 1e-3 after four steps (k = 5, eps = 1e-3)."""
    hist = Hy.kalos(5, 1e-3, 10.0, 7, mu0=0.8, iters=4)
    err = [abs(E + 0.5) for _, E in hist]
    print("E:", ["%.6f" % E for _, E in hist])
    assert all(b < a for a, b in zip(err, err[1:]))
    assert err[-1] < 1e-3
    # mu follows sqrt(-2 E)
    for (mu, E), (mu2, _) in zip(hist, hist[1:]):
        assert abs(mu2 - math.sqrt(-2.0 * E)) < 1e-15
