"""Pins of the d = 2 oracle (Alg. 3 in the plane; Sec. 3's representation with two dimensions): the
fitted kernel against Bessel closed forms and direct quadrature, Alg. 1's criterion, the plan's
symmetry and monotonicity, the modified form against the difference form and the dense operator,
and the apply against the fitted kernel applied in closed form."""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import mra
from oracle import ns2d as N


@pytest.mark.parametrize("mu,alpha", [(5.0, 1.0), (0.5, 1.0), (0.0, 0.5), (3.0, 0.7)])
def test_kernel_closed_form_against_its_integral(mu, alpha):
    for r in (0.01, 0.3, 1.2):
        val = integrate.quad(lambda s: math.exp(-r * r * math.exp(2 * s) - mu * mu * math.exp(-2 * s) / 4
                                                 + (2 - 2 * alpha) * s), -30, 30, limit=800, epsabs=0, epsrel=1e-13)[0]
        assert abs(N.c2_alpha(alpha) * val / float(N.kernel2d(mu, alpha, r)) - 1.0) < 1e-10


@pytest.mark.parametrize("mu,alpha,eps", [(5.0, 1.0, 1e-6), (1.0, 1.0, 1e-8), (0.0, 0.5, 1e-6), (3.0, 0.7, 1e-6)])
def test_fit_relative_error(mu, alpha, eps):
    delta, R = math.sqrt(eps) * 2.0 ** -8, math.sqrt(2.0)
    tau, w = N.fit_kernel2d(mu, alpha, eps, delta, R)
    r = np.exp(np.random.default_rng(1).uniform(math.log(delta), math.log(R), 4000))
    got = (w[None, :] * np.exp(-tau[None, :] * r[:, None] ** 2)).sum(1)
    assert np.max(np.abs(got / N.kernel2d(mu, alpha, r) - 1.0)) <= eps
    assert np.all(tau > 0) and np.all(w > 0)


def _case(seed=4, k=6, eps=1e-5, n=3, jmax=7):
    rng = np.random.default_rng(seed)
    xy = rng.uniform(0.3, 0.7, (n, 2))
    a = 10 ** rng.uniform(1.5, 3.0, n)
    c = rng.normal(size=n)
    return k, eps, xy, a, c, jmax


def test_alg1_criterion_and_wide_source():
    """Every leaf below jmax passes the interpolation test at its children's nodes, every internal node
    fails it (checked with an independent tensor evaluation); a wide Gaussian stays one box."""
    k, eps, xy, a, c, jmax = _case()
    tr = N.project2d(k, eps, 1, jmax, xy, a, c)
    thr = eps * N.source_norm2d(xy, a, c)
    x, _ = mra.gauss_legendre01(k)
    for i in range(tr.keys.size):
        j, (lx, ly) = int(tr.level[i]), tr.l[i]
        if j >= jmax or j < 1:
            continue
        s = N._box_coeffs(k, j, lx, ly, lambda X, Y: N.gauss2d(X, Y, xy, a, c))
        err = 0.0
        for sx, sy in itertools.product((0, 1), repeat=2):
            u = (2 * lx + sx + x) / 2.0 ** (j + 1)
            v = (2 * ly + sy + x) / 2.0 ** (j + 1)
            px = mra.phi(k, u * 2.0 ** j - lx)
            py = mra.phi(k, v * 2.0 ** j - ly)
            poly = 2.0 ** j * np.einsum("qa,ab,rb->qr", px, s, py)
            U, V = np.meshgrid(u, v, indexing="ij")
            err = max(err, float(np.abs(poly - N.gauss2d(U, V, xy, a, c)).max()))
        assert (err > thr) == (tr.leaf[i] == 0), (j, lx, ly)
    wide = N.project2d(k, 1e-3, 0, 6, [[0.5, 0.5]], [0.5], [1.0])
    assert wide.keys.size == 1


def test_plan_symmetric_monotone_and_full():
    k = 6
    tau, w = N.fit_kernel2d(5.0, 1.0, 1e-6, 1e-6, math.sqrt(2.0))
    F = mra.F_table(k, tau, 5)
    H0, H1 = mra.two_scale_filters(k)
    R6, _ = N.make_plan2d(F, H0, H1, w, 1e-6, 5)
    R4, _ = N.make_plan2d(F, H0, H1, w, 1e-4, 5)
    for j in range(1, 6):
        for L in itertools.product(range(-3, 4), repeat=2):
            r = tuple(R6[j, L[0] + 3, L[1] + 3])
            for P in ((L[1], L[0]), (-L[0], L[1]), (L[0], -L[1])):
                assert tuple(R6[j, P[0] + 3, P[1] + 3]) == r
            a4, b4 = R4[j, L[0] + 3, L[1] + 3]
            if b4 >= a4:       # a looser eps keeps a sub-range
                assert r[0] <= a4 and b4 <= r[1]
    full = N.full_plan2d(tau.size, 5)
    assert np.all(full[1:, ..., 0] == 0) and np.all(full[1:, ..., 1] == tau.size - 1)


def test_modified_equals_difference_form_and_dense():
    """eq. apply_algo against eq. g_scales_band (after assembly, at the leaves) on an adaptive tree
    with the screened plan and with a random plan; with screening off on a uniform level-3 tree the
    modified form is the dense P_3 T P_3."""
    k, eps, xy, a, c, jmax = _case(k=4, jmax=6)
    tr = N.project2d(k, eps, 2, jmax, xy, a, c)
    tau, w = N.fit_kernel2d(5.0, 1.0, eps, math.sqrt(eps) * 2.0 ** -tr.depth, math.sqrt(2.0))
    F = mra.F_table(k, tau, tr.depth)
    H0, H1 = mra.two_scale_filters(k)
    R, _ = N.make_plan2d(F, H0, H1, w, eps, tr.depth)
    rng = np.random.default_rng(2)
    Rr = R.copy()
    for j in range(1, tr.depth + 1):
        for L in itertools.product(range(7), repeat=2):
            m1 = int(rng.integers(0, tau.size))
            Rr[j, L[0], L[1]] = (m1, min(tau.size - 1, m1 + int(rng.integers(0, 20)))) if rng.random() < 0.8 else (0, -1)
    lf = tr.leaf == 1
    for plan in (R, Rr):
        g = N.assemble2d(tr, N.apply_modified2d(tr, F, w, plan))
        gd = N.assemble2d(tr, N.apply_difference2d(tr, F, w, plan, H0, H1))
        assert np.abs(g[lf] - gd[lf]).max() <= 1e-13 * np.abs(g[lf]).max()
    leaves = {(3, x, y): rng.normal(size=(4, 4)) for x in range(8) for y in range(8)}
    tu = N.redundant_tree2(4, leaves)
    F2 = mra.F_table(4, tau[:30], 3)
    gu = N.assemble2d(tu, N.apply_modified2d(tu, F2, w[:30], N.full_plan2d(30, 3)))
    dense = N.dense_uniform2d(tu, F2, w[:30])
    assert max(np.abs(gu[i] - dense[i]).max() for i in dense) < 1e-13 * max(np.abs(v).max() for v in dense.values())


def test_apply_against_fitted_kernel_closed_form():
    """The applied potential at grid points against the fitted kernel applied exactly to the
    square-truncated source (per term and source two 1-D erf integrals): within eps ||f||_2."""
    k, eps, xy, a, c, jmax = _case()
    tr = N.project2d(k, eps, 2, jmax, xy, a, c)
    tau, w = N.fit_kernel2d(5.0, 1.0, eps, math.sqrt(eps) * 2.0 ** -tr.depth, math.sqrt(2.0))
    F = mra.F_table(k, tau, tr.depth)
    H0, H1 = mra.two_scale_filters(k)
    R, _ = N.make_plan2d(F, H0, H1, w, eps, tr.depth)
    g = N.assemble2d(tr, N.apply_modified2d(tr, F, w, R))
    gx, gy = np.linspace(0.05, 0.95, 13), np.linspace(0.07, 0.93, 11)
    ref = N.fitted_truncated2d(tau, w, xy, a, c, gx, gy)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    val = N.evaluate2d(tr, g, np.stack([X.ravel(), Y.ravel()], 1)).reshape(ref.shape)
    assert np.abs(val - ref).max() <= eps * N.source_norm2d(xy, a, c)


def test_evaluation_inverts_the_projection_at_nodes():
    k, eps, xy, a, c, jmax = _case(k=5, jmax=5)
    tr = N.project2d(k, eps, 2, jmax, xy, a, c)
    x, _ = mra.gauss_legendre01(k)
    for i in np.nonzero(tr.leaf)[0][:20]:
        j, (lx, ly) = int(tr.level[i]), tr.l[i]
        X, Y = np.meshgrid((lx + x) / 2.0 ** j, (ly + x) / 2.0 ** j, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel()], 1)
        want = N.gauss2d(X, Y, xy, a, c).ravel()
        got = N.evaluate2d(tr, tr.coef, pts)
        # at the nodes the polynomial equals f (the k-point rule interpolates)
        assert np.abs(got - want).max() <= 1e-10 * max(1.0, np.abs(want).max())
