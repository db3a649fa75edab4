"""Pins of the oracle's 1-D tables (App. A.1-A.4, eq. KernelFactor) against facts the paper and
the mathematics fix, independently of how the oracle computes them."""
import numpy as np
import pytest

from oracle import mra


@pytest.mark.parametrize("k", [1, 2, 6, 8, 10])
def test_gauss_legendre_exact_for_degree_2k_minus_1(k):
    x, w = mra.gauss_legendre01(k)
    for d in range(2 * k):
        assert abs(np.sum(w * x ** d) - 1.0 / (d + 1)) < 1e-14


def test_gauss_legendre_two_points():
    x, w = mra.gauss_legendre01(2)
    assert np.allclose(np.sort(x), [0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)], atol=1e-15)
    assert np.allclose(w, 0.5)


@pytest.mark.parametrize("k", [4, 8, 10])
def test_scaling_functions_orthonormal_and_end_values(k):
    # orthonormality on [0,1] (App. A.1), checked with a much finer independent rule
    t, wt = np.polynomial.legendre.leggauss(64)
    x, w = 0.5 * (t + 1), 0.5 * wt
    P = mra.phi(k, x)
    assert np.abs(P.T @ (w[:, None] * P) - np.eye(k)).max() < 1e-13
    # P_a(1) = 1, P_a(-1) = (-1)^a ; zero outside [0,1]
    a = np.arange(k)
    assert np.allclose(mra.phi(k, 1.0), np.sqrt(2 * a + 1))
    assert np.allclose(mra.phi(k, 0.0), (-1.0) ** a * np.sqrt(2 * a + 1))
    assert np.all(mra.phi(k, np.array([-0.1, 1.1])) == 0.0)
    # phi_2(x) = sqrt5 (6x^2 - 6x + 1)
    assert abs(mra.phi(k, 0.3)[2] - np.sqrt(5) * (6 * 0.09 - 1.8 + 1)) < 1e-14


def test_haar_filters():
    H0, H1 = mra.two_scale_filters(1)
    assert np.allclose(H0, 1 / np.sqrt(2)) and np.allclose(H1, 1 / np.sqrt(2))


@pytest.mark.parametrize("k", [2, 6, 8, 10])
def test_filters_orthogonality_and_symmetry(k):
    H0, H1 = mra.two_scale_filters(k)
    assert np.abs(H0 @ H0.T + H1 @ H1.T - np.eye(k)).max() < 1e-13
    D = np.diag((-1.0) ** np.arange(k))
    assert np.abs(H1 - D @ H0 @ D).max() < 1e-14


@pytest.mark.parametrize("k", [3, 6, 8])
def test_filters_reproduce_polynomials_across_scales(k):
    """A polynomial of degree < k lies in V_0: its level-1 coefficients (projected directly on each
    half by an independent quadrature) decompose to its level-0 coefficients and are recovered
    from them by zero-detail reconstruction (eqs. decomp_scaling, recon_even/odd)."""
    rng = np.random.default_rng(1)
    p = np.polynomial.Polynomial(rng.normal(size=k))
    t, wt = np.polynomial.legendre.leggauss(40)
    x, w = 0.5 * (t + 1), 0.5 * wt
    s0 = (w * p(x)) @ mra.phi(k, x)                     # <p, phi_a>
    s1 = []
    for half in (0, 1):                                  # <p, phi^1_{a,half}> = 2^{1/2} int p(x) phi_a(2x - half)
        y = 0.5 * (x + half)
        s1.append(np.sqrt(2.0) * 0.5 * (w * p(y)) @ mra.phi(k, x))
    H0, H1 = mra.two_scale_filters(k)
    assert np.abs(H0 @ s1[0] + H1 @ s1[1] - s0).max() < 1e-13
    assert np.abs(H0.T @ s0 - s1[0]).max() < 1e-13
    assert np.abs(H1.T @ s0 - s1[1]).max() < 1e-13


def _gegenbauer_m_half(n, t):
    """C_n^(-1/2)(t) by the Gegenbauer three-term recurrence with lambda = -1/2."""
    lam = -0.5
    c0, c1 = np.ones_like(t), 2 * lam * t
    if n == 0:
        return c0
    for m in range(2, n + 1):
        c0, c1 = c1, (2 * (m + lam - 1) * t * c1 - (m + 2 * lam - 2) * c0) / m
    return c1


@pytest.mark.parametrize("k", [4, 8])
def test_crosscorrelation_properties(k):
    """Prop. 1, items 1-7 (App. A.4)."""
    x = np.linspace(0.0, 1.0, 41)
    Pp = mra.crosscorr(k, x)
    Pm = mra.crosscorr(k, -x[1:])
    sgn = (-1.0) ** np.add.outer(np.arange(k), np.arange(k))
    # 1. transposition
    allx = np.linspace(-1, 1, 81)
    Pa = mra.crosscorr(k, allx)
    assert np.abs(Pa - sgn * np.swapaxes(Pa, -1, -2)).max() < 1e-13
    # 2. Phi^-(-x) = (-1)^{a+b} Phi^+(x)
    assert np.abs(Pm - sgn * Pp[1:]).max() < 1e-13
    # 3. values at 0
    assert np.abs(mra.crosscorr(k, 0.0)[0] - np.eye(k)).max() < 1e-13
    # 4. bounded by 1
    assert np.abs(Pa).max() <= 1.0 + 1e-13
    # 5. Gegenbauer forms
    assert np.abs(Pp[:, 0, 0] - (0.5 * _gegenbauer_m_half(1, 2 * x - 1) + 0.5)).max() < 1e-14
    assert np.abs(Pp[:, 0, 0] - (1 - x)).max() < 1e-14
    assert np.abs(Pp[:, 1, 0] - np.sqrt(3) * x * (1 - x)).max() < 1e-14
    for l in range(1, k):
        ref = 0.5 * np.sqrt(2 * l + 1) * _gegenbauer_m_half(l + 1, 2 * x - 1)
        assert np.abs(Pp[:, l, 0] - ref).max() < 1e-12
    # 7. vanishing moments, with an independent fine rule on each half
    t, wt = np.polynomial.legendre.leggauss(40)
    u, wu = 0.5 * (t + 1), 0.5 * wt
    Pu, Pmu = mra.crosscorr(k, u), mra.crosscorr(k, u - 1)
    for q in range(2 * k):
        mom = np.einsum("i,iab->ab", wu * u ** q, Pu) + np.einsum("i,iab->ab", wu * (u - 1) ** q, Pmu)
        for a in range(k):
            for b in range(k):
                if a + b >= 1 and q <= a + b - 1:
                    assert abs(mom[a, b]) < 1e-13
    mom0 = np.sum(wu * Pu[:, 0, 0]) + np.sum(wu * Pmu[:, 0, 0])
    assert abs(mom0 - 1.0) < 1e-14


@pytest.mark.parametrize("k,j,tau,l", [(6, 0, 30.0, 0), (6, 1, 300.0, 1), (8, 2, 5e3, -2), (8, 0, 2.0, 3),
                                       (10, 3, 1e5, 1), (6, 2, 1e4, -1)])
def test_F_block_against_direct_2d_quadrature(k, j, tau, l):
    """<phi^j_{a,l}, e^{-tau (x-y)^2} phi^j_{b,0}> by a brute-force tensor Gauss-Legendre rule over
    the two boxes (split in 16 panels each) equals F^{j;l}_ab (eq. KernelFactor derivation)."""
    F = mra.F_block(k, j, tau, l)
    t, wt = np.polynomial.legendre.leggauss(24)
    edges = np.linspace(0, 1, 17)
    u = np.concatenate([a + (b - a) * 0.5 * (t + 1) for a, b in zip(edges[:-1], edges[1:])])
    wu = np.concatenate([(b - a) * 0.5 * wt for a, b in zip(edges[:-1], edges[1:])])
    h = 2.0 ** -j
    x = h * (l + u)            # output box l
    y = h * u                  # input box 0
    K = np.exp(-tau * (x[:, None] - y[None, :]) ** 2)
    Pu = mra.phi(k, u) * np.sqrt(1 / h)   # phi^j_a = 2^{j/2} phi_a(2^j x - l)
    ref = h * h * np.einsum("i,q,iq,ia,qb->ab", wu, wu, K, Pu, Pu)
    assert np.abs(F - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("k", [2, 6, 10])
def test_crosscorr_coefficients_reproduce_phi(k):
    """The exact rational expansion of Phi^+- (App. A.4) reproduces Phi_ab(x) evaluated by the
    independent Gauss-Legendre integration in crosscorr(), on both halves; coefficients above
    degree a+b+1 are exactly zero."""
    Cp, Cm = mra.crosscorr_coeffs(k)
    x = np.linspace(0.003, 0.997, 11)
    basis = mra.phi(2 * k, x)
    assert np.abs(np.einsum("abn,in->iab", Cp, basis) - mra.crosscorr(k, x)).max() < 1e-14
    assert np.abs(np.einsum("abn,in->iab", Cm, basis) - mra.crosscorr(k, x - 1.0)).max() < 1e-14
    a, b, n = np.meshgrid(np.arange(k), np.arange(k), np.arange(2 * k), indexing="ij")
    assert np.all(Cp[n > a + b + 1] == 0.0) and np.all(Cm[n > a + b + 1] == 0.0)


def _G_adjacent(beta, l):
    """int_0^1 int_0^1 exp(-beta (u + l - v)^2) du dv for l = 0, 1 (the constant basis pair), by the
    triangular density of u - v: closed forms through erf."""
    from scipy.special import erf
    sb = np.sqrt(beta)
    if l == 0:
        return np.sqrt(np.pi / beta) * erf(sb) - (1.0 - np.exp(-beta)) / beta
    return ((1.0 - np.exp(-beta)) / (2.0 * beta) + np.sqrt(np.pi / beta) * (erf(2.0 * sb) - erf(sb))
            - (np.exp(-beta) - np.exp(-4.0 * beta)) / (2.0 * beta))


@pytest.mark.parametrize("k", [6, 8, 9, 10])
@pytest.mark.parametrize("j,tau", [(0, 1e3), (2, 1e4), (0, 1e6), (1, 7.1e8), (0, 1e10)])
def test_F_constant_pair_closed_form(k, j, tau):
    """F^{j;l}_00 = 2^-j G(tau/4^j, l) with G the closed form of the double integral of the Gaussian
    over two unit boxes at distance l (eq. KernelFactor with phi_0 = 1): to 1e-14 relative on the
    diagonal block also for very narrow Gaussians, where every high-degree moment of Phi is large,
    and to 1e-14 of that diagonal entry (the term's scale) for the neighbour; F^{j;0}_10 = 0 by the
    reflection x -> 1 - x."""
    beta = tau / 4.0 ** j
    F0 = mra.F_block(k, j, tau, 0)
    ref0 = _G_adjacent(beta, 0) / 2.0 ** j
    assert abs(F0[0, 0] - ref0) <= 1e-14 * ref0, (F0[0, 0], ref0)
    F1 = mra.F_block(k, j, tau, 1)
    assert abs(F1[0, 0] - _G_adjacent(beta, 1) / 2.0 ** j) <= 1e-14 * ref0
    assert abs(F0[1, 0]) <= 1e-15 * abs(F0[0, 0])


@pytest.mark.parametrize("k", [6, 8])
def test_F_symmetry_and_limits(k):
    D = np.diag((-1.0) ** np.arange(k))
    for j, tau in [(0, 10.0), (2, 1e3), (1, 1e7)]:
        ref0 = np.abs(mra.F_block(k, j, tau, 0)).max()
        for l in range(0, 8):
            Fp, Fm = mra.F_block(k, j, tau, l), mra.F_block(k, j, tau, -l)
            scale = ref0               # errors are measured against the term's largest block
            assert np.abs(Fm - Fp.T).max() <= 1e-13 * scale
            assert np.abs(Fm - D @ Fp @ D).max() <= 1e-13 * scale
    # wide Gaussian: F -> 2^{-j} e0 e0^T since int Phi_ab = delta_a0 delta_b0
    for j in (0, 3):
        F = mra.F_block(k, j, 1e-12, 2)
        ref = np.zeros((k, k)); ref[0, 0] = 2.0 ** -j
        assert np.abs(F - ref).max() < 1e-10
    # narrow Gaussian at l = 0: F -> 2^{-j} sqrt(pi 4^j / tau) I, up to O(4^j / tau)
    tau = 1e14
    for j in (0, 2):
        beta = tau / 4 ** j
        F = mra.F_block(k, j, tau, 0)
        assert np.abs(F * 2 ** j / np.sqrt(np.pi / beta) - np.eye(k)).max() < 1e-4


@pytest.mark.parametrize("k,tau", [(6, 40.0), (8, 3e3), (8, 1e6)])
def test_F_two_scale_consistency(k, tau):
    """T_{j-1} = P_{j-1} T_j P_{j-1}: F^{j-1;L} = sum_{s,s'} H^s F^{j;2L+s-s'} H^{s'}^T."""
    H = mra.two_scale_filters(k)
    for j in (1, 3):
        for L in (-2, 0, 1, 3):
            lhs = mra.F_block(k, j - 1, tau, L)
            rhs = sum(H[s] @ mra.F_block(k, j, tau, 2 * L + s - sp) @ H[sp].T for s in (0, 1) for sp in (0, 1))
            assert np.abs(lhs - rhs).max() < 1e-13 * max(1.0, np.abs(lhs).max())
