"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds only the input recipes (source Gaussians, kernel parameters, accuracy,
basis order, tree limits, sample points).  It contains none of the method's arithmetic, so
both the HIP library's callers and the CPU oracle may use it.

Random draws use numpy.random.Generator(PCG64(seed)) in the order listed for each recipe.
Sources are sums of unit-mass Gaussians c_i (a_i/pi)^{3/2} exp(-a_i |x - x_i|^2).
Kernels are (-Delta + mu^2)^(-alpha): Poisson (mu=0, alpha=1, 1/(4 pi r)), Yukawa / bound-state
Helmholtz (alpha=1, e^{-mu r}/(4 pi r)) and fractional (mu=0).
"""
import json
import os

import numpy as np

__all__ = ["Workload", "c1", "c2", "c3", "c4_draw", "c4_member", "c5", "cot1d_example", "cot1d_many", "ns2d", "small_adaptive", "points"]


class Workload(dict):
    """Recipe: k, eps, j0, jmax, mu, alpha, xyz (n,3), a (n,), c (n,), name, seed."""

    def __getattr__(self, name):
        try:
            return self[name]
        except KeyError:
            raise AttributeError(name)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def c1():
    """3-D Poisson, k=6, uniform level 3 (512 leaves), eps=1e-4; one unit-mass Gaussian with
    exponent 100 at the centre of the cube (no randomness)."""
    return Workload(name="poisson_k6_uniform_n3", seed=None, k=6, eps=1e-4, j0=3, jmax=3, mu=0.0, alpha=1.0,
                    xyz=np.array([[0.5, 0.5, 0.5]]), a=np.array([100.0]), c=np.array([1.0]))


def _gauss_sum(rng, n, log10_lo, log10_hi):
    a = 10.0 ** rng.uniform(log10_lo, log10_hi, n)      # exponents, log-uniform
    xyz = rng.uniform(0.2, 0.8, (n, 3))                 # centres in [0.2, 0.8]^3
    c = rng.normal(0.0, 1.0, n)                         # weights N(0,1)
    return xyz, a, c


def c2(seed=2, n=50):
    """3-D Poisson, k=8, eps=1e-6, adaptive from j0=2 up to jmax=12; 50 Gaussians with
    exponents log-uniform in [10, 1e4], centres uniform in [0.2, 0.8]^3, weights N(0,1)."""
    rng = _rng(seed)
    xyz, a, c = _gauss_sum(rng, n, 1.0, 4.0)
    return Workload(name="poisson_k8_eps1e-6_50gauss", seed=seed, k=8, eps=1e-6, j0=2, jmax=12, mu=0.0,
                    alpha=1.0, xyz=xyz, a=a, c=c)


def c3(seed=3, n=20):
    """Bound-state Helmholtz e^{-mu r}/(4 pi r), mu ~ U[1,10] (drawn first), k=10, eps=1e-8,
    20 Gaussians with the ranges of c2."""
    rng = _rng(seed)
    mu = rng.uniform(1.0, 10.0)
    xyz, a, c = _gauss_sum(rng, n, 1.0, 4.0)
    return Workload(name="yukawa_k10_eps1e-8_20gauss", seed=seed, k=10, eps=1e-8, j0=2, jmax=12, mu=float(mu),
                    alpha=1.0, xyz=xyz, a=a, c=c)


C4_POOL = 1024                 # Gaussians drawn per batch member; a member uses a prefix of them
C4_LEAVES = (1e3, 2e5)         # range of the members' leaf counts (log-uniform targets)
C4_SIZES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_sizes.json")


def c4_draw(i):
    """The random part of batch member i (0..63), in draw order: kernel uniform over {Poisson,
    Yukawa mu~U[0.5,10], fractional alpha~U(0.2,1.4)}; (k, eps) uniform over (6,1e-4), (8,1e-6),
    (10,1e-8); a target leaf count log-uniform in C4_LEAVES; the exponents' upper limit 10^u with u
    rising linearly from 2 to 5 over the log of that range (more leaves need narrower Gaussians);
    a pool of C4_POOL Gaussians (exponents log-uniform in [10, 10^u], centres in [0.2, 0.8]^3,
    weights N(0,1))."""
    rng = _rng(1000 + i)
    kind = int(rng.integers(0, 3))
    mu, alpha = 0.0, 1.0
    if kind == 1:
        mu = float(rng.uniform(0.5, 10.0))
    elif kind == 2:
        alpha = float(rng.uniform(0.2, 1.4))
    k, eps = [(6, 1e-4), (8, 1e-6), (10, 1e-8)][int(rng.integers(0, 3))]
    lo, hi = np.log10(C4_LEAVES[0]), np.log10(C4_LEAVES[1])
    target = float(10.0 ** rng.uniform(lo, hi))
    u = 2.0 + 3.0 * (np.log10(target) - lo) / (hi - lo)
    xyz, a, c = _gauss_sum(rng, C4_POOL, 1.0, u)
    return Workload(seed=1000 + i, k=k, eps=eps, j0=2, jmax=12, mu=mu, alpha=alpha, target=target, u=u,
                    xyz=xyz, a=a, c=c)


def c4_member(i, n=None):
    """Member i of the batch of uneven solves: the first n Gaussians of c4_draw(i)'s pool, n as
    calibrated per member (stored in c4_sizes.json by calibrate_c4.py, beside this file) so that
    the members' leaf counts spread log-uniformly over C4_LEAVES."""
    d = c4_draw(i)
    if n is None:
        with open(C4_SIZES) as fh:
            n = int(json.load(fh)["members"][str(i)]["n"])
    return Workload(name="batch_member_%d" % i, seed=d.seed, k=d.k, eps=d.eps, j0=d.j0, jmax=d.jmax, mu=d.mu,
                    alpha=d.alpha, xyz=d.xyz[:n], a=d.a[:n], c=d.c[:n])


def c5(seed=5, n=500):
    """3-D Poisson, k=10, eps=1e-10; 500 Gaussians, exponents log-uniform in [10, 1e5],
    centres uniform in [0.2, 0.8]^3, weights N(0,1)."""
    rng = _rng(seed)
    xyz, a, c = _gauss_sum(rng, n, 1.0, 5.0)
    return Workload(name="poisson_k10_eps1e-10_500gauss", seed=seed, k=10, eps=1e-10, j0=2, jmax=14, mu=0.0,
                    alpha=1.0, xyz=xyz, a=a, c=c)


def cot1d_example(k, eps):
    """The 1-D cotangent example (Sec. 2.4.2): f(x) = sum_n exp(-300 (x + n - 1/2)^2) on the periodic
    unit interval, order k, accuracy eps (also the absolute refinement threshold), from level 2."""
    return Workload(name="cot1d_gauss300_k%d" % k, seed=None, k=k, eps=eps, thr=eps, j0=2, jmax=30,
                    centers=np.array([0.5]), exps=np.array([300.0]), weights=np.array([1.0]))


def cot1d_many(seed=11, n=128):
    """A larger 1-D input for the cotangent operator: n periodized Gaussians with exponents
    log-uniform in [1e2, 1e7], centres uniform in [0,1), weights N(0,1); k = 10, eps = 1e-9."""
    rng = _rng(seed)
    exps = 10.0 ** rng.uniform(2.0, 7.0, n)
    centers = rng.uniform(0.0, 1.0, n)
    weights = rng.normal(0.0, 1.0, n)
    return Workload(name="cot1d_%dgauss_k10" % n, seed=seed, k=10, eps=1e-9, thr=1e-9, j0=2, jmax=30,
                    centers=centers, exps=exps, weights=weights)


def ns2d(seed=2, n=50, log10_hi=4.0, k=8, eps=1e-6, mu=5.0):
    """A 2-D input for Alg. 3 in the plane: n unit-mass Gaussians (a/pi) exp(-a |p - p_i|^2) with
    exponents log-uniform in [10, 10^log10_hi], centres uniform in [0.2, 0.8]^2, weights N(0,1); the
    plane's bound-state Helmholtz kernel K_0(mu r) / (2 pi); order k, accuracy eps, j0 = 2, jmax = 12."""
    rng = _rng(seed)
    a = 10.0 ** rng.uniform(1.0, log10_hi, n)
    xy = rng.uniform(0.2, 0.8, (n, 2))
    c = rng.normal(0.0, 1.0, n)
    return Workload(name="ns2d_yukawa_k%d_%dgauss" % (k, n), seed=seed, k=k, eps=eps, j0=2, jmax=12, mu=mu, alpha=1.0,
                    xy=xy, a=a, c=c)


def small_adaptive(seed, k=6, eps=1e-4, n=3, jmax=6, mu=0.0, alpha=1.0):
    """A few Gaussians (exponents log-uniform in [10, 10^2.5], centres in [0.3, 0.7]^3, weights
    N(0,1)) giving small adaptive trees for fast parity cases."""
    rng = _rng(seed)
    a = 10.0 ** rng.uniform(1.0, 2.5, n)
    xyz = rng.uniform(0.3, 0.7, (n, 3))
    c = rng.normal(0.0, 1.0, n)
    return Workload(name="small_adaptive_%d" % seed, seed=seed, k=k, eps=eps, j0=1, jmax=jmax, mu=mu,
                    alpha=alpha, xyz=xyz, a=a, c=c)


def points(n=10000, seed=6):
    """n evaluation points uniform in [0,1]^3."""
    return _rng(seed).uniform(0.0, 1.0, (n, 3))
