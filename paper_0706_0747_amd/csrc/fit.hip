// Gaussian-sum fit of the kernels of (-Delta + mu^2)^(-alpha) (host, FP64).
//
// K_{mu,alpha}(r) = C_alpha int exp(-r^2 e^{2s}) exp(-mu^2 e^{-2s}/4 + (3-2alpha) s) ds      (Sec. 3, eq. IntegralRepr)
// C_alpha = 2 * 2^{-2 alpha} pi^{-3/2} / Gamma(alpha); the trapezoidal rule with s_m = A + m h,
// m = 1..M, h = (B-A)/M gives tau_m = e^{2 s_m}, w_m = h C_alpha e^{-mu^2 e^{-2 s_m}/4 + (3-2alpha) s_m}
// (eq. KernelApproxByGaussians), accurate to eps K_{0,alpha}(r) on [delta, R].
// The paper takes A, B, h from a reference it does not reproduce; this library uses (nu = 3/2 - alpha):
//   h0 = pi^2 / (2 (ln(1/eps) + ln 8))          trapezoid error ~ e^{-pi^2/(2h)} (strip |Im s| < pi/4)
//   A  = ln(eps Gamma(nu+1)/4) / (2 nu) - ln R   the discarded lower tail is <= eps/4 of K_0 on [delta,R]
//   B  = ln(t_B / delta^2) / 2                    Gamma(nu, t_B)/Gamma(nu) <= eps/4 (upper tail)
// and h = h0 * 0.9^i, i = 0, 1, ..., until the relative error on 64 points per decade over
// [delta, R] is at most eps/2.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mwns_internal.h"

namespace {

double c_alpha(double alpha) { return 2.0 * std::pow(2.0, -2.0 * alpha) * std::pow(M_PI, -1.5) / std::tgamma(alpha); }

double upper_t(double nu, double eps) {
    if (nu <= 1.0) return std::max(1.0, std::log(4.0 / (eps * std::tgamma(nu))));
    double base = std::log(8.0 / (eps * std::tgamma(nu)));
    double t = base;
    for (int i = 0; i < 8; ++i) t = base + (nu - 1.0) * std::log(t);
    return std::max(t, 2.0 * (nu - 1.0));
}

}  // namespace

using namespace mwns;

extern "C" mwns_status mwns_fit_kernel(double mu, double alpha, double scale, double eps, double delta, double R,
                                       int cap, int* M, double* tau, double* w) {
    MWNS_GUARD_BEGIN
    if (!M) fail(MWNS_EINVAL, "M is NULL");
    if (!(alpha > 0.0 && alpha < 1.5) || !(mu >= 0.0) || !(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < R) ||
        !(scale > 0.0) || !std::isfinite(R) || !std::isfinite(mu))
        fail(MWNS_EINVAL, "fit parameters out of range");
    const double nu = 1.5 - alpha;
    const double h0 = M_PI * M_PI / (2.0 * (std::log(1.0 / eps) + std::log(8.0)));
    const double A = std::log(eps * std::tgamma(nu + 1.0) / 4.0) / (2.0 * nu) - std::log(R);
    const double B = 0.5 * std::log(upper_t(nu, eps) / (delta * delta));
    const double C = c_alpha(alpha);
    // check grid: 64 points per decade on [delta, R]
    const int ngrid = (int)std::ceil(64.0 * std::log10(R / delta));
    std::vector<double> r(ngrid + 1), ref(ngrid + 1), ref0(ngrid + 1);
    // the kernel at the check points, K(r) = c1 (mu/r)^nu K_nu(mu r), and its mu = 0 form
    // K0(r) = c0 / (2 r^{3-2 alpha}), with the constant factors formed once
    const double c0 = std::tgamma(1.5 - alpha) * c_alpha(alpha);
    const double c1 = std::pow(2.0, alpha - 1.5) * c_alpha(alpha);
    for (int i = 0; i <= ngrid; ++i) {
        r[i] = (i == ngrid) ? R : delta * std::pow(10.0, i / 64.0);
        ref0[i] = scale * (c0 / (2.0 * std::pow(r[i], 3.0 - 2.0 * alpha)));
        ref[i] = mu == 0.0 ? ref0[i] : scale * (c1 * std::pow(mu / r[i], nu) * std::cyl_bessel_k(nu, mu * r[i]));
    }
    std::vector<double> t, ww;
    for (int it = 0; it < 40; ++it) {
        int m = (int)std::ceil((B - A) / (h0 * std::pow(0.9, it)));
        double h = (B - A) / m;
        t.resize(m);
        ww.resize(m);
        for (int i = 0; i < m; ++i) {
            double s = A + h * (i + 1);
            t[i] = std::exp(2.0 * s);
            ww[i] = scale * h * C * std::exp(-mu * mu * std::exp(-2.0 * s) / 4.0 + (3.0 - 2.0 * alpha) * s);
        }
        double emax = 0.0;
        for (int g = 0; g <= ngrid; ++g) {
            // t grows with i; once t_i r^2 > 746, exp(-t_i r^2) is below half the smallest
            // subnormal and rounds to +0, so the remaining terms add nothing to the sum
            double acc = 0.0;
            for (int i = 0; i < m && t[i] * r[g] * r[g] <= 746.0; ++i) acc += ww[i] * std::exp(-t[i] * r[g] * r[g]);
            emax = std::max(emax, std::fabs(ref[g] - acc) / ref0[g]);
        }
        if (emax <= 0.5 * eps) {
            if (m > cap) {
                *M = m;
                set_error("fit needs " + std::to_string(m) + " terms, capacity is " + std::to_string(cap));
                return MWNS_ERANGE;
            }
            if (!tau || !w) fail(MWNS_EINVAL, "tau or w is NULL");
            std::copy(t.begin(), t.end(), tau);
            std::copy(ww.begin(), ww.end(), w);
            *M = m;
            return MWNS_OK;
        }
    }
    fail(MWNS_ERANGE, "Gaussian-sum fit did not reach the requested accuracy");
    MWNS_GUARD_END
}
