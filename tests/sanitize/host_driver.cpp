// Host-side code of libmwns run under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only,
// no device call): the Gaussian-sum fit through its C entry point, including its error paths, and
// the 1-D tables (Gauss-Legendre rule, scaling functions, two-scale filters, cross-correlation
// coefficients) for every basis order.  Exit status 0 when every call behaved as documented.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_0706_0747_amd/csrc/mwns_internal.h"

// Context creation (host_common) looks up the allocation-free evaluation's array, which lives
// with the tree kernels; this driver creates no context, so the lookup is never reached.
void mwns::noalloc_scratch_init(int) {}

int main() {
    int bad = 0;
    std::vector<double> tau(2000), w(2000);
    struct Case { double mu, alpha, eps, delta; };
    const Case cases[] = {{0, 1, 1e-4, 1e-3}, {4, 1, 1e-8, 1e-5}, {0, 0.7, 1e-6, 1e-4}, {0, 1, 1e-10, 1e-7}, {0.5, 1.3, 1e-6, 1e-4}};
    for (const Case& c : cases) {
        int M = 0;
        const mwns_status s = mwns_fit_kernel(c.mu, c.alpha, 1.0, c.eps, c.delta, 1.8, 2000, &M, tau.data(), w.data());
        if (s != MWNS_OK || M < 1) { std::printf("fit failed: %d %s\n", (int)s, mwns_last_error()); bad = 1; }
        for (int m = 0; m < M; ++m)
            if (!(tau[m] > 0.0) || !std::isfinite(w[m])) bad = 1;
    }
    int M = 0;
    if (mwns_fit_kernel(0, 1, 1.0, 1e-10, 1e-7, 1.8, 3, &M, tau.data(), w.data()) != MWNS_ERANGE || M <= 3) bad = 1;
    if (mwns_fit_kernel(0, 2, 1.0, 1e-6, 1e-3, 1.8, 2000, &M, tau.data(), w.data()) != MWNS_EINVAL) bad = 1;
    if (mwns_fit_kernel(0, 1, 1.0, 1e-6, 2.0, 1.0, 2000, &M, tau.data(), w.data()) != MWNS_EINVAL) bad = 1;
    if (mwns_fit_kernel(0, 1, 1.0, 1e-6, 1e-3, 1.8, 2000, nullptr, tau.data(), w.data()) != MWNS_EINVAL) bad = 1;
    for (int k = 1; k <= mwns::KMAX; ++k) {
        const mwns::Quad q = mwns::gauss_legendre01(k);
        double sw = 0.0;
        for (double x : q.w) sw += x;
        if (std::fabs(sw - 1.0) > 1e-14) bad = 1;
        std::vector<double> phi(k), H0(k * k), H1(k * k), C((size_t)k * k * 2 * k);
        for (double x : q.x) mwns::legendre_phi(k, x, phi.data());
        mwns::two_scale_filters(k, H0.data(), H1.data());
        double orth = 0.0;     // H0 H0^T + H1 H1^T = I
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                double s = 0.0;
                for (int c = 0; c < k; ++c) s += H0[a * k + c] * H0[b * k + c] + H1[a * k + c] * H1[b * k + c];
                orth = std::fmax(orth, std::fabs(s - (a == b ? 1.0 : 0.0)));
            }
        if (orth > 1e-13) bad = 1;
        mwns::crosscorr_plus_coeffs(k, C.data());
        for (double x : C)
            if (!std::isfinite(x)) bad = 1;
    }
    std::printf("host driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
