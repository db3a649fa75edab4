// Host-side runtime of libmwns: status plumbing, contexts, device allocation and the small 1-D
// tables (Gauss-Legendre rule, Legendre scaling functions, two-scale filters, cross-correlation
// expansions) that the kernels consume.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "mwns_internal.h"

namespace mwns {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

void fail(mwns_status st, const std::string& msg) { throw Failure{st, msg}; }

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(MWNS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device blocks are kept after they are freed and reused for later requests of the same size
// class (four classes per power of two, so at most 25% is wasted).  All of a context's work is
// ordered on its stream, so a block freed by earlier work is free for later work on that stream.
// Reuse spares the allocator (for the Python binding, a callback into torch) on every apply.
size_t size_class(size_t bytes) {
    if (bytes <= 256) return 256;
    int e = 63 - __builtin_clzll((unsigned long long)(bytes - 1));      // 2^e < bytes <= 2^(e+1)
    const size_t step = (size_t)1 << (e - 1);                          // quarter octave
    return (bytes + step - 1) / step * step;
}

void release_cache(mwns_ctx* ctx) {
    for (auto& c : ctx->cache) {
        if (ctx->free_fn) ctx->free_fn(c.second, ctx->user);
        else (void)hipFree(c.second);
        ctx->in_use -= c.first;
    }
    ctx->cache.clear();
    ctx->cached = 0;
}

void ctx_release(mwns_ctx* ctx) {
    if (--ctx->refs > 0) return;
    (void)hipStreamSynchronize(ctx->stream);
    release_cache(ctx);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

void* pinned_staging(mwns_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->pinned_bytes) return ctx->pinned;
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->pinned) {
        MWNS_HIP(hipHostFree(ctx->pinned));
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
    }
    size_t cap = (size_t)1 << 20;
    while (cap < bytes) cap <<= 1;
    void* p = nullptr;
    MWNS_HIP(hipHostMalloc(&p, cap, hipHostMallocDefault));
    ctx->pinned = p;
    ctx->pinned_bytes = cap;
    return p;
}

void* dalloc(mwns_ctx* ctx, size_t bytes) {
    if (bytes == 0) return nullptr;
    const size_t cls = size_class(bytes);
    for (size_t i = ctx->cache.size(); i-- > 0;)
        if (ctx->cache[i].first == cls) {
            void* p = ctx->cache[i].second;
            ctx->cache.erase(ctx->cache.begin() + (std::ptrdiff_t)i);
            ctx->cached -= cls;
            return p;
        }
    if (ctx->budget && ctx->in_use + cls > ctx->budget) release_cache(ctx);
    if (ctx->budget && ctx->in_use + cls > ctx->budget)
        fail(MWNS_ENOMEM, "context byte budget exceeded (" + std::to_string(ctx->in_use + cls) + " > " +
                              std::to_string(ctx->budget) + ")");
    void* p = nullptr;
    if (ctx->alloc) {
        p = ctx->alloc(cls, ctx->user);
        if (!p) {
            release_cache(ctx);
            p = ctx->alloc(cls, ctx->user);
        }
        if (!p) fail(MWNS_ENOMEM, "device allocator returned NULL for " + std::to_string(cls) + " bytes");
    } else {
        hipError_t e = hipMalloc(&p, cls);
        if (e != hipSuccess || !p) {
            release_cache(ctx);
            e = hipMalloc(&p, cls);
        }
        if (e != hipSuccess || !p) fail(MWNS_ENOMEM, "hipMalloc of " + std::to_string(cls) + " bytes failed");
    }
    ctx->in_use += cls;
    return p;
}

void dfree(mwns_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    const size_t cls = size_class(bytes);
    ctx->cache.push_back({cls, p});
    ctx->cached += cls;
}

// n-point Gauss-Legendre rule on [0,1]: nodes are the roots of P_n(2x-1) (App. A.1), found by
// Newton's method on P_n from the Chebyshev-like initial guesses; weights 1/((1-t^2) P_n'(t)^2).
Quad gauss_legendre01(int n) {
    Quad q;
    q.x.resize(n);
    q.w.resize(n);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2 * m - 1) * t * p1 - (m - 1) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        {   // final derivative at the converged root
            double p0 = 1.0, p1 = t;
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2 * m - 1) * t * p1 - (m - 1) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
        }
        double wt = 2.0 / ((1.0 - t * t) * dp * dp);
        // t is the i-th largest root; map to [0,1] in ascending order
        q.x[n - 1 - i] = 0.5 * (1.0 + t);
        q.x[i] = 0.5 * (1.0 - t);
        q.w[n - 1 - i] = 0.5 * wt;
        q.w[i] = 0.5 * wt;
    }
    return q;
}

// phi_a(x) = sqrt(2a+1) P_a(2x-1) (App. A.1, eq. scalingFNC), evaluated without the support cut.
void legendre_phi(int k, double x, double* out) {
    double t = 2.0 * x - 1.0, p0 = 1.0, p1 = t;
    out[0] = 1.0;
    if (k > 1) out[1] = t;
    for (int a = 2; a < k; ++a) {
        double p2 = ((2 * a - 1) * t * p1 - (a - 1) * p0) / a;
        out[a] = p2;
        p0 = p1;
        p1 = p2;
    }
    for (int a = 0; a < k; ++a) out[a] *= std::sqrt(2.0 * a + 1.0);
}

// h^(s)_ab = 2^{-1/2} int_0^1 phi_a((u+s)/2) phi_b(u) du: the coefficients of the two-scale relation
// phi_a(x) = sqrt2 sum_b (h0_ab phi_b(2x) + h1_ab phi_b(2x-1)) (App. A.3); exact with k points.
void two_scale_filters(int k, double* H0, double* H1) {
    Quad q = gauss_legendre01(k);
    double pa[64], pb[64];
    double* H[2] = {H0, H1};
    for (int s = 0; s < 2; ++s) {
        std::fill(H[s], H[s] + k * k, 0.0);
        for (int i = 0; i < k; ++i) {
            legendre_phi(k, 0.5 * (q.x[i] + s), pa);
            legendre_phi(k, q.x[i], pb);
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) H[s][a * k + b] += q.w[i] * pa[a] * pb[b];
        }
        for (int i = 0; i < k * k; ++i) H[s][i] *= M_SQRT1_2;
    }
}

// G^(0), G^(1): the wavelets' two-scale coefficients (App. A.2-A.3).  The paper defines them only
// through a reference it does not reproduce; any orthonormal basis of the complement of V_0 in V_1
// serves here, since only the norm of the detail coefficients is used.  The k columns of [H0 H1]^T
// are orthonormal in R^{2k}; Householder reflections that triangularise them give an orthogonal
// Q = P_0 ... P_{k-1} whose last k columns span their orthogonal complement: G = those columns^T.
void wavelet_filters(int k, double* G0, double* G1) {
    const int n = 2 * k;
    std::vector<double> H(2 * k * k), A(n * k), Q(n * n, 0.0), v(n);
    two_scale_filters(k, H.data(), H.data() + k * k);
    for (int c = 0; c < k; ++c)
        for (int b = 0; b < k; ++b) {
            A[b * k + c] = H[c * k + b];                 // rows 0..k-1: H0^T
            A[(k + b) * k + c] = H[k * k + c * k + b];   // rows k..2k-1: H1^T
        }
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    for (int c = 0; c < k; ++c) {
        double norm = 0.0;
        for (int i = c; i < n; ++i) norm += A[i * k + c] * A[i * k + c];
        norm = std::sqrt(norm);
        const double alpha = A[c * k + c] > 0.0 ? -norm : norm;
        std::fill(v.begin(), v.end(), 0.0);
        for (int i = c; i < n; ++i) v[i] = A[i * k + c];
        v[c] -= alpha;
        double vv = 0.0;
        for (int i = c; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        // A <- (I - 2 v v^T / v^T v) A ; Q <- Q (I - 2 v v^T / v^T v)
        for (int cc = c; cc < k; ++cc) {
            double d = 0.0;
            for (int i = c; i < n; ++i) d += v[i] * A[i * k + cc];
            d *= 2.0 / vv;
            for (int i = c; i < n; ++i) A[i * k + cc] -= d * v[i];
        }
        for (int r = 0; r < n; ++r) {
            double d = 0.0;
            for (int i = c; i < n; ++i) d += Q[r * n + i] * v[i];
            d *= 2.0 / vv;
            for (int i = c; i < n; ++i) Q[r * n + i] -= d * v[i];
        }
    }
    for (int r = 0; r < k; ++r)
        for (int b = 0; b < k; ++b) {
            G0[r * k + b] = Q[b * n + k + r];
            G1[r * k + b] = Q[(k + b) * n + k + r];
        }
}

// Phi^+_ab(x) = int_0^{1-x} phi_a(x+y) phi_b(y) dy on [0,1] is a polynomial of degree <= 2k-1
// (App. A.4), so Phi^+_ab = sum_{n<2k} C[a][b][n] phi_n with C from a 2k-point rule; the inner
// integral uses the k-point rule on [0, 1-x] (exact, degree a+b <= 2k-2).
void crosscorr_plus_coeffs(int k, double* C) {
    const int K2 = 2 * k;
    Quad outer = gauss_legendre01(K2);
    Quad inner = gauss_legendre01(k);
    std::fill(C, C + k * k * K2, 0.0);
    std::vector<double> phiv(K2), pa(k), pb(k), Phi(k * k);
    for (int q = 0; q < K2; ++q) {
        double x = outer.x[q], len = 1.0 - x;
        std::fill(Phi.begin(), Phi.end(), 0.0);
        for (int i = 0; i < k; ++i) {
            double y = len * inner.x[i];
            legendre_phi(k, x + y, pa.data());
            legendre_phi(k, y, pb.data());
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) Phi[a * k + b] += len * inner.w[i] * pa[a] * pb[b];
        }
        legendre_phi(K2, x, phiv.data());
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                for (int n = 0; n <= std::min(a + b + 1, K2 - 1); ++n) C[(a * k + b) * K2 + n] += outer.w[q] * Phi[a * k + b] * phiv[n];
    }
    // Phi^+_ab is a polynomial of degree a + b + 1 (App. A.4): its coefficients of higher degree
    // are exactly zero (never accumulated above), so the large high-degree Gaussian moments of
    // narrow terms meet no quadrature noise.
}

DevArray<double> upload_filters(mwns_ctx* ctx, int k) {
    std::vector<double> H(2 * k * k);
    two_scale_filters(k, H.data(), H.data() + k * k);
    DevArray<double> d(ctx, H.size());
    d.upload(H.data(), H.size(), ctx->stream);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    return d;
}

}  // namespace mwns

using namespace mwns;

extern "C" {

const char* mwns_last_error(void) { return g_last_error.c_str(); }
int mwns_abi_version(void) { return MWNS_ABI_VERSION; }

mwns_status mwns_ctx_create(int device, void* stream, mwns_alloc_fn alloc, mwns_free_fn free_fn, void* user,
                            size_t byte_budget, mwns_ctx** out) {
    MWNS_GUARD_BEGIN
    if (!out) fail(MWNS_EINVAL, "out is NULL");
    if ((alloc == nullptr) != (free_fn == nullptr)) fail(MWNS_EINVAL, "alloc and free must be given together");
    int n = 0;
    MWNS_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) fail(MWNS_EINVAL, "device " + std::to_string(device) + " not present");
    MWNS_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    MWNS_HIP(hipGetDeviceProperties(&prop, device));
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
        fail(MWNS_EDEVICE, std::string("libmwns is built for gfx950, device is ") + prop.gcnArchName);
    noalloc_scratch_init(device);
    auto* c = new mwns_ctx;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    c->budget = byte_budget;
    *out = c;
    return MWNS_OK;
    MWNS_GUARD_END
}

void mwns_ctx_destroy(mwns_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    release_cache(ctx);
    mwns::ctx_release(ctx);     // trees, operators and plans of the context may still hold it
}

mwns_status mwns_ctx_release_cache(mwns_ctx* ctx) {
    MWNS_GUARD_BEGIN
    if (!ctx) fail(MWNS_EINVAL, "ctx is NULL");
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    release_cache(ctx);
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_ctx_synchronize(mwns_ctx* ctx) {
    MWNS_GUARD_BEGIN
    if (!ctx) fail(MWNS_EINVAL, "ctx is NULL");
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    return MWNS_OK;
    MWNS_GUARD_END
}

size_t mwns_ctx_bytes_in_use(const mwns_ctx* ctx) { return ctx ? ctx->in_use - ctx->cached : 0; }
size_t mwns_ctx_bytes_cached(const mwns_ctx* ctx) { return ctx ? ctx->cached : 0; }

}  // extern "C"
