// The 1-D modified ns-form of the periodic cotangent operator (Sec. 2.4, Alg. 2; the numerical
// example of Sec. 2.4.2):  (C f)(y) = p.v. int_0^1 cot(pi (y - x)) f(x) dx on the periodic unit
// interval, f given as a sum of periodized Gaussians.
//
//   * operator: blocks r^{j;l}_ab = 2^-j p.v. int_{-1}^{1} cot(pi 2^-j (x + l)) Phi_ab(x) dx
//     (eq. cot.01) for l = -LR1..LR1 at every scale, by a 64-point Gauss-Legendre rule over the two
//     polynomial pieces of Phi (App. A.4), whose combined integrand is regular at the poles of the
//     cotangent on [0,1]; bands B_j from the Frobenius norms of the difference super-blocks
//     S^{j;L} - [H0 H1]^T r^{j-1;L} [H0 H1] (Sec. 2.3-2.4).
//   * projection: Alg. 1 in one dimension with an absolute threshold; compression to the
//     redundant tree (eq. decomp_scaling).
//   * apply: the output tree is the redundant tree of f with every leaf refined whose whole band
//     holds an internal node of f of its scale (and so on for the added children); input blocks from the tree or from the nearest ancestor by
//     zero-detail reconstruction (Alg. 2 Step 2); the banded contraction of eq. apply_algo (leaf:
//     coarse distance <= B_j; internal: minus fine distance <= B_{j+1}); assembly (eq. g_assemble).
//   * evaluation at points (App. A.1).
// Keys: level << 57 | translation; nodes sorted by key, i.e. by (level, translation).
#include <algorithm>
#include <cmath>
#include <memory>
#include <unordered_map>

#include "mwns_internal.h"

namespace mwns {
namespace {

constexpr int K1MAX = 16;               // largest basis order of the 1-D path
constexpr int DMAX1 = 32;               // largest coarse distance entering the band choice
constexpr int LR1 = 2 * DMAX1 + 1;      // blocks are tabulated for l = -LR1..LR1
constexpr int NLR1 = 2 * LR1 + 1;
constexpr int NGL1 = 64;                // quadrature points of the blocks
constexpr int MAXLEV1 = 40;

inline uint64_t key1(int j, int64_t l) { return ((uint64_t)j << 57) | (uint64_t)l; }
inline int key1_level(uint64_t key) { return (int)(key >> 57); }
inline int64_t key1_trans(uint64_t key) { return (int64_t)(key & ((1ull << 57) - 1)); }
inline int64_t pdist(int64_t l, int64_t n) {
    int64_t m = ((l % n) + n) % n;
    return std::min(m, n - m);
}

__device__ inline void phi_dev(int k, double x, double* out) {
    const double t = 2.0 * x - 1.0;
    double p0 = 1.0, p1 = t;
    out[0] = 1.0;
    if (k > 1) out[1] = t;
    for (int a = 2; a < k; ++a) {
        const double p2 = ((2 * a - 1) * t * p1 - (a - 1) * p0) / a;
        out[a] = p2;
        p0 = p1;
        p1 = p2;
    }
    for (int a = 0; a < k; ++a) out[a] *= sqrt(2.0 * a + 1.0);
}

// One thread per entry (j, l, a, b): r = 2^-j sum_q w_q [cot(pi 2^-j (l + t_q)) Phi^+_ab(t_q) +
// cot(pi 2^-j (l - t_q)) Phi^-_ab(-t_q)], with Phi^-_ab(-t) = Phi^+_ba(t).
__global__ void cot_blocks_kernel(int k, int nlev, const double* __restrict__ tq, const double* __restrict__ wq,
                                  const double* __restrict__ php, double* __restrict__ R) {
    const int64_t n = (int64_t)nlev * NLR1 * k * k;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = (int)(i % k), a = (int)((i / k) % k);
    const int li = (int)((i / (k * k)) % NLR1), j = (int)(i / ((int64_t)k * k * NLR1));
    const double s = ldexp(1.0, -j), l = (double)(li - LR1);
    double acc = 0.0;
    for (int q = 0; q < NGL1; ++q) {
        const double t = tq[q];
        const double cp = 1.0 / tan(M_PI * s * (l + t)), cm = 1.0 / tan(M_PI * s * (l - t));
        acc += wq[q] * (cp * php[(q * k + a) * k + b] + cm * php[(q * k + b) * k + a]);
    }
    R[i] = s * acc;
}

// One workgroup per (j, L): || S^{j;L} - Hc^T r^{j-1;L} Hc ||_F^2 with Hc = [H0 H1] (k x 2k);
// S's block (so, si) is r^{j; 2L + so - si} (rows: output child so).
__global__ void diffnorm_kernel(int k, const int2* __restrict__ jl, const double* __restrict__ R,
                                const double* __restrict__ H, double* __restrict__ out) {
    __shared__ double red[256];
    const int j = jl[blockIdx.x].x, L = jl[blockIdx.x].y;
    const int n2 = 2 * k;
    const double* Rc = R + ((int64_t)(j - 1) * NLR1 + (L + LR1)) * k * k;
    double s2 = 0.0;
    for (int e = threadIdx.x; e < n2 * n2; e += blockDim.x) {
        const int u = e / n2, v = e % n2;
        const int so = u / k, a = u % k, si = v / k, b = v % k;
        const double S = R[((int64_t)j * NLR1 + (2 * L + so - si + LR1)) * k * k + a * k + b];
        double U = 0.0;
        for (int c = 0; c < k; ++c) {
            double t = 0.0;
            for (int d = 0; d < k; ++d) t += Rc[c * k + d] * H[(si * k + d) * k + b];
            U += H[(so * k + c) * k + a] * t;
        }
        const double dlt = S - U;
        s2 += dlt * dlt;
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// f(x) = sum_i w_i sum_n exp(-a_i (x + n - c_i)^2), images |n| <= ceil(sqrt(45/a_i)) + 1
__device__ double pgauss(double x, int ng, const double* __restrict__ gc, const double* __restrict__ ga,
                         const double* __restrict__ gw) {
    double f = 0.0;
    for (int i = 0; i < ng; ++i) {
        const int nimg = (int)ceil(sqrt(45.0 / ga[i])) + 1;
        for (int n = -nimg; n <= nimg; ++n) {
            const double d = x + n - gc[i];
            f += gw[i] * exp(-ga[i] * d * d);
        }
    }
    return f;
}

// One workgroup of 64 threads per candidate box (level j, translation l): its coefficients
// s_a = 2^{-j/2} sum_q w_q f(x_q) phi_a(x_q) (eq. fvals2coefs) and the largest difference between f
// and the box's polynomial at both children's nodes (Alg. 1).
__global__ void project1_kernel(int k, int j, const int64_t* __restrict__ cand, int ng, const double* __restrict__ gc,
                                const double* __restrict__ ga, const double* __restrict__ gw,
                                const double* __restrict__ xq, const double* __restrict__ wq,
                                const double* __restrict__ phiq, const double* __restrict__ phich,
                                double* __restrict__ coef, double* __restrict__ err) {
    __shared__ double fv[3 * K1MAX], s[K1MAX], dv[2 * K1MAX];
    const int64_t l = cand[blockIdx.x];
    const int t = threadIdx.x;
    const double h = ldexp(1.0, -j);
    if (t < 3 * k) {
        double x;
        if (t < k) x = h * ((double)l + xq[t]);
        else {
            const int c = (t - k) / k, q = (t - k) % k;
            x = 0.5 * h * ((double)(2 * l + c) + xq[q]);
        }
        fv[t] = pgauss(x, ng, gc, ga, gw);
    }
    __syncthreads();
    if (t < k) {
        double acc = 0.0;
        for (int q = 0; q < k; ++q) acc += wq[q] * fv[q] * phiq[q * k + t];
        s[t] = sqrt(h) * acc;
        coef[blockIdx.x * k + t] = s[t];
    }
    __syncthreads();
    if (t < 2 * k) {
        const int c = t / k, q = t % k;
        double v = 0.0;
        for (int a = 0; a < k; ++a) v += s[a] * phich[(c * k + q) * k + a];
        dv[t] = fabs(v / sqrt(h) - fv[k + t]);
    }
    __syncthreads();
    if (t == 0) {
        double m = 0.0;
        for (int i = 0; i < 2 * k; ++i) m = fmax(m, dv[i]);
        err[blockIdx.x] = m;
    }
}

// parent = H0 child0 + H1 child1 (eq. decomp_scaling), one thread per (parent, a)
__global__ void compress1_kernel(int k, int n, const int64_t* __restrict__ par, const int64_t* __restrict__ ch0,
                                 const double* __restrict__ H, double* __restrict__ coef) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int p = i / k, a = i % k;
    const double* c0 = coef + ch0[p] * k;
    const double* c1 = c0 + k;
    double acc = 0.0;
    for (int b = 0; b < k; ++b) acc += H[a * k + b] * c0[b] + H[k * k + a * k + b] * c1[b];
    coef[par[p] * k + a] = acc;
}

// Input blocks: x = H^(s_1)^T ... H^(s_up)^T f[anc], the path bits read from the translation from
// the top (Alg. 2 Step 2); up = 0 copies the node.  One thread per block.
__global__ void gather1_kernel(int k, int n, const int64_t* __restrict__ anc, const int* __restrict__ up,
                               const int64_t* __restrict__ trans, const double* __restrict__ H,
                               const double* __restrict__ f, double* __restrict__ X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s[K1MAX], t[K1MAX];
    for (int a = 0; a < k; ++a) s[a] = f[anc[i] * k + a];
    for (int step = up[i]; step > 0; --step) {
        const int sig = (int)((trans[i] >> (step - 1)) & 1);
        const double* Hs = H + sig * k * k;
        for (int b = 0; b < k; ++b) {
            double acc = 0.0;
            for (int a = 0; a < k; ++a) acc += Hs[a * k + b] * s[a];
            t[b] = acc;
        }
        for (int b = 0; b < k; ++b) s[b] = t[b];
    }
    for (int a = 0; a < k; ++a) X[(int64_t)i * k + a] = s[a];
}

// ghat[node][a] = sum over the node's jobs of c * sum_b R[j][l][a][b] X[in][b]; one thread per
// (node, a), jobs in CSR order (fixed summation order).
__global__ void contract1_kernel(int k, int n, const int* __restrict__ nlev, const int64_t* __restrict__ off,
                                 const int64_t* __restrict__ jin, const int* __restrict__ jli, const int* __restrict__ jc,
                                 const double* __restrict__ R, const double* __restrict__ X, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int node = i / k, a = i % k;
    const int j = nlev[node];
    double acc = 0.0;
    for (int64_t e = off[node]; e < off[node + 1]; ++e) {
        const double* r = R + ((int64_t)j * NLR1 + jli[e]) * k * k + a * k;
        const double* x = X + jin[e] * k;
        double v = 0.0;
        for (int b = 0; b < k; ++b) v += r[b] * x[b];
        acc += jc[e] * v;
    }
    out[(int64_t)node * k + a] = acc;
}

// g[i] = ghat[i] + H^(s)^T g[parent] for the nodes of one level (eq. g_assemble)
__global__ void assemble1_kernel(int k, int n, const int64_t* __restrict__ node, const int64_t* __restrict__ par,
                                 const int* __restrict__ sig, const double* __restrict__ H, double* __restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int p = i / k, b = i % k;
    const double* Hs = H + sig[p] * k * k;
    const double* gp = g + par[p] * k;
    double acc = 0.0;
    for (int a = 0; a < k; ++a) acc += Hs[a * k + b] * gp[a];
    g[node[p] * k + b] += acc;
}

// value at x: the leaf containing x (walk down from the root), then 2^{j/2} sum_a g_a phi_a(2^j x - l)
__global__ void eval1_kernel(int k, int64_t nn, const uint64_t* __restrict__ keys, const uint8_t* __restrict__ leaf,
                             const double* __restrict__ g, int64_t np, const double* __restrict__ x,
                             double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const double xv = x[i];
    double ph[K1MAX];
    for (int j = 0; j < MAXLEV1; ++j) {
        const int64_t n = (int64_t)1 << j;
        int64_t l = (int64_t)floor(xv * (double)n);
        l = l < 0 ? 0 : (l > n - 1 ? n - 1 : l);
        const int64_t p = find_sorted(keys, nn, ((uint64_t)j << 57) | (uint64_t)l);
        if (p < 0) break;
        if (leaf[p]) {
            phi_dev(k, xv * (double)n - (double)l, ph);
            double v = 0.0;
            for (int a = 0; a < k; ++a) v += g[p * k + a] * ph[a];
            out[i] = sqrt((double)n) * v;
            return;
        }
    }
    out[i] = NAN;
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace mwns

using namespace mwns;

struct mwns_op1 {
    CtxHold hold;
    mwns_ctx* ctx = nullptr;
    int k = 0, max_level = 0;
    double eps = 0.0;
    std::vector<int32_t> band;     // [max_level + 2]: B_j (j >= 1), band[max_level + 1] = 0
    DevArray<double> R;            // [max_level + 1][NLR1][k][k], l = -LR1..LR1
    DevArray<double> H;            // [2][k][k]
};

struct mwns_tree1 {
    CtxHold hold;
    mwns_ctx* ctx = nullptr;
    int k = 0, depth = 0;
    int64_t nleaves = 0;
    std::vector<uint64_t> keys;    // sorted
    std::vector<uint8_t> leaf;
    DevArray<uint64_t> dkeys;
    DevArray<uint8_t> dleaf;
    DevArray<double> coef;         // [nodes][k]
};

namespace {

void check_ctx1(mwns_ctx* ctx) {
    if (!ctx) fail(MWNS_EINVAL, "NULL context");
    MWNS_HIP(hipSetDevice(ctx->device));
}

std::vector<double> upload_h(mwns_ctx* ctx, int k, DevArray<double>& dH) {
    std::vector<double> H(2 * k * k);
    two_scale_filters(k, H.data(), H.data() + k * k);
    dH.reset(ctx, H.size());
    dH.upload(H.data(), H.size(), ctx->stream);
    return H;
}

// tree from sorted keys, leaf flags and the leaves' coefficients on the device (internal nodes
// compressed); checks that the leaves tile [0,1) and siblings come in pairs
std::unique_ptr<mwns_tree1> build_tree1(mwns_ctx* ctx, int k, std::vector<uint64_t> keys, std::vector<uint8_t> leaf,
                                       DevArray<double>&& coef, const double* dH, bool compress) {
    auto t = std::make_unique<mwns_tree1>();
    t->hold.set(ctx);
    t->ctx = ctx;
    t->k = k;
    const int64_t n = (int64_t)keys.size();
    for (int64_t i = 0; i < n; ++i) {
        const int j = key1_level(keys[i]);
        t->depth = std::max(t->depth, j);
        if (i && keys[i] <= keys[i - 1]) fail(MWNS_EINVAL, "keys are not sorted and distinct");
        if (j > 0) {
            const uint64_t pk = key1(j - 1, key1_trans(keys[i]) >> 1);
            const int64_t p = find_sorted(keys.data(), n, pk);
            if (p < 0 || leaf[p]) fail(MWNS_EINVAL, "a node without an internal parent");
            if (find_sorted(keys.data(), n, keys[i] ^ 1ull) < 0) fail(MWNS_EINVAL, "a node without its sibling");
        }
        if (!leaf[i] && find_sorted(keys.data(), n, key1(j + 1, 2 * key1_trans(keys[i]))) < 0)
            fail(MWNS_EINVAL, "an internal node without children");
        t->nleaves += leaf[i] ? 1 : 0;
    }
    if (n == 0 || keys[0] != key1(0, 0)) fail(MWNS_EINVAL, "the tree has no root");
    t->keys = std::move(keys);
    t->leaf = std::move(leaf);
    t->coef = std::move(coef);
    if (compress) {
        for (int j = t->depth - 1; j >= 0; --j) {
            std::vector<int64_t> par, ch0;
            for (int64_t i = 0; i < n; ++i)
                if (key1_level(t->keys[i]) == j && !t->leaf[i]) {
                    par.push_back(i);
                    ch0.push_back(find_sorted(t->keys.data(), n, key1(j + 1, 2 * key1_trans(t->keys[i]))));
                }
            if (par.empty()) continue;
            DevArray<int64_t> dp(ctx, par.size()), dc(ctx, ch0.size());
            dp.upload(par.data(), par.size(), ctx->stream);
            dc.upload(ch0.data(), ch0.size(), ctx->stream);
            compress1_kernel<<<blocks_for((int64_t)par.size() * k, 256), 256, 0, ctx->stream>>>(
                k, (int)par.size(), dp.p, dc.p, dH, t->coef.p);
            MWNS_HIP(hipGetLastError());
            MWNS_HIP(hipStreamSynchronize(ctx->stream));
        }
    }
    t->dkeys.reset(ctx, n);
    t->dkeys.upload(t->keys.data(), n, ctx->stream);
    t->dleaf.reset(ctx, n);
    t->dleaf.upload(t->leaf.data(), n, ctx->stream);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    return t;
}

}  // namespace

extern "C" {

mwns_status mwns_cot1d_op_create(mwns_ctx* ctx, int k, double eps, int max_level, mwns_op1** out) {
    MWNS_GUARD_BEGIN
    check_ctx1(ctx);
    if (!out) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > K1MAX) fail(MWNS_EINVAL, "k must be in 1..16");
    if (!(eps > 0.0) || !std::isfinite(eps)) fail(MWNS_EINVAL, "eps must be finite and > 0");
    if (max_level < 0 || max_level > MAXLEV1) fail(MWNS_EINVAL, "max_level must be in 0..40");
    auto op = std::make_unique<mwns_op1>();
    op->hold.set(ctx);
    op->ctx = ctx;
    op->k = k;
    op->max_level = max_level;
    op->eps = eps;
    const int nlev = max_level + 1;
    // Phi^+_ab(t_q) = int_0^{1-t} phi_a(t + y) phi_b(y) dy at the block rule's nodes (k-point rule, exact)
    const Quad qo = gauss_legendre01(NGL1), qi = gauss_legendre01(k);
    std::vector<double> php((size_t)NGL1 * k * k, 0.0), pa(K1MAX), pb(K1MAX);
    for (int q = 0; q < NGL1; ++q) {
        const double t = qo.x[q], len = 1.0 - t;
        for (int i = 0; i < k; ++i) {
            const double y = len * qi.x[i];
            legendre_phi(k, t + y, pa.data());
            legendre_phi(k, y, pb.data());
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) php[((size_t)q * k + a) * k + b] += len * qi.w[i] * pa[a] * pb[b];
        }
    }
    DevArray<double> dt(ctx, NGL1), dw(ctx, NGL1), dphp(ctx, php.size());
    dt.upload(qo.x.data(), NGL1, ctx->stream);
    dw.upload(qo.w.data(), NGL1, ctx->stream);
    dphp.upload(php.data(), php.size(), ctx->stream);
    op->R.reset(ctx, (size_t)nlev * NLR1 * k * k);
    const int64_t ne = (int64_t)nlev * NLR1 * k * k;
    cot_blocks_kernel<<<blocks_for(ne, 256), 256, 0, ctx->stream>>>(k, nlev, dt.p, dw.p, dphp.p, op->R.p);
    MWNS_HIP(hipGetLastError());
    upload_h(ctx, k, op->H);
    // difference norms per (j, representative L) and the bands
    std::vector<int2> jl;
    std::vector<int> dist;
    for (int j = 1; j <= max_level; ++j) {
        const int64_t nc = (int64_t)1 << (j - 1);
        if (nc <= 2 * DMAX1 + 1) {
            for (int64_t L = 0; L < nc; ++L) {
                const int64_t Lr = (2 * L <= nc) ? L : L - nc;
                jl.push_back(make_int2(j, (int)Lr));
                dist.push_back((int)pdist(L, nc));
            }
        } else {
            for (int L = -DMAX1; L <= DMAX1; ++L) {
                jl.push_back(make_int2(j, L));
                dist.push_back(std::abs(L));
            }
        }
    }
    std::vector<double> n2(jl.size());
    if (!jl.empty()) {
        DevArray<int2> djl(ctx, jl.size());
        DevArray<double> dn(ctx, jl.size());
        djl.upload(jl.data(), jl.size(), ctx->stream);
        diffnorm_kernel<<<(unsigned)jl.size(), 256, 0, ctx->stream>>>(k, djl.p, op->R.p, op->H.p, dn.p);
        MWNS_HIP(hipGetLastError());
        dn.download(n2.data(), n2.size(), ctx->stream);
    }
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    op->band.assign(max_level + 2, 0);
    size_t pos = 0;
    for (int j = 1; j <= max_level; ++j) {
        const int64_t full = ((int64_t)1 << (j - 1)) / 2;
        std::map<int, double> byd;
        while (pos < jl.size() && jl[pos].x == j) {
            byd[dist[pos]] += std::sqrt(n2[pos]);
            ++pos;
        }
        int64_t b = full;
        while (b > 0) {
            double s = 0.0;
            for (const auto& kv : byd)
                if (kv.first > b - 1) s += kv.second;
            if (!(s <= eps)) break;
            --b;
        }
        if (b > DMAX1) fail(MWNS_ERANGE, "the band at scale " + std::to_string(j) + " is wider than the tabulated blocks");
        op->band[j] = (int32_t)b;
    }
    *out = op.release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_cot1d_op_bands(const mwns_op1* op, int32_t* bands, int* count) {
    MWNS_GUARD_BEGIN
    if (!op || !count) fail(MWNS_EINVAL, "NULL argument");
    if (bands) {
        if (*count < (int)op->band.size()) fail(MWNS_ERANGE, "bands array too small");
        std::copy(op->band.begin(), op->band.end(), bands);
    }
    *count = (int)op->band.size();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_cot1d_op_set_bands(mwns_op1* op, const int32_t* bands, int count) {
    MWNS_GUARD_BEGIN
    if (!op || !bands) fail(MWNS_EINVAL, "NULL argument");
    if (count != (int)op->band.size()) fail(MWNS_EINVAL, "count must be max_level + 2");
    for (int j = 1; j <= op->max_level; ++j)
        if (bands[j] < 0 || bands[j] > DMAX1) fail(MWNS_EINVAL, "bands must be in 0..32");
    std::copy(bands, bands + count, op->band.begin());
    op->band[0] = 0;
    op->band[op->max_level + 1] = 0;
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_cot1d_op_blocks(mwns_ctx* ctx, const mwns_op1* op, double* R, size_t* count) {
    MWNS_GUARD_BEGIN
    check_ctx1(ctx);
    if (!op || !count) fail(MWNS_EINVAL, "NULL argument");
    const size_t n = op->R.n;
    if (R) {
        if (*count < n) fail(MWNS_ERANGE, "blocks array too small");
        op->R.download(R, n, ctx->stream);
        MWNS_HIP(hipStreamSynchronize(ctx->stream));
    }
    *count = n;
    return MWNS_OK;
    MWNS_GUARD_END
}

void mwns_cot1d_op_destroy(mwns_op1* op) { delete op; }

mwns_status mwns_cot1d_project(mwns_ctx* ctx, int k, double thr, int j0, int jmax, int n, const double* centers,
                               const double* exps, const double* weights, mwns_tree1** out) {
    MWNS_GUARD_BEGIN
    check_ctx1(ctx);
    if (!out || (n > 0 && (!centers || !exps || !weights))) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > K1MAX) fail(MWNS_EINVAL, "k must be in 1..16");
    if (!(thr >= 0.0) || !std::isfinite(thr)) fail(MWNS_EINVAL, "thr must be finite and >= 0");
    if (j0 < 0 || jmax < j0 || jmax > MAXLEV1) fail(MWNS_EINVAL, "need 0 <= j0 <= jmax <= 40");
    if (n < 0) fail(MWNS_EINVAL, "n must be >= 0");
    for (int i = 0; i < n; ++i)
        if (!(exps[i] > 0.0) || !std::isfinite(exps[i]) || !std::isfinite(centers[i]) || !std::isfinite(weights[i]))
            fail(MWNS_EINVAL, "Gaussian exponents must be > 0 and all parameters finite");
    const Quad q = gauss_legendre01(k);
    std::vector<double> phiq(k * k), phich(2 * k * k), tmp(K1MAX);
    for (int i = 0; i < k; ++i) {
        legendre_phi(k, q.x[i], tmp.data());
        for (int a = 0; a < k; ++a) phiq[i * k + a] = tmp[a];
        for (int c = 0; c < 2; ++c) {
            legendre_phi(k, 0.5 * (q.x[i] + c), tmp.data());
            for (int a = 0; a < k; ++a) phich[(c * k + i) * k + a] = tmp[a];
        }
    }
    DevArray<double> dx(ctx, k), dwq(ctx, k), dphi(ctx, phiq.size()), dphc(ctx, phich.size());
    DevArray<double> dgc(ctx, std::max(n, 1)), dga(ctx, std::max(n, 1)), dgw(ctx, std::max(n, 1));
    dx.upload(q.x.data(), k, ctx->stream);
    dwq.upload(q.w.data(), k, ctx->stream);
    dphi.upload(phiq.data(), phiq.size(), ctx->stream);
    dphc.upload(phich.data(), phich.size(), ctx->stream);
    dgc.upload(centers, n, ctx->stream);
    dga.upload(exps, n, ctx->stream);
    dgw.upload(weights, n, ctx->stream);
    std::vector<std::pair<uint64_t, std::vector<double>>> leaves;
    std::vector<int64_t> cand;
    for (int64_t l = 0; l < ((int64_t)1 << j0); ++l) cand.push_back(l);
    for (int j = j0; !cand.empty(); ++j) {
        const int nc = (int)cand.size();
        DevArray<int64_t> dc(ctx, nc);
        DevArray<double> dco(ctx, (size_t)nc * k), der(ctx, nc);
        dc.upload(cand.data(), nc, ctx->stream);
        project1_kernel<<<nc, 64, 0, ctx->stream>>>(k, j, dc.p, n, dgc.p, dga.p, dgw.p, dx.p, dwq.p, dphi.p, dphc.p,
                                                    dco.p, der.p);
        MWNS_HIP(hipGetLastError());
        std::vector<double> co((size_t)nc * k), er(nc);
        dco.download(co.data(), co.size(), ctx->stream);
        der.download(er.data(), nc, ctx->stream);
        MWNS_HIP(hipStreamSynchronize(ctx->stream));
        std::vector<int64_t> next;
        for (int i = 0; i < nc; ++i) {
            if (j < jmax && er[i] > thr) {
                next.push_back(2 * cand[i]);
                next.push_back(2 * cand[i] + 1);
            } else {
                leaves.emplace_back(key1(j, cand[i]), std::vector<double>(co.begin() + (size_t)i * k, co.begin() + (size_t)(i + 1) * k));
            }
        }
        cand.swap(next);
    }
    // all nodes: leaves and their ancestors
    std::vector<uint64_t> keys;
    for (const auto& lv : leaves) {
        uint64_t kk = lv.first;
        keys.push_back(kk);
        for (int j = key1_level(kk); j > 0; --j) keys.push_back(key1(j - 1, key1_trans(kk) >> (key1_level(kk) - j + 1)));
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::vector<uint8_t> leaf(keys.size(), 0);
    std::vector<double> hc(keys.size() * k, 0.0);
    for (const auto& lv : leaves) {
        const int64_t p = find_sorted(keys.data(), (int64_t)keys.size(), lv.first);
        leaf[p] = 1;
        std::copy(lv.second.begin(), lv.second.end(), hc.begin() + p * k);
    }
    DevArray<double> coef(ctx, hc.size());
    coef.upload(hc.data(), hc.size(), ctx->stream);
    DevArray<double> dH;
    upload_h(ctx, k, dH);
    *out = build_tree1(ctx, k, std::move(keys), std::move(leaf), std::move(coef), dH.p, true).release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_cot1d_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* lkeys, const double* coeffs,
                                   mwns_tree1** out) {
    MWNS_GUARD_BEGIN
    check_ctx1(ctx);
    if (!out || nleaves <= 0 || !lkeys || !coeffs) fail(MWNS_EINVAL, "NULL argument or no leaves");
    if (k < 1 || k > K1MAX) fail(MWNS_EINVAL, "k must be in 1..16");
    std::vector<uint64_t> keys;
    for (int64_t i = 0; i < nleaves; ++i) {
        const uint64_t kk = lkeys[i];
        const int jl = key1_level(kk);
        if (jl > MAXLEV1 || key1_trans(kk) >= ((int64_t)1 << jl)) fail(MWNS_EINVAL, "invalid leaf key");
        keys.push_back(kk);
        for (int j = jl; j > 0; --j) keys.push_back(key1(j - 1, key1_trans(kk) >> (jl - j + 1)));
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::vector<uint8_t> leaf(keys.size(), 0);
    std::vector<double> hc(keys.size() * k, 0.0);
    for (int64_t i = 0; i < nleaves; ++i) {
        const int64_t p = find_sorted(keys.data(), (int64_t)keys.size(), lkeys[i]);
        if (leaf[p]) fail(MWNS_EINVAL, "duplicate leaf key");
        leaf[p] = 1;
        std::copy(coeffs + i * k, coeffs + (i + 1) * k, hc.begin() + p * k);
    }
    for (size_t i = 0; i < keys.size(); ++i)
        if (leaf[i] && i + 1 < keys.size()) {
            // a leaf must not have descendants among the keys
            const int j = key1_level(keys[i]);
            if (find_sorted(keys.data(), (int64_t)keys.size(), key1(j + 1, 2 * key1_trans(keys[i]))) >= 0)
                fail(MWNS_EINVAL, "a leaf has descendants");
        }
    DevArray<double> coef(ctx, hc.size());
    coef.upload(hc.data(), hc.size(), ctx->stream);
    DevArray<double> dH;
    upload_h(ctx, k, dH);
    *out = build_tree1(ctx, k, std::move(keys), std::move(leaf), std::move(coef), dH.p, true).release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_cot1d_apply(mwns_ctx* ctx, const mwns_op1* op, const mwns_tree1* f, mwns_tree1** g,
                             double* ms_contract) {
    MWNS_GUARD_BEGIN
    check_ctx1(ctx);
    if (!op || !f || !g) fail(MWNS_EINVAL, "NULL argument");
    if (op->ctx != ctx || f->ctx != ctx) fail(MWNS_EINVAL, "operator or tree of another context");
    if (op->k != f->k) fail(MWNS_EINVAL, "the operator's and the tree's orders differ");
    if (f->depth > op->max_level) fail(MWNS_EINVAL, "the tree is deeper than the operator's max_level");
    const int k = f->k;
    const std::vector<int32_t>& B = op->band;
    // output tree: f's nodes; a leaf of scale j is refined when an internal node of f of scale j
    // lies in its whole band (parents at periodic distance <= B_j), and so on for the added children
    std::map<uint64_t, uint8_t> nodes;
    std::map<int, std::vector<int64_t>> ipar;   // per scale: parents of f's internal nodes, sorted
    for (size_t i = 0; i < f->keys.size(); ++i) {
        nodes[f->keys[i]] = f->leaf[i];
        if (!f->leaf[i] && key1_level(f->keys[i]) > 0)
            ipar[key1_level(f->keys[i])].push_back(key1_trans(f->keys[i]) >> 1);
    }
    for (auto& kv : ipar) {
        std::sort(kv.second.begin(), kv.second.end());
        kv.second.erase(std::unique(kv.second.begin(), kv.second.end()), kv.second.end());
    }
    // is there an entry cp of v with periodic distance |c - cp| <= b on nc boxes?
    auto near = [](const std::vector<int64_t>& v, int64_t c, int64_t b, int64_t nc) {
        if (2 * b + 1 >= nc) return !v.empty();
        auto any_in = [&](int64_t lo, int64_t hi) {
            auto it = std::lower_bound(v.begin(), v.end(), lo);
            return it != v.end() && *it <= hi;
        };
        const int64_t lo = c - b, hi = c + b;
        if (lo < 0) return any_in(0, hi) || any_in(lo + nc, nc - 1);
        if (hi >= nc) return any_in(lo, nc - 1) || any_in(0, hi - nc);
        return any_in(lo, hi);
    };
    std::vector<uint64_t> todo;
    for (const auto& kv : nodes)
        if (kv.second) todo.push_back(kv.first);
    while (!todo.empty()) {
        std::vector<uint64_t> next;
        for (uint64_t kk : todo) {
            const int j = key1_level(kk);
            auto it = ipar.find(j);
            if (j == 0 || it == ipar.end()) continue;
            if (!near(it->second, key1_trans(kk) >> 1, B[j], (int64_t)1 << (j - 1))) continue;
            if (j + 1 > op->max_level) fail(MWNS_ERANGE, "the output tree would be deeper than the operator's max_level");
            nodes[kk] = 0;
            for (int c = 0; c < 2; ++c) {
                const uint64_t ck = key1(j + 1, 2 * key1_trans(kk) + c);
                nodes[ck] = 1;
                next.push_back(ck);
            }
        }
        todo.swap(next);
    }
    std::vector<uint64_t> okeys;
    std::vector<uint8_t> oleaf;
    for (const auto& kv : nodes) {
        okeys.push_back(kv.first);
        oleaf.push_back(kv.second);
    }
    const int64_t no = (int64_t)okeys.size();
    // input blocks: every (j, b') a job reads, from f or from f's nearest ancestor
    std::unordered_map<uint64_t, int64_t> inidx;
    std::vector<int64_t> ianc, itrans;
    std::vector<int> iup;
    auto input = [&](int j, int64_t bp) -> int64_t {
        const uint64_t kk = key1(j, bp);
        auto it = inidx.find(kk);
        if (it != inidx.end()) return it->second;
        int up = 0;
        int64_t p;
        while ((p = find_sorted(f->keys.data(), (int64_t)f->keys.size(), key1(j - up, bp >> up))) < 0) ++up;
        const int64_t id = (int64_t)ianc.size();
        ianc.push_back(p);
        iup.push_back(up);
        itrans.push_back(bp);
        inidx.emplace(kk, id);
        return id;
    };
    std::vector<int64_t> off(1, 0), jin;
    std::vector<int> jli, jc, nlev(no);
    for (int64_t i = 0; i < no; ++i) {
        const int j = key1_level(okeys[i]);
        const int64_t b = key1_trans(okeys[i]);
        const bool lf = oleaf[i] != 0;
        nlev[i] = j;
        if (j == 0) {
            if (lf) {
                jin.push_back(input(0, 0));
                jli.push_back(LR1);
                jc.push_back(1);
            }
        } else {
            const int64_t n = (int64_t)1 << j;
            const int64_t reach = std::max<int64_t>(2 * B[j] + 1, lf ? 0 : B[j + 1]);
            std::vector<int64_t> seen;
            for (int64_t l = -reach; l <= reach; ++l) {
                const int64_t lm = ((l % n) + n) % n;
                if (std::find(seen.begin(), seen.end(), lm) != seen.end()) continue;
                seen.push_back(lm);
                const int64_t bp = ((b - l) % n + n) % n;
                const int64_t L = pdist((b >> 1) - (bp >> 1), n / 2);
                const int c = (L <= B[j] ? 1 : 0) - (lf ? 0 : (pdist(l, n) <= B[j + 1] ? 1 : 0));
                if (!c) continue;
                jin.push_back(input(j, bp));
                jli.push_back((int)(l + LR1));
                jc.push_back(c);
            }
        }
        off.push_back((int64_t)jin.size());
    }
    const int64_t nin = (int64_t)ianc.size(), nj = (int64_t)jin.size();
    hipStream_t st = ctx->stream;
    DevArray<int64_t> dianc(ctx, std::max<int64_t>(nin, 1)), ditr(ctx, std::max<int64_t>(nin, 1));
    DevArray<int> diup(ctx, std::max<int64_t>(nin, 1));
    DevArray<double> X(ctx, (size_t)std::max<int64_t>(nin, 1) * k);
    dianc.upload(ianc.data(), nin, st);
    ditr.upload(itrans.data(), nin, st);
    diup.upload(iup.data(), nin, st);
    if (nin) {
        gather1_kernel<<<blocks_for(nin, 128), 128, 0, st>>>(k, (int)nin, dianc.p, diup.p, ditr.p, op->H.p, f->coef.p, X.p);
        MWNS_HIP(hipGetLastError());
    }
    DevArray<int64_t> doff(ctx, off.size()), djin(ctx, std::max<int64_t>(nj, 1));
    DevArray<int> djli(ctx, std::max<int64_t>(nj, 1)), djc(ctx, std::max<int64_t>(nj, 1)), dnlev(ctx, no);
    doff.upload(off.data(), off.size(), st);
    djin.upload(jin.data(), nj, st);
    djli.upload(jli.data(), nj, st);
    djc.upload(jc.data(), nj, st);
    dnlev.upload(nlev.data(), no, st);
    DevArray<double> out(ctx, (size_t)no * k);
    hipEvent_t e0, e1;
    MWNS_HIP(hipEventCreate(&e0));
    MWNS_HIP(hipEventCreate(&e1));
    MWNS_HIP(hipEventRecord(e0, st));
    contract1_kernel<<<blocks_for(no * k, 128), 128, 0, st>>>(k, (int)no, dnlev.p, doff.p, djin.p, djli.p, djc.p,
                                                              op->R.p, X.p, out.p);
    MWNS_HIP(hipGetLastError());
    MWNS_HIP(hipEventRecord(e1, st));
    // assembly, level by level from the top
    int depth = 0;
    for (uint64_t kk : okeys) depth = std::max(depth, key1_level(kk));
    for (int j = 1; j <= depth; ++j) {
        std::vector<int64_t> nd, par;
        std::vector<int> sg;
        for (int64_t i = 0; i < no; ++i)
            if (key1_level(okeys[i]) == j) {
                nd.push_back(i);
                par.push_back(find_sorted(okeys.data(), no, key1(j - 1, key1_trans(okeys[i]) >> 1)));
                sg.push_back((int)(key1_trans(okeys[i]) & 1));
            }
        DevArray<int64_t> dnd(ctx, nd.size()), dpar(ctx, par.size());
        DevArray<int> dsg(ctx, sg.size());
        dnd.upload(nd.data(), nd.size(), st);
        dpar.upload(par.data(), par.size(), st);
        dsg.upload(sg.data(), sg.size(), st);
        assemble1_kernel<<<blocks_for((int64_t)nd.size() * k, 128), 128, 0, st>>>(k, (int)nd.size(), dnd.p, dpar.p,
                                                                                  dsg.p, op->H.p, out.p);
        MWNS_HIP(hipGetLastError());
        MWNS_HIP(hipStreamSynchronize(st));
    }
    MWNS_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    MWNS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_contract) *ms_contract = ms;
    *g = build_tree1(ctx, k, std::move(okeys), std::move(oleaf), std::move(out), op->H.p, false).release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_cot1d_export(mwns_ctx* ctx, const mwns_tree1* t, int64_t* nnodes, uint64_t* keys, uint8_t* is_leaf,
                              double* coeffs) {
    MWNS_GUARD_BEGIN
    check_ctx1(ctx);
    if (!t || !nnodes) fail(MWNS_EINVAL, "NULL argument");
    const int64_t n = (int64_t)t->keys.size();
    if (keys || is_leaf || coeffs) {
        if (*nnodes < n) fail(MWNS_ERANGE, "arrays too small");
        if (keys) std::copy(t->keys.begin(), t->keys.end(), keys);
        if (is_leaf) std::copy(t->leaf.begin(), t->leaf.end(), is_leaf);
        if (coeffs) {
            t->coef.download(coeffs, (size_t)n * t->k, ctx->stream);
            MWNS_HIP(hipStreamSynchronize(ctx->stream));
        }
    }
    *nnodes = n;
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_cot1d_eval(mwns_ctx* ctx, const mwns_tree1* t, int64_t npts, const double* x, double* out) {
    MWNS_GUARD_BEGIN
    check_ctx1(ctx);
    if (!t || (npts > 0 && (!x || !out))) fail(MWNS_EINVAL, "NULL argument");
    if (npts < 0) fail(MWNS_EINVAL, "npts must be >= 0");
    if (npts == 0) return MWNS_OK;
    for (int64_t i = 0; i < npts; ++i)
        if (!(x[i] >= 0.0 && x[i] <= 1.0)) fail(MWNS_EINVAL, "points must lie in [0, 1]");
    DevArray<double> dx(ctx, npts), dout(ctx, npts);
    dx.upload(x, npts, ctx->stream);
    eval1_kernel<<<blocks_for(npts, 128), 128, 0, ctx->stream>>>(t->k, (int64_t)t->keys.size(), t->dkeys.p, t->dleaf.p,
                                                               t->coef.p, npts, dx.p, dout.p);
    MWNS_HIP(hipGetLastError());
    dout.download(out, npts, ctx->stream);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    return MWNS_OK;
    MWNS_GUARD_END
}

void mwns_tree1_destroy(mwns_tree1* t) { delete t; }

}  // extern "C"
