// The hydrogen ground state by the iteration of Sec. 6.2: phi = -2 G_mu V phi with
// G_mu = (-Delta + mu^2)^{-1} (kernel e^{-mu r} / (4 pi r)), V = -Z / r, mu moved to sqrt(-2 E).
//
// Three device pieces beside the modified ns-form apply:
//   * the Coulomb product rho = c / r * f on a refinement of f's tree (the paper defers products of
//     adaptively represented functions to other work; the reading taken here: every leaf of f split
//     once, the boxes whose closure holds the nucleus split down to a finest level, and each new
//     leaf's block the k-point Gauss-Legendre rule of eq. fvals2coefs applied to c / r times f's
//     polynomial at the leaf's nodes; the nucleus sits at the cube's centre, a corner of boxes on
//     every scale, so no node falls on it);
//   * the inner product of two trees over the leaves of the first (the second holds every box of
//     those leaves, e.g. a product built on a refinement of the first, whose redundant tree stores
//     the projections onto all coarser boxes);
//   * the iteration driver.
// The physical cube [-L, L]^3 (nucleus at its centre) is the unit cube scaled by s = 2 L: physical
// integrals are s^3 times unit-cube ones and the physical kernel is s^2 e^{-(mu s) r_u} / (4 pi r_u)
// on the unit cube (the fit's scale s^2, its mu scaled by s).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <set>
#include <vector>

#include "mwns_internal.h"

using namespace mwns;

namespace {

__device__ inline int64_t brick_elem(int k, int child, int a, int b, int c) {
    const int P = 2 * k;
    return ((int64_t)((child & 1) * k + a) * P + ((child >> 1) & 1) * k + b) * P + ((child >> 2) & 1) * k + c;
}

// One output leaf of the product: where its block goes, and the leaf of f whose polynomial holds it.
struct ProdJob {
    int64_t src, dst;         // element offsets of the source / destination bricks
    int32_t src_child, dst_child;
    int32_t J, j;             // levels of f's leaf and of the output leaf
    int32_t L[3], l[3];       // their translations
};

constexpr int PT = 256;

// out[i0][i1][i2] = sum_m M[i_d][m] in[...m at position d...]: one mode product of a K^3 tensor in LDS.
// MT[o][i] is read as M[o * K + i] (row = output index).
template <int K, int D>
__device__ inline void mode_product(const double* M, const double* in, double* out) {
    constexpr int KK = K * K, K3 = KK * K;
    for (int e = threadIdx.x; e < K3; e += PT) {
        const int i0 = e / KK, i1 = (e / K) % K, i2 = e % K;
        const int o = D == 0 ? i0 : (D == 1 ? i1 : i2);
        const int base = D == 0 ? i1 * K + i2 : (D == 1 ? i0 * KK + i2 : i0 * KK + i1 * K);
        const int stride = D == 0 ? KK : (D == 1 ? K : 1);
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m) s += M[o * K + m] * in[base + m * stride];
        out[e] = s;
    }
}

// One block per output leaf.  Values of f at the leaf's K^3 Gauss-Legendre nodes from f's leaf
// block (eq. func_interp, three mode products with the scaling functions at the nodes' local
// coordinates in f's box), times w_q w_r w_t c / (s |x - 1/2|), then back to coefficients with the
// scaling functions at the nodes (eq. fvals2coefs, three mode products); written into the output
// tree's brick.
template <int K>
__global__ void __launch_bounds__(PT) coulomb_product_kernel(const ProdJob* __restrict__ jobs,
                                                             const double* __restrict__ fcoef,
                                                             double* __restrict__ gcoef,
                                                             const double* __restrict__ qx, const double* __restrict__ qw,
                                                             const double* __restrict__ phq, double c_over_s) {
    constexpr int KK = K * K, K3 = KK * K;
    __shared__ double bufA[K3], bufB[K3];
    __shared__ double P[3][KK];        // P[d][q * K + a] = phi_a(local coordinate in f's box of node q, dimension d)
    __shared__ double Ph[KK];          // Ph[a * K + q] = phi_a(x_q) (transposed: row = output degree)
    __shared__ double fac[3][K];       // per dimension: w_q and the node's coordinate offset from the centre
    __shared__ double off[3][K];
    const ProdJob& jb = jobs[blockIdx.x];      // read in place: a private copy indexed by d would spill
    const int tid = threadIdx.x;
    for (int e = tid; e < K3; e += PT) {
        const int a = e / KK, b = (e / K) % K, c = e % K;
        bufA[e] = fcoef[jb.src + brick_elem(K, jb.src_child, a, b, c)];
    }
    if (tid < 3 * K) {
        const int d = tid / K, q = tid % K;
        const double loc = ldexp((double)jb.l[d] + qx[q], jb.J - jb.j) - (double)jb.L[d];
        const double t = 2.0 * loc - 1.0;
        double p0 = 1.0, p1 = t;
        P[d][q * K] = 1.0;
        if (K > 1) P[d][q * K + 1] = sqrt(3.0) * t;
        for (int a = 2; a < K; ++a) {
            const double p2 = ((2 * a - 1) * t * p1 - (a - 1) * p0) / a;
            P[d][q * K + a] = sqrt(2.0 * a + 1.0) * p2;
            p0 = p1;
            p1 = p2;
        }
        fac[d][q] = qw[q];
        off[d][q] = ldexp((double)jb.l[d] + qx[q], -jb.j) - 0.5;
    }
    if (tid < KK) Ph[(tid % K) * K + tid / K] = phq[tid];
    __syncthreads();
    mode_product<K, 0>(P[0], bufA, bufB);
    __syncthreads();
    mode_product<K, 1>(P[1], bufB, bufA);
    __syncthreads();
    mode_product<K, 2>(P[2], bufA, bufB);
    __syncthreads();
    // 2^{3J/2} from f's basis, 2^{-3j/2} from the output's quadrature (eq. fvals2coefs)
    const double scale = exp2(1.5 * (double)(jb.J - jb.j)) * c_over_s;
    for (int e = tid; e < K3; e += PT) {
        const int q = e / KK, r = (e / K) % K, t = e % K;
        const double dx = off[0][q], dy = off[1][r], dz = off[2][t];
        const double rad = sqrt(dx * dx + dy * dy + dz * dz);
        bufB[e] = bufB[e] * (fac[0][q] * fac[1][r] * fac[2][t]) * (scale / rad);
    }
    __syncthreads();
    mode_product<K, 0>(Ph, bufB, bufA);
    __syncthreads();
    mode_product<K, 1>(Ph, bufA, bufB);
    __syncthreads();
    mode_product<K, 2>(Ph, bufB, bufA);
    __syncthreads();
    for (int e = tid; e < K3; e += PT) {
        const int a = e / KK, b = (e / K) % K, c = e % K;
        gcoef[jb.dst + brick_elem(K, jb.dst_child, a, b, c)] = bufA[e];
    }
}

struct DotPair {
    int64_t u, v;             // element offsets of the two bricks
    int32_t uc, vc;           // children within them
};

// One wavefront per pair: the dot product of the two k^3 blocks, reduced across the wave in a
// fixed order, into part[pair].
__global__ void __launch_bounds__(PT) block_dot_kernel(int64_t npairs, int k, const DotPair* __restrict__ pairs,
                                                       const double* __restrict__ ucoef,
                                                       const double* __restrict__ vcoef, double* __restrict__ part) {
    const int64_t p = (int64_t)blockIdx.x * (PT / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (p >= npairs) return;
    const DotPair pr = pairs[p];
    const int kk = k * k, k3 = kk * k;
    double s = 0.0;
    for (int e = lane; e < k3; e += 64) {
        const int a = e / kk, b = (e / k) % k, c = e % k;
        s += ucoef[pr.u + brick_elem(k, pr.uc, a, b, c)] * vcoef[pr.v + brick_elem(k, pr.vc, a, b, c)];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) part[p] = s;
}

// One block: the sum of part[0..n) in a fixed order (strided partial sums, then a tree in LDS).
__global__ void __launch_bounds__(1024) sum_kernel(int64_t n, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

template <int K>
void launch_product(const ProdJob* jobs, int64_t n, const double* f, double* g, const double* qx, const double* qw,
                    const double* phq, double c_over_s, hipStream_t st) {
    hipLaunchKernelGGL(coulomb_product_kernel<K>, dim3((unsigned)n), dim3(PT), 0, st, jobs, f, g, qx, qw, phq, c_over_s);
}

// Keys of the 8 boxes of level j >= 1 whose closure holds the cube's centre.
void nucleus_boxes(int j, uint64_t* out) {
    const int64_t h = (int64_t)1 << (j - 1);
    for (int s = 0; s < 8; ++s) out[s] = make_key(j, h - 1 + (s & 1), h - 1 + ((s >> 1) & 1), h - 1 + ((s >> 2) & 1));
}

void check_tree(mwns_ctx* ctx, const mwns_tree* t) {
    if (!t) fail(MWNS_EINVAL, "NULL tree");
    if (t->ctx != ctx) fail(MWNS_EINVAL, "tree belongs to another context");
}

mwns_tree* coulomb_product(mwns_ctx* ctx, const mwns_tree* f, double c, double s, int jmax) {
    const int k = f->k;
    if (f->depth + 1 > MAXLEV) fail(MWNS_EINVAL, "f's leaves are too deep to split");
    // children of f's leaves (sorted), then the nucleus boxes split level by level
    std::vector<uint64_t> base;
    base.reserve((size_t)f->nleaves * 8);
    for (int64_t i = 0; i < f->nnodes; ++i) {
        if (!f->leaf[i]) continue;
        const uint64_t key = f->keys[i];
        const int j = key_level(key);
        int64_t l[3];
        key_coords(key, l);
        for (int ch = 0; ch < 8; ++ch)
            base.push_back(make_key(j + 1, 2 * l[0] + (ch & 1), 2 * l[1] + ((ch >> 1) & 1), 2 * l[2] + ((ch >> 2) & 1)));
    }
    std::sort(base.begin(), base.end());
    std::set<uint64_t> removed, added;
    auto present = [&](uint64_t key) {
        return added.count(key) || (std::binary_search(base.begin(), base.end(), key) && !removed.count(key));
    };
    const int top = std::max(jmax, f->depth + 1);
    for (int lev = 1; lev <= top && lev < jmax; ++lev) {
        uint64_t nb[8];
        nucleus_boxes(lev, nb);
        for (uint64_t key : nb) {
            if (!present(key)) continue;
            if (added.erase(key) == 0) removed.insert(key);
            int64_t l[3];
            key_coords(key, l);
            for (int ch = 0; ch < 8; ++ch)
                added.insert(make_key(lev + 1, 2 * l[0] + (ch & 1), 2 * l[1] + ((ch >> 1) & 1), 2 * l[2] + ((ch >> 2) & 1)));
        }
    }
    std::vector<uint64_t> leaves;
    leaves.reserve(base.size() + added.size());
    for (uint64_t key : base)
        if (!removed.count(key)) leaves.push_back(key);
    leaves.insert(leaves.end(), added.begin(), added.end());
    std::sort(leaves.begin(), leaves.end());
    const int64_t n = (int64_t)leaves.size();
    std::vector<int64_t> order, pos;
    std::unique_ptr<mwns_tree> g = skeleton_from_leaves(ctx, k, n, leaves.data(), &order, &pos);
    std::vector<ProdJob> jobs(n);
    const int64_t be = brick_elems(k);
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t key = leaves[order[i]];
        ProdJob& jb = jobs[i];
        int64_t l[3];
        key_coords(key, l);
        jb.j = key_level(key);
        // f's leaf holding this box: the nearest ancestor that is a leaf of f
        int J = jb.j;
        int64_t L[3] = {l[0], l[1], l[2]};
        int64_t node = -1;
        while (J > 0) {
            --J;
            for (int d = 0; d < 3; ++d) L[d] >>= 1;
            node = find_sorted(f->keys.data(), f->nnodes, make_key(J, L[0], L[1], L[2]));
            if (node >= 0 && f->leaf[node]) break;
            node = -1;
        }
        if (node < 0) fail(MWNS_EINVAL, "product leaf without a leaf of f above it");
        int64_t brick;
        int child;
        node_brick(f, node, &brick, &child);
        jb.src = brick * be;
        jb.src_child = child;
        jb.J = J;
        node_brick(g.get(), pos[i], &brick, &child);
        jb.dst = brick * be;
        jb.dst_child = child;
        for (int d = 0; d < 3; ++d) {
            jb.L[d] = (int32_t)L[d];
            jb.l[d] = (int32_t)l[d];
        }
    }
    hipStream_t st = ctx->stream;
    const Quad gl = gauss_legendre01(k);
    std::vector<double> tab(2 * k + k * k);
    for (int q = 0; q < k; ++q) {
        tab[q] = gl.x[q];
        tab[k + q] = gl.w[q];
        legendre_phi(k, gl.x[q], &tab[2 * k + q * k]);
    }
    DevArray<double> dtab(ctx, tab.size());
    DevArray<ProdJob> djobs(ctx, n);
    dtab.upload(tab.data(), tab.size(), st);
    djobs.upload(jobs.data(), n, st);
    MWNS_HIP(hipMemsetAsync(g->coef.p, 0, g->coef.n * sizeof(double), st));
    const double* qx = dtab.p;
    const double* qw = dtab.p + k;
    const double* phq = dtab.p + 2 * k;
    switch (k) {
        case 1: launch_product<1>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 2: launch_product<2>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 3: launch_product<3>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 4: launch_product<4>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 5: launch_product<5>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 6: launch_product<6>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 7: launch_product<7>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 8: launch_product<8>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        case 9: launch_product<9>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
        default: launch_product<10>(djobs.p, n, f->coef.p, g->coef.p, qx, qw, phq, c / s, st); break;
    }
    MWNS_HIP(hipGetLastError());
    DevArray<double> dH = upload_filters(ctx, k);
    compress_tree(g.get(), dH.p);
    // the job and table arrays go back to the context's cache once the stream has used them
    MWNS_HIP(hipStreamSynchronize(st));
    return g.release();
}

double tree_dot(mwns_ctx* ctx, const mwns_tree* u, const mwns_tree* v) {
    if (u->k != v->k) fail(MWNS_EINVAL, "trees of different orders");
    const int64_t be = brick_elems(u->k);
    std::vector<DotPair> pairs;
    pairs.reserve(u->nleaves);
    for (int64_t i = 0; i < u->nnodes; ++i) {
        if (!u->leaf[i]) continue;
        const int64_t m = find_sorted(v->keys.data(), v->nnodes, u->keys[i]);
        if (m < 0) fail(MWNS_EINVAL, "the second tree lacks a box of the first tree's leaves");
        DotPair p;
        int64_t brick;
        int child;
        node_brick(u, i, &brick, &child);
        p.u = brick * be;
        p.uc = child;
        node_brick(v, m, &brick, &child);
        p.v = brick * be;
        p.vc = child;
        pairs.push_back(p);
    }
    const int64_t n = (int64_t)pairs.size();
    hipStream_t st = ctx->stream;
    DevArray<DotPair> dp(ctx, n);
    DevArray<double> part(ctx, n + 1);
    dp.upload(pairs.data(), n, st);
    const int64_t blocks = (n + PT / 64 - 1) / (PT / 64);
    hipLaunchKernelGGL(block_dot_kernel, dim3((unsigned)blocks), dim3(PT), 0, st, n, u->k, dp.p, u->coef.p, v->coef.p,
                       part.p);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, st, n, part.p, part.p + n);
    MWNS_HIP(hipGetLastError());
    double* h = static_cast<double*>(pinned_staging(ctx, sizeof(double)));
    MWNS_HIP(hipMemcpyAsync(h, part.p + n, sizeof(double), hipMemcpyDeviceToHost, st));
    MWNS_HIP(hipStreamSynchronize(st));
    return *h;
}

// Runs a library call from inside another: its error (already recorded) becomes this call's.
void call(mwns_status st) {
    if (st != MWNS_OK) throw Failure{st, mwns_last_error()};
}

struct TreeBox {
    mwns_tree* t = nullptr;
    TreeBox() = default;
    explicit TreeBox(mwns_tree* p) : t(p) {}
    TreeBox(const TreeBox&) = delete;
    TreeBox& operator=(const TreeBox&) = delete;
    void reset(mwns_tree* p) {
        if (t) mwns_tree_destroy(t);
        t = p;
    }
    ~TreeBox() { reset(nullptr); }
};

}  // namespace

extern "C" {

mwns_status mwns_tree_coulomb_product(mwns_ctx* ctx, const mwns_tree* f, double c, double s, int jmax,
                                      mwns_tree** out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !out) fail(MWNS_EINVAL, "NULL argument");
    check_tree(ctx, f);
    if (!std::isfinite(c) || !(s > 0.0) || !std::isfinite(s)) fail(MWNS_EINVAL, "c must be finite and s > 0");
    if (jmax < 1 || jmax > MAXLEV) fail(MWNS_EINVAL, "jmax out of range");
    MWNS_HIP(hipSetDevice(ctx->device));
    *out = coulomb_product(ctx, f, c, s, jmax);
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_dot(mwns_ctx* ctx, const mwns_tree* u, const mwns_tree* v, double* out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !out) fail(MWNS_EINVAL, "NULL argument");
    check_tree(ctx, u);
    check_tree(ctx, v);
    MWNS_HIP(hipSetDevice(ctx->device));
    *out = tree_dot(ctx, u, v);
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_hydrogen_kalos(mwns_ctx* ctx, int k, double eps, double L, int jmax, double mu0, double Z, int j0,
                                int iters, double* mu_out, double* E_out, int64_t* rho_leaves, double* ms_apply) {
    MWNS_GUARD_BEGIN
    if (!ctx || !mu_out || !E_out) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > KMAX) fail(MWNS_EINVAL, "k out of range");
    if (!(eps > 0.0 && eps < 1.0) || !(L > 0.0) || !std::isfinite(L) || !(mu0 > 0.0) || !std::isfinite(mu0) ||
        !(Z > 0.0) || !std::isfinite(Z))
        fail(MWNS_EINVAL, "need 0 < eps < 1 and L, mu0, Z > 0");
    if (jmax < 1 || jmax >= MAXLEV || j0 < 0 || j0 > jmax || iters < 1) fail(MWNS_EINVAL, "levels or iters out of range");
    MWNS_HIP(hipSetDevice(ctx->device));
    const double s = 2.0 * L, s3 = s * s * s, a = s * s;
    // phi_0 = (2/pi)^{3/4} e^{-r^2}, normalised: one Gaussian of exponent s^2 on the unit cube
    const double ctr[3] = {0.5, 0.5, 0.5};
    const double amp = std::pow(2.0 / M_PI, 0.75) * std::pow(M_PI / a, 1.5);
    TreeBox phi, rho;
    mwns_tree* t = nullptr;
    call(mwns_project_gaussians(ctx, k, eps, j0, jmax, 1, ctr, &a, &amp, &t));
    phi.reset(t);
    const double nphi = std::sqrt(s3 * tree_dot(ctx, phi.t, phi.t));
    rho.reset(coulomb_product(ctx, phi.t, 2.0 * Z / nphi, s, jmax));       // -2 V phi / ||phi||
    phi.reset(nullptr);
    double mu = mu0;
    std::vector<double> tau(4096), w(4096);
    std::vector<double> hmu(iters), hE(iters), hms(iters);
    std::vector<int64_t> hleaves(iters);
    for (int it = 0; it < iters; ++it) {
        const int depth = rho.t->depth;
        int M = 0;
        call(mwns_fit_kernel(mu * s, 1.0, s * s, eps, std::sqrt(eps) * std::ldexp(1.0, -depth), std::sqrt(3.0),
                             (int)tau.size(), &M, tau.data(), w.data()));
        mwns_op* op = nullptr;
        call(mwns_op_create(ctx, k, M, tau.data(), w.data(), eps, depth, nullptr, &op));
        TreeBox g;
        mwns_apply_stats stats;
        const mwns_status sa = mwns_apply(ctx, op, rho.t, MWNS_F64 | (ms_apply ? MWNS_TIMES_ONLY : 0), &t,
                                          ms_apply ? &stats : nullptr);
        mwns_op_destroy(op);
        call(sa);
        g.reset(t);                                                         // phi_new on rho's tree
        if (ms_apply) hms[it] = stats.ms_closure + stats.ms_contract + stats.ms_assemble;
        hleaves[it] = rho.t->nleaves;
        const double n2 = s3 * tree_dot(ctx, g.t, g.t);
        const double ip1 = s3 * tree_dot(ctx, g.t, rho.t);                  // <phi_new, rho>
        TreeBox phin;
        call(mwns_tree_discard(ctx, g.t, eps, &t, nullptr));
        phin.reset(t);
        g.reset(nullptr);
        TreeBox rnew(coulomb_product(ctx, phin.t, 2.0 * Z / std::sqrt(n2), s, jmax));   // -2 V phi_new / ||phi_new||
        const double ip2 = s3 * tree_dot(ctx, phin.t, rnew.t);              // <phi_new, rho_new>
        const double E = (0.5 * ip1 - 0.5 * mu * mu * n2 - 0.5 * std::sqrt(n2) * ip2) / n2;
        hmu[it] = mu;
        hE[it] = E;
        if (!(E < 0.0)) fail(MWNS_ERANGE, "the energy estimate is not negative: no bound state to follow");
        mu = std::sqrt(-2.0 * E);
        rho.reset(rnew.t);
        rnew.t = nullptr;
    }
    std::copy(hmu.begin(), hmu.end(), mu_out);
    std::copy(hE.begin(), hE.end(), E_out);
    if (rho_leaves) std::copy(hleaves.begin(), hleaves.end(), rho_leaves);
    if (ms_apply) std::copy(hms.begin(), hms.end(), ms_apply);
    return MWNS_OK;
    MWNS_GUARD_END
}

}  // extern "C"
