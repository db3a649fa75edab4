// Detail norms and l2 pruning of trees (App. A.2-A.3, Sec. 2.2, Alg. 3 Step 4).
//
// The detail coefficients of an internal node are the seven blocks that the orthogonal two-scale
// transform W = [[H0, H1], [G0, G1]] (per dimension) leaves besides the parent's own scaling block
// when applied to its sibling brick of children (eqs. decomp_scaling, decomp_wavelet).  Their
// squared norm is the node's contribution to ||f||_2^2 beyond its coarser approximation, so
// removing a sibling group whose children are leaves changes f by exactly that much in l2 norm.
// l2 pruning (Sec. 2.2) acts on the function that a tree's leaves represent, with the internal
// nodes rebuilt from the leaves: starting on the finest scale, sibling groups whose children are
// leaves are removed, in ascending order of their detail norm (ties by key), while the cumulative
// squared norm of what was removed stays within eta^2; the first group of a scale that would
// exceed it ends that scale and the rest of the budget carries to the next coarser one.  The kept
// nodes keep the rebuilt blocks.  Alg. 3 Step 4's discard is the same at eta = eps ||f||_2.
#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>

#include "mwns_internal.h"

namespace mwns {
namespace {

// Squared norm of the detail part of brick b (the children of internal node parent[b]): the
// brick goes through W along each of its three dimensions in LDS; entries with every transformed
// index below k are the scaling block, the others the details.  One workgroup per brick.
template <int K>
__global__ void __launch_bounds__(256) detail_norm_kernel(const double* __restrict__ coef, const int64_t* __restrict__ bricks,
                                                          const int64_t* __restrict__ parent, const double* __restrict__ Wg,
                                                          double* __restrict__ out) {
    constexpr int N = 2 * K;
    constexpr int E = N * N * N;
    __shared__ double A[E], Bf[E], W[N * N];
    __shared__ double part[256 / 64];
    const int64_t b = bricks[blockIdx.x];
    const double* x = coef + b * E;
    for (int e = threadIdx.x; e < E; e += 256) A[e] = x[e];
    for (int e = threadIdx.x; e < N * N; e += 256) W[e] = Wg[e];
    __syncthreads();
    // mode 1: B[r][u2][u3] = sum_u W[r][u] A[u][u2][u3]
    for (int e = threadIdx.x; e < E; e += 256) {
        const int r = e / (N * N), rest = e - r * N * N;
        double s = 0.0;
        for (int u = 0; u < N; ++u) s += W[r * N + u] * A[u * N * N + rest];
        Bf[e] = s;
    }
    __syncthreads();
    // mode 2: A[r1][r][u3] = sum_u W[r][u] B[r1][u][u3]
    for (int e = threadIdx.x; e < E; e += 256) {
        const int r1 = e / (N * N), r = (e / N) % N, u3 = e % N;
        double s = 0.0;
        for (int u = 0; u < N; ++u) s += W[r * N + u] * Bf[(r1 * N + u) * N + u3];
        A[e] = s;
    }
    __syncthreads();
    // mode 3 and the squares of the detail entries
    double acc = 0.0;
    for (int e = threadIdx.x; e < E; e += 256) {
        const int r1 = e / (N * N), r2 = (e / N) % N, r = e % N;
        if (r1 < K && r2 < K && r < K) continue;
        double s = 0.0;
        for (int u = 0; u < N; ++u) s += W[r * N + u] * A[(r1 * N + r2) * N + u];
        acc += s * s;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[parent[blockIdx.x]] = part[0] + part[1] + part[2] + part[3];
}

template <int K>
struct DetailLaunch {
    static void run(hipStream_t st, int64_t n, const double* coef, const int64_t* bricks, const int64_t* parent,
                    const double* W, double* out) {
        detail_norm_kernel<K><<<(unsigned)n, 256, 0, st>>>(coef, bricks, parent, W, out);
    }
};

// Copies brick map[i] of src to brick i of dst, (2k)^3 doubles each.
__global__ void gather_bricks_kernel(int64_t n, int64_t elems, const int64_t* __restrict__ map, const double* __restrict__ src,
                                     double* __restrict__ dst) {
    const int64_t i = blockIdx.y;
    const double* s = src + map[i] * elems;
    double* d = dst + i * elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems; e += (int64_t)gridDim.x * blockDim.x)
        d[e] = s[e];
    (void)n;
}

template <template <int> class Fn, class... Args>
void dispatch(int k, Args&&... args) {
    switch (k) {
        case 1: Fn<1>::run(args...); break;
        case 2: Fn<2>::run(args...); break;
        case 3: Fn<3>::run(args...); break;
        case 4: Fn<4>::run(args...); break;
        case 5: Fn<5>::run(args...); break;
        case 6: Fn<6>::run(args...); break;
        case 7: Fn<7>::run(args...); break;
        case 8: Fn<8>::run(args...); break;
        case 9: Fn<9>::run(args...); break;
        case 10: Fn<10>::run(args...); break;
        default: fail(MWNS_EINVAL, "unsupported k");
    }
}

// ||d||_2^2 of every node (0 at leaves), in node order, on the host.
std::vector<double> detail_norms(mwns_ctx* ctx, const mwns_tree* t) {
    const int k = t->k, N = 2 * k;
    std::vector<double> dn(t->nnodes, 0.0);
    const int64_t nb = t->nbricks - 1;      // bricks of levels 1..depth
    if (nb <= 0) return dn;
    std::vector<double> H(2 * k * k), G(2 * k * k), W(N * N);
    two_scale_filters(k, H.data(), H.data() + k * k);
    wavelet_filters(k, G.data(), G.data() + k * k);
    for (int r = 0; r < k; ++r)
        for (int b = 0; b < k; ++b) {
            W[r * N + b] = H[r * k + b];
            W[r * N + k + b] = H[k * k + r * k + b];
            W[(k + r) * N + b] = G[r * k + b];
            W[(k + r) * N + k + b] = G[k * k + r * k + b];
        }
    std::vector<int64_t> idx(2 * nb);
    for (int64_t b = 0; b < nb; ++b) {
        idx[b] = 1 + b;
        idx[nb + b] = t->brick_parent[1 + b];
    }
    hipStream_t st = ctx->stream;
    DevArray<int64_t> didx(ctx, idx.size());
    DevArray<double> dW(ctx, W.size()), dout(ctx, t->nnodes);
    didx.upload(idx.data(), idx.size(), st);
    dW.upload(W.data(), W.size(), st);
    MWNS_HIP(hipMemsetAsync(dout.p, 0, t->nnodes * sizeof(double), st));
    for (int64_t b0 = 0; b0 < nb; b0 += 1 << 30)
        dispatch<DetailLaunch>(k, st, std::min<int64_t>(nb - b0, 1 << 30), t->coef.p, didx.p + b0, didx.p + nb + b0, dW.p, dout.p);
    MWNS_HIP(hipGetLastError());
    dout.download(dn.data(), dn.size(), st);
    MWNS_HIP(hipStreamSynchronize(st));
    return dn;
}

// t with its internal nodes rebuilt from its leaves by the two-scale decomposition: the redundant
// tree of the function the leaves represent (a tree from an apply holds the assembled partial sums
// of the modified form at its internal nodes, which are not the leaves' coarse projections).
std::unique_ptr<mwns_tree> from_leaves_copy(mwns_ctx* ctx, const mwns_tree* t) {
    std::unique_ptr<mwns_tree> c(new mwns_tree);
    c->ctx = ctx;
    c->hold.set(ctx);
    c->k = t->k;
    c->keys = t->keys;
    c->leaf = t->leaf;
    c->threshold = t->threshold;
    c->min_margin = t->min_margin;
    finalize_structure(c.get());
    c->coef.reset(ctx, t->coef.n);
    MWNS_HIP(hipMemcpyAsync(c->coef.p, t->coef.p, t->coef.n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    DevArray<double> dH = upload_filters(ctx, t->k);
    compress_tree(c.get(), dH.p);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    return c;
}

// The pruned tree of the function that t's leaves represent, within eta (see above); *removed
// receives the removed squared norm.
mwns_tree* prune_tree(mwns_ctx* ctx, const mwns_tree* t0, double eta, double* removed) {
    const std::unique_ptr<mwns_tree> work = from_leaves_copy(ctx, t0);
    const mwns_tree* t = work.get();
    const std::vector<double> dn = detail_norms(ctx, t);
    const int64_t N = t->nnodes;
    std::vector<uint8_t> leaf(t->leaf);
    std::vector<uint8_t> alive(N, 1);
    // children brick of each internal node
    std::vector<int64_t> child_brick(N, -1);
    for (int64_t b = 1; b < t->nbricks; ++b) child_brick[t->brick_parent[b]] = b;
    auto first_child = [&](int64_t node) {   // node index of child 0 of an internal node
        const int64_t b = child_brick[node];
        const int j = key_level(t->keys[node]) + 1;
        return t->lev[j].node_off + 8 * (b - t->lev[j].brick_off);
    };
    const double budget = eta * eta;
    double used = 0.0;
    for (int j = t->depth - 1; j >= 0; --j) {
        const mwns_level& L = t->lev[j];
        std::vector<int64_t> cand;
        for (int64_t i = L.node_off; i < L.node_off + L.nnodes; ++i) {
            if (leaf[i] || !alive[i]) continue;
            const int64_t c0 = first_child(i);
            bool all = true;
            for (int s = 0; s < 8 && all; ++s) all = leaf[c0 + s] != 0;
            if (all) cand.push_back(i);
        }
        std::sort(cand.begin(), cand.end(), [&](int64_t a, int64_t b) {
            return dn[a] != dn[b] ? dn[a] < dn[b] : t->keys[a] < t->keys[b];
        });
        for (int64_t i : cand) {
            if (used + dn[i] > budget) break;
            used += dn[i];
            leaf[i] = 1;
            const int64_t c0 = first_child(i);
            for (int s = 0; s < 8; ++s) alive[c0 + s] = 0;
        }
    }
    std::unique_ptr<mwns_tree> p(new mwns_tree);
    p->ctx = ctx;
    p->hold.set(ctx);
    p->k = t->k;
    p->threshold = t->threshold;
    p->min_margin = t->min_margin;
    std::vector<int64_t> old_of;     // old node index of each kept node
    for (int64_t i = 0; i < N; ++i)
        if (alive[i]) {
            p->keys.push_back(t->keys[i]);
            p->leaf.push_back(leaf[i]);
            old_of.push_back(i);
        }
    finalize_structure(p.get());
    // brick map: the root brick, then every kept sibling group from its child 0 in the old tree
    std::vector<int64_t> map(p->nbricks, 0);
    for (int j = 1; j <= p->depth; ++j) {
        const mwns_level& L = p->lev[j];
        for (int64_t b = 0; b < L.nbricks; ++b) {
            const int64_t old = old_of[L.node_off + 8 * b];
            int64_t ob;
            int child;
            node_brick(t, old, &ob, &child);
            map[L.brick_off + b] = ob;
        }
    }
    hipStream_t st = ctx->stream;
    p->dkeys.reset(ctx, p->nnodes);
    p->dleaf.reset(ctx, p->nnodes);
    p->dkeys.upload(p->keys.data(), p->nnodes, st);
    p->dleaf.upload(p->leaf.data(), p->nnodes, st);
    const int64_t elems = brick_elems(p->k);
    p->coef.reset(ctx, (size_t)p->nbricks * elems);
    DevArray<int64_t> dmap(ctx, map.size());
    dmap.upload(map.data(), map.size(), st);
    for (int64_t b0 = 0; b0 < p->nbricks; b0 += 65535) {
        const int64_t nb = std::min<int64_t>(p->nbricks - b0, 65535);
        gather_bricks_kernel<<<dim3((unsigned)((elems + 255) / 256), (unsigned)nb), 256, 0, st>>>(nb, elems, dmap.p + b0, t->coef.p,
                                                                                              p->coef.p + b0 * elems);
    }
    MWNS_HIP(hipGetLastError());
    MWNS_HIP(hipStreamSynchronize(st));
    if (removed) *removed = used;
    return p.release();
}

// ||f||_2: the root block's norm plus every detail norm (Parseval over the orthonormal basis).
double tree_norm(mwns_ctx* ctx, const mwns_tree* t, const std::vector<double>& dn) {
    const int k = t->k, P = 2 * k;
    std::vector<double> root(brick_elems(k));
    MWNS_HIP(hipMemcpyAsync(root.data(), t->coef.p, root.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b)
            for (int c = 0; c < k; ++c) {
                const double v = root[((int64_t)a * P + b) * P + c];
                s += v * v;
            }
    for (double d : dn) s += d;
    return std::sqrt(s);
}

void check_tree(mwns_ctx* ctx, const mwns_tree* t) {
    if (!ctx || !t) fail(MWNS_EINVAL, "NULL argument");
    if (t->ctx != ctx) fail(MWNS_EINVAL, "tree belongs to another context");
}

}  // namespace
}  // namespace mwns

using namespace mwns;

extern "C" {

mwns_status mwns_tree_detail_norms(mwns_ctx* ctx, const mwns_tree* t, double* out) {
    MWNS_GUARD_BEGIN
    check_tree(ctx, t);
    if (!out) fail(MWNS_EINVAL, "NULL argument");
    const std::vector<double> dn = detail_norms(ctx, from_leaves_copy(ctx, t).get());
    std::copy(dn.begin(), dn.end(), out);
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_prune(mwns_ctx* ctx, const mwns_tree* t, double eta, mwns_tree** out, double* removed) {
    MWNS_GUARD_BEGIN
    check_tree(ctx, t);
    if (!out) fail(MWNS_EINVAL, "NULL argument");
    if (!(eta >= 0.0) || !std::isfinite(eta)) fail(MWNS_EINVAL, "eta must be finite and >= 0");
    *out = prune_tree(ctx, t, eta, removed);
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_discard(mwns_ctx* ctx, const mwns_tree* t, double eps, mwns_tree** out, double* removed) {
    MWNS_GUARD_BEGIN
    check_tree(ctx, t);
    if (!out) fail(MWNS_EINVAL, "NULL argument");
    if (!(eps >= 0.0) || !std::isfinite(eps)) fail(MWNS_EINVAL, "eps must be finite and >= 0");
    const std::unique_ptr<mwns_tree> work = from_leaves_copy(ctx, t);
    const double eta = eps * tree_norm(ctx, work.get(), detail_norms(ctx, work.get()));
    *out = prune_tree(ctx, t, eta, removed);
    return MWNS_OK;
    MWNS_GUARD_END
}

}  // extern "C"
