// Internal declarations of libmwns (HIP, gfx950).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mwns.h"

namespace mwns {

constexpr int KMAX = 10;         // largest basis order (2k <= 16: one MFMA tile per dimension; above: two)
constexpr int KNARROW = 8;       // largest order of the one-tile contraction kernel
constexpr int LF = 7;            // 1-D blocks are tabulated for l = -LF..LF
constexpr int NLF = 2 * LF + 1;
constexpr int LP = 3;            // the plan covers coarse displacements |L_d| <= LP
constexpr int NLP = 2 * LP + 1;
constexpr int NLP3 = NLP * NLP * NLP;
constexpr int MAXLEV = 19;

// Status plumbing -----------------------------------------------------------------------------
void set_error(const std::string& msg);
struct Failure {
    mwns_status st;
    std::string msg;
};
[[noreturn]] void fail(mwns_status st, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define MWNS_HIP(call) ::mwns::check_hip((call), #call)

// Every extern "C" entry point wraps its body in these: no exception crosses the ABI.
#define MWNS_GUARD_BEGIN try {
#define MWNS_GUARD_END                                   \
    }                                                    \
    catch (const Failure& f) {                           \
        set_error(f.msg);                                \
        return f.st;                                     \
    }                                                    \
    catch (const std::bad_alloc&) {                      \
        set_error("host allocation failed");             \
        return MWNS_ENOMEM;                              \
    }                                                    \
    catch (const std::exception& e) {                    \
        set_error(e.what());                             \
        return MWNS_EINVAL;                              \
    }


// Keys ----------------------------------------------------------------------------------------
__host__ __device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x7ffffull;                                     // 19 bits
    v = (v | (v << 32)) & 0x001f00000000ffffull;
    v = (v | (v << 16)) & 0x001f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
__host__ __device__ inline uint64_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x001f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x001f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x7ffffull;
    return v;
}
__host__ __device__ inline uint64_t make_key(int j, int64_t x, int64_t y, int64_t z) {
    return ((uint64_t)j << 57) | spread3((uint64_t)x) | (spread3((uint64_t)y) << 1) | (spread3((uint64_t)z) << 2);
}
__host__ __device__ inline int key_level(uint64_t key) { return (int)(key >> 57); }
__host__ __device__ inline void key_coords(uint64_t key, int64_t* l) {
    uint64_t m = key & ((1ull << 57) - 1);
    l[0] = (int64_t)compact3(m);
    l[1] = (int64_t)compact3(m >> 1);
    l[2] = (int64_t)compact3(m >> 2);
}
// index of key in sorted keys[0..n) or -1
__host__ __device__ inline int64_t find_sorted(const uint64_t* keys, int64_t n, uint64_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && keys[lo] == key) ? lo : -1;
}

// Host-side 1-D tables (App. A.1, A.3, A.4) ---------------------------------------------------
struct Quad {
    std::vector<double> x, w;   // nodes and weights on [0,1]
};
Quad gauss_legendre01(int n);
void legendre_phi(int k, double x, double* out);        // phi_a(x), a < k (no support cut)
void two_scale_filters(int k, double* H0, double* H1);  // k x k row-major
void wavelet_filters(int k, double* G0, double* G1);    // k x k row-major: [[H0 H1], [G0 G1]] orthogonal
void crosscorr_plus_coeffs(int k, double* C);          // C[a][b][n], Phi^+_ab = sum_n C phi_n on [0,1]

// Context / allocation -----------------------------------------------------------------------
}  // namespace mwns

struct mwns_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    mwns_alloc_fn alloc = nullptr;
    mwns_free_fn free_fn = nullptr;
    void* user = nullptr;
    size_t budget = 0;
    size_t in_use = 0;                                  // bytes held: live blocks and the cache
    size_t cached = 0;                                  // bytes of freed blocks kept for reuse
    std::vector<std::pair<size_t, void*>> cache;        // (size class, block), most recent last
    int variant[16] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};   // per basis order k
    int refs = 1;            // the handle itself plus every live tree, operator and plan of the context
    void* pinned = nullptr;  // pinned host staging of the host round trips (hipHostMalloc)
    size_t pinned_bytes = 0;
};

namespace mwns {
void* dalloc(mwns_ctx* ctx, size_t bytes);
void dfree(mwns_ctx* ctx, void* p, size_t bytes);
void release_cache(mwns_ctx* ctx);
// A pinned host block of at least `bytes` for the copies of one host round trip; the caller
// synchronises the stream before the next call (growing the block waits for the stream).
void* pinned_staging(mwns_ctx* ctx, size_t bytes);
// Looks up this GPU's device address of the fixed scratch array of mwns_tree_eval_noalloc (once
// per device; called by mwns_ctx_create with the device current).
void noalloc_scratch_init(int device);
// Drops one reference to ctx; the last one returns the cached blocks and frees the context.
void ctx_release(mwns_ctx* ctx);
// A tree, operator or plan keeps its context alive: declared as the object's first member, it is
// destroyed after every device array of the object has gone back to the context.
struct CtxHold {
    mwns_ctx* ctx = nullptr;
    CtxHold() = default;
    CtxHold(const CtxHold&) = delete;
    CtxHold& operator=(const CtxHold&) = delete;
    void set(mwns_ctx* c) {
        if (c) ++c->refs;
        if (ctx) ctx_release(ctx);
        ctx = c;
    }
    ~CtxHold() {
        if (ctx) ctx_release(ctx);
    }
};
template <class T>
struct DevArray {
    mwns_ctx* ctx = nullptr;
    T* p = nullptr;
    size_t n = 0;
    DevArray() = default;
    DevArray(mwns_ctx* c, size_t count) { reset(c, count); }
    DevArray(const DevArray&) = delete;
    DevArray& operator=(const DevArray&) = delete;
    DevArray(DevArray&& o) noexcept { swap(o); }
    DevArray& operator=(DevArray&& o) noexcept { release(); swap(o); return *this; }
    ~DevArray() { release(); }
    void swap(DevArray& o) { std::swap(ctx, o.ctx); std::swap(p, o.p); std::swap(n, o.n); }
    void reset(mwns_ctx* c, size_t count) {
        release();
        ctx = c;
        n = count;
        p = count ? static_cast<T*>(dalloc(c, count * sizeof(T))) : nullptr;
    }
    void release() {
        if (p) dfree(ctx, p, n * sizeof(T));
        p = nullptr;
        n = 0;
    }
    void upload(const T* h, size_t count, hipStream_t s) {
        if (count) MWNS_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void download(T* h, size_t count, hipStream_t s) const {
        if (count) MWNS_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
};
}  // namespace mwns

// Handles --------------------------------------------------------------------------------------
struct mwns_op {
    mwns::CtxHold hold;
    mwns_ctx* ctx = nullptr;
    int k = 0, M = 0, max_level = 0, group = 1;
    double eps = 0.0, theta = 0.0;
    std::vector<double> tau, w;
    mwns::DevArray<double> F;        // [max_level+1][M][NLF][k][k]
    mwns::DevArray<double> dw;       // [M]
    std::vector<int32_t> plan;       // [max_level+1][NLP^3][2]
    std::vector<double> fro;         // [max_level+1][M][NLF] Frobenius norms of the blocks F^{j;m,l}
    // for the precision routing: a host copy of F (made by the first routed apply) and upper
    // bounds of || sum_{L=lo..hi} |S^{j;m,L}| ||_2 keyed by (j, m, lo, hi, mlo, mhi)
    mutable std::vector<double> Fh;
    mutable std::map<std::array<int, 6>, double> absnorm;
};

struct mwns_level {
    int64_t node_off = 0, nnodes = 0;    // nodes of this level in canonical order
    int64_t brick_off = 0, nbricks = 0;  // sibling groups (bricks) of this level; level 0: 1 virtual brick
};

struct mwns_tree {
    mwns::CtxHold hold;
    mwns_ctx* ctx = nullptr;
    int k = 0, depth = 0;
    int64_t nnodes = 0, nleaves = 0, nbricks = 0;
    double threshold = 0.0, min_margin = 0.0;
    std::vector<mwns_level> lev;
    std::vector<uint64_t> keys;          // canonical order
    std::vector<uint8_t> leaf;
    std::vector<int64_t> brick_parent;   // node index of the parent of each brick (-1 for level 0)
    mwns::DevArray<uint64_t> dkeys;
    mwns::DevArray<uint8_t> dleaf;
    mwns::DevArray<double> coef;         // [nbricks][(2k)^3], brick layout u = s*k + a per dimension
};

namespace mwns {
// Brick layout helpers
inline int64_t brick_elems(int k) { return (int64_t)(2 * k) * (2 * k) * (2 * k); }
// node -> (brick, child); level 0 root -> (0, 0)
inline void node_brick(const mwns_tree* t, int64_t node, int64_t* brick, int* child) {
    int j = key_level(t->keys[node]);
    if (j == 0) { *brick = 0; *child = 0; return; }
    const mwns_level& L = t->lev[j];
    int64_t r = node - L.node_off;
    *brick = L.brick_off + r / 8;
    *child = (int)(r % 8);
}
// builds levels/brick tables from sorted keys + leaf flags (host); throws on malformed trees
void finalize_structure(mwns_tree* t);
// compress internal nodes bottom-up on the device (eq. decomp_scaling, three dimensions)
void compress_tree(mwns_tree* t, const double* dH /* H0,H1 device [2][k][k] */);
DevArray<double> upload_filters(mwns_ctx* ctx, int k);
// structure of the tree with leaves keys[nleaves] (any order); coefficients left to the caller
std::unique_ptr<mwns_tree> skeleton_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* keys,
                                               std::vector<int64_t>* order, std::vector<int64_t>* pos);
}  // namespace mwns
