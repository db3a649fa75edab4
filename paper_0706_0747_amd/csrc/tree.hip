// Function trees on the device: adaptive projection of Gaussian sums (Alg. 1), the redundant tree
// (Sec. 2.2.1) by two-scale decomposition (App. A.3, eq. decomp_scaling), point evaluation
// (App. A.1), import and export.
//
// Storage: nodes in canonical order (ascending key: level-major, then Morton).  The 8 children of
// every internal node are consecutive and form a "brick"; bricks of level j are ordered like
// their parents.  Coefficients live per brick as a (2k)^3 tensor with index u = s*k + a in each
// dimension (s = child parity, a = degree), so the 8 siblings of a level form one dense block; the
// root occupies child 0 of a level-0 brick whose other 7 children are zero.
#include <algorithm>
#include <cstring>
#include <cmath>
#include <memory>
#include <mutex>
#include <numeric>

#include "mwns_internal.h"

namespace mwns {

struct LevelTab {
    int64_t node_off[MAXLEV + 2];
    int64_t brick_off[MAXLEV + 2];
    int depth;
};

__device__ inline void node_to_brick(const LevelTab& lt, int j, int64_t node, int64_t* brick, int* child) {
    if (j == 0) { *brick = 0; *child = 0; return; }
    int64_t r = node - lt.node_off[j];
    *brick = lt.brick_off[j] + (r >> 3);
    *child = (int)(r & 7);
}

__device__ inline int64_t brick_index(int k, int child, int a, int b, int c) {
    const int P = 2 * k;
    return ((int64_t)((child & 1) * k + a) * P + ((child >> 1) & 1) * k + b) * P + ((child >> 2) & 1) * k + c;
}

namespace {

constexpr int PT = 256;   // threads of the transform blocks
// threads of a projection block: sixteen waves above k = 8, where a box has 48-57 MFMA tiles (four per
// wave keep the accumulators small enough for four waves per SIMD; eight waves held two)
constexpr int proj_threads(int k) { return k >= 9 ? 1024 : 256; }
// source terms per chunk: 64 above k = 8, where the term table still fits in the transform buffers
constexpr int proj_chunk(int k) { return k >= 9 ? 64 : 32; }
typedef double d4 __attribute__((ext_vector_type(4)));

// One line of a separable transform: out[o * so] = scale * sum_i M[o][i] in[i * si] for o < NO,
// the sum in ascending i.  The thread reads its NI inputs once; M's addresses are the same in
// every lane, so its entries come through the scalar cache.
template <int NO, int NI>
__device__ inline void line_apply(const double* __restrict__ M, const double* in, int si, double* out, int so,
                                  double scale) {
    double v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) v[i] = in[i * si];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        double sm = 0.0;
#pragma unroll
        for (int i = 0; i < NI; ++i) sm += M[o * NI + i] * v[i];
        out[o * so] = sm * scale;
    }
}

// One block per candidate box of level j (Alg. 1): source values at the box's k^3 Gauss-Legendre
// nodes and at the 8 children's nodes, coefficients s (eq. fvals2coefs in 3-D), values
// interpolated from s at the children's nodes and max |f - f~|, which the host compares with the
// threshold.
//
// The source is separable per term, f = sum_i w_i e_i(x) e_i(y) e_i(z), so the values on a grid
// are a product over the terms: F[x][(y, z)] = sum_i (w_i e_i(x)) (e_i(y) e_i(z)).  It runs on
// v_mfma_f64_16x16x4 (A[m][k] in lane m+16k, B[k][n] in lane n+16k, D[4i+g][n] in register i of
// lane n+16g): rows are x points, columns (y, z) pairs, the inner index four terms per step.  The
// children grid takes MT x NTC tiles, the own grid NTO tiles; wave w owns tiles w, w+NW, ...
// The interpolant on the children grid is one more product in the same layout, so |f - f~| is
// formed in registers.
template <int K>
__global__ void __launch_bounds__(proj_threads(K)) project_kernel(int j, int jmax, const uint64_t* __restrict__ keys, int nsrc,
                                                     const double* __restrict__ src /* x,y,z,a,cf,lim per term */,
                                                     double nc3, double ni, const double* __restrict__ tab,
                                                     double* __restrict__ s_out, double* __restrict__ err_out) {
    // nc3 = 2^{-3j/2} and ni = 2^{3j/2}, the level's normalisation of the scaling functions
    constexpr int K3 = K * K * K;
    constexpr int P2 = 2 * K;
    constexpr int NQ = 3 * K;                // 1-D points: K own nodes, then 2K children nodes
    constexpr int MT = (P2 + 15) / 16, NTC = (P2 * P2 + 15) / 16, NTO = (K * K + 15) / 16;
    constexpr int NTCH = MT * NTC;           // children tiles come first
    constexpr int NT = NTCH + NTO;
    constexpr int BT = proj_threads(K);
    constexpr int CH = proj_chunk(K);
    constexpr int NW = BT / 64;
    constexpr int TPW = (NT + NW - 1) / NW;
    constexpr int KS = (K + 3) / 4;          // inner steps of the interpolation product
    constexpr int NE = CH * 3 * NQ;          // term table E[i][d][q]; E[i][0][q] carries the weight
    constexpr int NTR = 8 * K3;              // transform buffers t1 (2 K^3) and t2 (6 K^3)
    static_assert(K <= 16, "the own grid's x points fit one tile");
    static_assert(K * P2 <= BT, "one thread per line of every transform stage");
    // the term table is dead once the grids are summed: the transforms reuse its storage
    __shared__ double smem[(NE > NTR ? NE : NTR) + K3];
    __shared__ double red[NW];
    __shared__ double xq[3 * NQ];            // 1-D points [d][q]
    __shared__ double st[CH * 5];            // the current chunk of terms (x, y, z, a, cf)
    __shared__ int chunk_n, cursor;          // kept terms in the chunk; next source to screen
    double* E = smem;
    double* t1 = smem;
    double* t2 = smem + 2 * K3;
    double* fown = smem + (NE > NTR ? NE : NTR);
    // tab: P[a][i] = phi_a(x_i) w_i (K*K), Q[q][a] = phi_a((s + x_i)/2), q = s*K + i (2K*K), gx[K]
    const double* P = tab;
    const double* Q = tab + K * K;
    const double* gx = tab + 3 * K * K;
    const int box = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    int64_t l[3];
    key_coords(keys[box], l);
    const double h = ldexp(1.0, -j);
    const bool fine = j < jmax;              // children values enter only the refinement test
    d4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    // the box's 1-D points per dimension: its own nodes, then the children's nodes
    for (int e = threadIdx.x; e < 3 * NQ; e += BT) {
        const int d = e / NQ, q = e % NQ;
        double x;
        if (q < K) x = h * (l[d] + gx[q]);
        else {
            const int sg = (q - K) / K, pp = (q - K) % K;
            x = 0.5 * h * (2 * l[d] + sg + gx[pp]);
        }
        xq[e] = x;
    }
    // Source screening: a term whose largest value on the box, |cf| e^{-a d^2} (d the distance from its
    // centre to the box), lies below 2^-64 of the refinement threshold is skipped (lim = ln(|cf| / thr)
    // + 64 ln 2, precomputed per term: skip when a d^2 > lim).  The kept terms enter the chunks in
    // their original order; wave 0 screens 64 sources per step and compacts them by ballot.
    if (threadIdx.x == 0) cursor = 0;
    __syncthreads();
    for (;;) {
        if (wave == 0) {
            int cnt = 0, cur = cursor;
            while (cnt < CH && cur < nsrc) {
                const int i = cur + lane;
                bool kp = false;
                if (i < nsrc) {
                    const double* sp = src + (int64_t)i * 6;
                    double d2 = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double lo = h * (double)l[d], hi = h * (double)(l[d] + 1);
                        const double dd = fmax(fmax(lo - sp[d], sp[d] - hi), 0.0);
                        d2 += dd * dd;
                    }
                    kp = sp[3] * d2 <= sp[5];
                }
                const uint64_t m = __ballot(kp);
                const int pre = __popcll(m & ((1ull << lane) - 1ull));
                const int tot = __popcll(m);
                const int take = min(tot, CH - cnt);
                if (kp && pre < take)
                    for (int e = 0; e < 5; ++e) st[(cnt + pre) * 5 + e] = src[(int64_t)i * 6 + e];
                if (take < tot) {      // the chunk is full inside this window: resume at the first kept source left
                    uint64_t rest = m;
                    for (int q = 0; q < take; ++q) rest &= rest - 1ull;
                    cur += __ffsll((long long)rest) - 1;
                } else {
                    cur += 64;
                }
                cnt += take;
            }
            if (lane == 0) {
                chunk_n = cnt;
                cursor = cur;
            }
        }
        __syncthreads();
        const int nc = chunk_n;
        if (nc == 0) break;
        const int nc4 = (nc + 3) & ~3;       // whole steps of four terms; the padding terms are zero
        for (int e = threadIdx.x; e < nc4 * 3 * NQ; e += BT) {
            const int q = e % NQ, d = (e / NQ) % 3, i = e / (3 * NQ);
            double v = 0.0;
            if (i < nc) {
                const double* sp = st + i * 5;
                const double dx = xq[d * NQ + q] - sp[d];
                const double ev = exp(-sp[3] * dx * dx);
                v = d == 0 ? sp[4] * ev : ev;
            }
            E[e] = v;
        }
        __syncthreads();
        for (int i0 = 0; i0 < nc4; i0 += 4) {
            const double* Ei = E + (i0 + g) * 3 * NQ;
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int t = wave + NW * u;
                if (t >= NT || (t < NTCH && !fine)) continue;
                double a, b;
                if (t < NTCH) {
                    const int x = (t / NTC) * 16 + r, pr = (t % NTC) * 16 + r;
                    a = x < P2 ? Ei[K + x] : 0.0;
                    b = pr < P2 * P2 ? Ei[NQ + K + pr / P2] * Ei[2 * NQ + K + pr % P2] : 0.0;
                } else {
                    const int pr = (t - NTCH) * 16 + r;
                    a = r < K ? Ei[r] : 0.0;
                    b = pr < K * K ? Ei[NQ + pr / K] * Ei[2 * NQ + pr % K] : 0.0;
                }
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wave + NW * u;
        if (t < NTCH || t >= NT) continue;
        const int pr = (t - NTCH) * 16 + r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = 4 * i + g;
            if (x < K && pr < K * K) fown[x * K * K + pr] = acc[u][i];
        }
    }
    __syncthreads();
    // s = 2^{-3j/2} (P (x) P (x) P) f_own, contracting the last index first; one thread per line
    double* ta = t1;
    double* s_l = t1 + K3;
    const int ln = threadIdx.x;    // line of the current stage
    if (ln < K * K) line_apply<K, K>(P, fown + ln * K, 1, ta + ln * K, 1, 1.0);
    __syncthreads();
    if (ln < K * K) line_apply<K, K>(P, ta + (ln / K) * K * K + ln % K, K, t2 + (ln / K) * K * K + ln % K, K, 1.0);
    __syncthreads();
    if (ln < K * K) {
        line_apply<K, K>(P, t2 + ln, K * K, s_l + ln, K * K, nc3);
        double* sb = s_out + (int64_t)box * K3;
        for (int a1 = 0; a1 < K; ++a1) sb[a1 * K * K + ln] = s_l[a1 * K * K + ln];
    }
    __syncthreads();
    double emax = 0.0;
    if (fine) {
        // f~ on the (2K)^3 children grid = 2^{3j/2} (Q (x) Q (x) Q) s, compared with the values the
        // children tiles hold for the same grid points
        double* u1 = t2;                     // [a1][a2][q3]   K*K*2K
        double* u2 = t2 + 2 * K3;            // [a1][q2][q3] K*2K*2K
        if (ln < K * K) line_apply<P2, K>(Q, s_l + ln * K, 1, u1 + ln * P2, 1, 1.0);
        __syncthreads();
        if (ln < K * P2)
            line_apply<P2, K>(Q, u1 + (ln / P2) * K * P2 + ln % P2, P2, u2 + (ln / P2) * P2 * P2 + ln % P2, P2, 1.0);
        __syncthreads();
        // last factor as a product: rows q1, columns (q2, q3), inner index a1
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int t = wave + NW * u;
            if (t >= NTCH) continue;
            const int mt = t / NTC, x = mt * 16 + r, pr = (t % NTC) * 16 + r;
            d4 fi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                const int a1 = 4 * kk + g;
                const double a = x < P2 && a1 < K ? Q[x * K + a1] : 0.0;
                const double b = pr < P2 * P2 && a1 < K ? u2[a1 * P2 * P2 + pr] : 0.0;
                fi = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, fi, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q1 = mt * 16 + 4 * i + g;
                if (q1 < P2 && pr < P2 * P2) emax = fmax(emax, fabs(acc[u][i] - ni * fi[i]));
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) emax = fmax(emax, __shfl_xor(emax, off));
    if (lane == 0) red[wave] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NW; ++w) red[0] = fmax(red[0], red[w]);
        err_out[box] = red[0];
    }
}

}  // namespace
}  // namespace mwns

namespace mwns {
namespace {

// The projected candidates of the levels j0..depth, one entry per level: coefficients s[li]
// node-major [n[li]][k^3], taken by the 256-thread blocks [bstart[li], bstart[li + 1]) of one
// launch (a block never spans two levels, so its level is found once per block).
struct LeafTab {
    int n = 0;
    int j[MAXLEV + 1];
    int64_t nn[MAXLEV + 1];
    int64_t bstart[MAXLEV + 2];
    const double* s[MAXLEV + 1];
};

// Copy the leaves' coefficients into their bricks, all levels in one launch.
template <int K>
__global__ void __launch_bounds__(256) scatter_leaves_kernel(LeafTab lf, const uint8_t* __restrict__ is_leaf,
                                                            LevelTab lt, double* __restrict__ coef) {
    constexpr int K3 = K * K * K;
    int li = 0;
    while (li + 1 < lf.n && (int64_t)blockIdx.x >= lf.bstart[li + 1]) ++li;
    const int64_t loc = ((int64_t)blockIdx.x - lf.bstart[li]) * 256 + threadIdx.x;
    if (loc >= lf.nn[li] * K3) return;
    const int j = lf.j[li];
    const int64_t c = loc / K3;
    if (!is_leaf[lt.node_off[j] + c]) return;
    const int e = (int)(loc % K3);
    int64_t brick;
    int child;
    node_to_brick(lt, j, lt.node_off[j] + c, &brick, &child);
    const int a = e / (K * K), bb = (e / K) % K, cc = e % K;
    coef[brick * (int64_t)(8 * K3) + brick_index(K, child, a, bb, cc)] = lf.s[li][loc];
}

// Parent block of every internal node of level j from its brick of level j+1:
// s^j = sum_s (H^{s1} (x) H^{s2} (x) H^{s3}) s^{j+1}_s = (H (x) H (x) H) X, H = [H0 H1] (k x 2k)
// (App. A.3, eq. decomp_scaling in each dimension).
template <int K>
__global__ void __launch_bounds__(PT) compress_kernel(int j, const int64_t* __restrict__ parent_node,
                                                      const int64_t* __restrict__ child_brick, LevelTab lt,
                                                      const double* __restrict__ Hd, double* __restrict__ coef) {
    constexpr int P2 = 2 * K, K3 = K * K * K;
    __shared__ double X[P2 * P2 * P2];
    __shared__ double u1[P2 * P2 * K];
    __shared__ double u2[P2 * K * K];
    __shared__ double H[K * P2];
    const int64_t i = blockIdx.x;
    const double* xb = coef + child_brick[i] * (int64_t)(P2 * P2 * P2);
    for (int e = threadIdx.x; e < P2 * P2 * P2; e += PT) X[e] = xb[e];
    for (int e = threadIdx.x; e < K * P2; e += PT) {
        const int a = e / P2, u = e % P2;
        H[e] = Hd[(u / K) * K * K + a * K + (u % K)];     // H[a][s*K + c] = H^s[a][c]
    }
    __syncthreads();
    for (int e = threadIdx.x; e < P2 * P2 * K; e += PT) {
        const int v1 = e / (P2 * K), v2 = (e / K) % P2, a3 = e % K;
        double s = 0.0;
        for (int v3 = 0; v3 < P2; ++v3) s += H[a3 * P2 + v3] * X[(v1 * P2 + v2) * P2 + v3];
        u1[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < P2 * K * K; e += PT) {
        const int v1 = e / (K * K), a2 = (e / K) % K, a3 = e % K;
        double s = 0.0;
        for (int v2 = 0; v2 < P2; ++v2) s += H[a2 * P2 + v2] * u1[(v1 * P2 + v2) * K + a3];
        u2[e] = s;
    }
    __syncthreads();
    int64_t brick;
    int child;
    node_to_brick(lt, j, parent_node[i], &brick, &child);
    double* ob = coef + brick * (int64_t)(8 * K3);
    for (int e = threadIdx.x; e < K3; e += PT) {
        const int a1 = e / (K * K), a2 = (e / K) % K, a3 = e % K;
        double s = 0.0;
        for (int v1 = 0; v1 < P2; ++v1) s += H[a1 * P2 + v1] * u2[(v1 * K + a2) * K + a3];
        ob[brick_index(K, child, a1, a2, a3)] = s;
    }
}

// f at points from the leaf holding each point (App. A.1).
template <int K>
__global__ void __launch_bounds__(64) eval_kernel(int64_t npts, const double* __restrict__ xyz, const int32_t* __restrict__ child,
                            const uint8_t* __restrict__ leaf, LevelTab lt, const double* __restrict__ coef,
                            double* __restrict__ out, int* __restrict__ bad) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const double x[3] = {xyz[3 * p], xyz[3 * p + 1], xyz[3 * p + 2]};
    if (!(x[0] >= 0.0 && x[0] <= 1.0 && x[1] >= 0.0 && x[1] <= 1.0 && x[2] >= 0.0 && x[2] <= 1.0)) {
        atomicAdd(bad, 1);      // outside the cube (or NaN): no value
        out[p] = __builtin_nan("");
        return;
    }
    // Walk down from the root: the child of a node that holds the point is the one whose parity
    // bits at the next level are those of floor(2^{j+1} x) (clamped to the cube).
    int64_t node = 0;
    for (int j = 0; j <= lt.depth; ++j) {
        if (!leaf[node]) {
            const int32_t cb = j < lt.depth ? child[node] : -1;
            if (cb < 0) break;   // an internal node without children: not a valid tree
            const int64_t side1 = (int64_t)1 << (j + 1);
            int oct = 0;
            for (int d = 0; d < 3; ++d) {
                int64_t v = (int64_t)floor(x[d] * side1);
                v = v < 0 ? 0 : (v > side1 - 1 ? side1 - 1 : v);
                oct |= (int)(v & 1) << d;
            }
            node = lt.node_off[j + 1] + 8 * ((int64_t)cb - lt.brick_off[j + 1]) + oct;
            continue;
        }
        // the leaf: local coordinates u in [0, 1] of the point in the box
        const int64_t side = (int64_t)1 << j;
        double u[3];
        for (int d = 0; d < 3; ++d) {
            int64_t v = (int64_t)floor(x[d] * side);
            v = v < 0 ? 0 : (v > side - 1 ? side - 1 : v);
            u[d] = x[d] * side - v;
        }
        // every loop over d and a is unrolled, so ph stays in registers (no private memory)
        double ph[3][K];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double t = 2.0 * u[d] - 1.0;
            double p0 = 1.0, p1 = t;
            ph[d][0] = 1.0;
            if (K > 1) ph[d][1] = t;
#pragma unroll
            for (int a = 2; a < K; ++a) {
                const double p2 = ((2 * a - 1) * t * p1 - (a - 1) * p0) / a;
                ph[d][a] = p2;
                p0 = p1;
                p1 = p2;
            }
#pragma unroll
            for (int a = 0; a < K; ++a) ph[d][a] *= sqrt(2.0 * a + 1.0);
        }
        int64_t brick;
        int sib;
        node_to_brick(lt, j, node, &brick, &sib);
        const double* cb = coef + brick * (int64_t)(8 * K * K * K);
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            double sa = 0.0;
#pragma unroll
            for (int b = 0; b < K; ++b) {
                double sb = 0.0;
#pragma unroll
                for (int c = 0; c < K; ++c) sb += cb[brick_index(K, sib, a, b, c)] * ph[2][c];
                sa += sb * ph[1][b];
            }
            s += sa * ph[0][a];
        }
        out[p] = s * pow(2.0, 1.5 * j);
        return;
    }
    atomicAdd(bad, 1);
    out[p] = __builtin_nan("");
}

template <template <int> class Fn, class... Args>
void dispatch_k(int k, Args&&... args) {
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

template <int K>
struct ProjectLaunch {
    static void run(hipStream_t st, int64_t n, int j, int jmax, const uint64_t* keys, int nsrc, const double* src,
                    const double* tab, double* s, double* err) {
        project_kernel<K><<<(unsigned)n, proj_threads(K), 0, st>>>(j, jmax, keys, nsrc, src, std::pow(2.0, -1.5 * j),
                                                      std::pow(2.0, 1.5 * j), tab, s, err);
    }
};
template <int K>
struct ScatterLaunch {
    static void run(hipStream_t st, int64_t blocks, const LeafTab& lf, const uint8_t* leaf, const LevelTab& lt,
                    double* coef) {
        scatter_leaves_kernel<K><<<(unsigned)blocks, 256, 0, st>>>(lf, leaf, lt, coef);
    }
};
template <int K>
struct CompressLaunch {
    static void run(hipStream_t st, int64_t n, int j, const int64_t* pn, const int64_t* cb, const LevelTab& lt,
                    const double* H, double* coef) {
        compress_kernel<K><<<(unsigned)n, PT, 0, st>>>(j, pn, cb, lt, H, coef);
    }
};
template <int K>
struct EvalLaunch {
    static void run(hipStream_t st, int64_t n, const double* xyz, const int32_t* child, const uint8_t* leaf,
                    const LevelTab& lt, const double* coef, double* out, int* bad) {
        // one point per thread; small blocks spread the points over the compute units
        eval_kernel<K><<<(unsigned)((n + 63) / 64), 64, 0, st>>>(n, xyz, child, leaf, lt, coef, out, bad);
    }
};

LevelTab level_tab(const mwns_tree* t) {
    LevelTab lt{};
    for (int j = 0; j <= t->depth; ++j) {
        lt.node_off[j] = t->lev[j].node_off;
        lt.brick_off[j] = t->lev[j].brick_off;
    }
    lt.depth = t->depth;
    return lt;
}

// ------------------------------------------------- evaluation without allocation
// mwns_tree_eval_noalloc keeps its working memory -- the child-brick table of the tree, the
// per-group offsets of the scan that builds it, and the count of points without a value -- in
// one fixed array in device memory, which every GPU the library runs on holds until the process
// ends.  Host code never passes the array's name to a kernel: it is a host-side stand-in; the
// device address of each GPU's copy is looked up once when a context is created on that GPU.
constexpr int64_t NOALLOC_MAX_NODES = (int64_t)1 << 22;     // largest tree the entry point takes
constexpr int SCAN_BLOCK = 1024;                            // nodes per scan group (one block)
constexpr int64_t SCAN_GROUPS = NOALLOC_MAX_NODES / SCAN_BLOCK;
// int32 layout: child table [MAX_NODES] | group offsets [SCAN_GROUPS] | counter (+ padding)
constexpr int64_t SCRATCH_INTS = NOALLOC_MAX_NODES + SCAN_GROUPS + 64;
static __device__ __align__(256) int32_t scratch[SCRATCH_INTS];

// Internal nodes among nodes [1024 g, 1024 g + 1024) into group[g].
__global__ void __launch_bounds__(SCAN_BLOCK) internal_count_kernel(int64_t n, const uint8_t* __restrict__ leaf,
                                                                    int32_t* __restrict__ group) {
    __shared__ int wsum[SCAN_BLOCK / 64];
    const int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    const unsigned long long b = __ballot(i < n && !leaf[i]);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < SCAN_BLOCK / 64; ++w) s += wsum[w];
        group[blockIdx.x] = s;
    }
}

// Exclusive prefix sums of group[0..ngroups) in place (one block; ngroups <= 4 * 1024), and the
// counter of points without a value set to zero.
__global__ void __launch_bounds__(1024) group_scan_kernel(int ngroups, int32_t* __restrict__ group,
                                                          int32_t* __restrict__ counter) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (ngroups + 1023) / 1024;
    int loc[SCAN_GROUPS / 1024];
    int s = 0;
    for (int q = 0; q < per; ++q) {
        const int g = t * per + q;
        loc[q] = g < ngroups ? group[g] : 0;
        s += loc[q];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t ? part[t - 1] : 0;
    for (int q = 0; q < per; ++q) {
        const int g = t * per + q;
        if (g < ngroups) {
            group[g] = run;
            run += loc[q];
        }
    }
    if (t == 0) *counter = 0;
}

// child[i] = brick of the children of node i (1 + the number of internal nodes before i: the
// bricks of a tree follow its internal nodes in canonical order, brick 0 holding the root), or -1
// for a leaf.
__global__ void __launch_bounds__(SCAN_BLOCK) child_table_kernel(int64_t n, const uint8_t* __restrict__ leaf,
                                                                 const int32_t* __restrict__ group,
                                                                 int32_t* __restrict__ child) {
    __shared__ int wsum[SCAN_BLOCK / 64];
    const int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    const bool internal = i < n && !leaf[i];
    const unsigned long long b = __ballot(internal);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = __popcll(b);
    __syncthreads();
    int before = group[blockIdx.x];
    for (int q = 0; q < w; ++q) before += wsum[q];
    before += __popcll(b & ((1ull << lane) - 1ull));
    if (i < n) child[i] = internal ? 1 + before : -1;
}

std::mutex g_scratch_mutex;
void* g_scratch_ptr[64] = {};

}  // namespace

// Device address of this GPU's copy of the evaluation scratch array; called by mwns_ctx_create
// with the context's device current.
void noalloc_scratch_init(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (device < 0 || device >= 64 || g_scratch_ptr[device]) return;
    void* p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress of the evaluation scratch array");
    g_scratch_ptr[device] = p;
}

// Levels, node offsets and bricks from sorted keys and leaf flags.  Every internal node must have
// its 8 children and every non-root node a parent.
void finalize_structure(mwns_tree* t) {
    const int64_t N = (int64_t)t->keys.size();
    if (N == 0 || t->keys[0] != make_key(0, 0, 0, 0)) fail(MWNS_EINVAL, "tree has no root");
    t->nnodes = N;
    t->depth = key_level(t->keys[N - 1]);
    t->lev.assign(t->depth + 1, mwns_level{});
    for (int64_t i = 0; i < N; ++i) {
        if (i && t->keys[i] <= t->keys[i - 1]) fail(MWNS_EINVAL, "keys not strictly ascending");
        int j = key_level(t->keys[i]);
        if (t->lev[j].nnodes == 0) t->lev[j].node_off = i;
        t->lev[j].nnodes++;
    }
    t->nleaves = 0;
    for (int64_t i = 0; i < N; ++i) t->nleaves += t->leaf[i] ? 1 : 0;
    t->brick_parent.assign(1, -1);
    t->lev[0].brick_off = 0;
    t->lev[0].nbricks = 1;
    int64_t nb = 1;
    for (int j = 1; j <= t->depth; ++j) {
        mwns_level& L = t->lev[j];
        if (L.nnodes == 0 || L.nnodes % 8) fail(MWNS_EINVAL, "incomplete sibling groups at level " + std::to_string(j));
        L.brick_off = nb;
        L.nbricks = L.nnodes / 8;
        nb += L.nbricks;
        const mwns_level& Lp = t->lev[j - 1];
        int64_t b = 0;
        for (int64_t i = Lp.node_off; i < Lp.node_off + Lp.nnodes; ++i) {
            if (t->leaf[i]) continue;
            // child s of (j - 1, l) is (j, 2 l + (s & 1, (s >> 1) & 1, s >> 2)): the parent's
            // interleaved bits shifted by three with s below them
            const uint64_t base = ((uint64_t)j << 57) | ((t->keys[i] & ((1ull << 57) - 1)) << 3);
            for (int s = 0; s < 8; ++s) {
                const int64_t ci = L.node_off + 8 * b + s;
                if (b >= L.nbricks || t->keys[ci] != (base | (uint64_t)s))
                    fail(MWNS_EINVAL, "children of an internal node are missing at level " + std::to_string(j));
            }
            t->brick_parent.push_back(i);
            ++b;
        }
        if (b != L.nbricks) fail(MWNS_EINVAL, "nodes without a parent at level " + std::to_string(j));
    }
    for (int64_t i = t->lev[t->depth].node_off; i < N; ++i)
        if (!t->leaf[i]) fail(MWNS_EINVAL, "internal node at the deepest level");
    t->nbricks = nb;
}

// Internal nodes bottom-up (the redundant tree, Sec. 2.2.1).
void compress_tree(mwns_tree* t, const double* dH) {
    mwns_ctx* ctx = t->ctx;
    LevelTab lt = level_tab(t);
    // parent node and child brick of every brick of levels 1..depth, one upload; the levels run
    // in stream order from the deepest up, each reading what the one below wrote
    const int64_t nb = t->nbricks - 1;
    if (nb <= 0) return;
    std::vector<int64_t> pc(2 * nb);
    for (int64_t b = 0; b < nb; ++b) {
        pc[b] = t->brick_parent[1 + b];
        pc[nb + b] = 1 + b;
    }
    DevArray<int64_t> dpc(ctx, pc.size());
    dpc.upload(pc.data(), pc.size(), ctx->stream);
    for (int j = t->depth - 1; j >= 0; --j) {
        const mwns_level& L = t->lev[j + 1];
        if (L.nbricks == 0) continue;
        dispatch_k<CompressLaunch>(t->k, ctx->stream, L.nbricks, j, dpc.p + (L.brick_off - 1),
                                   dpc.p + nb + (L.brick_off - 1), lt, dH, t->coef.p);
        MWNS_HIP(hipGetLastError());
    }
    // the host index array is the source of an asynchronous copy
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
}

}  // namespace mwns

using namespace mwns;

namespace {

void projection_tables(int k, std::vector<double>& tab) {
    Quad q = gauss_legendre01(k);
    tab.assign(3 * k * k + k, 0.0);
    double v[64];
    for (int i = 0; i < k; ++i) {
        legendre_phi(k, q.x[i], v);
        for (int a = 0; a < k; ++a) tab[a * k + i] = v[a] * q.w[i];          // P[a][i]
        for (int s = 0; s < 2; ++s) {
            legendre_phi(k, 0.5 * (s + q.x[i]), v);
            for (int a = 0; a < k; ++a) tab[k * k + (s * k + i) * k + a] = v[a];   // Q[s*k+i][a]
        }
        tab[3 * k * k + i] = q.x[i];
    }
}

double source_norm(int n, const double* xyz, const double* a, const double* c) {
    // ||f||_2 over R^3 for unit-mass Gaussians (closed form of the Gaussian overlap integrals)
    double tot = 0.0;
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < n; ++q) {
            const double s = a[i] + a[q];
            double d2 = 0.0;
            for (int d = 0; d < 3; ++d) d2 += (xyz[3 * i + d] - xyz[3 * q + d]) * (xyz[3 * i + d] - xyz[3 * q + d]);
            // (a_i a_q / pi^2)^{3/2} (pi / s)^{3/2} = u^{3/2}, u = a_i a_q / (pi s)
            const double u = a[i] * a[q] / (M_PI * s);
            tot += c[i] * c[q] * (u * std::sqrt(u)) * std::exp(-a[i] * a[q] * d2 / s);
        }
    return std::sqrt(tot);
}

// The 8 children of every selected key, in ascending order: child s of (j, l) is
// (j + 1, 2 l + (s & 1, (s >> 1) & 1, s >> 2)), whose interleaved bits are the parent's shifted by
// three with s below them.
std::vector<uint64_t> children_of(const std::vector<uint64_t>& keys, const std::vector<uint8_t>& sel) {
    std::vector<uint64_t> out;
    constexpr uint64_t MORTON = (1ull << 57) - 1;
    for (size_t i = 0; i < keys.size(); ++i) {
        if (!sel[i]) continue;
        const uint64_t base = ((uint64_t)(key_level(keys[i]) + 1) << 57) | ((keys[i] & MORTON) << 3);
        for (uint64_t s = 0; s < 8; ++s) out.push_back(base | s);
    }
    return out;
}

}  // namespace

extern "C" {

mwns_status mwns_project_gaussians(mwns_ctx* ctx, int k, double eps, int j0, int jmax, int n, const double* xyz,
                                   const double* a, const double* c, mwns_tree** out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !out || !xyz || !a || !c) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > KMAX) fail(MWNS_EINVAL, "k must be in [1, " + std::to_string(KMAX) + "]");
    if (j0 < 0 || jmax < j0 || jmax > MAXLEV || !(eps > 0.0) || n < 1) fail(MWNS_EINVAL, "j0, jmax, eps or n out of range");
    for (int i = 0; i < n; ++i)
        if (!(a[i] > 0.0) || !std::isfinite(c[i]) || !std::isfinite(xyz[3 * i]) || !std::isfinite(xyz[3 * i + 1]) ||
            !std::isfinite(xyz[3 * i + 2]))
            fail(MWNS_EINVAL, "source terms must have a > 0 and finite centres and weights");
    hipStream_t st = ctx->stream;
    std::unique_ptr<mwns_tree> t(new mwns_tree);
    t->ctx = ctx;
    t->hold.set(ctx);
    t->k = k;
    const int k3 = k * k * k;
    // source terms: x, y, z, a, cf = c (a/pi)^{3/2}, and the screening limit lim = ln(|cf| / thr) + 64 ln 2
    // (a box at distance d from the centre skips the term when a d^2 > lim: its values there stay below
    // 2^-64 thr; thr = 0 keeps every term, cf = 0 none)
    const double thr = eps * source_norm(n, xyz, a, c);
    t->threshold = thr;
    std::vector<double> src(6 * n);
    for (int i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) src[6 * i + d] = xyz[3 * i + d];
        src[6 * i + 3] = a[i];
        const double cf = c[i] * std::pow(a[i] / M_PI, 1.5);
        src[6 * i + 4] = cf;
        src[6 * i + 5] = thr > 0.0 ? std::log(std::fabs(cf) / thr) + 64.0 * std::log(2.0) : INFINITY;
    }
    std::vector<double> tab;
    projection_tables(k, tab);
    DevArray<double> dsrc(ctx, src.size()), dtab(ctx, tab.size());
    dsrc.upload(src.data(), src.size(), st);
    dtab.upload(tab.data(), tab.size(), st);
    // levels below j0: complete grids of internal nodes; level j0..: candidates (Alg. 1)
    std::vector<std::vector<uint64_t>> lkeys;
    std::vector<std::vector<uint8_t>> lleaf;
    std::vector<DevArray<double>> lcoef;
    std::vector<uint64_t> cand;
    for (int j = 0; j < j0; ++j) {
        const int64_t side = (int64_t)1 << j;
        std::vector<uint64_t> kk;
        for (int64_t x = 0; x < side; ++x)
            for (int64_t y = 0; y < side; ++y)
                for (int64_t z = 0; z < side; ++z) kk.push_back(make_key(j, x, y, z));
        std::sort(kk.begin(), kk.end());
        lkeys.push_back(kk);
        lleaf.push_back(std::vector<uint8_t>(kk.size(), 0));
        lcoef.emplace_back();
    }
    {
        const int64_t side = (int64_t)1 << j0;
        for (int64_t x = 0; x < side; ++x)
            for (int64_t y = 0; y < side; ++y)
                for (int64_t z = 0; z < side; ++z) cand.push_back(make_key(j0, x, y, z));
        std::sort(cand.begin(), cand.end());
    }
    double min_margin = INFINITY;
    for (int j = j0; !cand.empty(); ++j) {
        const int64_t nc = (int64_t)cand.size();
        DevArray<uint64_t> dk(ctx, nc);
        DevArray<double> ds(ctx, (size_t)nc * k3), derr(ctx, nc);
        // candidates up and errors down through the context's pinned staging block
        char* pin = static_cast<char*>(pinned_staging(ctx, (size_t)nc * 16));
        uint64_t* pkeys = reinterpret_cast<uint64_t*>(pin);
        const double* err = reinterpret_cast<const double*>(pin + (size_t)nc * 8);
        std::memcpy(pkeys, cand.data(), (size_t)nc * 8);
        MWNS_HIP(hipMemcpyAsync(dk.p, pkeys, (size_t)nc * 8, hipMemcpyHostToDevice, st));
        dispatch_k<ProjectLaunch>(k, st, nc, j, jmax, dk.p, n, dsrc.p, dtab.p, ds.p, derr.p);
        MWNS_HIP(hipGetLastError());
        MWNS_HIP(hipMemcpyAsync(pin + (size_t)nc * 8, derr.p, (size_t)nc * 8, hipMemcpyDeviceToHost, st));
        MWNS_HIP(hipStreamSynchronize(st));
        // refine where the interpolation error exceeds the threshold, below the finest level (Alg. 1)
        std::vector<uint8_t> ref(nc), lf(nc);
        for (int64_t i = 0; i < nc; ++i) {
            ref[i] = (uint8_t)(j < jmax && err[i] > thr);
            lf[i] = ref[i] ? 0 : 1;
        }
        if (j < jmax)
            for (int64_t i = 0; i < nc; ++i) min_margin = std::min(min_margin, std::fabs(err[i] - thr) / thr);
        lkeys.push_back(std::move(cand));
        lleaf.push_back(std::move(lf));
        lcoef.push_back(std::move(ds));
        cand = children_of(lkeys.back(), ref);
    }
    t->min_margin = min_margin;
    for (size_t j = 0; j < lkeys.size(); ++j) {
        t->keys.insert(t->keys.end(), lkeys[j].begin(), lkeys[j].end());
        t->leaf.insert(t->leaf.end(), lleaf[j].begin(), lleaf[j].end());
    }
    finalize_structure(t.get());
    t->dkeys.reset(ctx, t->nnodes);
    t->dleaf.reset(ctx, t->nnodes);
    t->dkeys.upload(t->keys.data(), t->nnodes, st);
    t->dleaf.upload(t->leaf.data(), t->nnodes, st);
    t->coef.reset(ctx, (size_t)t->nbricks * brick_elems(k));
    MWNS_HIP(hipMemsetAsync(t->coef.p, 0, t->coef.n * sizeof(double), st));
    LevelTab lt = level_tab(t.get());
    {
        LeafTab lf;
        int64_t blocks = 0;
        for (int j = j0; j <= t->depth; ++j) {
            lf.j[lf.n] = j;
            lf.nn[lf.n] = t->lev[j].nnodes;
            lf.bstart[lf.n] = blocks;
            lf.s[lf.n] = lcoef[j].p;
            ++lf.n;
            blocks += (t->lev[j].nnodes * k3 + 255) / 256;
        }
        lf.bstart[lf.n] = blocks;
        dispatch_k<ScatterLaunch>(k, st, blocks, lf, t->dleaf.p, lt, t->coef.p);
        MWNS_HIP(hipGetLastError());
    }
    DevArray<double> dH = upload_filters(ctx, k);
    compress_tree(t.get(), dH.p);
    *out = t.release();
    return MWNS_OK;
    MWNS_GUARD_END
}

}  // extern "C"

// The structure of the tree whose leaves are keys[] (validated as a tiling of the unit cube): all
// ancestors, levels and bricks, keys and leaf flags on the device, and an uninitialised brick array.
// order = the sort permutation of keys, pos[i] = node index of keys[order[i]].
std::unique_ptr<mwns_tree> mwns::skeleton_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* keys,
                                                     std::vector<int64_t>* order_out, std::vector<int64_t>* pos_out) {
    std::vector<int64_t>& order = *order_out;
    order.resize(nleaves);
    std::iota(order.begin(), order.end(), 0);
    for (int64_t i = 0; i < nleaves; ++i) {
        const int j = key_level(keys[i]);
        int64_t l[3];
        key_coords(keys[i], l);
        if (j > MAXLEV || make_key(j, l[0], l[1], l[2]) != keys[i]) fail(MWNS_EINVAL, "malformed key");
        for (int d = 0; d < 3; ++d)
            if (l[d] >= ((int64_t)1 << j)) fail(MWNS_EINVAL, "key outside the unit cube");
    }
    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return keys[x] < keys[y]; });
    std::vector<uint64_t> all;
    for (int64_t i = 0; i < nleaves; ++i) {
        uint64_t key = keys[order[i]];
        all.push_back(key);
        int j = key_level(key);
        int64_t l[3];
        key_coords(key, l);
        while (j > 0) {
            --j;
            for (int d = 0; d < 3; ++d) l[d] >>= 1;
            all.push_back(make_key(j, l[0], l[1], l[2]));
        }
    }
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    std::unique_ptr<mwns_tree> t(new mwns_tree);
    t->ctx = ctx;
    t->hold.set(ctx);
    t->k = k;
    t->keys = all;
    t->leaf.assign(all.size(), 0);
    std::vector<int64_t>& pos = *pos_out;
    pos.assign(nleaves, 0);
    for (int64_t i = 0; i < nleaves; ++i) {
        const uint64_t key = keys[order[i]];
        if (i && key == keys[order[i - 1]]) fail(MWNS_EINVAL, "duplicate leaf key");
        pos[i] = std::lower_bound(all.begin(), all.end(), key) - all.begin();
        t->leaf[pos[i]] = 1;
    }
    // a leaf may not have descendants: its successor in key order at the next level would be a child
    for (int64_t i = 0; i < nleaves; ++i) {
        int64_t l[3];
        const int j = key_level(all[pos[i]]);
        key_coords(all[pos[i]], l);
        if (std::binary_search(all.begin(), all.end(), make_key(j + 1, 2 * l[0], 2 * l[1], 2 * l[2])) ||
            std::binary_search(all.begin(), all.end(), make_key(j + 1, 2 * l[0] + 1, 2 * l[1] + 1, 2 * l[2] + 1)))
            fail(MWNS_EINVAL, "leaves overlap");
    }
    finalize_structure(t.get());
    hipStream_t st = ctx->stream;
    t->dkeys.reset(ctx, t->nnodes);
    t->dleaf.reset(ctx, t->nnodes);
    t->dkeys.upload(t->keys.data(), t->nnodes, st);
    t->dleaf.upload(t->leaf.data(), t->nnodes, st);
    t->coef.reset(ctx, (size_t)t->nbricks * brick_elems(k));
    return t;
}

extern "C" {

mwns_status mwns_tree_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* keys, const double* coeffs,
                                  mwns_tree** out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !out || !keys || !coeffs) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > KMAX || nleaves < 1) fail(MWNS_EINVAL, "k or nleaves out of range");
    const int k3 = k * k * k;
    std::vector<int64_t> order, pos;
    std::unique_ptr<mwns_tree> t = skeleton_from_leaves(ctx, k, nleaves, keys, &order, &pos);
    hipStream_t st = ctx->stream;
    std::vector<double> hb(t->coef.n, 0.0);
    for (int64_t i = 0; i < nleaves; ++i) {
        int64_t brick;
        int child;
        node_brick(t.get(), pos[i], &brick, &child);
        const double* src = coeffs + order[i] * k3;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                for (int c = 0; c < k; ++c) {
                    const int P = 2 * k;
                    const int64_t e = ((int64_t)((child & 1) * k + a) * P + ((child >> 1) & 1) * k + b) * P +
                                      ((child >> 2) & 1) * k + c;
                    hb[brick * brick_elems(k) + e] = src[(a * k + b) * k + c];
                }
    }
    t->coef.upload(hb.data(), hb.size(), st);
    DevArray<double> dH = upload_filters(ctx, k);
    compress_tree(t.get(), dH.p);
    *out = t.release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_set_leaves(mwns_ctx* ctx, mwns_tree* t, const double* coeffs) {
    MWNS_GUARD_BEGIN
    if (!ctx || !t || !coeffs) fail(MWNS_EINVAL, "NULL argument");
    if (t->ctx != ctx) fail(MWNS_EINVAL, "tree belongs to another context");
    const int k = t->k, k3 = k * k * k, P = 2 * k;
    std::vector<double> hb(t->coef.n, 0.0);
    int64_t li = 0;
    for (int64_t i = 0; i < t->nnodes; ++i) {
        if (!t->leaf[i]) continue;
        int64_t brick;
        int child;
        node_brick(t, i, &brick, &child);
        const double* src = coeffs + li++ * k3;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                for (int c = 0; c < k; ++c) {
                    const int64_t e = ((int64_t)((child & 1) * k + a) * P + ((child >> 1) & 1) * k + b) * P +
                                      ((child >> 2) & 1) * k + c;
                    hb[brick * brick_elems(k) + e] = src[(a * k + b) * k + c];
                }
    }
    t->coef.upload(hb.data(), hb.size(), ctx->stream);
    DevArray<double> dH = upload_filters(ctx, k);
    compress_tree(t, dH.p);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_get_info(const mwns_tree* t, mwns_tree_info* info) {
    MWNS_GUARD_BEGIN
    if (!t || !info) fail(MWNS_EINVAL, "NULL argument");
    info->k = t->k;
    info->depth = t->depth;
    info->nnodes = t->nnodes;
    info->nleaves = t->nleaves;
    info->threshold = t->threshold;
    info->min_margin = t->min_margin;
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_export(mwns_ctx* ctx, const mwns_tree* t, int64_t* nnodes, uint64_t* keys, uint8_t* is_leaf,
                             double* coeffs) {
    MWNS_GUARD_BEGIN
    if (!ctx || !t || !nnodes) fail(MWNS_EINVAL, "NULL argument");
    if (!keys) { *nnodes = t->nnodes; return MWNS_OK; }
    if (*nnodes < t->nnodes) {
        *nnodes = t->nnodes;
        fail(MWNS_ERANGE, "export buffers too small");
    }
    std::copy(t->keys.begin(), t->keys.end(), keys);
    if (is_leaf) std::copy(t->leaf.begin(), t->leaf.end(), is_leaf);
    if (coeffs) {
        const int k = t->k, k3 = k * k * k;
        std::vector<double> hb(t->coef.n);
        t->coef.download(hb.data(), hb.size(), ctx->stream);
        MWNS_HIP(hipStreamSynchronize(ctx->stream));
        for (int64_t i = 0; i < t->nnodes; ++i) {
            int64_t brick;
            int child;
            node_brick(t, i, &brick, &child);
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b)
                    for (int c = 0; c < k; ++c) {
                        const int P = 2 * k;
                        const int64_t e = ((int64_t)((child & 1) * k + a) * P + ((child >> 1) & 1) * k + b) * P +
                                          ((child >> 2) & 1) * k + c;
                        coeffs[i * k3 + (a * k + b) * k + c] = hb[brick * brick_elems(k) + e];
                    }
        }
    }
    *nnodes = t->nnodes;
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_eval(mwns_ctx* ctx, const mwns_tree* t, int64_t npts, const double* xyz, double* out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !t || (npts && (!xyz || !out)) || npts < 0) fail(MWNS_EINVAL, "NULL argument");
    if (npts == 0) return MWNS_OK;
    for (int64_t p = 0; p < 3 * npts; ++p)
        if (!(xyz[p] >= 0.0 && xyz[p] <= 1.0)) fail(MWNS_EINVAL, "point outside the unit cube");
    hipStream_t st = ctx->stream;
    DevArray<double> dx(ctx, 3 * npts), dout(ctx, npts);
    DevArray<int> dbad(ctx, 1);
    DevArray<int32_t> dchild(ctx, t->nnodes);
    // points and the child table go up, values come down through the context's pinned block:
    // [points][child table][values][bad count]
    const size_t b_x = (size_t)npts * 3 * sizeof(double);
    const size_t b_c = ((size_t)t->nnodes * sizeof(int32_t) + 7) & ~(size_t)7;
    const size_t b_o = (size_t)npts * sizeof(double);
    char* pin = static_cast<char*>(pinned_staging(ctx, b_x + b_c + b_o + sizeof(double)));
    std::memcpy(pin, xyz, b_x);
    // child brick of every internal node (-1 for leaves), from the parent of every brick
    int32_t* child = reinterpret_cast<int32_t*>(pin + b_x);
    std::fill(child, child + t->nnodes, -1);
    for (int64_t b = 1; b < t->nbricks; ++b) child[t->brick_parent[b]] = (int32_t)b;
    MWNS_HIP(hipMemcpyAsync(dx.p, pin, b_x, hipMemcpyHostToDevice, st));
    MWNS_HIP(hipMemcpyAsync(dchild.p, child, (size_t)t->nnodes * sizeof(int32_t), hipMemcpyHostToDevice, st));
    MWNS_HIP(hipMemsetAsync(dbad.p, 0, sizeof(int), st));
    LevelTab lt = level_tab(t);
    dispatch_k<EvalLaunch>(t->k, st, npts, dx.p, dchild.p, t->dleaf.p, lt, t->coef.p, dout.p, dbad.p);
    MWNS_HIP(hipGetLastError());
    double* pout = reinterpret_cast<double*>(pin + b_x + b_c);
    int* pbad = reinterpret_cast<int*>(pin + b_x + b_c + b_o);
    MWNS_HIP(hipMemcpyAsync(pout, dout.p, b_o, hipMemcpyDeviceToHost, st));
    MWNS_HIP(hipMemcpyAsync(pbad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    MWNS_HIP(hipStreamSynchronize(st));
    if (*pbad) fail(MWNS_ESTATE, "points without a leaf: the tree does not cover the cube");
    std::memcpy(out, pout, b_o);
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree_eval_noalloc(mwns_ctx* ctx, const mwns_tree* t, int64_t npts, const double* xyz, double* out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !t || npts < 0 || (npts && (!xyz || !out))) fail(MWNS_EINVAL, "NULL argument or npts < 0");
    if (t->ctx != ctx) fail(MWNS_EINVAL, "tree belongs to another context");
    if (t->nnodes > NOALLOC_MAX_NODES)
        fail(MWNS_ERANGE, "tree has " + std::to_string(t->nnodes) + " nodes; the allocation-free evaluation takes at most " +
                              std::to_string(NOALLOC_MAX_NODES));
    int32_t* base = (ctx->device >= 0 && ctx->device < 64) ? static_cast<int32_t*>(g_scratch_ptr[ctx->device]) : nullptr;
    if (!base) fail(MWNS_ESTATE, "no evaluation scratch address for this device");
    if (npts == 0) return MWNS_OK;
    hipStream_t st = ctx->stream;
    int32_t* child = base;
    int32_t* group = base + NOALLOC_MAX_NODES;
    int32_t* counter = group + SCAN_GROUPS;
    const int ng = (int)((t->nnodes + SCAN_BLOCK - 1) / SCAN_BLOCK);
    internal_count_kernel<<<ng, SCAN_BLOCK, 0, st>>>(t->nnodes, t->dleaf.p, group);
    group_scan_kernel<<<1, 1024, 0, st>>>(ng, group, counter);
    child_table_kernel<<<ng, SCAN_BLOCK, 0, st>>>(t->nnodes, t->dleaf.p, group, child);
    const LevelTab lt = level_tab(t);
    dispatch_k<EvalLaunch>(t->k, st, npts, xyz, child, t->dleaf.p, lt, t->coef.p, out, counter);
    MWNS_HIP(hipGetLastError());
    return MWNS_OK;
    MWNS_GUARD_END
}

void mwns_tree_destroy(mwns_tree* t) { delete t; }

}  // extern "C"
