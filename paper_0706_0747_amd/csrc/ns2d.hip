// The d = 2 version of the modified ns-form apply (Alg. 3, written in the paper for d = 2; Sec. 6.1
// notes the apply exists for d = 2 as well): the plane's kernels of (-Delta + mu^2)^(-alpha) as
// Gaussian sums, the screening of Sec. 4 with two factors, Alg. 1 with four children, the apply of
// eq. apply_algo on quadtrees, assembly and evaluation.
//
//   * fit (host FP64): K(r) = C2 int exp(-r^2 e^{2s} - mu^2 e^{-2s}/4 + (2 - 2 alpha) s) ds,
//     C2 = 2^{1 - 2 alpha} / (pi Gamma(alpha)) (Sec. 3's representation in two dimensions); the
//     trapezoidal rule s_m = A + m h; accuracy relative to K itself on [delta, R].
//   * operator: the 1-D blocks F^{j;m,l} are those of the 3-D operator (eq. KernelFactor does not
//     depend on the dimension) and come from its device builder; the plan: theta = eps sum_m w_m
//     ||F^{0;m,0}||_F^2, per L the estimate 1/2 sym[N_dif N_F + N_upF N_dif] of eq.
//     NormEstimateUsing1DBlocks with two factors, term ranges as in 3-D (prefix and suffix below
//     theta/2 dropped, empty below theta), grouped by the number of |L_d| > 1.
//   * projection (Alg. 1): a box is refined when f and the box's polynomial differ by more than
//     eps ||f||_2 at some child's k x k Gauss-Legendre nodes; compression (eq. decomp_scaling).
//   * apply: every node of f's tree (Alg. 3 Step 1), fine displacements l in [-7, 7]^2 with the input
//     inside the square, terms R_j(L) with + and, at internal nodes, R_{j+1}(l) with - (their common
//     part cancels and is skipped); inputs missing from the tree by zero-detail reconstruction from
//     the nearest ancestor (Step 2); per term y += c w_m F^{j;m,l1} X F^{j;m,l2}^T (Step 3); assembly
//     from the root (Step 4, eq. g_assemble).
// Keys: level << 57 | morton(x, y) with x in bit 0; blocks [k][k], a = degree in x, b = degree in y.
#include <algorithm>
#include <cmath>
#include <exception>
#include <memory>
#include <thread>
#include <unordered_map>

#include "mwns_internal.h"

namespace mwns {
namespace {

constexpr int K2MAX = 10;
constexpr int MAXLEV2 = MAXLEV;        // the 1-D blocks' builder covers scales 0..19
constexpr int LP2 = 3, NLP2 = 7;

__host__ __device__ inline uint64_t spread2(uint64_t v) {
    v &= 0xfffffffull;                                   // 28 bits
    v = (v | (v << 16)) & 0x0000ffff0000ffffull;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}
__host__ __device__ inline uint64_t compact2(uint64_t v) {
    v &= 0x5555555555555555ull;
    v = (v ^ (v >> 1)) & 0x3333333333333333ull;
    v = (v ^ (v >> 2)) & 0x0f0f0f0f0f0f0f0full;
    v = (v ^ (v >> 4)) & 0x00ff00ff00ff00ffull;
    v = (v ^ (v >> 8)) & 0x0000ffff0000ffffull;
    v = (v ^ (v >> 16)) & 0x00000000ffffffffull;
    return v;
}
__host__ __device__ inline uint64_t key2(int j, int64_t x, int64_t y) {
    return ((uint64_t)j << 57) | spread2((uint64_t)x) | (spread2((uint64_t)y) << 1);
}
inline int key2_level(uint64_t k) { return (int)(k >> 57); }
inline void key2_xy(uint64_t k, int64_t* x, int64_t* y) {
    const uint64_t m = k & ((1ull << 57) - 1);
    *x = (int64_t)compact2(m);
    *y = (int64_t)compact2(m >> 1);
}

__device__ inline void phi2_dev(int k, double x, double* out) {
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

__device__ double gsum2(double x, double y, int ng, const double* __restrict__ g) {
    // g: [ng][4] = (x_i, y_i, a_i, c_i); f = sum c_i (a_i / pi) exp(-a_i |p - p_i|^2)
    double f = 0.0;
    for (int i = 0; i < ng; ++i) {
        const double dx = x - g[4 * i], dy = y - g[4 * i + 1], a = g[4 * i + 2];
        f += g[4 * i + 3] * (a * M_1_PI) * exp(-a * (dx * dx + dy * dy));
    }
    return f;
}

// One workgroup of 256 threads per candidate box (j, x, y): values at the box's k x k nodes and at
// the children's 4 k^2 nodes, the box's coefficients s_ab = 2^-j sum w_q w_r f phi_a(x_q) phi_b(x_r),
// and the largest |f - polynomial| over the children's nodes.
__global__ void project2_kernel(int k, int j, const int64_t* __restrict__ cand, int ng, const double* __restrict__ g,
                                const double* __restrict__ xq, const double* __restrict__ wq,
                                const double* __restrict__ phiq, const double* __restrict__ phich,
                                double* __restrict__ coef, double* __restrict__ err) {
    __shared__ double fv[5 * K2MAX * K2MAX], s[K2MAX * K2MAX], red[256];
    const int64_t bx = cand[2 * blockIdx.x], by = cand[2 * blockIdx.x + 1];
    const double h = ldexp(1.0, -j);
    const int kk = k * k;
    for (int t = threadIdx.x; t < 5 * kk; t += blockDim.x) {
        double x, y;
        if (t < kk) {
            x = h * ((double)bx + xq[t / k]);
            y = h * ((double)by + xq[t % k]);
        } else {
            const int c = (t - kk) / kk, q = ((t - kk) % kk) / k, r = (t - kk) % k;
            x = 0.5 * h * ((double)(2 * bx + (c & 1)) + xq[q]);
            y = 0.5 * h * ((double)(2 * by + (c >> 1)) + xq[r]);
        }
        fv[t] = gsum2(x, y, ng, g);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kk; t += blockDim.x) {
        const int a = t / k, b = t % k;
        double acc = 0.0;
        for (int q = 0; q < k; ++q)
            for (int r = 0; r < k; ++r) acc += wq[q] * wq[r] * fv[q * k + r] * phiq[q * k + a] * phiq[r * k + b];
        s[t] = h * acc;
        coef[(int64_t)blockIdx.x * kk + t] = h * acc;
    }
    __syncthreads();
    double m = 0.0;
    for (int t = threadIdx.x; t < 4 * kk; t += blockDim.x) {
        const int c = t / kk, q = (t % kk) / k, r = t % k;
        const double* px = phich + ((c & 1) * k + q) * k;
        const double* py = phich + ((c >> 1) * k + r) * k;
        double v = 0.0;
        for (int a = 0; a < k; ++a) {
            double u = 0.0;
            for (int b = 0; b < k; ++b) u += s[a * k + b] * py[b];
            v += px[a] * u;
        }
        m = fmax(m, fabs(v / h - fv[kk + t]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) err[blockIdx.x] = red[0];
}

// parent = sum_{sx,sy} H^(sx) child H^(sy)^T; one thread per (parent, a, b); ch: the four children's
// node indices in child order s = sx + 2 sy
__global__ void compress2_kernel(int k, int n, const int64_t* __restrict__ par, const int64_t* __restrict__ ch,
                                 const double* __restrict__ H, double* __restrict__ coef) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = k * k;
    if (i >= n * kk) return;
    const int p = i / kk, a = (i % kk) / k, b = i % k;
    double acc = 0.0;
    for (int s = 0; s < 4; ++s) {
        const double* C = coef + ch[4 * p + s] * kk;
        const double* Hx = H + (s & 1) * kk;
        const double* Hy = H + (s >> 1) * kk;
        for (int c = 0; c < k; ++c) {
            double u = 0.0;
            for (int d = 0; d < k; ++d) u += C[c * k + d] * Hy[b * k + d];
            acc += Hx[a * k + c] * u;
        }
    }
    coef[par[p] * kk + (a * k + b)] = acc;
}

// Input blocks: from node anc, up steps of zero-detail reconstruction s <- H^(sx)^T s H^(sy) with
// the path bits of (x, y) from the top.  One workgroup of 128 threads per block.
__global__ void gather2_kernel(int k, const int64_t* __restrict__ anc, const int* __restrict__ up,
                               const int64_t* __restrict__ xy, const double* __restrict__ H,
                               const double* __restrict__ f, double* __restrict__ X) {
    __shared__ double s[K2MAX * K2MAX], t[K2MAX * K2MAX];
    const int i = blockIdx.x, kk = k * k;
    for (int e = threadIdx.x; e < kk; e += blockDim.x) s[e] = f[anc[i] * kk + e];
    __syncthreads();
    for (int step = up[i]; step > 0; --step) {
        const int sx = (int)((xy[2 * i] >> (step - 1)) & 1), sy = (int)((xy[2 * i + 1] >> (step - 1)) & 1);
        const double* Hx = H + sx * kk;
        const double* Hy = H + sy * kk;
        for (int e = threadIdx.x; e < kk; e += blockDim.x) {
            const int a = e / k, b = e % k;
            double acc = 0.0;
            for (int c = 0; c < k; ++c) {
                double u = 0.0;
                for (int d = 0; d < k; ++d) u += s[c * k + d] * Hy[d * k + b];
                acc += Hx[c * k + a] * u;
            }
            t[e] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kk; e += blockDim.x) s[e] = t[e];
        __syncthreads();
    }
    for (int e = threadIdx.x; e < kk; e += blockDim.x) X[(int64_t)i * kk + e] = s[e];
}

// Job: input block, fine displacement (l1, l2), inclusive term range, sign.
struct Job2 {
    int64_t in;
    int l1, l2, m1, m2, sign, pad;
};

// Orders 9, 10: one workgroup per output node: for each job and term, T = X F2^T, then
// y += c w_m F1 T, with F1 = F^{j;m,l1}, F2 = F^{j;m,l2} (row = output degree); jobs and terms in a
// fixed order.
__global__ void contract2_kernel(int k, int M, const int* __restrict__ nlev, const int64_t* __restrict__ off,
                                 const Job2* __restrict__ jobs, const double* __restrict__ F, const double* __restrict__ w,
                                 const double* __restrict__ X, double* __restrict__ out) {
    __shared__ double xs[K2MAX * K2MAX], ts[K2MAX * K2MAX];
    const int node = blockIdx.x, kk = k * k, e = threadIdx.x;
    const int a = e / k, b = e % k;
    const int j = nlev[node];
    double acc = 0.0;
    for (int64_t q = off[node]; q < off[node + 1]; ++q) {
        const Job2 jb = jobs[q];
        __syncthreads();
        if (e < kk) xs[e] = X[jb.in * kk + e];
        for (int m = jb.m1; m <= jb.m2; ++m) {
            const double* F1 = F + (((int64_t)j * M + m) * 15 + (jb.l1 + 7)) * kk;
            const double* F2 = F + (((int64_t)j * M + m) * 15 + (jb.l2 + 7)) * kk;
            __syncthreads();
            if (e < kk) {
                double u = 0.0;
                for (int d = 0; d < k; ++d) u += xs[a * k + d] * F2[b * k + d];
                ts[e] = u;
            }
            __syncthreads();
            if (e < kk) {
                double v = 0.0;
                for (int c = 0; c < k; ++c) v += F1[a * k + c] * ts[c * k + b];
                acc += jb.sign * w[m] * v;
            }
        }
    }
    if (e < kk) out[(int64_t)node * kk + e] = acc;
}

// Orders k <= 8 (k^2 <= 64): one wavefront per output node, four nodes per workgroup, no workgroup
// barriers.  Lane e = a k + b holds y[a][b]; per job the lane keeps row a of X (gathered by lane
// shuffles).  The blocks F1 and F2 of four terms at a time go to the wave's own LDS region (lane e
// loads element e of each; the next four terms' blocks are loaded into registers while these are
// used); per term the lane forms T[a][b] = sum_d X[a][d] F2[b][d] and reads column b of T from
// lanes c k + b by shuffles for y[a][b] += c w sum_c F1[a][c] T[c][b].  Lanes e >= k^2 compute on row
// and column 0 and write nothing.
template <int K>
__global__ void __launch_bounds__(256) contract2_wave_kernel(int n, int M, const int* __restrict__ nlev,
                                                             const int64_t* __restrict__ off, const Job2* __restrict__ jobs,
                                                             const double* __restrict__ F, const double* __restrict__ w,
                                                             const double* __restrict__ X, double* __restrict__ out) {
    constexpr int KK = K * K, C = 4;
    __shared__ double fs[4][2][C][KK];
    const int wv = threadIdx.x >> 6;
    const int node = blockIdx.x * 4 + wv;
    if (node >= n) return;                          // whole waves only: no workgroup barrier below
    const int e = threadIdx.x & 63;
    const bool act = e < KK;
    const int a = act ? e / K : 0, b = act ? e % K : 0;
    const int j = nlev[node];
    const int64_t stride = (int64_t)15 * KK;        // from term m to m + 1
    double (*f1s)[KK] = fs[wv][0];
    double (*f2s)[KK] = fs[wv][1];
    double acc = 0.0;
    for (int64_t q = off[node]; q < off[node + 1]; ++q) {
        const Job2 jb = jobs[q];
        const double x = X[jb.in * KK + (act ? e : 0)];
        double xr[K];
#pragma unroll
        for (int d = 0; d < K; ++d) xr[d] = __shfl(x, a * K + d);
        const double* F1b = F + (((int64_t)j * M) * 15 + (jb.l1 + 7)) * KK + (act ? e : 0);
        const double* F2b = F + (((int64_t)j * M) * 15 + (jb.l2 + 7)) * KK + (act ? e : 0);
        double p1[C], p2[C];
        auto fetch = [&](int m0) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int m = m0 + c <= jb.m2 ? m0 + c : jb.m2;
                p1[c] = F1b[m * stride];
                p2[c] = F2b[m * stride];
            }
        };
        fetch(jb.m1);
        for (int m0 = jb.m1; m0 <= jb.m2; m0 += C) {
            __builtin_amdgcn_wave_barrier();         // the previous chunk's reads of this region are done
#pragma unroll
            for (int c = 0; c < C; ++c) {
                f1s[c][e < KK ? e : 0] = p1[c];
                f2s[c][e < KK ? e : 0] = p2[c];
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);      // lgkmcnt(0): this wave's LDS writes are done
            __builtin_amdgcn_wave_barrier();
            if (m0 + C <= jb.m2) fetch(m0 + C);
            const int nc = jb.m2 - m0 + 1 < C ? jb.m2 - m0 + 1 : C;
            for (int c = 0; c < nc; ++c) {
                double t = 0.0;
#pragma unroll
                for (int d = 0; d < K; ++d) t += xr[d] * f2s[c][b * K + d];
                double v = 0.0;
#pragma unroll
                for (int cc = 0; cc < K; ++cc) v += f1s[c][a * K + cc] * __shfl(t, cc * K + b);
                acc += jb.sign * w[m0 + c] * v;
            }
        }
    }
    if (act) out[(int64_t)node * KK + e] = acc;
}

// Orders 5..8 on the matrix cores: one workgroup of four wavefronts per output node; wave w takes
// the (job, term) pairs of the node whose running index is w mod 4, and the four partial sums are
// added in wave order at the end.  The k x k blocks are padded to 8 x 8 (zeros) and cut into 2 x 2
// blocks of 4 x 4, one per block of the four-block v_mfma_f64_4x4x4 (A[i][k] of block b in lane
// i + 4b + 16k, B[k][j] in lane j + 4b + 16k, D[i][j] in lane j + 4b + 16i); block b = 2 bi + bj is the
// output block (rows 4 bi.., columns 4 bj..), and lane (x, b, y) = x + 4b + 16y.  Per job the lane
// holds X[4 bi + x][4 kk + y] (kk = 0, 1); per term, with the wave's next term of the job loaded
// meanwhile:
//   T = X F2^T in two steps kk (B = F2[4 bj + x][4 kk + y]), which leaves T[4 bi + y][4 bj + x] in
//   the lane;
//   y += c w F1 T in two steps kk (A = c w F1[4 bi + x][4 kk + y], B = T[4 kk + y][4 bj + x], taken
//   by a shuffle from the lane of block (kk, bj)).
template <int K>
__global__ void __launch_bounds__(256) contract2_mfma_kernel(int n, int M, const int* __restrict__ nlev,
                                                             const int64_t* __restrict__ off, const Job2* __restrict__ jobs,
                                                             const double* __restrict__ F, const double* __restrict__ w,
                                                             const double* __restrict__ X, double* __restrict__ out) {
    static_assert(K > 4 && K <= 8, "two 4 x 4 blocks per dimension");
    constexpr int KK = K * K, NW = 4;
    __shared__ double part[NW][64];
    const int node = blockIdx.x;
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int x = lane & 3, bk = (lane >> 2) & 3, y = lane >> 4;
    const int bi = bk >> 1, bj = bk & 1;
    const int ra = 4 * bi + x, rb = 4 * bj + x;     // rows of the A operands (X, F1) and of F2
    const bool va0 = ra < K && y < K, va1 = ra < K && 4 + y < K;
    const bool vb0 = rb < K && y < K, vb1 = rb < K && 4 + y < K;
    const int oa0 = va0 ? ra * K + y : 0, oa1 = va1 ? ra * K + 4 + y : 0;
    const int ob0 = vb0 ? rb * K + y : 0, ob1 = vb1 ? rb * K + 4 + y : 0;
    const int s0 = x + 4 * bj + 16 * y, s1 = x + 4 * (2 + bj) + 16 * y;   // lanes of blocks (0, bj), (1, bj)
    const int j = nlev[node];
    const int64_t stride = (int64_t)15 * KK;        // from term m to m + 1
    double acc = 0.0;
    int base = 0;                                   // running index of the node's (job, term) pairs
    for (int64_t q = off[node]; q < off[node + 1]; ++q) {
        const Job2 jb = jobs[q];
        const int cnt = jb.m2 - jb.m1 + 1;
        const int t0 = ((wv - base) % NW + NW) % NW;
        base += cnt;
        if (t0 >= cnt) continue;
        const double* Xb = X + jb.in * KK;
        const double xa0 = va0 ? Xb[oa0] : 0.0, xa1 = va1 ? Xb[oa1] : 0.0;
        const double* F1b = F + (((int64_t)j * M) * 15 + (jb.l1 + 7)) * KK;
        const double* F2b = F + (((int64_t)j * M) * 15 + (jb.l2 + 7)) * KK;
        double f10, f11, f20, f21;
        auto load = [&](int m, double& a0, double& a1, double& b0, double& b1) {
            const double* p1 = F1b + m * stride;
            const double* p2 = F2b + m * stride;
            a0 = va0 ? p1[oa0] : 0.0;
            a1 = va1 ? p1[oa1] : 0.0;
            b0 = vb0 ? p2[ob0] : 0.0;
            b1 = vb1 ? p2[ob1] : 0.0;
        };
        load(jb.m1 + t0, f10, f11, f20, f21);
        for (int m = jb.m1 + t0; m <= jb.m2; m += NW) {
            double n10, n11, n20, n21;
            load(m + NW <= jb.m2 ? m + NW : m, n10, n11, n20, n21);
            double t = __builtin_amdgcn_mfma_f64_4x4x4f64(xa0, f20, 0.0, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f64_4x4x4f64(xa1, f21, t, 0, 0, 0);
            const double cw = jb.sign * w[m];
            const double t0v = __shfl(t, s0), t1v = __shfl(t, s1);
            acc = __builtin_amdgcn_mfma_f64_4x4x4f64(cw * f10, t0v, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_4x4x4f64(cw * f11, t1v, acc, 0, 0, 0);
            f10 = n10;
            f11 = n11;
            f20 = n20;
            f21 = n21;
        }
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0) {
        const double sum = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        const int ro = 4 * bi + y, co = 4 * bj + x;
        if (ro < K && co < K) out[(int64_t)node * KK + ro * K + co] = sum;
    }
}

// g[node] += H^(sx)^T g[parent] H^(sy) for the nodes of one level
__global__ void assemble2_kernel(int k, int n, const int64_t* __restrict__ node, const int64_t* __restrict__ par,
                                 const int* __restrict__ sg, const double* __restrict__ H, double* __restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = k * k;
    if (i >= n * kk) return;
    const int p = i / kk, a = (i % kk) / k, b = i % k;
    const double* Hx = H + (sg[p] & 1) * kk;
    const double* Hy = H + (sg[p] >> 1) * kk;
    const double* G = g + par[p] * kk;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) {
        double u = 0.0;
        for (int d = 0; d < k; ++d) u += G[c * k + d] * Hy[d * k + b];
        acc += Hx[c * k + a] * u;
    }
    g[node[p] * kk + a * k + b] += acc;
}

__global__ void eval2_kernel(int k, int64_t nn, const uint64_t* __restrict__ keys, const uint8_t* __restrict__ leaf,
                             const double* __restrict__ g, int64_t np, const double* __restrict__ pts, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const double x = pts[2 * i], y = pts[2 * i + 1];
    double px[K2MAX], py[K2MAX];
    for (int j = 0; j <= MAXLEV2; ++j) {
        const int64_t n = (int64_t)1 << j;
        int64_t lx = (int64_t)floor(x * (double)n), ly = (int64_t)floor(y * (double)n);
        lx = lx < 0 ? 0 : (lx > n - 1 ? n - 1 : lx);
        ly = ly < 0 ? 0 : (ly > n - 1 ? n - 1 : ly);
        const int64_t p = find_sorted(keys, nn, key2(j, lx, ly));
        if (p < 0) break;
        if (leaf[p]) {
            phi2_dev(k, x * (double)n - (double)lx, px);
            phi2_dev(k, y * (double)n - (double)ly, py);
            double v = 0.0;
            for (int a = 0; a < k; ++a) {
                double u = 0.0;
                for (int b = 0; b < k; ++b) u += g[p * k * k + a * k + b] * py[b];
                v += px[a] * u;
            }
            out[i] = (double)n * v;
            return;
        }
    }
    out[i] = NAN;
}

unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace mwns

using namespace mwns;

struct mwns_op2 {
    CtxHold hold;
    mwns_ctx* ctx = nullptr;
    int k = 0, M = 0, max_level = 0;
    double eps = 0.0, theta = 0.0;
    std::vector<double> w;
    DevArray<double> F;            // [max_level + 1][M][15][k][k]
    DevArray<double> dw;
    DevArray<double> H;            // [2][k][k]
    std::vector<int32_t> plan;     // [max_level + 1][7][7][2]
};

struct mwns_tree2 {
    CtxHold hold;
    mwns_ctx* ctx = nullptr;
    int k = 0, depth = 0;
    int64_t nleaves = 0;
    std::vector<uint64_t> keys;    // sorted
    std::vector<uint8_t> leaf;
    DevArray<uint64_t> dkeys;
    DevArray<uint8_t> dleaf;
    DevArray<double> coef;         // [n][k][k]
};

namespace {

void check_ctx2(mwns_ctx* ctx) {
    if (!ctx) fail(MWNS_EINVAL, "NULL context");
    MWNS_HIP(hipSetDevice(ctx->device));
}

double c2_alpha(double alpha) { return 2.0 * std::pow(2.0, -2.0 * alpha) / (M_PI * std::tgamma(alpha)); }

// the plane's kernel: (2 pi)^-1 2^{1-alpha} / Gamma(alpha) (mu/r)^{1-alpha} K_{1-alpha}(mu r) for
// mu > 0; Gamma(1 - alpha) / (4^alpha pi Gamma(alpha)) r^{2 alpha - 2} for mu = 0
double kernel2(double mu, double alpha, double r) {
    if (mu > 0.0) {
        const double nu = 1.0 - alpha;
        return std::pow(2.0, 1.0 - alpha) / (2.0 * M_PI * std::tgamma(alpha)) * std::pow(mu / r, nu) *
               std::cyl_bessel_k(nu, mu * r);
    }
    return std::tgamma(1.0 - alpha) / (std::pow(4.0, alpha) * M_PI * std::tgamma(alpha)) * std::pow(r, 2.0 * alpha - 2.0);
}

void two_h(int k, std::vector<double>& H) {
    H.resize(2 * k * k);
    two_scale_filters(k, H.data(), H.data() + k * k);
}

std::unique_ptr<mwns_tree2> build_tree2(mwns_ctx* ctx, int k, std::vector<uint64_t> keys, std::vector<uint8_t> leaf,
                                        DevArray<double>&& coef, const double* dH, bool compress) {
    auto t = std::make_unique<mwns_tree2>();
    t->hold.set(ctx);
    t->ctx = ctx;
    t->k = k;
    const int64_t n = (int64_t)keys.size();
    if (n == 0 || keys[0] != key2(0, 0, 0)) fail(MWNS_EINVAL, "the tree has no root");
    for (int64_t i = 0; i < n; ++i) {
        if (i && keys[i] <= keys[i - 1]) fail(MWNS_EINVAL, "keys are not sorted and distinct");
        const int j = key2_level(keys[i]);
        t->depth = std::max(t->depth, j);
        int64_t x, y;
        key2_xy(keys[i], &x, &y);
        if (j > 0) {
            const int64_t p = find_sorted(keys.data(), n, key2(j - 1, x >> 1, y >> 1));
            if (p < 0 || leaf[p]) fail(MWNS_EINVAL, "a node without an internal parent");
        }
        if (!leaf[i])
            for (int s = 0; s < 4; ++s)
                if (find_sorted(keys.data(), n, key2(j + 1, 2 * x + (s & 1), 2 * y + (s >> 1))) < 0)
                    fail(MWNS_EINVAL, "an internal node without its four children");
        t->nleaves += leaf[i] ? 1 : 0;
    }
    t->keys = std::move(keys);
    t->leaf = std::move(leaf);
    t->coef = std::move(coef);
    if (compress) {
        for (int j = t->depth - 1; j >= 0; --j) {
            std::vector<int64_t> par, ch;
            for (int64_t i = 0; i < n; ++i)
                if (key2_level(t->keys[i]) == j && !t->leaf[i]) {
                    int64_t x, y;
                    key2_xy(t->keys[i], &x, &y);
                    par.push_back(i);
                    for (int s = 0; s < 4; ++s)
                        ch.push_back(find_sorted(t->keys.data(), n, key2(j + 1, 2 * x + (s & 1), 2 * y + (s >> 1))));
                }
            if (par.empty()) continue;
            DevArray<int64_t> dp(ctx, par.size()), dc(ctx, ch.size());
            dp.upload(par.data(), par.size(), ctx->stream);
            dc.upload(ch.data(), ch.size(), ctx->stream);
            compress2_kernel<<<nblk((int64_t)par.size() * k * k, 256), 256, 0, ctx->stream>>>(k, (int)par.size(), dp.p, dc.p,
                                                                                             dH, t->coef.p);
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

// per-L term range of the 2-D plan (the 3-D plan's rule): prefix and suffix whose cumulative sums
// stay <= theta/2 dropped; empty when the whole sum is <= theta
void term_range2(const std::vector<double>& e, double theta, int32_t* r) {
    double tot = 0.0;
    for (double v : e) tot += v;
    if (tot <= theta) { r[0] = 0; r[1] = -1; return; }
    double c = 0.0;
    int m1 = 0;
    for (int m = 0; m < (int)e.size(); ++m) {
        c += e[m];
        if (c > 0.5 * theta) { m1 = m; break; }
    }
    c = 0.0;
    int m2 = (int)e.size() - 1;
    for (int m = (int)e.size() - 1; m >= 0; --m) {
        c += e[m];
        if (c > 0.5 * theta) { m2 = m; break; }
    }
    r[0] = m1;
    r[1] = m2;
}

}  // namespace

extern "C" {

mwns_status mwns_fit_kernel2d(double mu, double alpha, double eps, double delta, double R, int cap, int* M, double* tau,
                              double* w) {
    MWNS_GUARD_BEGIN
    if (!M) fail(MWNS_EINVAL, "NULL argument");
    if (!(alpha > 0.0 && alpha <= 1.0) || !(mu >= 0.0) || (mu == 0.0 && alpha >= 1.0) || !(eps > 0.0 && eps < 1.0) ||
        !(delta > 0.0 && delta < R))
        fail(MWNS_EINVAL, "need 0 < alpha <= 1, mu >= 0 (mu > 0 when alpha = 1), 0 < eps < 1, 0 < delta < R");
    double h = M_PI * M_PI / (2.0 * (std::log(1.0 / eps) + std::log(8.0)));
    double A = 1e300;
    if (mu > 0.0) A = std::min(A, std::log(mu) - 0.5 * std::log(4.0 * std::log(1e30 / eps)));
    if (alpha < 1.0) {
        const double g = 2.0 - 2.0 * alpha;
        A = std::min(A, std::log(eps * kernel2(mu, alpha, R) * g / (c2_alpha(alpha) * M_E)) / g);
    }
    double B = 0.5 * std::log(std::log(4.0 / eps) / (delta * delta)) + 1.0;
    const int ndec = std::max(1, (int)std::ceil(std::log10(R / delta)));
    std::vector<double> tt, ww;
    auto max_err = [&](int npd) {
        double e = 0.0;
        const int n = npd * ndec + 1;
        for (int i = 0; i < n; ++i) {
            const double r = std::exp(std::log(delta) + (std::log(R) - std::log(delta)) * i / (n - 1));
            double s = 0.0;
            for (size_t m = 0; m < tt.size(); ++m) s += ww[m] * std::exp(-tt[m] * r * r);
            const double ref = kernel2(mu, alpha, r);
            e = std::max(e, std::fabs(ref - s) / ref);
        }
        return e;
    };
    for (int it = 0; it < 40; ++it) {
        const int n = std::max(1, (int)std::ceil((B - A) / h));
        tt.clear();
        ww.clear();
        const double hh = (A + n * h - A) / n;
        for (int m = 1; m <= n; ++m) {
            const double s = A + hh * m;
            const double wm = hh * c2_alpha(alpha) * std::exp(-mu * mu * std::exp(-2.0 * s) / 4.0 + (2.0 - 2.0 * alpha) * s);
            if (wm > 0.0) {             // weights that underflow to zero contribute nothing
                tt.push_back(std::exp(2.0 * s));
                ww.push_back(wm);
            }
        }
        if (max_err(64) <= eps && max_err(256) <= eps) {
            const int need = (int)tt.size();
            if (tau && w) {
                if (cap < need) { *M = need; fail(MWNS_ERANGE, "cap smaller than the number of terms"); }
                std::copy(tt.begin(), tt.end(), tau);
                std::copy(ww.begin(), ww.end(), w);
            }
            *M = need;
            return MWNS_OK;
        }
        h *= 0.9;
        A -= 1.0;
        B += 1.0;
    }
    fail(MWNS_ERANGE, "the fit did not converge");
    MWNS_GUARD_END
}

mwns_status mwns_op2d_create(mwns_ctx* ctx, int k, int M, const double* tau, const double* w, double eps, int max_level,
                             int allow_band_overflow, mwns_op2** out) {
    MWNS_GUARD_BEGIN
    check_ctx2(ctx);
    if (!out || !tau || !w) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > K2MAX) fail(MWNS_EINVAL, "k must be in 1..10");
    if (max_level < 0 || max_level > MAXLEV2) fail(MWNS_EINVAL, "max_level must be in 0..19");
    // the 1-D blocks come from the 3-D operator's device builder (its 3-D plan is not used)
    mwns_op_opts o{};
    o.group_regions = 1;
    o.allow_band_overflow = 1;
    mwns_op* op3 = nullptr;
    const mwns_status st3 = mwns_op_create(ctx, k, M, tau, w, eps, max_level, &o, &op3);
    if (st3 != MWNS_OK) return st3;
    std::unique_ptr<mwns_op> hold3(op3);
    auto op = std::make_unique<mwns_op2>();
    op->hold.set(ctx);
    op->ctx = ctx;
    op->k = k;
    op->M = M;
    op->max_level = max_level;
    op->eps = eps;
    op->w.assign(w, w + M);
    op->F = std::move(op3->F);
    op->dw = std::move(op3->dw);
    const int nlev = max_level + 1, kk = k * k;
    std::vector<double> H;
    two_h(k, H);
    op->H.reset(ctx, H.size());
    op->H.upload(H.data(), H.size(), ctx->stream);
    std::vector<double> Fh(op->F.n);
    op->F.download(Fh.data(), Fh.size(), ctx->stream);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    auto blk = [&](int j, int m, int l) { return Fh.data() + (((size_t)j * M + m) * 15 + (l + 7)) * kk; };
    double theta = 0.0;
    for (int m = 0; m < M; ++m) {
        double f2 = 0.0;
        for (int e = 0; e < kk; ++e) f2 += blk(0, m, 0)[e] * blk(0, m, 0)[e];
        theta += w[m] * f2;
    }
    op->theta = theta * eps;
    op->plan.assign((size_t)nlev * NLP2 * NLP2 * 2, 0);
    for (size_t i = 1; i < op->plan.size(); i += 2) op->plan[i] = -1;
    op->plan[((LP2 * NLP2) + LP2) * 2] = 0;
    op->plan[((LP2 * NLP2) + LP2) * 2 + 1] = M - 1;
    const int n2 = 2 * k;
    std::vector<double> S(n2 * n2), U(n2 * n2), T(kk);
    for (int j = 1; j < nlev; ++j) {
        // norms N_F, N_upF, N_dif of the 2k x 2k super-blocks at L = 0..3
        std::vector<double> NF((size_t)M * 4), NU((size_t)M * 4), ND((size_t)M * 4);
        for (int m = 0; m < M; ++m)
            for (int L = 0; L <= LP2; ++L) {
                for (int so = 0; so < 2; ++so)
                    for (int si = 0; si < 2; ++si) {
                        const double* f = blk(j, m, 2 * L + so - si);
                        for (int a = 0; a < k; ++a)
                            for (int b = 0; b < k; ++b) S[(so * k + a) * n2 + si * k + b] = f[a * k + b];
                    }
                const double* c = blk(j - 1, m, L);
                for (int so = 0; so < 2; ++so)
                    for (int si = 0; si < 2; ++si)
                        for (int a = 0; a < k; ++a)
                            for (int b = 0; b < k; ++b) {
                                double acc = 0.0;
                                for (int p = 0; p < k; ++p)
                                    for (int q = 0; q < k; ++q)
                                        acc += H[so * kk + p * k + a] * c[p * k + q] * H[si * kk + q * k + b];
                                U[(so * k + a) * n2 + si * k + b] = acc;
                            }
                double nf = 0.0, nu = 0.0, nd = 0.0;
                for (int e = 0; e < n2 * n2; ++e) {
                    nf += S[e] * S[e];
                    nu += U[e] * U[e];
                    nd += (S[e] - U[e]) * (S[e] - U[e]);
                }
                NF[m * 4 + L] = std::sqrt(nf);
                NU[m * 4 + L] = std::sqrt(nu);
                ND[m * 4 + L] = std::sqrt(nd);
            }
        int32_t rng[4][4][2];
        for (int p = 0; p <= LP2; ++p)
            for (int q = p; q <= LP2; ++q) {
                std::vector<double> e(M);
                for (int m = 0; m < M; ++m) {
                    double est = ND[m * 4 + p] * NF[m * 4 + q] + NU[m * 4 + p] * ND[m * 4 + q];
                    if (q != p) est += ND[m * 4 + q] * NF[m * 4 + p] + NU[m * 4 + q] * ND[m * 4 + p];
                    else est *= 2.0;
                    e[m] = w[m] * est / 2.0;
                }
                term_range2(e, op->theta, rng[p][q]);
                rng[q][p][0] = rng[p][q][0];
                rng[q][p][1] = rng[p][q][1];
                if (q == LP2 && rng[p][q][1] >= rng[p][q][0] && !allow_band_overflow)
                    fail(MWNS_ERANGE, "band overflow: level " + std::to_string(j) + " keeps terms at the edge |L_d| = 3");
            }
        // grouping: hull of the ranges of the classes with 0, 1, 2 coordinates |L_d| > 1
        int hull[3][2] = {{M, -1}, {M, -1}, {M, -1}};
        for (int p = 0; p <= LP2; ++p)
            for (int q = p; q <= LP2; ++q) {
                const int g = (p > 1) + (q > 1);
                if (rng[p][q][1] >= rng[p][q][0]) {
                    hull[g][0] = std::min(hull[g][0], rng[p][q][0]);
                    hull[g][1] = std::max(hull[g][1], rng[p][q][1]);
                }
            }
        for (int x = -LP2; x <= LP2; ++x)
            for (int y = -LP2; y <= LP2; ++y) {
                const int g = (std::abs(x) > 1) + (std::abs(y) > 1);
                int32_t* r = op->plan.data() + (((size_t)j * NLP2 + (x + LP2)) * NLP2 + (y + LP2)) * 2;
                r[0] = hull[g][1] >= hull[g][0] ? hull[g][0] : 0;
                r[1] = hull[g][1] >= hull[g][0] ? hull[g][1] : -1;
            }
    }
    *out = op.release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_op2d_plan_export(const mwns_op2* op, int32_t* plan, size_t* count) {
    MWNS_GUARD_BEGIN
    if (!op || !count) fail(MWNS_EINVAL, "NULL argument");
    if (plan) {
        if (*count < op->plan.size()) fail(MWNS_ERANGE, "plan array too small");
        std::copy(op->plan.begin(), op->plan.end(), plan);
    }
    *count = op->plan.size();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_op2d_plan_import(mwns_op2* op, const int32_t* plan, size_t count) {
    MWNS_GUARD_BEGIN
    if (!op || !plan) fail(MWNS_EINVAL, "NULL argument");
    if (count != op->plan.size()) fail(MWNS_EINVAL, "plan size must be (max_level + 1) * 7 * 7 * 2");
    for (size_t i = 0; i < count; i += 2)
        if (plan[i + 1] >= plan[i] && (plan[i] < 0 || plan[i + 1] >= op->M)) fail(MWNS_EINVAL, "term range out of range");
    std::copy(plan, plan + count, op->plan.begin());
    return MWNS_OK;
    MWNS_GUARD_END
}

void mwns_op2d_destroy(mwns_op2* op) { delete op; }

mwns_status mwns_project2d(mwns_ctx* ctx, int k, double eps, int j0, int jmax, int n, const double* xy, const double* a,
                           const double* c, mwns_tree2** out) {
    MWNS_GUARD_BEGIN
    check_ctx2(ctx);
    if (!out || (n > 0 && (!xy || !a || !c))) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > K2MAX) fail(MWNS_EINVAL, "k must be in 1..10");
    if (!(eps > 0.0) || j0 < 0 || jmax < j0 || jmax > MAXLEV2 || n < 0) fail(MWNS_EINVAL, "eps, j0, jmax or n out of range");
    for (int i = 0; i < n; ++i)
        if (!(a[i] > 0.0) || !std::isfinite(a[i]) || !std::isfinite(c[i]) || !std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1]))
            fail(MWNS_EINVAL, "exponents must be > 0 and all parameters finite");
    // threshold eps ||f||_2 with the closed-form norm of the Gaussian sum
    double f2 = 0.0;
    for (int i = 0; i < n; ++i)
        for (int i2 = 0; i2 < n; ++i2) {
            const double dx = xy[2 * i] - xy[2 * i2], dy = xy[2 * i + 1] - xy[2 * i2 + 1];
            f2 += c[i] * c[i2] * (a[i] * a[i2] / (M_PI * M_PI)) * (M_PI / (a[i] + a[i2])) *
                  std::exp(-a[i] * a[i2] / (a[i] + a[i2]) * (dx * dx + dy * dy));
        }
    const double thr = eps * std::sqrt(std::max(f2, 0.0));
    const Quad q = gauss_legendre01(k);
    std::vector<double> phiq(k * k), phich(2 * k * k), tmp(16), g(4 * std::max(n, 1));
    for (int i = 0; i < k; ++i) {
        legendre_phi(k, q.x[i], tmp.data());
        for (int b = 0; b < k; ++b) phiq[i * k + b] = tmp[b];
        for (int s = 0; s < 2; ++s) {
            legendre_phi(k, 0.5 * (q.x[i] + s), tmp.data());
            for (int b = 0; b < k; ++b) phich[(s * k + i) * k + b] = tmp[b];
        }
    }
    for (int i = 0; i < n; ++i) {
        g[4 * i] = xy[2 * i];
        g[4 * i + 1] = xy[2 * i + 1];
        g[4 * i + 2] = a[i];
        g[4 * i + 3] = c[i];
    }
    DevArray<double> dx(ctx, k), dwq(ctx, k), dphi(ctx, phiq.size()), dphc(ctx, phich.size()), dg(ctx, g.size());
    dx.upload(q.x.data(), k, ctx->stream);
    dwq.upload(q.w.data(), k, ctx->stream);
    dphi.upload(phiq.data(), phiq.size(), ctx->stream);
    dphc.upload(phich.data(), phich.size(), ctx->stream);
    dg.upload(g.data(), g.size(), ctx->stream);
    const int kk = k * k;
    std::vector<std::pair<uint64_t, std::vector<double>>> leaves;
    std::vector<int64_t> cand;
    for (int64_t x = 0; x < ((int64_t)1 << j0); ++x)
        for (int64_t y = 0; y < ((int64_t)1 << j0); ++y) {
            cand.push_back(x);
            cand.push_back(y);
        }
    for (int j = j0; !cand.empty(); ++j) {
        const int nc = (int)cand.size() / 2;
        DevArray<int64_t> dc(ctx, cand.size());
        DevArray<double> dco(ctx, (size_t)nc * kk), der(ctx, nc);
        dc.upload(cand.data(), cand.size(), ctx->stream);
        project2_kernel<<<nc, 256, 0, ctx->stream>>>(k, j, dc.p, n, dg.p, dx.p, dwq.p, dphi.p, dphc.p, dco.p, der.p);
        MWNS_HIP(hipGetLastError());
        std::vector<double> co((size_t)nc * kk), er(nc);
        dco.download(co.data(), co.size(), ctx->stream);
        der.download(er.data(), nc, ctx->stream);
        MWNS_HIP(hipStreamSynchronize(ctx->stream));
        std::vector<int64_t> next;
        for (int i = 0; i < nc; ++i) {
            const int64_t x = cand[2 * i], y = cand[2 * i + 1];
            if (j < jmax && er[i] > thr) {
                for (int s = 0; s < 4; ++s) {
                    next.push_back(2 * x + (s & 1));
                    next.push_back(2 * y + (s >> 1));
                }
            } else {
                leaves.emplace_back(key2(j, x, y), std::vector<double>(co.begin() + (size_t)i * kk, co.begin() + (size_t)(i + 1) * kk));
            }
        }
        cand.swap(next);
    }
    std::vector<uint64_t> keys;
    for (const auto& lv : leaves) {
        int64_t x, y;
        key2_xy(lv.first, &x, &y);
        const int jl = key2_level(lv.first);
        for (int j = jl; j >= 0; --j) keys.push_back(key2(j, x >> (jl - j), y >> (jl - j)));
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::vector<uint8_t> leaf(keys.size(), 0);
    std::vector<double> hc(keys.size() * kk, 0.0);
    for (const auto& lv : leaves) {
        const int64_t p = find_sorted(keys.data(), (int64_t)keys.size(), lv.first);
        leaf[p] = 1;
        std::copy(lv.second.begin(), lv.second.end(), hc.begin() + p * kk);
    }
    DevArray<double> coef(ctx, hc.size());
    coef.upload(hc.data(), hc.size(), ctx->stream);
    std::vector<double> H;
    two_h(k, H);
    DevArray<double> dH(ctx, H.size());
    dH.upload(H.data(), H.size(), ctx->stream);
    *out = build_tree2(ctx, k, std::move(keys), std::move(leaf), std::move(coef), dH.p, true).release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree2d_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* lkeys, const double* coeffs,
                                    mwns_tree2** out) {
    MWNS_GUARD_BEGIN
    check_ctx2(ctx);
    if (!out || nleaves <= 0 || !lkeys || !coeffs) fail(MWNS_EINVAL, "NULL argument or no leaves");
    if (k < 1 || k > K2MAX) fail(MWNS_EINVAL, "k must be in 1..10");
    const int kk = k * k;
    std::vector<uint64_t> keys;
    for (int64_t i = 0; i < nleaves; ++i) {
        const int jl = key2_level(lkeys[i]);
        int64_t x, y;
        key2_xy(lkeys[i], &x, &y);
        if (jl > MAXLEV2 || x >= ((int64_t)1 << jl) || y >= ((int64_t)1 << jl) || key2(jl, x, y) != lkeys[i])
            fail(MWNS_EINVAL, "invalid leaf key");
        for (int j = jl; j >= 0; --j) keys.push_back(key2(j, x >> (jl - j), y >> (jl - j)));
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::vector<uint8_t> leaf(keys.size(), 0);
    std::vector<double> hc(keys.size() * kk, 0.0);
    for (int64_t i = 0; i < nleaves; ++i) {
        const int64_t p = find_sorted(keys.data(), (int64_t)keys.size(), lkeys[i]);
        if (leaf[p]) fail(MWNS_EINVAL, "duplicate leaf key");
        leaf[p] = 1;
        std::copy(coeffs + i * kk, coeffs + (i + 1) * kk, hc.begin() + p * kk);
    }
    for (size_t i = 0; i < keys.size(); ++i)
        if (leaf[i]) {
            int64_t x, y;
            key2_xy(keys[i], &x, &y);
            if (find_sorted(keys.data(), (int64_t)keys.size(), key2(key2_level(keys[i]) + 1, 2 * x, 2 * y)) >= 0)
                fail(MWNS_EINVAL, "a leaf has descendants");
        }
    DevArray<double> coef(ctx, hc.size());
    coef.upload(hc.data(), hc.size(), ctx->stream);
    std::vector<double> H;
    two_h(k, H);
    DevArray<double> dH(ctx, H.size());
    dH.upload(H.data(), H.size(), ctx->stream);
    *out = build_tree2(ctx, k, std::move(keys), std::move(leaf), std::move(coef), dH.p, true).release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_apply2d(mwns_ctx* ctx, const mwns_op2* op, const mwns_tree2* f, mwns_tree2** g, double* ms_contract,
                         double* flops) {
    MWNS_GUARD_BEGIN
    check_ctx2(ctx);
    if (!op || !f || !g) fail(MWNS_EINVAL, "NULL argument");
    if (op->ctx != ctx || f->ctx != ctx) fail(MWNS_EINVAL, "operator or tree of another context");
    if (op->k != f->k) fail(MWNS_EINVAL, "the operator's and the tree's orders differ");
    if (f->depth > op->max_level) fail(MWNS_EINVAL, "the tree is deeper than the operator's max_level");
    const int k = f->k, kk = k * k, nlev = op->max_level + 1;
    const int64_t no = (int64_t)f->keys.size();
    auto range = [&](int j, int L1, int L2, int* m1, int* m2) {
        if (j >= nlev || std::abs(L1) > LP2 || std::abs(L2) > LP2) { *m1 = 0; *m2 = -1; return; }
        const int32_t* r = op->plan.data() + (((size_t)j * NLP2 + (L1 + LP2)) * NLP2 + (L2 + LP2)) * 2;
        *m1 = r[0];
        *m2 = r[1];
    };
    // The job lists, built by several host threads over contiguous node ranges.  Each range keeps its
    // own table of inputs (an input box seen by two ranges is gathered twice, with the same values),
    // and the ranges are joined in node order, so the result does not depend on the thread count.
    struct Part {
        std::vector<Job2> jobs;
        std::vector<int64_t> ends;                   // jobs.size() after each node of the range
        std::unordered_map<uint64_t, int64_t> inidx;
        std::vector<int64_t> ianc, ixy;
        std::vector<int> iup;
        double fl = 0.0;
    };
    std::vector<int> nl(no);
    auto build = [&](int64_t lo, int64_t hi, Part& P) {
        auto input = [&](int j, int64_t x, int64_t y) -> int64_t {
            const uint64_t kk2 = key2(j, x, y);
            auto it = P.inidx.find(kk2);
            if (it != P.inidx.end()) return it->second;
            int up = 0;
            int64_t p;
            while ((p = find_sorted(f->keys.data(), no, key2(j - up, x >> up, y >> up))) < 0) ++up;
            const int64_t id = (int64_t)P.ianc.size();
            P.ianc.push_back(p);
            P.iup.push_back(up);
            P.ixy.push_back(x);
            P.ixy.push_back(y);
            P.inidx.emplace(kk2, id);
            return id;
        };
        auto add = [&](int64_t in, int l1, int l2, int a, int b, int sign) {
            if (b < a) return;
            P.jobs.push_back(Job2{in, l1, l2, a, b, sign, 0});
            P.fl += (double)(b - a + 1) * 4.0 * k * kk;
        };
        for (int64_t i = lo; i < hi; ++i) {
            const int j = key2_level(f->keys[i]);
            int64_t bx, by;
            key2_xy(f->keys[i], &bx, &by);
            const bool lf = f->leaf[i] != 0;
            nl[i] = j;
            if (j == 0) {
                int a1, b1, a2 = 0, b2 = -1;
                range(0, 0, 0, &a1, &b1);
                if (!lf) range(1, 0, 0, &a2, &b2);
                const int64_t in = input(0, 0, 0);
                // [a1, b1] minus [a2, b2] (R_1(0) lies inside R_0 = all terms)
                if (b2 < a2) add(in, 0, 0, a1, b1, 1);
                else {
                    add(in, 0, 0, a1, std::min(b1, a2 - 1), 1);
                    add(in, 0, 0, std::max(a1, b2 + 1), b1, 1);
                    add(in, 0, 0, std::max(a2, b1 + 1), b2, -1);
                    add(in, 0, 0, a2, std::min(b2, a1 - 1), -1);
                }
            } else {
                const int64_t n = (int64_t)1 << j;
                for (int l1 = -7; l1 <= 7; ++l1)
                    for (int l2 = -7; l2 <= 7; ++l2) {
                        const int64_t px = bx - l1, py = by - l2;
                        if (px < 0 || px >= n || py < 0 || py >= n) continue;
                        int a1, b1, a2 = 0, b2 = -1;
                        range(j, (int)((bx >> 1) - (px >> 1)), (int)((by >> 1) - (py >> 1)), &a1, &b1);
                        if (!lf) range(j + 1, l1, l2, &a2, &b2);
                        if (b1 < a1 && b2 < a2) continue;
                        const int64_t in = input(j, px, py);
                        if (b2 < a2 || b1 < a1 || b1 < a2 || b2 < a1) {        // disjoint or one empty
                            add(in, l1, l2, a1, b1, 1);
                            add(in, l1, l2, a2, b2, -1);
                        } else {                                               // the overlap cancels
                            add(in, l1, l2, a1, std::min(b1, a2 - 1), 1);
                            add(in, l1, l2, std::max(a1, b2 + 1), b1, 1);
                            add(in, l1, l2, a2, std::min(b2, a1 - 1), -1);
                            add(in, l1, l2, std::max(a2, b1 + 1), b2, -1);
                        }
                    }
            }
            P.ends.push_back((int64_t)P.jobs.size());
        }
    };
    const int nth = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)std::max(1u, std::thread::hardware_concurrency()), 16,
                                                                (no + 511) / 512}));
    std::vector<Part> parts(nth);
    {
        std::vector<std::exception_ptr> errs(nth);
        std::vector<std::thread> pool;
        for (int t = 0; t < nth; ++t)
            pool.emplace_back([&, t] {
                try {
                    build(no * t / nth, no * (t + 1) / nth, parts[t]);
                } catch (...) {
                    errs[t] = std::current_exception();
                }
            });
        for (auto& th : pool) th.join();
        for (auto& e : errs)
            if (e) std::rethrow_exception(e);
    }
    // the jobs of all ranges, their inputs renumbered, written by the same threads straight into the
    // context's pinned staging block (one DMA to the device)
    std::vector<int64_t> jbase(nth + 1, 0), ibase(nth + 1, 0);
    for (int t = 0; t < nth; ++t) {
        jbase[t + 1] = jbase[t] + (int64_t)parts[t].jobs.size();
        ibase[t + 1] = ibase[t] + (int64_t)parts[t].ianc.size();
    }
    const int64_t njobs = jbase[nth];
    Job2* hjobs = static_cast<Job2*>(pinned_staging(ctx, (size_t)std::max<int64_t>(njobs, 1) * sizeof(Job2)));
    {
        std::vector<std::thread> pool;
        for (int t = 0; t < nth; ++t)
            pool.emplace_back([&, t] {
                Job2* dst = hjobs + jbase[t];
                for (const Job2& jb : parts[t].jobs) {
                    *dst = jb;
                    dst->in += ibase[t];
                    ++dst;
                }
            });
        for (auto& th : pool) th.join();
    }
    std::vector<int64_t> off(1, 0), ianc, ixy;
    std::vector<int> iup;
    double fl = 0.0;
    for (int t = 0; t < nth; ++t) {
        Part& P = parts[t];
        for (int64_t e : P.ends) off.push_back(jbase[t] + e);
        ianc.insert(ianc.end(), P.ianc.begin(), P.ianc.end());
        ixy.insert(ixy.end(), P.ixy.begin(), P.ixy.end());
        iup.insert(iup.end(), P.iup.begin(), P.iup.end());
        fl += P.fl;
        P = Part();
    }
    const int64_t nin = (int64_t)ianc.size();
    hipStream_t st = ctx->stream;
    DevArray<double> X(ctx, (size_t)std::max<int64_t>(nin, 1) * kk);
    if (nin) {
        DevArray<int64_t> da(ctx, nin), dxy(ctx, 2 * nin);
        DevArray<int> du(ctx, nin);
        da.upload(ianc.data(), nin, st);
        dxy.upload(ixy.data(), 2 * nin, st);
        du.upload(iup.data(), nin, st);
        gather2_kernel<<<(unsigned)nin, 128, 0, st>>>(k, da.p, du.p, dxy.p, op->H.p, f->coef.p, X.p);
        MWNS_HIP(hipGetLastError());
        MWNS_HIP(hipStreamSynchronize(st));
    }
    DevArray<int64_t> doff(ctx, off.size());
    DevArray<Job2> djobs(ctx, (size_t)std::max<int64_t>(njobs, 1));
    DevArray<int> dnl(ctx, no);
    doff.upload(off.data(), off.size(), st);
    djobs.upload(hjobs, (size_t)njobs, st);
    dnl.upload(nl.data(), no, st);
    DevArray<double> out(ctx, (size_t)no * kk);
    hipEvent_t e0, e1;
    MWNS_HIP(hipEventCreate(&e0));
    MWNS_HIP(hipEventCreate(&e1));
    MWNS_HIP(hipEventRecord(e0, st));
    switch (k) {
#define MWNS_C2W(KV) \
    case KV: \
        contract2_wave_kernel<KV><<<(unsigned)((no + 3) / 4), 256, 0, st>>>((int)no, op->M, dnl.p, doff.p, djobs.p, op->F.p, \
                                                                          op->dw.p, X.p, out.p); \
        break;
        MWNS_C2W(1) MWNS_C2W(2) MWNS_C2W(3) MWNS_C2W(4)
#undef MWNS_C2W
#define MWNS_C2M(KV) \
    case KV: \
        contract2_mfma_kernel<KV><<<(unsigned)no, 256, 0, st>>>((int)no, op->M, dnl.p, doff.p, djobs.p, op->F.p, \
                                                                          op->dw.p, X.p, out.p); \
        break;
        MWNS_C2M(5) MWNS_C2M(6) MWNS_C2M(7) MWNS_C2M(8)
#undef MWNS_C2M
        default:
            contract2_kernel<<<(unsigned)no, 128, 0, st>>>(k, op->M, dnl.p, doff.p, djobs.p, op->F.p, op->dw.p, X.p, out.p);
    }
    MWNS_HIP(hipGetLastError());
    MWNS_HIP(hipEventRecord(e1, st));
    for (int j = 1; j <= f->depth; ++j) {
        std::vector<int64_t> nd, par;
        std::vector<int> sg;
        for (int64_t i = 0; i < no; ++i)
            if (key2_level(f->keys[i]) == j) {
                int64_t x, y;
                key2_xy(f->keys[i], &x, &y);
                nd.push_back(i);
                par.push_back(find_sorted(f->keys.data(), no, key2(j - 1, x >> 1, y >> 1)));
                sg.push_back((int)((x & 1) + 2 * (y & 1)));
            }
        DevArray<int64_t> dnd(ctx, nd.size()), dpar(ctx, par.size());
        DevArray<int> dsg(ctx, sg.size());
        dnd.upload(nd.data(), nd.size(), st);
        dpar.upload(par.data(), par.size(), st);
        dsg.upload(sg.data(), sg.size(), st);
        assemble2_kernel<<<nblk((int64_t)nd.size() * kk, 128), 128, 0, st>>>(k, (int)nd.size(), dnd.p, dpar.p, dsg.p,
                                                                            op->H.p, out.p);
        MWNS_HIP(hipGetLastError());
        MWNS_HIP(hipStreamSynchronize(st));
    }
    MWNS_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    MWNS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_contract) *ms_contract = ms;
    if (flops) *flops = fl;
    std::vector<uint64_t> keys = f->keys;
    std::vector<uint8_t> leaf = f->leaf;
    *g = build_tree2(ctx, k, std::move(keys), std::move(leaf), std::move(out), op->H.p, false).release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree2d_export(mwns_ctx* ctx, const mwns_tree2* t, int64_t* nnodes, uint64_t* keys, uint8_t* is_leaf,
                               double* coeffs) {
    MWNS_GUARD_BEGIN
    check_ctx2(ctx);
    if (!t || !nnodes) fail(MWNS_EINVAL, "NULL argument");
    const int64_t n = (int64_t)t->keys.size();
    if (keys || is_leaf || coeffs) {
        if (*nnodes < n) fail(MWNS_ERANGE, "arrays too small");
        if (keys) std::copy(t->keys.begin(), t->keys.end(), keys);
        if (is_leaf) std::copy(t->leaf.begin(), t->leaf.end(), is_leaf);
        if (coeffs) {
            t->coef.download(coeffs, (size_t)n * t->k * t->k, ctx->stream);
            MWNS_HIP(hipStreamSynchronize(ctx->stream));
        }
    }
    *nnodes = n;
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_tree2d_eval(mwns_ctx* ctx, const mwns_tree2* t, int64_t npts, const double* pts, double* out) {
    MWNS_GUARD_BEGIN
    check_ctx2(ctx);
    if (!t || (npts > 0 && (!pts || !out))) fail(MWNS_EINVAL, "NULL argument");
    if (npts < 0) fail(MWNS_EINVAL, "npts must be >= 0");
    if (npts == 0) return MWNS_OK;
    for (int64_t i = 0; i < 2 * npts; ++i)
        if (!(pts[i] >= 0.0 && pts[i] <= 1.0)) fail(MWNS_EINVAL, "points must lie in [0, 1]^2");
    DevArray<double> dp(ctx, 2 * npts), dout(ctx, npts);
    dp.upload(pts, 2 * npts, ctx->stream);
    eval2_kernel<<<nblk(npts, 128), 128, 0, ctx->stream>>>(t->k, (int64_t)t->keys.size(), t->dkeys.p, t->dleaf.p, t->coef.p,
                                                          npts, dp.p, dout.p);
    MWNS_HIP(hipGetLastError());
    dout.download(out, npts, ctx->stream);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    return MWNS_OK;
    MWNS_GUARD_END
}

void mwns_tree2d_destroy(mwns_tree2* t) { delete t; }

}  // extern "C"
