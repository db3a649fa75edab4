// g = T f in the modified ns-form (eq. apply_algo, Alg. 3) on FP64 MFMA.
//
// Work is organised by sibling groups ("bricks"): the 8 children of a node form a (2k)^3 tensor
// with index u = s*k + a per dimension.  Between the brick of parent P and the brick of parent
// P - L (coarse displacement L) the fine displacement is l = 2L + s - s', so one Gaussian term acts
// per dimension as the 2k x 2k super-block
//     S^{j;m,L} = [[F^{j;m,2L}, F^{j;m,2L-1}], [F^{j;m,2L+1}, F^{j;m,2L}]]      (rows: output parity)
// and a term applied over a box of displacements L in [lo1,hi1] x [lo2,hi2] x [lo3,hi3] factorises
// (Sec. 5, the nested-loop factorisation with the term sum last):
//     Y += c w_m sum_{L1} S^{L1} x_1 [ sum_{L2} S^{L2} x_2 [ sum_{L3} S^{L3} x_3 X_{P-L} ] ].
// Per output node b and input b - l the method's coefficient of term m is
//     c_m = [m in R_j(L)] - [b internal] [m in R_{j+1}(l)],
// so each level runs "whole-band" jobs over boxes of L from the plan row j (all children) and
// "down-band" jobs from row j+1 expressed on fine l (masked super-blocks, internal children only,
// c = -1).  The boxes are the cells of the coarsest partition of [-3,3] per dimension on which the
// plan's ranges are constant (Core / Boundary sets, Sec. 4).
//
// MFMA mapping (v_mfma_f64_16x16x4: A[m][k] in lane m+16k, B[k][n] in lane n+16k, D[4i+g][n] in
// lane 16g+n, register i): 2k <= 16 is padded to one 16 x 16 tile per dimension.  Wave w owns the
// input slices v1 in {w*TPW..}: mode 3 (contract v3, A = X slice with K index 4g+kk loaded as 4
// consecutive doubles, B = S3), mode 2 straight from the mode-3 accumulators (their register i
// holds contraction index 4i+g), an LDS transpose, then mode 1 into the per-wave output tiles.
#include <algorithm>
#include <array>
#include <cmath>
#include <memory>

#include "mwns_internal.h"

namespace mwns {

struct LevelTab2 {
    int64_t node_off[MAXLEV + 2];
    int64_t brick_off[MAXLEV + 2];
    int depth;
};

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct Tpl {
    int lo[3], hi[3];      // coarse displacement box
    int mlo[3], mhi[3];    // fine displacement mask per dimension
    int m1, m2;            // inclusive term range
    int dpart;             // 0: whole band (all children, +), 1: down band (internal children, -)
};

constexpr int AT = 256;            // threads per block of the transform kernels
constexpr int T2S_V1 = 272;        // LDS strides of the mode-2 result [v1][u2][u3] (conflict-free)
constexpr int T2S_U2 = 16;
constexpr int NMAX = 4;            // largest box extent per dimension of one job (the host splits boxes)
constexpr int S3_V = 36;           // LDS stride of the staged mode-3 operand [L][v][u]

// One level of the apply as seen by the contraction kernel.
struct LevelDesc {
    const double* Xr;        // real input bricks of the level (the level's own bricks)
    const double* Xg;        // ghost input bricks
    const int32_t* nbr;      // [brick][(2Lr+1)^3] input index, -1 outside the cube
    const uint8_t* cmask;    // [brick] bit s set when child s is internal
    const Tpl* tpl;          // jobs of the level
    const double* Fj;        // F^{j;m,l} of the level [M][NLF][k][k]
    double* out;             // output bricks of the level
    int64_t nreal;
    int Lr, valid, ntpl, pad;
};

// Masked super-block entry S^{m,L}[u][v]: F^{j;m,2L+su-sv}_{a b} when the fine displacement lies in
// [mlo, mhi], else 0; u = su*K + a (output), v = sv*K + b (input); rows/columns >= 2K are padding.
template <int K>
__device__ inline double sop(const double* __restrict__ Fm, int L, int mlo, int mhi, int u, int v) {
    if (u >= 2 * K || v >= 2 * K) return 0.0;
    const int su = u >= K, sv = v >= K;
    const int l = 2 * L + su - sv;
    if (l < mlo || l > mhi) return 0.0;
    return Fm[(l + LF) * K * K + (u - su * K) * K + (v - sv * K)];
}

// Byte offset of lane (g, r)'s four consecutive doubles X[v1][r][4g..4g+3] in a brick; rows,
// slices and column groups outside the 2K extent get an offset past the buffer (loads return 0).
template <int K>
__device__ inline uint32_t slice_offset(int v1, int g, int r) {
    constexpr int D = 2 * K;
    if (v1 >= D || r >= D || 4 * g >= D) return 0x40000000u;
    return (uint32_t)((((v1 * D) + r) * D + 4 * g) * 8);
}

template <int K, int TPW>
__device__ inline void load_slices(const double* __restrict__ X, int nbytes, const uint32_t (&off)[TPW], double (&x)[TPW][4]) {
    constexpr int D = 2 * K;
    // nbytes = 0 turns every load into an out-of-range one that returns zeros without touching memory
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, nbytes, 0x00020000);
    typedef double dv2 __attribute__((ext_vector_type(2)));
    for (int t = 0; t < TPW; ++t) {
        if constexpr (D % 4 == 0) {
            const dv2 a = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, off[t], 0, 0));
            const dv2 b = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, off[t] + 16, 0, 0));
            x[t][0] = a.x; x[t][1] = a.y; x[t][2] = b.x; x[t][3] = b.y;
        } else {
            // a 4-column group may cross the end of a row: load the valid columns one by one
            const uint32_t o = off[t];
            const int col = (int)((o / 8) % D);
            for (int kk = 0; kk < 4; ++kk) {
                const uint32_t ok = (o < 0x40000000u && col + kk < D) ? o + 8 * kk : 0x40000000u;
                x[t][kk] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, ok, 0, 0));
            }
        }
    }
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, not for its
// vector-memory loads, so prefetched input slices stay in flight across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One block per output brick, over all levels at once (order[] lists (level, brick)).  CW waves
// per block, each owning TPW input slices; PF steps of input slices are prefetched into registers.
// For every job the in-cube cells of its box are first compacted into an LDS list (ascending L1,
// L2, L3), so the term loop and the cell loop fuse into one stream of steps whose input bricks
// are known PF steps ahead (the same list repeats for every term of the job).
template <int K, int CW, int PF, int WPE>
__global__ void __launch_bounds__(64 * CW) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
ns_apply_kernel(const LevelDesc* __restrict__ levels, const int2* __restrict__ order, const double* __restrict__ w) {
    constexpr int CT = 64 * CW;
    constexpr int D = 2 * K;
    constexpr int TPW = (D + CW - 1) / CW;
    constexpr bool FULL = (CW * TPW == D);     // every wave owns TPW real slices
    constexpr int64_t E = (int64_t)D * D * D;
    constexpr int NB = PF + 1;
    __shared__ double T2s[16 * T2S_V1];
    __shared__ double S3s[NMAX * 16 * S3_V];
    __shared__ double S2s[NMAX * 256];
    __shared__ double S1s[NMAX * 256];
    __shared__ int2 steps[NMAX * NMAX * NMAX];
    __shared__ int nsteps_s;
    // wave index and every neighbour index are uniform per wave: keep them in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int2 job = order[blockIdx.x];
    const LevelDesc lv = levels[job.x];
    const int64_t b = job.y;
    const int Lr = lv.Lr;
    const int NL = 2 * Lr + 1;
    const int32_t* nb = lv.nbr + b * NL * NL * NL;
    const int cmb = lv.cmask[b];
    d4 Y[TPW];
    uint32_t xoff[TPW];
    for (int t = 0; t < TPW; ++t) {
        Y[t] = (d4){0.0, 0.0, 0.0, 0.0};
        xoff[t] = slice_offset<K>(wave * TPW + t, g, r);
    }
    for (int ti = 0; ti < lv.ntpl; ++ti) {
        const Tpl tp = lv.tpl[ti];
        if (tp.dpart && cmb == 0) continue;     // no internal child receives the down band
        const int n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
        // compact list of the box's in-cube cells: (input index, q1 << 4 | q2 << 2 | q3)
        lds_barrier();
        if (threadIdx.x < 64) {
            const int t = threadIdx.x;
            int idx = -1, q1 = 0, q2 = 0, q3 = 0;
            if (t < n1 * n2 * n3) {
                q1 = t / (n2 * n3);
                q2 = (t / n3) % n2;
                q3 = t % n3;
                idx = nb[((tp.lo[0] + q1 + Lr) * NL + (tp.lo[1] + q2 + Lr)) * NL + tp.lo[2] + q3 + Lr];
            }
            const unsigned long long in = __ballot(idx >= 0);
            if (idx >= 0) steps[__popcll(in & ((1ull << t) - 1ull))] = make_int2(idx, (q1 << 4) | (q2 << 2) | q3);
            if (t == 0) nsteps_s = __popcll(in);
        }
        lds_barrier();
        const int ns = __builtin_amdgcn_readfirstlane(nsteps_s);
        if (ns == 0) continue;
        const int total = __builtin_amdgcn_readfirstlane((tp.m2 - tp.m1 + 1) * ns);
        auto brick = [&](int si) -> const double* {
            const int idx = __builtin_amdgcn_readfirstlane(steps[si].x);
            return idx < lv.nreal ? lv.Xr + idx * E : lv.Xg + (idx - lv.nreal) * E;
        };
        // Loads are issued unconditionally (past the end with nbytes = 0) so that the compiler's
        // wait counts see one load group per step on every path.
        double xb[NB][TPW][4];
        int pf = 0;   // cell of the next prefetch
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const bool live = u < total;
            load_slices<K, TPW>(brick(pf), live ? (int)(E * 8) : 0, xoff, xb[u]);
            if (live && ++pf == ns) pf = 0;
        }
        int m = tp.m1, si = 0;
        d4 T1[TPW], T2[TPW];
        for (int t = 0; t < TPW; ++t) T1[t] = T2[t] = (d4){0.0, 0.0, 0.0, 0.0};
        for (int s0 = 0; s0 < total; s0 += NB) {
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (s0 + u >= total) break;
                if (si == 0) {
                    // stage this term's masked super-blocks in LDS (conflict-free reads; cw folded
                    // into S1) before the next prefetch, so waiting for these loads does not wait
                    // for it
                    const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
                    const double cw = tp.dpart ? -w[m] : w[m];
                    for (int e = threadIdx.x; e < (n1 + n2 + n3) * 256; e += CT) {
                        const int sb = e >> 8, v = (e >> 4) & 15, uu = e & 15;
                        if (sb < n1) S1s[sb * 256 + v * 16 + uu] = cw * sop<K>(Fm, tp.lo[0] + sb, tp.mlo[0], tp.mhi[0], uu, v);
                        else if (sb < n1 + n2) {
                            const int q = sb - n1;
                            S2s[q * 256 + v * 16 + uu] = sop<K>(Fm, tp.lo[1] + q, tp.mlo[1], tp.mhi[1], uu, v);
                        } else {
                            const int q = sb - n1 - n2;
                            S3s[q * 16 * S3_V + v * S3_V + uu] = sop<K>(Fm, tp.lo[2] + q, tp.mlo[2], tp.mhi[2], uu, v);
                        }
                    }
                    lds_barrier();
                }
                if (PF > 0) {
                    const bool live = s0 + u + PF < total;
                    load_slices<K, TPW>(brick(pf), live ? (int)(E * 8) : 0, xoff, xb[(u + PF) % NB]);
                    if (live && ++pf == ns) pf = 0;
                } else {
                    load_slices<K, TPW>(brick(si), (int)(E * 8), xoff, xb[u]);
                }
                const int cell = __builtin_amdgcn_readfirstlane(steps[si].y);
                const int next = si + 1 < ns ? __builtin_amdgcn_readfirstlane(steps[si + 1].y) : -1;
                // mode 3: T1 += X x_3 S3^{L3}
                {
                    const double* s3p = S3s + (cell & 3) * 16 * S3_V + r;
                    double s3[4];
                    for (int kk = 0; kk < 4; ++kk) s3[kk] = s3p[(4 * g + kk) * S3_V];
                    for (int kk = 0; kk < 4; ++kk)
                        for (int t = 0; t < TPW; ++t)
                            if (FULL || wave * TPW + t < D) T1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[u][t][kk], s3[kk], T1[t], 0, 0, 0);
                }
                if (next < 0 || (next >> 2) != (cell >> 2)) {
                    // end of an (L1, L2) row -- mode 2: T2 += S2^{L2} x_2 T1
                    const double* s2p = S2s + ((cell >> 2) & 3) * 256 + r;
                    double s2[4];
                    for (int i = 0; i < 4; ++i) s2[i] = s2p[(4 * i + g) * 16];
                    for (int i = 0; i < 4; ++i)
                        for (int t = 0; t < TPW; ++t)
                            if (FULL || wave * TPW + t < D) T2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(s2[i], T1[t][i], T2[t], 0, 0, 0);
                    for (int t = 0; t < TPW; ++t) T1[t] = (d4){0.0, 0.0, 0.0, 0.0};
                }
                if (next < 0 || (next >> 4) != (cell >> 4)) {
                    // end of an L1 plane -- mode 1 through an LDS transpose: Y += S1^{L1} x_1 T2
                    for (int t = 0; t < TPW; ++t) {
                        const int v1 = wave * TPW + t;
                        if (!FULL && v1 >= D) break;
                        for (int i = 0; i < 4; ++i) T2s[v1 * T2S_V1 + (4 * i + g) * T2S_U2 + r] = T2[t][i];
                    }
                    lds_barrier();
                    const double* s1p = S1s + (cell >> 4) * 256 + r;
                    double s1[4];
                    for (int kk = 0; kk < 4; ++kk) s1[kk] = s1p[(4 * kk + g) * 16];
                    for (int t = 0; t < TPW; ++t) {
                        const int u2 = wave * TPW + t;
                        if (!FULL && u2 >= D) break;
                        // the down band reaches only internal children: accumulate it apart, add it masked
                        d4 acc = tp.dpart ? (d4){0.0, 0.0, 0.0, 0.0} : Y[t];
                        for (int kk = 0; kk < 4; ++kk) {
                            const int v1 = 4 * kk + g;
                            const double bv = v1 < D ? T2s[v1 * T2S_V1 + u2 * T2S_U2 + r] : 0.0;
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s1[kk], bv, acc, 0, 0, 0);
                        }
                        if (tp.dpart) {
                            for (int i = 0; i < 4; ++i) {
                                const int child = (4 * i + g >= K) + 2 * (u2 >= K) + 4 * (r >= K);
                                if ((cmb >> child) & 1) Y[t][i] += acc[i];
                            }
                        } else {
                            Y[t] = acc;
                        }
                    }
                    for (int t = 0; t < TPW; ++t) T2[t] = (d4){0.0, 0.0, 0.0, 0.0};
                    lds_barrier();
                }
                if (++si == ns) {
                    si = 0;
                    ++m;
                }
            }
        }
    }
    double* ob = lv.out + b * E;
    for (int t = 0; t < TPW; ++t) {
        const int u2 = wave * TPW + t;
        if (u2 >= D) break;
        for (int i = 0; i < 4; ++i) {
            const int u1 = 4 * i + g, u3 = r;
            if (u1 >= D || u3 >= D) continue;
            const int child = (u1 >= K) + 2 * (u2 >= K) + 4 * (u3 >= K);
            ob[((int64_t)u1 * D + u2) * D + u3] = ((lv.valid >> child) & 1) ? Y[t][i] : 0.0;
        }
    }
}

// ---------------------------------------------------------------- closure
// For every output brick of level j (parent P at level j-1) and L in [-Lr,Lr]^3: index of the
// brick whose parent is P - L among the level's real bricks, -1 outside the cube, -2 when P - L is
// not an internal node (the key is written to miss[] for interpolation).
__global__ void closure_kernel(int64_t nout, int jm1, const uint64_t* __restrict__ pkeys, int Lr,
                               int32_t* __restrict__ nbr, uint64_t* __restrict__ miss) {
    const int NL = 2 * Lr + 1, NL3 = NL * NL * NL;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nout * NL3) return;
    const int64_t b = idx / NL3;
    const int e = (int)(idx % NL3);
    const int L[3] = {e / (NL * NL) - Lr, (e / NL) % NL - Lr, e % NL - Lr};
    int64_t p[3];
    key_coords(pkeys[b], p);
    const int64_t side = (int64_t)1 << jm1;
    int64_t q[3];
    bool inside = true;
    for (int d = 0; d < 3; ++d) {
        q[d] = p[d] - L[d];
        inside = inside && q[d] >= 0 && q[d] < side;
    }
    miss[idx] = ~0ull;
    if (!inside) { nbr[idx] = -1; return; }
    const uint64_t key = make_key(jm1, q[0], q[1], q[2]);
    const int64_t f = find_sorted(pkeys, nout, key);
    if (f >= 0) { nbr[idx] = (int32_t)f; return; }
    nbr[idx] = -2;
    miss[idx] = key;
}

__global__ void closure_fill_kernel(int64_t n, const uint64_t* __restrict__ miss, const uint64_t* __restrict__ gkeys,
                                    int64_t ng, int64_t nreal, int32_t* __restrict__ nbr) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n || nbr[idx] != -2) return;
    nbr[idx] = (int32_t)(nreal + find_sorted(gkeys, ng, miss[idx]));
}

// LDS helpers for the two-scale transforms with zero details (App. A.3, eqs. recon_even/odd).
// out = (A1 (x) A2 (x) A3) in, A_d given as Ht[s][a] = H^(s)^T ... applied per dimension.
template <int K>
__device__ void up_one(const double* __restrict__ Ht, const double* in, double* out, double* tmp1, double* tmp2, int s1,
                       int s2, int s3) {
    // child s of a block: (H^{s1}^T (x) H^{s2}^T (x) H^{s3}^T) in ; Ht = [H0^T ; H1^T] as [2][K][K] (row = child degree)
    constexpr int K3 = K * K * K;
    const double* A1 = Ht + s1 * K * K;
    const double* A2 = Ht + s2 * K * K;
    const double* A3 = Ht + s3 * K * K;
    for (int e = threadIdx.x; e < K3; e += AT) {
        const int c1 = e / (K * K), c2 = (e / K) % K, a3 = e % K;
        double s = 0.0;
        for (int c3 = 0; c3 < K; ++c3) s += A3[a3 * K + c3] * in[(c1 * K + c2) * K + c3];
        tmp1[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K3; e += AT) {
        const int c1 = e / (K * K), a2 = (e / K) % K, a3 = e % K;
        double s = 0.0;
        for (int c2 = 0; c2 < K; ++c2) s += A2[a2 * K + c2] * tmp1[(c1 * K + c2) * K + a3];
        tmp2[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K3; e += AT) {
        const int a1 = e / (K * K), a2 = (e / K) % K, a3 = e % K;
        double s = 0.0;
        for (int c1 = 0; c1 < K; ++c1) s += A1[a1 * K + c1] * tmp2[(c1 * K + a2) * K + a3];
        out[e] = s;
    }
    __syncthreads();
}

// brick (2K)^3 += or = (Ht (x) Ht (x) Ht) in, Ht = [H0^T; H1^T] (2K x K): all 8 children at once.
template <int K>
__device__ void up_brick(const double* __restrict__ Ht, const double* in, double* __restrict__ brick, bool add, double* tmp1,
                         double* tmp2) {
    constexpr int P = 2 * K;
    for (int e = threadIdx.x; e < K * K * P; e += AT) {
        const int c1 = e / (K * P), c2 = (e / P) % K, u3 = e % P;
        double s = 0.0;
        for (int c3 = 0; c3 < K; ++c3) s += Ht[u3 * K + c3] * in[(c1 * K + c2) * K + c3];
        tmp1[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * P * P; e += AT) {
        const int c1 = e / (P * P), u2 = (e / P) % P, u3 = e % P;
        double s = 0.0;
        for (int c2 = 0; c2 < K; ++c2) s += Ht[u2 * K + c2] * tmp1[(c1 * K + c2) * P + u3];
        tmp2[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < P * P * P; e += AT) {
        const int u1 = e / (P * P), u2 = (e / P) % P, u3 = e % P;
        double s = 0.0;
        for (int c1 = 0; c1 < K; ++c1) s += Ht[u1 * K + c1] * tmp2[(c1 * P + u2) * P + u3];
        brick[e] = add ? brick[e] + s : s;
    }
    __syncthreads();
}

template <int K>
__device__ void load_block(const double* __restrict__ brick, int child, double* out) {
    constexpr int P = 2 * K, K3 = K * K * K;
    const int s1 = child & 1, s2 = (child >> 1) & 1, s3 = child >> 2;
    for (int e = threadIdx.x; e < K3; e += AT) {
        const int a = e / (K * K), b = (e / K) % K, c = e % K;
        out[e] = brick[((s1 * K + a) * P + s2 * K + b) * P + s3 * K + c];
    }
    __syncthreads();
}

// Ghost bricks: the children of a node Q of level j-1 that is not internal, interpolated from the
// deepest existing ancestor (a leaf) by repeated zero-detail reconstruction (Alg. 3 Step 2).
template <int K>
__global__ void __launch_bounds__(AT) ghost_kernel(int jm1, const uint64_t* __restrict__ gkeys, const uint64_t* __restrict__ keys,
                                                   int64_t nnodes, LevelTab2 lt, const double* __restrict__ coef,
                                                   const double* __restrict__ Htg, double* __restrict__ gout) {
    constexpr int P = 2 * K, K3 = K * K * K;
    __shared__ double Ht[2 * K * K];
    __shared__ double blk[K3], tmp1[K * P * P], tmp2[K * P * P];
    for (int e = threadIdx.x; e < 2 * K * K; e += AT) Ht[e] = Htg[e];
    __syncthreads();
    const uint64_t q = gkeys[blockIdx.x];
    int64_t l[3];
    key_coords(q, l);
    int i = jm1;
    int64_t node = -1;
    for (; i >= 0; --i) {
        node = find_sorted(keys, nnodes, make_key(i, l[0] >> (jm1 - i), l[1] >> (jm1 - i), l[2] >> (jm1 - i)));
        if (node >= 0) break;
    }
    double* go = gout + (int64_t)blockIdx.x * P * P * P;
    if (node < 0) {   // cannot happen for a tree with a root; keep the brick defined
        for (int e = threadIdx.x; e < P * P * P; e += AT) go[e] = 0.0;
        return;
    }
    int64_t brick;
    int child;
    if (i == 0) { brick = 0; child = 0; }
    else {
        const int64_t r = node - lt.node_off[i];
        brick = lt.brick_off[i] + (r >> 3);
        child = (int)(r & 7);
    }
    load_block<K>(coef + brick * (int64_t)P * P * P, child, blk);
    for (int t = i + 1; t <= jm1; ++t) {
        const int sh = jm1 - t;
        up_one<K>(Ht, blk, blk, tmp1, tmp2, (l[0] >> sh) & 1, (l[1] >> sh) & 1, (l[2] >> sh) & 1);
    }
    up_brick<K>(Ht, blk, go, false, tmp1, tmp2);
}

// Assembly (eq. g_assemble): every brick of level j += the 8-child upsampling of its parent's g.
template <int K>
__global__ void __launch_bounds__(AT) assemble_kernel(int j, const int64_t* __restrict__ parent_brick,
                                                      const int* __restrict__ parent_child, int64_t brick_off,
                                                      const double* __restrict__ Htg, double* __restrict__ coef) {
    constexpr int P = 2 * K, K3 = K * K * K;
    __shared__ double Ht[2 * K * K];
    __shared__ double blk[K3], tmp1[K * P * P], tmp2[K * P * P];
    for (int e = threadIdx.x; e < 2 * K * K; e += AT) Ht[e] = Htg[e];
    __syncthreads();
    const int64_t b = blockIdx.x;
    load_block<K>(coef + parent_brick[b] * (int64_t)P * P * P, parent_child[b], blk);
    up_brick<K>(Ht, blk, coef + (brick_off + b) * (int64_t)P * P * P, true, tmp1, tmp2);
}

// Number of (node, l, m) triples with a non-zero coefficient, one thread per output node of
// level j.  Coefficients are c_m = [m in R_j(L)] - [internal][m in R_{j+1}(l)]; per node
//   sum_l |W(l) sym-diff D(l)| = sum_l |W(l)| + [internal] sum_{|l|<=3} (|D(l)| - 2 |W(l) & D(l)|),
// and sum_l |W(l)| = 8 sum_L |R_j(L)| over coarse L with P - L inside the cube (each coarse L
// carries the 8 children of P - L); at level 0 the only input is the root itself.
__device__ inline int range_len(const int32_t* r) { return r[1] >= r[0] ? r[1] - r[0] + 1 : 0; }

__global__ void count_kernel(int64_t nout, int j, const uint64_t* __restrict__ pkeys, const uint8_t* __restrict__ cmask,
                             int valid, const int32_t* __restrict__ Rj, const int32_t* __restrict__ Rj1,
                             unsigned long long* __restrict__ total) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nout * 8) return;
    const int64_t b = t >> 3;
    const int child = (int)(t & 7);
    if (!((valid >> child) & 1)) return;
    const int internal = (cmask[b] >> child) & 1;
    auto at = [](const int32_t* R, int x, int y, int z) {
        return R + (((x + LP) * NLP + (y + LP)) * NLP + (z + LP)) * 2;
    };
    long long cnt = 0;
    if (j == 0) {
        const int32_t* w = at(Rj, 0, 0, 0);
        cnt = range_len(w);
        if (internal && Rj1) {
            const int32_t* d = at(Rj1, 0, 0, 0);
            const int ov = (range_len(w) && range_len(d)) ? max(0, min(w[1], d[1]) - max(w[0], d[0]) + 1) : 0;
            cnt += range_len(d) - 2 * ov;
        }
        atomicAdd(total, (unsigned long long)cnt);
        return;
    }
    int64_t p[3];
    key_coords(pkeys[b], p);
    const int64_t pside = (int64_t)1 << (j - 1), side = (int64_t)1 << j;
    for (int x = -LP; x <= LP; ++x)
        for (int y = -LP; y <= LP; ++y)
            for (int z = -LP; z <= LP; ++z) {
                const int64_t q[3] = {p[0] - x, p[1] - y, p[2] - z};
                if (q[0] < 0 || q[0] >= pside || q[1] < 0 || q[1] >= pside || q[2] < 0 || q[2] >= pside) continue;
                cnt += 8 * range_len(at(Rj, x, y, z));
            }
    if (internal && Rj1) {
        const int64_t o[3] = {2 * p[0] + (child & 1), 2 * p[1] + ((child >> 1) & 1), 2 * p[2] + (child >> 2)};
        for (int e1 = -LP; e1 <= LP; ++e1)
            for (int e2 = -LP; e2 <= LP; ++e2)
                for (int e3 = -LP; e3 <= LP; ++e3) {
                    const int64_t q[3] = {o[0] - e1, o[1] - e2, o[2] - e3};
                    if (q[0] < 0 || q[0] >= side || q[1] < 0 || q[1] >= side || q[2] < 0 || q[2] >= side) continue;
                    const int L[3] = {(int)((o[0] >> 1) - (q[0] >> 1)), (int)((o[1] >> 1) - (q[1] >> 1)),
                                      (int)((o[2] >> 1) - (q[2] >> 1))};
                    const int32_t* w = at(Rj, L[0], L[1], L[2]);   // |L_d| <= 2 here
                    const int32_t* d = at(Rj1, e1, e2, e3);
                    const int ov = (range_len(w) && range_len(d)) ? max(0, min(w[1], d[1]) - max(w[0], d[0]) + 1) : 0;
                    cnt += range_len(d) - 2 * ov;
                }
    }
    atomicAdd(total, (unsigned long long)cnt);
}

// Tile variants of the contraction kernel: (waves per block, prefetch depth, waves per SIMD).
struct Variant {
    int cw, pf, wpe;
};
constexpr Variant VARIANTS[] = {{8, 0, 4}, {8, 1, 2}, {8, 2, 2}, {16, 1, 4}, {16, 2, 4}, {16, 3, 4}};
constexpr int NVARIANTS = sizeof(VARIANTS) / sizeof(VARIANTS[0]);

template <int K, int V>
void launch_variant(hipStream_t st, int64_t nblocks, const LevelDesc* levels, const int2* order, const double* w) {
    constexpr Variant v = VARIANTS[V];
    ns_apply_kernel<K, v.cw, v.pf, v.wpe><<<(unsigned)nblocks, 64 * v.cw, 0, st>>>(levels, order, w);
}

template <int K>
struct ApplyLaunch {
    static void run(hipStream_t st, int variant, int64_t nblocks, const LevelDesc* levels, const int2* order,
                    const double* w) {
        switch (variant) {
            case 0: launch_variant<K, 0>(st, nblocks, levels, order, w); break;
            case 1: launch_variant<K, 1>(st, nblocks, levels, order, w); break;
            case 2: launch_variant<K, 2>(st, nblocks, levels, order, w); break;
            case 3: launch_variant<K, 3>(st, nblocks, levels, order, w); break;
            case 4: launch_variant<K, 4>(st, nblocks, levels, order, w); break;
            case 5: launch_variant<K, 5>(st, nblocks, levels, order, w); break;
            default: fail(MWNS_EINVAL, "unknown contraction kernel variant");
        }
    }
};
template <int K>
struct GhostLaunch {
    static void run(hipStream_t st, int64_t ng, int jm1, const uint64_t* gk, const uint64_t* keys, int64_t nn,
                    const LevelTab2& lt, const double* coef, const double* Ht, double* gout) {
        ghost_kernel<K><<<(unsigned)ng, AT, 0, st>>>(jm1, gk, keys, nn, lt, coef, Ht, gout);
    }
};
template <int K>
struct AssembleLaunch {
    static void run(hipStream_t st, int64_t nb, int j, const int64_t* pb, const int* pc, int64_t off, const double* Ht,
                    double* coef) {
        assemble_kernel<K><<<(unsigned)nb, AT, 0, st>>>(j, pb, pc, off, Ht, coef);
    }
};

constexpr int DEFAULT_VARIANT = 0;   // (8 waves, no prefetch, 4 waves per SIMD): fastest on the k = 8 Poisson workload

int variant_for(const mwns_ctx* ctx, int k) {
    const int v = ctx->variant[k];
    return v >= 0 ? v : DEFAULT_VARIANT;
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
        default: fail(MWNS_EINVAL, "unsupported k");
    }
}

// Coarsest per-dimension partition of [-LP, LP] on which a plan row is constant; returns cells.
std::vector<std::array<int, 2>> segments(const int32_t* row, int d) {
    auto slice_equal = [&](int t) {   // plan slices at coordinate t and t+1 along dimension d
        for (int a = -LP; a <= LP; ++a)
            for (int b = -LP; b <= LP; ++b) {
                int c0[3], c1[3];
                c0[d] = t; c1[d] = t + 1;
                const int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
                c0[o1] = c1[o1] = a;
                c0[o2] = c1[o2] = b;
                const int32_t* r0 = row + (((c0[0] + LP) * NLP + (c0[1] + LP)) * NLP + (c0[2] + LP)) * 2;
                const int32_t* r1 = row + (((c1[0] + LP) * NLP + (c1[1] + LP)) * NLP + (c1[2] + LP)) * 2;
                const bool e0 = r0[1] < r0[0], e1 = r1[1] < r1[0];
                if (e0 != e1) return false;
                if (!e0 && (r0[0] != r1[0] || r0[1] != r1[1])) return false;
            }
        return true;
    };
    std::vector<std::array<int, 2>> seg;
    int start = -LP;
    for (int t = -LP; t < LP; ++t)
        if (!slice_equal(t)) {
            seg.push_back({start, t});
            start = t + 1;
        }
    seg.push_back({start, LP});
    return seg;
}

void append_templates(const int32_t* row, bool down, std::vector<Tpl>& out) {
    std::vector<std::array<int, 2>> s[3];
    for (int d = 0; d < 3; ++d) s[d] = segments(row, d);
    for (auto& a : s[0])
        for (auto& b : s[1])
            for (auto& c : s[2]) {
                const int32_t* rr = row + (((a[0] + LP) * NLP + (b[0] + LP)) * NLP + (c[0] + LP)) * 2;
                if (rr[1] < rr[0]) continue;
                Tpl t{};
                const std::array<int, 2>* cell[3] = {&a, &b, &c};
                for (int d = 0; d < 3; ++d) {
                    const int lo = (*cell[d])[0], hi = (*cell[d])[1];
                    if (down) {   // fine l in [lo, hi]  <=>  coarse L in [ceil((lo-1)/2), floor((hi+1)/2)]
                        t.lo[d] = (int)std::ceil((lo - 1) / 2.0);
                        t.hi[d] = (int)std::floor((hi + 1) / 2.0);
                        t.mlo[d] = lo;
                        t.mhi[d] = hi;
                    } else {
                        t.lo[d] = lo;
                        t.hi[d] = hi;
                        t.mlo[d] = -LF;
                        t.mhi[d] = LF;
                    }
                }
                t.m1 = rr[0];
                t.m2 = rr[1];
                t.dpart = down ? 1 : 0;
                out.push_back(t);
            }
}

LevelTab2 level_tab2(const mwns_tree* t) {
    LevelTab2 lt{};
    for (int j = 0; j <= t->depth; ++j) {
        lt.node_off[j] = t->lev[j].node_off;
        lt.brick_off[j] = t->lev[j].brick_off;
    }
    lt.depth = t->depth;
    return lt;
}

struct Timer {
    hipEvent_t a, b;
    hipStream_t st;
    explicit Timer(hipStream_t s) : st(s) {
        MWNS_HIP(hipEventCreate(&a));
        MWNS_HIP(hipEventCreate(&b));
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    void start() { MWNS_HIP(hipEventRecord(a, st)); }
    void stop() { MWNS_HIP(hipEventRecord(b, st)); }
    double ms() {
        MWNS_HIP(hipEventSynchronize(b));
        float v = 0.f;
        MWNS_HIP(hipEventElapsedTime(&v, a, b));
        return v;
    }
};

}  // namespace
}  // namespace mwns

using namespace mwns;

extern "C" int mwns_num_variants(void) { return NVARIANTS; }

extern "C" mwns_status mwns_ctx_set_variant(mwns_ctx* ctx, int k, int variant) {
    MWNS_GUARD_BEGIN
    if (!ctx) fail(MWNS_EINVAL, "ctx is NULL");
    if (k < 1 || k > KMAX) fail(MWNS_EINVAL, "k out of range");
    if (variant < -1 || variant >= NVARIANTS) fail(MWNS_EINVAL, "variant out of range");
    ctx->variant[k] = variant;
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_ctx_get_variant(const mwns_ctx* ctx, int k, int* variant) {
    MWNS_GUARD_BEGIN
    if (!ctx || !variant) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > KMAX) fail(MWNS_EINVAL, "k out of range");
    *variant = ctx->variant[k];
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_apply(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, int mode, mwns_tree** g,
                                  mwns_apply_stats* stats) {
    MWNS_GUARD_BEGIN
    if (!ctx || !op || !f || !g) fail(MWNS_EINVAL, "NULL argument");
    if ((mode & 0xff) != MWNS_F64) fail(MWNS_EINVAL, "unsupported precision mode");
    if (op->k != f->k) fail(MWNS_EINVAL, "operator and tree have different k");
    if (op->max_level < f->depth) fail(MWNS_EINVAL, "operator max_level is below the tree depth");
    const int k = f->k;
    const int64_t E = brick_elems(k);
    hipStream_t st = ctx->stream;
    std::unique_ptr<mwns_tree> out(new mwns_tree);
    out->ctx = ctx;
    out->k = k;
    out->depth = f->depth;
    out->nnodes = f->nnodes;
    out->nleaves = f->nleaves;
    out->nbricks = f->nbricks;
    out->lev = f->lev;
    out->keys = f->keys;
    out->leaf = f->leaf;
    out->brick_parent = f->brick_parent;
    out->dkeys.reset(ctx, f->nnodes);
    out->dleaf.reset(ctx, f->nnodes);
    MWNS_HIP(hipMemcpyAsync(out->dkeys.p, f->dkeys.p, f->nnodes * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    MWNS_HIP(hipMemcpyAsync(out->dleaf.p, f->dleaf.p, f->nnodes, hipMemcpyDeviceToDevice, st));
    out->coef.reset(ctx, (size_t)f->nbricks * E);
    LevelTab2 lt = level_tab2(f);
    std::vector<double> Ht(2 * k * k);
    {
        std::vector<double> H(2 * k * k);
        two_scale_filters(k, H.data(), H.data() + k * k);
        for (int s = 0; s < 2; ++s)
            for (int a = 0; a < k; ++a)
                for (int c = 0; c < k; ++c) Ht[s * k * k + c * k + a] = H[s * k * k + a * k + c];
    }
    DevArray<double> dHt(ctx, Ht.size());
    dHt.upload(Ht.data(), Ht.size(), st);
    const int depth = f->depth;
    const int64_t planrow = (int64_t)NLP3 * 2;
    struct LevelWork {
        std::vector<Tpl> tpl;
        std::vector<uint8_t> cm;
        std::vector<uint64_t> pk;
        int Lr = 0;
        int64_t nout = 0, nghost = 0, nleafonly = 0, miss_off = 0;
        int valid = 0xff;
        DevArray<int32_t> nbr;
        DevArray<uint8_t> cmask;
        DevArray<Tpl> dtpl;
        DevArray<double> ghosts;
        DevArray<uint64_t> pkeys, gkeys;
    };
    std::vector<LevelWork> W(depth + 1);
    Timer tclos(st), tcon(st), tasm(st);
    tclos.start();
    // ---- jobs of every level: whole band from plan row j, down band from row j+1
    int64_t miss_total = 0;
    for (int j = 0; j <= depth; ++j) {
        LevelWork& lw = W[j];
        const mwns_level& L = f->lev[j];
        lw.nout = L.nbricks;
        std::vector<Tpl> raw;
        if (j == 0) {
            Tpl t{};
            for (int d = 0; d < 3; ++d) { t.lo[d] = t.hi[d] = 0; t.mlo[d] = -LF; t.mhi[d] = LF; }
            const int32_t* r0 = op->plan.data() + (((LP * NLP) + LP) * NLP + LP) * 2;
            t.m1 = r0[0];
            t.m2 = r0[1];
            if (t.m2 >= t.m1) raw.push_back(t);
            lw.valid = 0x01;
        } else {
            append_templates(op->plan.data() + (int64_t)j * planrow, false, raw);
        }
        if (j < depth && j + 1 <= op->max_level) append_templates(op->plan.data() + (int64_t)(j + 1) * planrow, true, raw);
        for (const Tpl& t : raw) {   // split boxes so that every extent is <= NMAX
            int cuts[3][8][2], nc[3];
            for (int d = 0; d < 3; ++d) {
                nc[d] = 0;
                for (int a = t.lo[d]; a <= t.hi[d]; a += NMAX) {
                    cuts[d][nc[d]][0] = a;
                    cuts[d][nc[d]][1] = std::min(t.hi[d], a + NMAX - 1);
                    ++nc[d];
                }
            }
            for (int x = 0; x < nc[0]; ++x)
                for (int y = 0; y < nc[1]; ++y)
                    for (int z = 0; z < nc[2]; ++z) {
                        Tpl q = t;
                        q.lo[0] = cuts[0][x][0]; q.hi[0] = cuts[0][x][1];
                        q.lo[1] = cuts[1][y][0]; q.hi[1] = cuts[1][y][1];
                        q.lo[2] = cuts[2][z][0]; q.hi[2] = cuts[2][z][1];
                        lw.tpl.push_back(q);
                    }
        }
        int Lr = 0;
        for (const Tpl& t : lw.tpl)
            for (int d = 0; d < 3; ++d) Lr = std::max(Lr, std::max(std::abs(t.lo[d]), std::abs(t.hi[d])));
        lw.Lr = Lr;
        const int NL = 2 * Lr + 1, NL3 = NL * NL * NL;
        lw.cm.assign(lw.nout, 0);
        if (j == 0) lw.cm[0] = f->leaf[0] ? 0 : 1;
        else
            for (int64_t b = 0; b < lw.nout; ++b)
                for (int s = 0; s < 8; ++s)
                    if (!f->leaf[L.node_off + 8 * b + s]) lw.cm[b] |= (uint8_t)(1 << s);
        for (int64_t b = 0; b < lw.nout; ++b) lw.nleafonly += lw.cm[b] == 0;
        lw.cmask.reset(ctx, lw.nout);
        lw.cmask.upload(lw.cm.data(), lw.nout, st);
        lw.nbr.reset(ctx, (size_t)lw.nout * NL3);
        if (j > 0) {
            lw.pk.resize(lw.nout);
            for (int64_t b = 0; b < lw.nout; ++b) lw.pk[b] = f->keys[f->brick_parent[L.brick_off + b]];
            lw.pkeys.reset(ctx, lw.nout);
            lw.pkeys.upload(lw.pk.data(), lw.nout, st);
        }
        if (lw.tpl.empty()) continue;
        if (j == 0) {
            std::vector<int32_t> nb(NL3, -1);
            nb[(Lr * NL + Lr) * NL + Lr] = 0;
            lw.nbr.upload(nb.data(), NL3, st);
            continue;
        }
        lw.miss_off = miss_total;
        miss_total += lw.nout * NL3;
    }
    // ---- neighbour closure: all levels, one host round trip for the missing-key sets
    DevArray<uint64_t> miss(ctx, std::max<int64_t>(1, miss_total));
    for (int j = 1; j <= depth; ++j) {
        LevelWork& lw = W[j];
        if (lw.tpl.empty()) continue;
        const int NL = 2 * lw.Lr + 1;
        const int64_t n = lw.nout * NL * NL * NL;
        closure_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(lw.nout, j - 1, lw.pkeys.p, lw.Lr, lw.nbr.p,
                                                                    miss.p + lw.miss_off);
        MWNS_HIP(hipGetLastError());
    }
    std::vector<uint64_t> hm(miss_total);
    miss.download(hm.data(), miss_total, st);
    MWNS_HIP(hipStreamSynchronize(st));
    int64_t total_ghosts = 0;
    for (int j = 1; j <= depth; ++j) {
        LevelWork& lw = W[j];
        if (lw.tpl.empty()) continue;
        const int NL = 2 * lw.Lr + 1;
        const int64_t n = lw.nout * NL * NL * NL;
        std::vector<uint64_t> gk;
        for (int64_t i = 0; i < n; ++i)
            if (hm[lw.miss_off + i] != ~0ull) gk.push_back(hm[lw.miss_off + i]);
        std::sort(gk.begin(), gk.end());
        gk.erase(std::unique(gk.begin(), gk.end()), gk.end());
        lw.nghost = (int64_t)gk.size();
        total_ghosts += lw.nghost;
        if (!lw.nghost) continue;
        lw.gkeys.reset(ctx, gk.size());
        lw.gkeys.upload(gk.data(), gk.size(), st);
        closure_fill_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, miss.p + lw.miss_off, lw.gkeys.p, lw.nghost,
                                                                         lw.nout, lw.nbr.p);
        MWNS_HIP(hipGetLastError());
        lw.ghosts.reset(ctx, (size_t)lw.nghost * E);
        dispatch_k<GhostLaunch>(k, st, lw.nghost, j - 1, lw.gkeys.p, f->dkeys.p, f->nnodes, lt, f->coef.p, dHt.p,
                                lw.ghosts.p);
        MWNS_HIP(hipGetLastError());
    }
    tclos.stop();
    // ---- contractions: one launch over every output brick of every level, costliest first
    std::vector<LevelDesc> descs(depth + 1);
    std::vector<std::pair<double, int2>> cost;
    int64_t jobs = 0;
    double flops = 0.0;
    for (int j = 0; j <= depth; ++j) {
        LevelWork& lw = W[j];
        double* outj = out->coef.p + f->lev[j].brick_off * E;
        LevelDesc& d = descs[j];
        d = LevelDesc{};
        d.out = outj;
        if (lw.tpl.empty()) {
            MWNS_HIP(hipMemsetAsync(outj, 0, lw.nout * E * sizeof(double), st));
            continue;
        }
        lw.dtpl.reset(ctx, lw.tpl.size());
        lw.dtpl.upload(lw.tpl.data(), lw.tpl.size(), st);
        d.Xr = f->coef.p + f->lev[j].brick_off * E;
        d.Xg = lw.ghosts.p;
        d.nbr = lw.nbr.p;
        d.cmask = lw.cmask.p;
        d.tpl = lw.dtpl.p;
        d.Fj = op->F.p + (int64_t)j * op->M * NLF * k * k;
        d.nreal = lw.nout;
        d.Lr = lw.Lr;
        d.valid = lw.valid;
        d.ntpl = (int)lw.tpl.size();
        const int64_t pside = j > 0 ? ((int64_t)1 << (j - 1)) : 1;
        for (int64_t b = 0; b < lw.nout; ++b) {
            int64_t p[3] = {0, 0, 0};
            if (j > 0) key_coords(lw.pk[b], p);
            double c = 0.0;
            for (const Tpl& t : lw.tpl) {
                if (t.dpart && lw.cm[b] == 0) continue;
                double nin[3];
                for (int dd = 0; dd < 3; ++dd) {
                    int cnt = 0;
                    for (int Lx = t.lo[dd]; Lx <= t.hi[dd]; ++Lx) cnt += (p[dd] - Lx >= 0 && p[dd] - Lx < pside);
                    nin[dd] = cnt;
                }
                const double nt = t.m2 - t.m1 + 1;
                c += nt * (nin[0] * nin[1] * nin[2] + nin[0] * nin[1] + nin[0]);
                const double D2 = 2.0 * k;
                const double n1 = t.hi[0] - t.lo[0] + 1, n2 = t.hi[1] - t.lo[1] + 1, n3 = t.hi[2] - t.lo[2] + 1;
                (void)n2;
                (void)n3;
                (void)n1;
                jobs += (int64_t)nt;
                flops += nt * 2.0 * D2 * D2 * D2 * D2 * (nin[0] * nin[1] * nin[2] + nin[0] * nin[1] + nin[0]);
            }
            cost.push_back({c, make_int2(j, (int)b)});
        }
    }
    // Launch order.  Workgroups are dealt round-robin to the 8 XCDs, each with its own L2, and the
    // input sibling groups of neighbouring output bricks overlap: so levels go costliest first,
    // each level is cut into 8 contiguous Morton ranges of equal length, and block 8i + x takes
    // the i-th brick of range x, keeping every XCD on one compact region of the tree at a time.
    std::vector<int2> order;
    order.reserve(cost.size());
    {
        std::vector<std::pair<double, int>> lev_cost;   // (cost per brick, level)
        size_t pos = 0;
        std::vector<size_t> lev_begin(depth + 2, 0);
        for (int j = 0; j <= depth; ++j) {
            lev_begin[j] = pos;
            double c = 0.0;
            size_t n = 0;
            while (pos < cost.size() && cost[pos].second.x == j) { c += cost[pos].first; ++pos; ++n; }
            if (n) lev_cost.push_back({c / n, j});
        }
        lev_begin[depth + 1] = pos;
        std::stable_sort(lev_cost.begin(), lev_cost.end(),
                         [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first > b.first; });
        constexpr int NXCD = 8;
        for (const auto& lc : lev_cost) {
            const int j = lc.second;
            const size_t b0 = lev_begin[j];
            size_t n = 0;
            while (b0 + n < cost.size() && cost[b0 + n].second.x == j) ++n;
            const size_t per = (n + NXCD - 1) / NXCD;
            for (size_t i = 0; i < per; ++i)
                for (int x = 0; x < NXCD; ++x) {
                    const size_t idx = x * per + i;
                    if (idx < n) order.push_back(cost[b0 + idx].second);
                }
        }
    }
    DevArray<LevelDesc> ddesc(ctx, descs.size());
    ddesc.upload(descs.data(), descs.size(), st);
    DevArray<int2> dorder(ctx, std::max<size_t>(1, order.size()));
    dorder.upload(order.data(), order.size(), st);
    tcon.start();
    if (!order.empty()) {
        dispatch_k<ApplyLaunch>(k, st, variant_for(ctx, k), (int64_t)order.size(), ddesc.p, dorder.p, op->dw.p);
        MWNS_HIP(hipGetLastError());
    }
    tcon.stop();
    // ---- assembly (eq. g_assemble), level by level on the stream
    tasm.start();
    std::vector<DevArray<int64_t>> apb(depth + 1);
    std::vector<DevArray<int>> apc(depth + 1);
    if (!(mode & MWNS_NO_ASSEMBLY)) {
        for (int j = 1; j <= depth; ++j) {
            const mwns_level& L = f->lev[j];
            std::vector<int64_t> pb(L.nbricks);
            std::vector<int> pc(L.nbricks);
            for (int64_t b = 0; b < L.nbricks; ++b) node_brick(f, f->brick_parent[L.brick_off + b], &pb[b], &pc[b]);
            apb[j].reset(ctx, pb.size());
            apc[j].reset(ctx, pc.size());
            apb[j].upload(pb.data(), pb.size(), st);
            apc[j].upload(pc.data(), pc.size(), st);
            dispatch_k<AssembleLaunch>(k, st, L.nbricks, j, apb[j].p, apc[j].p, L.brick_off, dHt.p, out->coef.p);
            MWNS_HIP(hipGetLastError());
        }
    }
    tasm.stop();
    if (stats) {
        mwns_apply_stats s{};
        DevArray<unsigned long long> tot(ctx, 1);
        MWNS_HIP(hipMemsetAsync(tot.p, 0, sizeof(unsigned long long), st));
        DevArray<int32_t> dplan(ctx, op->plan.size());
        dplan.upload(op->plan.data(), op->plan.size(), st);
        for (int j = 0; j <= depth; ++j) {
            const LevelWork& lw = W[j];
            const int32_t* Rj1 = (j + 1 <= op->max_level) ? dplan.p + (int64_t)(j + 1) * planrow : nullptr;
            count_kernel<<<(unsigned)((lw.nout * 8 + 255) / 256), 256, 0, st>>>(lw.nout, j, lw.pkeys.p, lw.cmask.p, lw.valid,
                                                                                dplan.p + (int64_t)j * planrow, Rj1, tot.p);
            MWNS_HIP(hipGetLastError());
        }
        unsigned long long c = 0;
        tot.download(&c, 1, st);
        MWNS_HIP(hipStreamSynchronize(st));
        s.contractions = (int64_t)c;
        s.brick_jobs = jobs;
        s.ghost_bricks = total_ghosts;
        s.useful_flops = flops;
        s.ms_closure = tclos.ms();
        s.ms_contract = tcon.ms();
        s.ms_assemble = tasm.ms();
        *stats = s;
    } else {
        MWNS_HIP(hipStreamSynchronize(st));
    }
    *g = out.release();
    return MWNS_OK;
    MWNS_GUARD_END
}
