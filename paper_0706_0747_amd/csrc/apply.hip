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
    int prec;              // precision class of the job's terms (PREC_*)
};

// Precision classes of a job.  Every class accumulates into the FP64 output; the reduced ones
// take their inputs from FP32 or split-BF16 copies of the input bricks and accumulate each
// mode product in FP32.
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16C = 2, PREC_BF16 = 3, NPREC = 4 };

constexpr int AT = 256;            // threads per block of the transform kernels
constexpr int T2S_V1 = 272;        // LDS strides of the FP64 mode-2 result [v1][u2][u3] (conflict-free)
constexpr int T2S_U2 = 16;
constexpr int T2F_V1 = 324;        // the same for the FP32 mode-2 result (64 distinct banks per access)
constexpr int T2F_U2 = 20;
constexpr int NMAX = 4;            // largest box extent per dimension of one job (the host splits boxes)
constexpr int S3_V = 36;           // LDS stride of the staged FP64 mode-3 operand [L][v][u]
constexpr int SF_V = 20;           // LDS stride of the staged FP32 operands [L][v][u]
// LDS of the contraction kernel, in doubles: the FP64 layout is the largest of the classes.
constexpr int SM_T2 = 16 * T2S_V1, SM_S3 = NMAX * 16 * S3_V, SM_S2 = NMAX * 256, SM_S1 = NMAX * 256;
constexpr int SMEM_DOUBLES = SM_T2 + SM_S3 + SM_S2 + SM_S1;
static_assert(16 * T2F_V1 / 2 + 3 * NMAX * 16 * SF_V / 2 <= SMEM_DOUBLES, "FP32 LDS layout");
static_assert(16 * T2F_V1 / 2 + 3 * NMAX * 16 * 4 * 2 <= SMEM_DOUBLES, "BF16 LDS layout");

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// One level of the apply as seen by the contraction kernel.
struct LevelDesc {
    const double* Xr;        // real input bricks of the level (the level's own bricks)
    const double* Xg;        // ghost input bricks
    const float* Xr32;       // FP32 copies, rows padded to 16: [brick][v1][v2][16]  (or null)
    const float* Xg32;
    const u4* Xrb;           // split-BF16 copies: [brick][v1][v2][4 groups] of (4 hi, 4 lo)  (or null)
    const u4* Xgb;
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

// Byte offset of lane (g, r)'s 16-byte group in the padded reduced-precision copies (FP32 or
// split BF16; both hold 64 bytes per (v1, v2) row).
template <int K>
__device__ inline uint32_t slice_offset_lp(int v1, int g, int r) {
    constexpr int D = 2 * K;
    if (v1 >= D || r >= D) return 0x40000000u;
    return (uint32_t)(((v1 * D) + r) * 64 + 16 * g);
}

template <int K, int TPW>
__device__ inline void load_slices(const double* __restrict__ X, int nbytes, const uint32_t (&off)[TPW], d4 (&x)[TPW]) {
    constexpr int D = 2 * K;
    // nbytes = 0 turns every load into an out-of-range one that returns zeros without touching memory
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, nbytes, 0x00020000);
    typedef double dv2 __attribute__((ext_vector_type(2)));
    for (int t = 0; t < TPW; ++t) {
        if constexpr (D % 4 == 0) {
            const dv2 a = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, off[t], 0, 0));
            const dv2 b = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, off[t] + 16, 0, 0));
            x[t] = (d4){a.x, a.y, b.x, b.y};
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

template <int TPW>
__device__ inline void load_slices_lp(const void* __restrict__ X, int nbytes, const uint32_t (&off)[TPW], u4 (&x)[TPW]) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, nbytes, 0x00020000);
    for (int t = 0; t < TPW; ++t) x[t] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(rs, off[t], 0, 0));
}

// Split of four FP32 values into BF16 hi and lo parts (hi + lo carries 16 significant bits):
// returns (hi0 hi1 | hi2 hi3 | lo0 lo1 | lo2 lo3) packed two per dword.
__device__ inline u4 split4(f4 x) {
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    bf2 h01 = {(__bf16)x[0], (__bf16)x[1]}, h23 = {(__bf16)x[2], (__bf16)x[3]};
    bf2 l01 = {(__bf16)(x[0] - (float)h01[0]), (__bf16)(x[1] - (float)h01[1])};
    bf2 l23 = {(__bf16)(x[2] - (float)h23[0]), (__bf16)(x[3] - (float)h23[1])};
    return (u4){__builtin_bit_cast(unsigned, h01), __builtin_bit_cast(unsigned, h23), __builtin_bit_cast(unsigned, l01),
                __builtin_bit_cast(unsigned, l23)};
}

// A x B over 16 contraction slots per operand pair with split-BF16 operands a = (4 hi | 4 lo) and
// b = (4 hi | 4 lo) of the same 4 contraction indices: the 16x16x32 BF16 MFMA sees the slots
// (a_hi b_hi | a_lo b_hi) and, when compensated, (a_hi b_lo | a_lo b_lo): all four partial
// products, exact in FP32, summed in FP32.  Uncompensated: (a_hi + a_lo) b_hi.
template <bool COMP>
__device__ inline f4 mfma_bf16x(u4 a, u4 b, f4 c) {
    const bf8 A = __builtin_bit_cast(bf8, a);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf8, (u4){b[0], b[1], b[0], b[1]}), c, 0, 0, 0);
    if constexpr (COMP) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf8, (u4){b[2], b[3], b[2], b[3]}), c, 0, 0, 0);
    return c;
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, not for its
// vector-memory loads, so prefetched input slices stay in flight across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Rows of the FP32 mode-1 operand: output row m of the MFMA tile holds u1 = perm_row(m), so that
// register i of lane (g, r) holds u1 = 4i + g as in the FP64 layout of the output accumulators.
__device__ inline int perm_row(int m) { return 4 * (m & 3) + (m >> 2); }

template <int PREC>
struct ClassTypes;
template <>
struct ClassTypes<PREC_F64> { using Acc = d4; using XV = d4; };
template <int PREC>
struct ClassTypes { using Acc = f4; using XV = u4; };

// The terms of one job for one output brick (see the kernel below), in precision class PREC.
template <int K, int CW, int PF, int PREC>
__device__ __forceinline__ void run_job(const LevelDesc& lv, const Tpl& tp, const double* __restrict__ w, int ns,
                                        const int2* steps, double* smem, int wave, int g, int r, int cmb,
                                        d4 (&Y)[(2 * K + CW - 1) / CW]) {
    constexpr int CT = 64 * CW;
    constexpr int D = 2 * K;
    constexpr int TPW = (D + CW - 1) / CW;
    constexpr bool FULL = (CW * TPW == D);
    constexpr int64_t E = (int64_t)D * D * D;
    constexpr int64_t ELP = (int64_t)D * D * 64;   // bytes of a reduced-precision brick
    constexpr int NB = PF + 1;
    using Acc = typename ClassTypes<PREC>::Acc;
    using XV = typename ClassTypes<PREC>::XV;
    const int n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
    const int total = __builtin_amdgcn_readfirstlane((tp.m2 - tp.m1 + 1) * ns);
    // LDS carve-up of this class
    double* T2s = smem;
    double* S3s = smem + SM_T2;
    double* S2s = S3s + SM_S3;
    double* S1s = S2s + SM_S2;
    float* T2f = reinterpret_cast<float*>(smem);
    float* S3f = T2f + 16 * T2F_V1;
    float* S2f = S3f + NMAX * 16 * SF_V;
    float* S1f = S2f + NMAX * 16 * SF_V;
    u4* S3b = reinterpret_cast<u4*>(T2f + 16 * T2F_V1);   // [L][u][4 groups] of (4 hi | 4 lo)
    u4* S2b = S3b + NMAX * 64;
    u4* S1b = S2b + NMAX * 64;
    uint32_t xoff[TPW];
    for (int t = 0; t < TPW; ++t)
        xoff[t] = PREC == PREC_F64 ? slice_offset<K>(wave * TPW + t, g, r) : slice_offset_lp<K>(wave * TPW + t, g, r);
    auto load = [&](int si, bool live, XV (&x)[TPW]) {
        const int idx = __builtin_amdgcn_readfirstlane(steps[si].x);
        const bool real = idx < lv.nreal;
        const int64_t q = real ? idx : idx - lv.nreal;
        if constexpr (PREC == PREC_F64) {
            load_slices<K, TPW>((real ? lv.Xr : lv.Xg) + q * E, live ? (int)(E * 8) : 0, xoff, x);
        } else if constexpr (PREC == PREC_F32) {
            load_slices_lp<TPW>((const char*)(real ? lv.Xr32 : lv.Xg32) + q * ELP, live ? (int)ELP : 0, xoff, x);
        } else {
            load_slices_lp<TPW>((const char*)(real ? lv.Xrb : lv.Xgb) + q * ELP, live ? (int)ELP : 0, xoff, x);
        }
    };
    XV xb[NB][TPW];
    int pf = 0;   // cell of the next prefetch
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const bool live = u < total;
        load(pf, live, xb[u]);
        if (live && ++pf == ns) pf = 0;
    }
    int m = tp.m1, si = 0;
    Acc T1[TPW], T2[TPW];
    for (int t = 0; t < TPW; ++t) T1[t] = T2[t] = Acc{};
    for (int s0 = 0; s0 < total; s0 += NB) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            if (s0 + u >= total) break;
            if (si == 0) {
                // stage this term's masked super-blocks in LDS (cw folded into S1), before the next
                // prefetch so that waiting for these loads does not wait for it
                const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
                const double cw = tp.dpart ? -w[m] : w[m];
                if constexpr (PREC == PREC_F64 || PREC == PREC_F32) {
                    for (int e = threadIdx.x; e < (n1 + n2 + n3) * 256; e += CT) {
                        const int sb = e >> 8, v = (e >> 4) & 15, uu = e & 15;
                        int q, d;
                        if (sb < n1) { q = sb; d = 0; }
                        else if (sb < n1 + n2) { q = sb - n1; d = 1; }
                        else { q = sb - n1 - n2; d = 2; }
                        const double val = (d == 0 ? cw : 1.0) * sop<K>(Fm, tp.lo[d] + q, tp.mlo[d], tp.mhi[d], uu, v);
                        if constexpr (PREC == PREC_F64) {
                            double* dst = d == 0 ? S1s + q * 256 + v * 16 : d == 1 ? S2s + q * 256 + v * 16 : S3s + q * 16 * S3_V + v * S3_V;
                            dst[uu] = val;
                        } else {
                            float* dst = (d == 0 ? S1f : d == 1 ? S2f : S3f) + (q * 16 + v) * SF_V;
                            dst[uu] = (float)val;
                        }
                    }
                } else {
                    // split BF16: one thread per (super-block, row u, group of 4 contraction indices)
                    for (int e = threadIdx.x; e < (n1 + n2 + n3) * 64; e += CT) {
                        const int sb = e >> 6, uu = (e >> 2) & 15, gg = e & 3;
                        int q, d;
                        if (sb < n1) { q = sb; d = 0; }
                        else if (sb < n1 + n2) { q = sb - n1; d = 1; }
                        else { q = sb - n1 - n2; d = 2; }
                        const double sc = d == 0 ? cw : 1.0;
                        f4 v4;
                        for (int c = 0; c < 4; ++c) v4[c] = (float)(sc * sop<K>(Fm, tp.lo[d] + q, tp.mlo[d], tp.mhi[d], uu, 4 * gg + c));
                        (d == 0 ? S1b : d == 1 ? S2b : S3b)[(q * 16 + uu) * 4 + gg] = split4(v4);
                    }
                }
                lds_barrier();
            }
            if (PF > 0) {
                const bool live = s0 + u + PF < total;
                load(pf, live, xb[(u + PF) % NB]);
                if (live && ++pf == ns) pf = 0;
            } else {
                load(si, true, xb[u]);
            }
            const int cell = __builtin_amdgcn_readfirstlane(steps[si].y);
            const int next = si + 1 < ns ? __builtin_amdgcn_readfirstlane(steps[si + 1].y) : -1;
            const int q1 = cell >> 4, q2 = (cell >> 2) & 3, q3 = cell & 3;
            // mode 3: T1 += X x_3 S3^{L3}
            if constexpr (PREC == PREC_F64) {
                const double* s3p = S3s + q3 * 16 * S3_V + r;
                double s3[4];
                for (int kk = 0; kk < 4; ++kk) s3[kk] = s3p[(4 * g + kk) * S3_V];
                for (int kk = 0; kk < 4; ++kk)
                    for (int t = 0; t < TPW; ++t)
                        if (FULL || wave * TPW + t < D) T1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[u][t][kk], s3[kk], T1[t], 0, 0, 0);
            } else if constexpr (PREC == PREC_F32) {
                const float* s3p = S3f + q3 * 16 * SF_V + r;
                float s3[4];
                for (int kk = 0; kk < 4; ++kk) s3[kk] = s3p[(4 * g + kk) * SF_V];
                // reinterpret the whole vector: a bit_cast of one subscripted vector element is
                // miscompiled (it reads element 0 whatever the subscript)
                f4 xf[TPW];
                for (int t = 0; t < TPW; ++t) xf[t] = __builtin_bit_cast(f4, xb[u][t]);
                for (int kk = 0; kk < 4; ++kk)
                    for (int t = 0; t < TPW; ++t)
                        if (FULL || wave * TPW + t < D) T1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xf[t][kk], s3[kk], T1[t], 0, 0, 0);
            } else {
                const u4 s3 = S3b[(q3 * 16 + r) * 4 + g];
                for (int t = 0; t < TPW; ++t)
                    if (FULL || wave * TPW + t < D) T1[t] = mfma_bf16x<PREC == PREC_BF16C>(xb[u][t], s3, T1[t]);
            }
            if (next < 0 || (next >> 2) != (cell >> 2)) {
                // end of an (L1, L2) row -- mode 2: T2 += S2^{L2} x_2 T1
                if constexpr (PREC == PREC_F64) {
                    const double* s2p = S2s + q2 * 256 + r;
                    double s2[4];
                    for (int i = 0; i < 4; ++i) s2[i] = s2p[(4 * i + g) * 16];
                    for (int i = 0; i < 4; ++i)
                        for (int t = 0; t < TPW; ++t)
                            if (FULL || wave * TPW + t < D) T2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(s2[i], T1[t][i], T2[t], 0, 0, 0);
                } else if constexpr (PREC == PREC_F32) {
                    const float* s2p = S2f + q2 * 16 * SF_V + r;
                    float s2[4];
                    for (int i = 0; i < 4; ++i) s2[i] = s2p[(4 * g + i) * SF_V];
                    for (int i = 0; i < 4; ++i)
                        for (int t = 0; t < TPW; ++t)
                            if (FULL || wave * TPW + t < D) T2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(s2[i], T1[t][i], T2[t], 0, 0, 0);
                } else {
                    const u4 s2 = S2b[(q2 * 16 + r) * 4 + g];
                    for (int t = 0; t < TPW; ++t)
                        if (FULL || wave * TPW + t < D) T2[t] = mfma_bf16x<PREC == PREC_BF16C>(s2, split4(T1[t]), T2[t]);
                }
                for (int t = 0; t < TPW; ++t) T1[t] = Acc{};
            }
            if (next < 0 || (next >> 4) != (cell >> 4)) {
                // end of an L1 plane -- mode 1 through an LDS transpose: Y += S1^{L1} x_1 T2
                for (int t = 0; t < TPW; ++t) {
                    const int v1 = wave * TPW + t;
                    if (!FULL && v1 >= D) break;
                    for (int i = 0; i < 4; ++i) {
                        if constexpr (PREC == PREC_F64) T2s[v1 * T2S_V1 + (4 * i + g) * T2S_U2 + r] = T2[t][i];
                        else T2f[v1 * T2F_V1 + (4 * g + i) * T2F_U2 + r] = T2[t][i];
                    }
                }
                lds_barrier();
                for (int t = 0; t < TPW; ++t) {
                    const int u2 = wave * TPW + t;
                    if (!FULL && u2 >= D) break;
                    d4 add;
                    if constexpr (PREC == PREC_F64) {
                        const double* s1p = S1s + q1 * 256 + r;
                        // the down band reaches only internal children: accumulate it apart, add it masked
                        d4 acc = tp.dpart ? (d4){0.0, 0.0, 0.0, 0.0} : Y[t];
                        for (int kk = 0; kk < 4; ++kk) {
                            const int v1 = 4 * kk + g;
                            const double bv = v1 < D ? T2s[v1 * T2S_V1 + u2 * T2S_U2 + r] : 0.0;
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s1p[(4 * kk + g) * 16], bv, acc, 0, 0, 0);
                        }
                        if (!tp.dpart) { Y[t] = acc; continue; }
                        add = acc;
                    } else {
                        f4 acc = {0.f, 0.f, 0.f, 0.f};
                        if constexpr (PREC == PREC_F32) {
                            const float* s1p = S1f + q1 * 16 * SF_V + perm_row(r);
                            for (int kk = 0; kk < 4; ++kk) {
                                const int v1 = 4 * g + kk;
                                const float bv = v1 < D ? T2f[v1 * T2F_V1 + u2 * T2F_U2 + r] : 0.f;
                                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(s1p[v1 * SF_V], bv, acc, 0, 0, 0);
                            }
                        } else {
                            f4 bv;
                            for (int j = 0; j < 4; ++j) {
                                const int v1 = 4 * g + j;
                                bv[j] = v1 < D ? T2f[v1 * T2F_V1 + u2 * T2F_U2 + r] : 0.f;
                            }
                            acc = mfma_bf16x<PREC == PREC_BF16C>(S1b[(q1 * 16 + perm_row(r)) * 4 + g], split4(bv), acc);
                        }
                        add = (d4){(double)acc[0], (double)acc[1], (double)acc[2], (double)acc[3]};
                        if (!tp.dpart) { Y[t] += add; continue; }
                    }
                    for (int i = 0; i < 4; ++i) {
                        const int child = (4 * i + g >= K) + 2 * (u2 >= K) + 4 * (r >= K);
                        if ((cmb >> child) & 1) Y[t][i] += add[i];
                    }
                }
                for (int t = 0; t < TPW; ++t) T2[t] = Acc{};
                lds_barrier();
            }
            if (++si == ns) {
                si = 0;
                ++m;
            }
        }
    }
}

// One block per output brick, over all levels at once (order[] lists (level, brick)).  CW waves
// per block, each owning TPW input slices; PF steps of input slices are prefetched into registers.
// For every job the in-cube cells of its box are first compacted into an LDS list (ascending L1,
// L2, L3), so the term loop and the cell loop fuse into one stream of steps whose input bricks
// are known PF steps ahead (the same list repeats for every term of the job).
//
// MFMA mapping of the FP64 class (v_mfma_f64_16x16x4: A[m][k] in lane m+16k, B[k][n] in lane
// n+16k, D[4i+g][n] in lane 16g+n, register i): wave w owns the input slices v1 in {w*TPW..}: mode 3
// (contract v3, A = X slice with K index 4g+kk loaded as 4 consecutive doubles, B = S3), mode 2
// straight from the mode-3 accumulators (their register i holds contraction index 4i+g), an LDS
// transpose, then mode 1 into the per-wave output tiles.  The FP32 class (v_mfma_f32_16x16x4,
// D[4g+i][n]) follows the same chain with the contraction slots permuted to match; the BF16
// classes (v_mfma_f32_16x16x32_bf16, lane 16g+n holding K slots 8g..8g+7) give every lane the 4
// contraction indices 4g..4g+3 as (4 hi | 4 lo) halves, which is exactly what the FP32 mode-3
// accumulators of the lane hold, so mode 2 again needs no data movement.
template <int K, int CW, int PF, int WPE>
__global__ void __launch_bounds__(64 * CW) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
ns_apply_kernel(const LevelDesc* __restrict__ levels, const int2* __restrict__ order, const double* __restrict__ w) {
    constexpr int D = 2 * K;
    constexpr int TPW = (D + CW - 1) / CW;
    constexpr int64_t E = (int64_t)D * D * D;
    __shared__ double smem[SMEM_DOUBLES];
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
    for (int t = 0; t < TPW; ++t) Y[t] = (d4){0.0, 0.0, 0.0, 0.0};
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
        switch (__builtin_amdgcn_readfirstlane(tp.prec)) {
            case PREC_F64: run_job<K, CW, PF, PREC_F64>(lv, tp, w, ns, steps, smem, wave, g, r, cmb, Y); break;
            case PREC_F32: run_job<K, CW, PF, PREC_F32>(lv, tp, w, ns, steps, smem, wave, g, r, cmb, Y); break;
            case PREC_BF16C: run_job<K, CW, PF, PREC_BF16C>(lv, tp, w, ns, steps, smem, wave, g, r, cmb, Y); break;
            default: run_job<K, CW, PF, PREC_BF16>(lv, tp, w, ns, steps, smem, wave, g, r, cmb, Y); break;
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

// Reduced-precision copies of input bricks: one thread per (brick, v1, v2, group of 4 columns)
// writes 16 bytes -- four FP32 values (F32) or their split BF16 (hi | lo) (BF16); columns at or
// beyond 2K are zero.
template <int K, bool BF>
__global__ void convert_kernel(int64_t nbricks, const double* __restrict__ X, u4* __restrict__ out) {
    constexpr int D = 2 * K;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbricks * D * D * 4) return;
    const int gg = (int)(i & 3);
    const int64_t row = i >> 2;     // (brick, v1, v2)
    const double* x = X + row * D;
    f4 v;
    for (int c = 0; c < 4; ++c) v[c] = 4 * gg + c < D ? (float)x[4 * gg + c] : 0.f;
    out[i] = BF ? split4(v) : __builtin_bit_cast(u4, v);
}

// Sum of squares of every brick element of one level (real and ghost inputs): one 256-thread
// block per brick, reduced in LDS and added to *acc.
template <int K>
__global__ void __launch_bounds__(256) sumsq_kernel(const double* __restrict__ X, double* __restrict__ acc) {
    constexpr int E = 8 * K * K * K;
    __shared__ double red[256];
    const double* x = X + (int64_t)blockIdx.x * E;
    double s = 0.0;
    for (int e = threadIdx.x; e < E; e += 256) s += x[e] * x[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(acc, red[0]);
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

template <int K>
struct SumsqLaunch {
    static void run(hipStream_t st, int64_t nb, const double* X, double* acc) {
        if (nb > 0) sumsq_kernel<K><<<(unsigned)nb, 256, 0, st>>>(X, acc);
    }
};
template <int K>
struct ConvertLaunch {
    static void run(hipStream_t st, int64_t nb, const double* X, u4* out, bool bf) {
        const int64_t n = nb * 2 * K * 2 * K * 4;
        if (n == 0) return;
        if (bf) convert_kernel<K, true><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(nb, X, out);
        else convert_kernel<K, false><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(nb, X, out);
    }
};

// Sum of squares of the coefficients of the leaves among the 8 children of every brick of one
// level (level 0: only child 0, the root): one 256-thread block per brick.
template <int K>
__global__ void __launch_bounds__(256) leafsq_kernel(int64_t node_off, int nchild, const uint8_t* __restrict__ leaf,
                                                     const double* __restrict__ coef, double* __restrict__ acc) {
    constexpr int P = 2 * K, K3 = K * K * K;
    __shared__ double red[256];
    const double* brick = coef + (int64_t)blockIdx.x * P * P * P;
    double s = 0.0;
    for (int e = threadIdx.x; e < nchild * K3; e += 256) {
        const int child = e / K3, q = e % K3;
        if (!leaf[node_off + (int64_t)blockIdx.x * 8 + child]) continue;
        const int a = q / (K * K), bb = (q / K) % K, c = q % K;
        const double x = brick[(((child & 1) * K + a) * P + ((child >> 1) & 1) * K + bb) * P + (child >> 2) * K + c];
        s += x * x;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(acc, red[0]);
}
template <int K>
struct LeafsqLaunch {
    static void run(hipStream_t st, int64_t nb, int64_t node_off, int nchild, const uint8_t* leaf, const double* coef,
                    double* acc) {
        if (nb > 0) leafsq_kernel<K><<<(unsigned)nb, 256, 0, st>>>(node_off, nchild, leaf, coef, acc);
    }
};

__global__ void fill_kernel(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- precision routing
// Rounding-error factors of the classes: a three-mode chain whose every mode has relative
// operand errors a (matrix) and b (input) and an FP32 accumulation over at most 16 * NMAX products
// computes (|S1| (x) |S2| (x) |S3|) |X| up to the factor ((1 + a + b + n u32)^3 - 1).
constexpr double U32 = 0x1p-24, UBF = 0x1p-8, USPLIT = 0x1p-16;
constexpr double cube_minus_one(double d) { return (1.0 + d) * (1.0 + d) * (1.0 + d) - 1.0; }
constexpr double NACC = 16.0 * NMAX * U32;
constexpr double GAMMA[NPREC] = {0.0, cube_minus_one(2.0 * U32 + NACC), cube_minus_one(2.0 * (USPLIT + U32) + NACC),
                                 cube_minus_one(UBF + USPLIT + 2.0 * U32 + NACC)};
// Relative time per unit of work, for the routing objective only.
constexpr double COST[NPREC] = {1.0, 0.6, 0.3, 0.2};

struct RouteItem {
    int j, t, m, cls;
    double beta, work;
};

// Chooses a class for every (level, job, term) minimising the modelled time subject to
// sum gamma_class * beta <= tol (Lagrangian relaxation, bisection on the multiplier); beta bounds
// the FP64 contribution of the item over its whole level:
//   || sum_b sum_{L in box} (S1 (x) S2 (x) S3) X_{b-L} || <= |w_m| prod_d sum_{L_d} ||S_d^{m,L_d}||_F ||X_level||,
// each input brick feeding one output brick per displacement.  Returns the bound reached.
double route(std::vector<RouteItem>& items, double tol, int allowed) {
    auto eval = [&](double lam, bool commit) {
        double err = 0.0;
        for (RouteItem& it : items) {
            int best = PREC_F64;
            double bv = it.work * COST[PREC_F64];
            for (int p = 1; p < NPREC; ++p) {
                if (!((allowed >> (p - 1)) & 1)) continue;
                const double v = it.work * COST[p] + lam * GAMMA[p] * it.beta;
                if (v < bv) { bv = v; best = p; }
            }
            err += GAMMA[best] * it.beta;
            if (commit) it.cls = best;
        }
        return err;
    };
    if (!(tol > 0.0) || items.empty()) {
        for (RouteItem& it : items) it.cls = PREC_F64;
        return 0.0;
    }
    double lo = -60.0, hi = 80.0;     // log10 of the multiplier; at 10^80 every item is FP64
    if (eval(std::pow(10.0, lo), false) <= tol) return eval(std::pow(10.0, lo), true);
    for (int it = 0; it < 100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (eval(std::pow(10.0, mid), false) <= tol) hi = mid;
        else lo = mid;
    }
    return eval(std::pow(10.0, hi), true);
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

namespace {

// The apply behind both entry points; mixed == nullptr is the all-FP64 apply.
void apply_impl(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, int mode, const mwns_mixed_opts* mixed,
                mwns_tree** g, mwns_apply_stats* stats) {
    if (!ctx || !op || !f || !g) fail(MWNS_EINVAL, "NULL argument");
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
    // ---- precision routing (mixed apply): per-level input norms, classes, reduced-precision inputs
    double err_bound = 0.0;
    std::vector<DevArray<u4>> xr32(depth + 1), xg32(depth + 1), xrb(depth + 1), xgb(depth + 1);
    if (mixed) {
        DevArray<double> lsq(ctx, depth + 1);
        fill_kernel<<<1, 64, 0, st>>>(lsq.p, depth + 1, 0.0);
        for (int j = 0; j <= depth; ++j) {
            const LevelWork& lw = W[j];
            if (lw.tpl.empty()) continue;
            dispatch_k<SumsqLaunch>(k, st, lw.nout, f->coef.p + f->lev[j].brick_off * E, lsq.p + j);
            dispatch_k<SumsqLaunch>(k, st, lw.nghost, lw.ghosts.p, lsq.p + j);
        }
        MWNS_HIP(hipGetLastError());
        std::vector<double> hsq(depth + 1);
        lsq.download(hsq.data(), depth + 1, st);
        MWNS_HIP(hipStreamSynchronize(st));
        std::vector<RouteItem> items;
        const int M = op->M;
        for (int j = 0; j <= depth; ++j) {
            const LevelWork& lw = W[j];
            const double xn = std::sqrt(hsq[j]);
            int64_t ninternal = 0;
            for (int64_t b = 0; b < lw.nout; ++b) ninternal += lw.cm[b] != 0;
            for (int t = 0; t < (int)lw.tpl.size(); ++t) {
                const Tpl& tp = lw.tpl[t];
                const double nb = tp.dpart ? (double)ninternal : (double)lw.nout;
                const double n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
                for (int m = tp.m1; m <= tp.m2; ++m) {
                    const double* fr = op->fro.data() + ((int64_t)j * M + m) * NLF;
                    double beta = std::fabs(op->w[m]) * xn;
                    for (int d = 0; d < 3; ++d) {
                        double a = 0.0;
                        for (int L = tp.lo[d]; L <= tp.hi[d]; ++L) {
                            double s2 = 0.0;
                            for (int su = 0; su < 2; ++su)
                                for (int sv = 0; sv < 2; ++sv) {
                                    const int l = 2 * L + su - sv;
                                    if (l >= tp.mlo[d] && l <= tp.mhi[d]) s2 += fr[l + LF] * fr[l + LF];
                                }
                            a += std::sqrt(s2);
                        }
                        beta *= a;
                    }
                    items.push_back(RouteItem{j, t, m, PREC_F64, beta, nb * (n1 * n2 * n3 + n1 * n2 + n1)});
                }
            }
        }
        err_bound = route(items, mixed->tol, mixed->classes);
        // split every job into runs of terms of one class
        size_t pos = 0;
        for (int j = 0; j <= depth; ++j) {
            LevelWork& lw = W[j];
            std::vector<Tpl> split;
            for (int t = 0; t < (int)lw.tpl.size(); ++t) {
                Tpl cur = lw.tpl[t];
                for (int m = lw.tpl[t].m1; m <= lw.tpl[t].m2; ++m, ++pos) {
                    const int c = items[pos].cls;
                    if (m == lw.tpl[t].m1) { cur.m1 = m; cur.prec = c; }
                    else if (c != cur.prec) {
                        cur.m2 = m - 1;
                        split.push_back(cur);
                        cur.m1 = m;
                        cur.prec = c;
                    }
                    cur.m2 = m;
                }
                split.push_back(cur);
            }
            lw.tpl.swap(split);
            bool need32 = false, needbf = false;
            for (const Tpl& t : lw.tpl) {
                need32 = need32 || t.prec == PREC_F32;
                needbf = needbf || t.prec == PREC_BF16C || t.prec == PREC_BF16;
            }
            const int64_t units = (int64_t)4 * 2 * k * 2 * k;     // 16-byte units per brick
            const double* xr = f->coef.p + f->lev[j].brick_off * E;
            if (need32) {
                xr32[j].reset(ctx, (size_t)lw.nout * units);
                dispatch_k<ConvertLaunch>(k, st, lw.nout, xr, xr32[j].p, false);
                if (lw.nghost) {
                    xg32[j].reset(ctx, (size_t)lw.nghost * units);
                    dispatch_k<ConvertLaunch>(k, st, lw.nghost, lw.ghosts.p, xg32[j].p, false);
                }
            }
            if (needbf) {
                xrb[j].reset(ctx, (size_t)lw.nout * units);
                dispatch_k<ConvertLaunch>(k, st, lw.nout, xr, xrb[j].p, true);
                if (lw.nghost) {
                    xgb[j].reset(ctx, (size_t)lw.nghost * units);
                    dispatch_k<ConvertLaunch>(k, st, lw.nghost, lw.ghosts.p, xgb[j].p, true);
                }
            }
            MWNS_HIP(hipGetLastError());
        }
    }
    tclos.stop();
    // ---- contractions: one launch over every output brick of every level, costliest first
    std::vector<LevelDesc> descs(depth + 1);
    std::vector<std::pair<double, int2>> cost;
    int64_t jobs = 0;
    double flops = 0.0, class_flops[NPREC] = {0.0, 0.0, 0.0, 0.0};
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
        d.Xr32 = reinterpret_cast<const float*>(xr32[j].p);
        d.Xg32 = reinterpret_cast<const float*>(xg32[j].p);
        d.Xrb = xrb[j].p;
        d.Xgb = xgb[j].p;
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
                if (nin[0] * nin[1] * nin[2] == 0) continue;     // the box lies outside the cube
                const double nt = t.m2 - t.m1 + 1;
                const double steps = nin[0] * nin[1] * nin[2] + nin[0] * nin[1] + nin[0];
                c += nt * steps * COST[t.prec];
                const double D2 = 2.0 * k;
                jobs += (int64_t)nt;
                const double fl = nt * 2.0 * D2 * D2 * D2 * D2 * steps;
                flops += fl;
                class_flops[t.prec] += fl;
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
        // ||g||_2: the leaves' scaling functions are orthonormal with disjoint supports
        DevArray<double> gsq(ctx, 1);
        fill_kernel<<<1, 64, 0, st>>>(gsq.p, 1, 0.0);
        if (!(mode & MWNS_NO_ASSEMBLY))
            for (int j = 0; j <= depth; ++j)
                dispatch_k<LeafsqLaunch>(k, st, f->lev[j].nbricks, f->lev[j].node_off, j == 0 ? 1 : 8, f->dleaf.p,
                                         out->coef.p + f->lev[j].brick_off * E, gsq.p);
        MWNS_HIP(hipGetLastError());
        unsigned long long c = 0;
        double g2 = 0.0;
        tot.download(&c, 1, st);
        gsq.download(&g2, 1, st);
        MWNS_HIP(hipStreamSynchronize(st));
        s.contractions = (int64_t)c;
        s.brick_jobs = jobs;
        s.ghost_bricks = total_ghosts;
        s.useful_flops = flops;
        s.ms_closure = tclos.ms();
        s.ms_contract = tcon.ms();
        s.ms_assemble = tasm.ms();
        s.err_bound = err_bound;
        s.g_norm = std::sqrt(g2);
        for (int p = 0; p < NPREC; ++p) s.class_flops[p] = class_flops[p];
        *stats = s;
    } else {
        MWNS_HIP(hipStreamSynchronize(st));
    }
    *g = out.release();
}

}  // namespace

extern "C" mwns_status mwns_apply(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, int mode, mwns_tree** g,
                                  mwns_apply_stats* stats) {
    MWNS_GUARD_BEGIN
    if ((mode & 0xff) != MWNS_F64 || (mode & ~(0xff | MWNS_NO_ASSEMBLY))) fail(MWNS_EINVAL, "unsupported mode");
    apply_impl(ctx, op, f, mode, nullptr, g, stats);
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_apply_mixed(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, const mwns_mixed_opts* opts,
                                        int flags, mwns_tree** g, mwns_apply_stats* stats) {
    MWNS_GUARD_BEGIN
    if (!opts) fail(MWNS_EINVAL, "opts is NULL");
    if (!(opts->tol >= 0.0) || !std::isfinite(opts->tol)) fail(MWNS_EINVAL, "tol must be finite and >= 0");
    if (opts->classes & ~(MWNS_CLASS_F32 | MWNS_CLASS_BF16C | MWNS_CLASS_BF16)) fail(MWNS_EINVAL, "unknown precision class");
    if (flags & ~MWNS_NO_ASSEMBLY) fail(MWNS_EINVAL, "unsupported flags");
    apply_impl(ctx, op, f, flags, opts, g, stats);
    return MWNS_OK;
    MWNS_GUARD_END
}
