// The contraction kernel of the apply (Alg. 3 Step 3 with the nested-loop factorisation of
// Sec. 5) on the MI355X matrix cores, in FP64 and in the reduced precision classes.
//
// Work is organised by sibling groups ("bricks"): the 8 children of a node form a (2k)^3 tensor
// with index u = s*k + a per dimension.  Between the brick of parent P and the brick of parent
// P - L (coarse displacement L) the fine displacement is l = 2L + s - s', so one Gaussian term acts
// per dimension as the 2k x 2k super-block
//     S^{j;m,L} = [[F^{j;m,2L}, F^{j;m,2L-1}], [F^{j;m,2L+1}, F^{j;m,2L}]]      (rows: output parity)
// and a term applied over a box of displacements L in [lo1,hi1] x [lo2,hi2] x [lo3,hi3] factorises
//     Y += c w_m sum_{L1} S^{L1} x_1 [ sum_{L2} S^{L2} x_2 [ sum_{L3} S^{L3} x_3 X_{P-L} ] ].
// 2k <= 16 is padded to one 16 x 16 MFMA tile per dimension.
#include <algorithm>
#include <type_traits>

#include "contract.h"

namespace mwns {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int T2S_V1 = 272;        // LDS strides of the FP64 mode-2 result [v1][u2][u3] (conflict-free)
constexpr int T2S_U2 = 16;
constexpr int T2F_V1 = 324;        // the same for the FP32 mode-2 result (64 distinct banks per access)
constexpr int T2F_U2 = 20;
constexpr int S3_V = 36;           // LDS stride of the staged FP64 mode-3 operand [L][v][u]
constexpr int SF_V = 20;           // LDS stride of the staged FP32 operands [L][v][u]
// LDS of the contraction kernel, in doubles: the FP64 layout is the largest of the classes.
constexpr int SM_T2 = 16 * T2S_V1, SM_S3 = NMAX * 16 * S3_V, SM_S2 = NMAX * 256, SM_S1 = NMAX * 256;
constexpr int SMEM_DOUBLES = SM_T2 + SM_S3 + SM_S2 + SM_S1;
// The reduced classes run GT terms of a job per pass over its cells (one input load, one step
// bookkeeping and one staging barrier for all of them); their LDS holds the FP32 mode-2 result
// once and the staged super-blocks of every term of the group.
template <int PREC, int K = 8>
struct LpShape {
    static constexpr bool BF = PREC != PREC_F32;
    // terms per pass: as many as the 128-register budget of two workgroups per CU holds unspilled
    static constexpr int GT = BF ? 2 : (K == 8 ? 2 : 1);
    static constexpr int TERM_BYTES = BF ? 3 * NMAX * 64 * 16 : 3 * NMAX * 16 * SF_V * 4;  // S1, S2, S3 of a term
    static constexpr int T2_BYTES = 16 * T2F_V1 * 4;
    static constexpr int SMEM = (T2_BYTES + GT * TERM_BYTES + 7) / 8;                  // doubles
};
// The FP64 class with G terms per pass keeps the staged super-blocks of every term of the group.
constexpr int SM_TERM = SM_S3 + SM_S2 + SM_S1;
template <int PREC, int K, int G = 1>
constexpr int smem_doubles() {
    if constexpr (PREC == PREC_F64) return SM_T2 + G * SM_TERM;
    else return LpShape<PREC, K>::SMEM;
}
static_assert(smem_doubles<PREC_F32, 8>() * 8 <= 80 * 1024 && smem_doubles<PREC_BF16C, 8>() * 8 <= 80 * 1024,
              "two workgroups per CU");

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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
                        const double val = (d == 0 ? cw : 1.0) * sop<K>(Fm, pick3(tp.lo, d) + q, pick3(tp.mlo, d), pick3(tp.mhi, d), uu, v);
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
                        for (int c = 0; c < 4; ++c) v4[c] = (float)(sc * sop<K>(Fm, pick3(tp.lo, d) + q, pick3(tp.mlo, d), pick3(tp.mhi, d), uu, 4 * gg + c));
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

// The terms of one job for one output brick in the FP64 class, G terms per pass (see run_job for
// the operand layouts): every step loads the input slices once and feeds them to the G terms'
// chains; the super-blocks of the G terms are staged side by side; mode 1 goes through the LDS
// transpose term by term.  The terms keep their order within each plane, but the plane results of
// consecutive terms interleave in Y, so the sums agree with run_job up to rounding.
template <int K, int CW, int G, int PF>
__device__ __forceinline__ void run_job_g(const LevelDesc& lv, const Tpl& tp, const double* __restrict__ w, int ns,
                                          const int2* steps, double* smem, int wave, int g, int r, int cmb,
                                          d4 (&Y)[(2 * K + CW - 1) / CW]) {
    constexpr int CT = 64 * CW;
    constexpr int D = 2 * K;
    constexpr int TPW = (D + CW - 1) / CW;
    constexpr bool FULL = (CW * TPW == D);
    constexpr int64_t E = (int64_t)D * D * D;
    const int n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
    double* T2s = smem;
    auto S3s = [&](int gi) { return smem + SM_T2 + gi * SM_TERM; };
    auto S2s = [&](int gi) { return S3s(gi) + SM_S3; };
    auto S1s = [&](int gi) { return S2s(gi) + SM_S2; };
    uint32_t xoff[TPW];
    for (int t = 0; t < TPW; ++t) xoff[t] = slice_offset<K>(wave * TPW + t, g, r);
    auto load = [&](int si, d4 (&x)[TPW]) {
        const int idx = __builtin_amdgcn_readfirstlane(steps[si].x);
        const bool real = idx < lv.nreal;
        const int64_t qi = real ? idx : idx - lv.nreal;
        load_slices<K, TPW>((real ? lv.Xr : lv.Xg) + qi * E, (int)(E * 8), xoff, x);
    };
    // PF = 1: the slices of the next step are loaded while the current one is computed (the step
    // list is the same for every pass of the job)
    d4 xn[TPW];
    if constexpr (PF > 0) load(0, xn);
    for (int m0 = tp.m1; m0 <= tp.m2; m0 += G) {
        const int gn = __builtin_amdgcn_readfirstlane(min(G, tp.m2 - m0 + 1));
        // stage the super-blocks of the pass's terms (the previous pass ended with a barrier)
        const int per = (n1 + n2 + n3) * 256;
        for (int e = threadIdx.x; e < gn * per; e += CT) {
            const int gi = e / per, ee = e % per;
            const int sb = ee >> 8, v = (ee >> 4) & 15, uu = ee & 15;
            const int m = m0 + gi;
            const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
            int q, d;
            if (sb < n1) { q = sb; d = 0; }
            else if (sb < n1 + n2) { q = sb - n1; d = 1; }
            else { q = sb - n1 - n2; d = 2; }
            const double sc = d == 0 ? (tp.dpart ? -w[m] : w[m]) : 1.0;
            double* dst = d == 0 ? S1s(gi) + q * 256 + v * 16 : d == 1 ? S2s(gi) + q * 256 + v * 16 : S3s(gi) + q * 16 * S3_V + v * S3_V;
            dst[uu] = sc * sop<K>(Fm, pick3(tp.lo, d) + q, pick3(tp.mlo, d), pick3(tp.mhi, d), uu, v);
        }
        lds_barrier();
        d4 T1[G][TPW], T2[G][TPW];
        for (int gi = 0; gi < G; ++gi)
            for (int t = 0; t < TPW; ++t) T1[gi][t] = T2[gi][t] = (d4){0.0, 0.0, 0.0, 0.0};
        for (int si = 0; si < ns; ++si) {
            const int cell = __builtin_amdgcn_readfirstlane(steps[si].y);
            const int next = si + 1 < ns ? __builtin_amdgcn_readfirstlane(steps[si + 1].y) : -1;
            const int q1 = cell >> 4, q2 = (cell >> 2) & 3, q3 = cell & 3;
            d4 x[TPW];
            if constexpr (PF > 0) {
                for (int t = 0; t < TPW; ++t) x[t] = xn[t];
                if (si + 1 < ns) load(si + 1, xn);
                else if (m0 + G <= tp.m2) load(0, xn);
            } else {
                load(si, x);
            }
            // mode 3 for every term of the pass
            for (int gi = 0; gi < G; ++gi) {
                if (gi >= gn) break;
                const double* s3p = S3s(gi) + q3 * 16 * S3_V + r;
                double s3[4];
                for (int kk = 0; kk < 4; ++kk) s3[kk] = s3p[(4 * g + kk) * S3_V];
                for (int kk = 0; kk < 4; ++kk)
                    for (int t = 0; t < TPW; ++t)
                        if (FULL || wave * TPW + t < D) T1[gi][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t][kk], s3[kk], T1[gi][t], 0, 0, 0);
            }
            if (next < 0 || (next >> 2) != (cell >> 2)) {
                // end of an (L1, L2) row -- mode 2 for every term
                for (int gi = 0; gi < G; ++gi) {
                    if (gi >= gn) break;
                    const double* s2p = S2s(gi) + q2 * 256 + r;
                    double s2[4];
                    for (int i = 0; i < 4; ++i) s2[i] = s2p[(4 * i + g) * 16];
                    for (int i = 0; i < 4; ++i)
                        for (int t = 0; t < TPW; ++t)
                            if (FULL || wave * TPW + t < D)
                                T2[gi][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(s2[i], T1[gi][t][i], T2[gi][t], 0, 0, 0);
                    for (int t = 0; t < TPW; ++t) T1[gi][t] = (d4){0.0, 0.0, 0.0, 0.0};
                }
            }
            if (next < 0 || (next >> 4) != (cell >> 4)) {
                // end of an L1 plane -- mode 1, term by term through the one LDS transpose buffer
                for (int gi = 0; gi < G; ++gi) {
                    if (gi >= gn) break;
                    for (int t = 0; t < TPW; ++t) {
                        const int v1 = wave * TPW + t;
                        if (!FULL && v1 >= D) break;
                        for (int i = 0; i < 4; ++i) T2s[v1 * T2S_V1 + (4 * i + g) * T2S_U2 + r] = T2[gi][t][i];
                    }
                    lds_barrier();
                    for (int t = 0; t < TPW; ++t) {
                        const int u2 = wave * TPW + t;
                        if (!FULL && u2 >= D) break;
                        const double* s1p = S1s(gi) + q1 * 256 + r;
                        d4 acc = tp.dpart ? (d4){0.0, 0.0, 0.0, 0.0} : Y[t];
                        for (int kk = 0; kk < 4; ++kk) {
                            const int v1 = 4 * kk + g;
                            const double bv = v1 < D ? T2s[v1 * T2S_V1 + u2 * T2S_U2 + r] : 0.0;
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s1p[(4 * kk + g) * 16], bv, acc, 0, 0, 0);
                        }
                        if (!tp.dpart) {
                            Y[t] = acc;
                            continue;
                        }
                        for (int i = 0; i < 4; ++i) {
                            const int child = (4 * i + g >= K) + 2 * (u2 >= K) + 4 * (r >= K);
                            if ((cmb >> child) & 1) Y[t][i] += acc[i];
                        }
                    }
                    for (int t = 0; t < TPW; ++t) T2[gi][t] = (d4){0.0, 0.0, 0.0, 0.0};
                    lds_barrier();
                }
            }
        }
    }
}

// The terms of one job for one output brick in a reduced class, GT terms per pass: every step
// loads the input slices once and feeds them to the GT terms' chains (FP32 or split-BF16; see
// run_job for the operand layouts); mode 1 goes through the LDS transpose term by term.
template <int K, int CW, int PREC>
__device__ __forceinline__ void run_job_lp(const LevelDesc& lv, const Tpl& tp, const double* __restrict__ w, int ns,
                                           const int2* steps, double* smem, int wave, int g, int r, int cmb,
                                           d4 (&Y)[(2 * K + CW - 1) / CW]) {
    using S = LpShape<PREC, K>;
    constexpr int GT = S::GT;
    constexpr bool BF = S::BF;
    constexpr int CT = 64 * CW;
    constexpr int D = 2 * K;
    constexpr int TPW = (D + CW - 1) / CW;
    constexpr bool FULL = (CW * TPW == D);
    constexpr int64_t ELP = (int64_t)D * D * 64;   // bytes of a reduced-precision brick
    const int n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
    float* T2f = reinterpret_cast<float*>(smem);
    char* sbase = reinterpret_cast<char*>(smem) + S::T2_BYTES;
    // staged operands of term gi of the pass
    auto S3f = [&](int gi) { return reinterpret_cast<float*>(sbase + gi * S::TERM_BYTES); };
    auto S2f = [&](int gi) { return S3f(gi) + NMAX * 16 * SF_V; };
    auto S1f = [&](int gi) { return S2f(gi) + NMAX * 16 * SF_V; };
    auto S3b = [&](int gi) { return reinterpret_cast<u4*>(sbase + gi * S::TERM_BYTES); };
    auto S2b = [&](int gi) { return S3b(gi) + NMAX * 64; };
    auto S1b = [&](int gi) { return S2b(gi) + NMAX * 64; };
    uint32_t xoff[TPW];
    for (int t = 0; t < TPW; ++t) xoff[t] = slice_offset_lp<K>(wave * TPW + t, g, r);
    for (int m0 = tp.m1; m0 <= tp.m2; m0 += GT) {
        const int gn = __builtin_amdgcn_readfirstlane(min(GT, tp.m2 - m0 + 1));
        // stage the super-blocks of the pass's terms (the previous pass ended with a barrier)
        if constexpr (!BF) {
            const int per = (n1 + n2 + n3) * 256;
            for (int e = threadIdx.x; e < gn * per; e += CT) {
                const int gi = e / per, ee = e % per;
                const int sb = ee >> 8, v = (ee >> 4) & 15, uu = ee & 15;
                const int m = m0 + gi;
                const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
                int q, d;
                if (sb < n1) { q = sb; d = 0; }
                else if (sb < n1 + n2) { q = sb - n1; d = 1; }
                else { q = sb - n1 - n2; d = 2; }
                const double sc = d == 0 ? (tp.dpart ? -w[m] : w[m]) : 1.0;
                float* dst = (d == 0 ? S1f(gi) : d == 1 ? S2f(gi) : S3f(gi)) + (q * 16 + v) * SF_V;
                dst[uu] = (float)(sc * sop<K>(Fm, pick3(tp.lo, d) + q, pick3(tp.mlo, d), pick3(tp.mhi, d), uu, v));
            }
        } else {
            const int per = (n1 + n2 + n3) * 64;
            for (int e = threadIdx.x; e < gn * per; e += CT) {
                const int gi = e / per, ee = e % per;
                const int sb = ee >> 6, uu = (ee >> 2) & 15, gg = ee & 3;
                const int m = m0 + gi;
                const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
                int q, d;
                if (sb < n1) { q = sb; d = 0; }
                else if (sb < n1 + n2) { q = sb - n1; d = 1; }
                else { q = sb - n1 - n2; d = 2; }
                const double sc = d == 0 ? (tp.dpart ? -w[m] : w[m]) : 1.0;
                f4 v4;
                for (int c = 0; c < 4; ++c) v4[c] = (float)(sc * sop<K>(Fm, pick3(tp.lo, d) + q, pick3(tp.mlo, d), pick3(tp.mhi, d), uu, 4 * gg + c));
                (d == 0 ? S1b(gi) : d == 1 ? S2b(gi) : S3b(gi))[(q * 16 + uu) * 4 + gg] = split4(v4);
            }
        }
        lds_barrier();
        f4 T1[GT][TPW], T2[GT][TPW];
        for (int gi = 0; gi < GT; ++gi)
            for (int t = 0; t < TPW; ++t) T1[gi][t] = T2[gi][t] = (f4){0.f, 0.f, 0.f, 0.f};
        for (int si = 0; si < ns; ++si) {
            const int idx = __builtin_amdgcn_readfirstlane(steps[si].x);
            const int cell = __builtin_amdgcn_readfirstlane(steps[si].y);
            const int next = si + 1 < ns ? __builtin_amdgcn_readfirstlane(steps[si + 1].y) : -1;
            const int q1 = cell >> 4, q2 = (cell >> 2) & 3, q3 = cell & 3;
            const bool real = idx < lv.nreal;
            const int64_t qi = real ? idx : idx - lv.nreal;
            const void* X = BF ? (const void*)((const char*)(real ? lv.Xrb : lv.Xgb) + qi * ELP)
                               : (const void*)((const char*)(real ? lv.Xr32 : lv.Xg32) + qi * ELP);
            u4 xb[TPW];
            load_slices_lp<TPW>(X, (int)ELP, xoff, xb);
            // mode 3 for every term of the pass
            if constexpr (!BF) {
                f4 xf[TPW];
                for (int t = 0; t < TPW; ++t) xf[t] = __builtin_bit_cast(f4, xb[t]);
                for (int gi = 0; gi < GT; ++gi) {
                    if (gi >= gn) break;
                    const float* s3p = S3f(gi) + q3 * 16 * SF_V + r;
                    float s3[4];
                    for (int kk = 0; kk < 4; ++kk) s3[kk] = s3p[(4 * g + kk) * SF_V];
                    for (int kk = 0; kk < 4; ++kk)
                        for (int t = 0; t < TPW; ++t)
                            if (FULL || wave * TPW + t < D)
                                T1[gi][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xf[t][kk], s3[kk], T1[gi][t], 0, 0, 0);
                }
            } else {
                for (int gi = 0; gi < GT; ++gi) {
                    if (gi >= gn) break;
                    const u4 s3 = S3b(gi)[(q3 * 16 + r) * 4 + g];
                    for (int t = 0; t < TPW; ++t)
                        if (FULL || wave * TPW + t < D) T1[gi][t] = mfma_bf16x<PREC == PREC_BF16C>(xb[t], s3, T1[gi][t]);
                }
            }
            if (next < 0 || (next >> 2) != (cell >> 2)) {
                // end of an (L1, L2) row -- mode 2 for every term
                for (int gi = 0; gi < GT; ++gi) {
                    if (gi >= gn) break;
                    if constexpr (!BF) {
                        const float* s2p = S2f(gi) + q2 * 16 * SF_V + r;
                        float s2[4];
                        for (int i = 0; i < 4; ++i) s2[i] = s2p[(4 * g + i) * SF_V];
                        for (int i = 0; i < 4; ++i)
                            for (int t = 0; t < TPW; ++t)
                                if (FULL || wave * TPW + t < D)
                                    T2[gi][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(s2[i], T1[gi][t][i], T2[gi][t], 0, 0, 0);
                    } else {
                        const u4 s2 = S2b(gi)[(q2 * 16 + r) * 4 + g];
                        for (int t = 0; t < TPW; ++t)
                            if (FULL || wave * TPW + t < D)
                                T2[gi][t] = mfma_bf16x<PREC == PREC_BF16C>(s2, split4(T1[gi][t]), T2[gi][t]);
                    }
                    for (int t = 0; t < TPW; ++t) T1[gi][t] = (f4){0.f, 0.f, 0.f, 0.f};
                }
            }
            if (next < 0 || (next >> 4) != (cell >> 4)) {
                // end of an L1 plane -- mode 1, term by term through the one LDS transpose buffer
                for (int gi = 0; gi < GT; ++gi) {
                    if (gi >= gn) break;
                    for (int t = 0; t < TPW; ++t) {
                        const int v1 = wave * TPW + t;
                        if (!FULL && v1 >= D) break;
                        for (int i = 0; i < 4; ++i) T2f[v1 * T2F_V1 + (4 * g + i) * T2F_U2 + r] = T2[gi][t][i];
                    }
                    lds_barrier();
                    for (int t = 0; t < TPW; ++t) {
                        const int u2 = wave * TPW + t;
                        if (!FULL && u2 >= D) break;
                        f4 acc = {0.f, 0.f, 0.f, 0.f};
                        if constexpr (!BF) {
                            const float* s1p = S1f(gi) + q1 * 16 * SF_V + perm_row(r);
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
                            acc = mfma_bf16x<PREC == PREC_BF16C>(S1b(gi)[(q1 * 16 + perm_row(r)) * 4 + g], split4(bv), acc);
                        }
                        const d4 add = (d4){(double)acc[0], (double)acc[1], (double)acc[2], (double)acc[3]};
                        if (!tp.dpart) {
                            Y[t] += add;
                            continue;
                        }
                        for (int i = 0; i < 4; ++i) {
                            const int child = (4 * i + g >= K) + 2 * (u2 >= K) + 4 * (r >= K);
                            if ((cmb >> child) & 1) Y[t][i] += add[i];
                        }
                    }
                    for (int t = 0; t < TPW; ++t) T2[gi][t] = (f4){0.f, 0.f, 0.f, 0.f};
                    lds_barrier();
                }
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
template <int K, int CW, int PF, int G, int PREC>
__device__ __forceinline__ void contract_brick(const LevelDesc* __restrict__ levels, int2 job, int accumulate, double* smem,
                                               int2* steps, int* nsteps) {
    constexpr int D = 2 * K;
    constexpr int TPW = (D + CW - 1) / CW;
    constexpr int64_t E = (int64_t)D * D * D;
    int& nsteps_s = *nsteps;
    // wave index and every neighbour index are uniform per wave: keep them in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const LevelDesc lv = levels[job.x];
    const double* __restrict__ w = lv.w;
    const int64_t b = job.y;
    const int Lr = lv.Lr;
    const int NL = 2 * Lr + 1;
    const int32_t* nb = lv.nbr + b * NL * NL * NL;
    const int cmb = lv.cmask[b];
    double* ob = lv.out + b * E;
    // this launch's class adds to what the launches of the other classes wrote (accumulate)
    d4 Y[TPW];
    for (int t = 0; t < TPW; ++t) {
        Y[t] = (d4){0.0, 0.0, 0.0, 0.0};
        const int u2 = wave * TPW + t;
        if (!accumulate || u2 >= D) continue;
        for (int i = 0; i < 4; ++i) {
            const int u1 = 4 * i + g, u3 = r;
            if (u1 < D && u3 < D) Y[t][i] = ob[((int64_t)u1 * D + u2) * D + u3];
        }
    }
    for (int ti = 0; ti < lv.ntpl; ++ti) {
        const Tpl tp = lv.tpl[ti];
        if (tp.prec != PREC) continue;          // another launch's class
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
        if constexpr (PREC == PREC_F64 && G > 1) run_job_g<K, CW, G, PF>(lv, tp, w, ns, steps, smem, wave, g, r, cmb, Y);
        else if constexpr (PREC == PREC_F64) run_job<K, CW, PF, PREC>(lv, tp, w, ns, steps, smem, wave, g, r, cmb, Y);
        else run_job_lp<K, CW, PREC>(lv, tp, w, ns, steps, smem, wave, g, r, cmb, Y);
    }
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

// One launch per precision class PREC: it runs the jobs of that class only (each class's chain
// alone keeps the register count low) and, with accumulate set, adds to the output the launches
// of the other classes wrote.
template <int K, int CW, int PF, int WPE, int G, int PREC>
__global__ void __launch_bounds__(64 * CW) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
ns_apply_kernel(const LevelDesc* __restrict__ levels, const int2* __restrict__ order, int* __restrict__ queues,
                int accumulate) {
    __shared__ double smem[smem_doubles<PREC, K, G>()];
    __shared__ int2 steps[NMAX * NMAX * NMAX];
    __shared__ int nsteps_s, pos_s;
    if (!queues) {
        contract_brick<K, CW, PF, G, PREC>(levels, order[blockIdx.x], accumulate, smem, steps, &nsteps_s);
        return;
    }
    // persistent: pull positions from this XCD's queue, then from the others; every workgroup
    // leaves once all 8 queues are drained (at most 8 failed pulls per workgroup)
    const int x0 = blockIdx.x % NXCD;
    int tried = 0;   // meaningful in thread 0 only
    for (;;) {
        if (threadIdx.x == 0) {
            int pos = -1;
            while (tried < NXCD) {
                const int q = (x0 + tried) % NXCD;
                const int i = atomicAdd(&queues[q], 1);
                if (queues[NXCD + q] + i < queues[2 * NXCD + q]) {
                    pos = queues[NXCD + q] + i;
                    break;
                }
                ++tried;
            }
            pos_s = pos;
        }
        __syncthreads();
        const int pos = pos_s;
        __syncthreads();
        if (pos < 0) break;
        contract_brick<K, CW, PF, G, PREC>(levels, order[pos], accumulate, smem, steps, &nsteps_s);
    }
}

// Reduced-precision copies of input bricks: one thread per (brick, v1, v2, group of 4 columns)
// writes 16 bytes -- four FP32 values or their split BF16 (hi | lo); columns at or beyond 2K are
// zero.  Every entry of the table has whole blocks, so a block's entry is uniform.
template <int K>
__global__ void __launch_bounds__(256) convert_kernel(ConvTab tb) {
    constexpr int D = 2 * K;
    int e = 0;
    while (e + 1 < tb.n && (int64_t)blockIdx.x >= tb.bstart[e + 1]) ++e;
    const int64_t i = ((int64_t)blockIdx.x - tb.bstart[e]) * 256 + threadIdx.x;
    if (i >= tb.nb[e] * D * D * 4) return;
    const int gg = (int)(i & 3);
    const int64_t row = i >> 2;     // (brick, v1, v2)
    const double* x = tb.X[e] + row * D;
    f4 v;
    for (int c = 0; c < 4; ++c) v[c] = 4 * gg + c < D ? (float)x[4 * gg + c] : 0.f;
    tb.out[e][i] = tb.bf[e] ? split4(v) : __builtin_bit_cast(u4, v);
}

// Tile variants of the contraction kernel: (waves per block, prefetch depth, waves per SIMD, FP64
// terms per pass over the cells).
struct Variant {
    int cw, pf, wpe, g;
};
constexpr Variant VARIANTS[] = {{8, 0, 4, 1},  {8, 1, 2, 1},  {8, 2, 2, 1},  {16, 1, 4, 1},
                                {16, 2, 4, 1}, {16, 3, 4, 1}, {16, 0, 4, 2}, {16, 1, 4, 2}};
constexpr int NVARIANTS = sizeof(VARIANTS) / sizeof(VARIANTS[0]);
// Default shape: (16 waves, one workgroup per CU, two FP64 terms per pass, the next step's slice
// prefetched) for 6 <= k <= 8, where it was fastest (k = 8 Poisson workload; k = 6, 7 adaptive
// trees); (8 waves, no prefetch, 4 waves per SIMD, one term per pass) below.
constexpr int default_variant(int k) { return k >= 6 && k <= 8 ? 7 : 0; }

template <int K, int V, int PREC>
void launch_variant(hipStream_t st, int64_t nblocks, const LevelDesc* levels, const int2* order, int* queues, int acc) {
    constexpr Variant v = VARIANTS[V];
    ns_apply_kernel<K, v.cw, v.pf, v.wpe, v.g, PREC><<<(unsigned)nblocks, 64 * v.cw, 0, st>>>(levels, order, queues, acc);
}

template <int K, int V, int PREC>
int64_t resident_variant(int device) {
    constexpr Variant v = VARIANTS[V];
    int per_cu = 0, ncu = 0;
    MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ns_apply_kernel<K, v.cw, v.pf, v.wpe, v.g, PREC>, 64 * v.cw, 0));
    MWNS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    return (int64_t)std::max(1, per_cu) * ncu;
}

// The FP64 class exists in every tile variant; the reduced classes in the shape of variant 0 only.
template <int K>
struct ApplyLaunch {
    static void run(hipStream_t st, int variant, int prec, int acc, int64_t nblocks, const LevelDesc* levels,
                    const int2* order, int* queues, int64_t* resident, int device) {
        auto go = [&](auto vt, auto pt) {
            constexpr int V = decltype(vt)::value, PR = decltype(pt)::value;
            if (resident) *resident = resident_variant<K, V, PR>(device);
            else launch_variant<K, V, PR>(st, nblocks, levels, order, queues, acc);
        };
        using I0 = std::integral_constant<int, 0>;
        switch (prec) {
            case PREC_F32: go(I0{}, std::integral_constant<int, PREC_F32>{}); return;
            case PREC_BF16C: go(I0{}, std::integral_constant<int, PREC_BF16C>{}); return;
            case PREC_BF16: go(I0{}, std::integral_constant<int, PREC_BF16>{}); return;
            default: break;
        }
        using F = std::integral_constant<int, PREC_F64>;
        switch (variant) {
            case 0: go(I0{}, F{}); break;
            case 1: go(std::integral_constant<int, 1>{}, F{}); break;
            case 2: go(std::integral_constant<int, 2>{}, F{}); break;
            case 3: go(std::integral_constant<int, 3>{}, F{}); break;
            case 4: go(std::integral_constant<int, 4>{}, F{}); break;
            case 5: go(std::integral_constant<int, 5>{}, F{}); break;
            case 6: go(std::integral_constant<int, 6>{}, F{}); break;
            case 7: go(std::integral_constant<int, 7>{}, F{}); break;
            default: fail(MWNS_EINVAL, "unknown contraction kernel variant");
        }
    }
};

template <int K>
struct ConvertLaunch {
    static void run(hipStream_t st, const ConvTab& tb) {
        if (tb.n == 0) return;
        convert_kernel<K><<<(unsigned)tb.bstart[tb.n], 256, 0, st>>>(tb);
    }
};

}  // namespace

int num_variants() { return NVARIANTS; }

int variant_for(const mwns_ctx* ctx, int k) {
    const int v = ctx->variant[k];
    // k = 9, 10: variant 3 (three workgroups per compute unit), the fastest on the k = 10 workloads
    return v >= 0 ? v : (k > KNARROW ? 3 : default_variant(k));
}

template <template <int> class Fn, class... Args>
void dispatch_narrow(int k, Args&&... args) {
    switch (k) {
        case 1: Fn<1>::run(args...); break;
        case 2: Fn<2>::run(args...); break;
        case 3: Fn<3>::run(args...); break;
        case 4: Fn<4>::run(args...); break;
        case 5: Fn<5>::run(args...); break;
        case 6: Fn<6>::run(args...); break;
        case 7: Fn<7>::run(args...); break;
        case 8: Fn<8>::run(args...); break;
        default: fail(MWNS_EINVAL, "the one-tile contraction kernel takes k <= 8");
    }
}

void launch_contract(int k, int variant, int prec, bool accumulate, hipStream_t st, int64_t nblocks,
                     const LevelDesc* levels, const int2* order, int* queues) {
    if (nblocks <= 0) return;
    dispatch_narrow<ApplyLaunch>(k, st, variant, prec, accumulate ? 1 : 0, nblocks, levels, order, queues, (int64_t*)nullptr, 0);
}

int64_t resident_blocks(int k, int variant, int prec, int device) {
    int64_t n = 0;
    dispatch_narrow<ApplyLaunch>(k, (hipStream_t) nullptr, variant, prec, 0, (int64_t)0, (const LevelDesc*)nullptr,
                            (const int2*)nullptr, (int*)nullptr, &n, device);
    return n;
}

void launch_convert(int k, hipStream_t st, const ConvTab& tb) {
    if (tb.n == 0) return;
    dispatch_narrow<ConvertLaunch>(k, st, tb);
}

}  // namespace mwns

using namespace mwns;

extern "C" int mwns_num_variants(void) { return NVARIANTS; }

extern "C" int mwns_num_variants_for(int k) { return k > KNARROW ? num_wide_variants() : (k >= 1 ? NVARIANTS : 0); }

extern "C" mwns_status mwns_variant_shape(int v, int* waves, int* prefetch, int* waves_per_simd, int* terms_per_pass) {
    MWNS_GUARD_BEGIN
    if (v < 0 || v >= NVARIANTS || !waves || !prefetch || !waves_per_simd || !terms_per_pass)
        fail(MWNS_EINVAL, "variant out of range or NULL output");
    *waves = VARIANTS[v].cw;
    *prefetch = VARIANTS[v].pf;
    *waves_per_simd = VARIANTS[v].wpe;
    *terms_per_pass = VARIANTS[v].g;
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_ctx_set_variant(mwns_ctx* ctx, int k, int variant) {
    MWNS_GUARD_BEGIN
    if (!ctx) fail(MWNS_EINVAL, "ctx is NULL");
    if (k < 1 || k > KMAX) fail(MWNS_EINVAL, "k out of range");
    if (variant < -1 || variant >= (k > KNARROW ? num_wide_variants() : NVARIANTS)) fail(MWNS_EINVAL, "variant out of range");
    ctx->variant[k] = variant;
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_ctx_get_variant(const mwns_ctx* ctx, int k, int* variant) {
    MWNS_GUARD_BEGIN
    if (!ctx || !variant) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > KMAX) fail(MWNS_EINVAL, "k out of range");
    *variant = variant_for(ctx, k);
    return MWNS_OK;
    MWNS_GUARD_END
}
