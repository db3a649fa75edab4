// The contraction kernel of the apply for 8 < k <= 10 (2k in (16, 20]): the FP64 class and the
// FP32 class of the precision routing.
//
// Same method as contract.hip (sibling-group bricks, 2k x 2k super-blocks S^{j;m,L} per
// dimension, the nested-loop factorisation of Sec. 5 over boxes of coarse displacements, the
// coefficient rule c_m = [m in R_j(L)] - [b internal][m in R_{j+1}(l)]).  Every dimension of the
// brick is split 16 + 4: the first 16 indices go through v_mfma_f64_16x16x4 (A[m][k] in lane
// m+16k, B[k][n] in lane n+16k, D[4i+g][n] in lane 16g+n, register i), the last (up to) 4 through
// v_mfma_f64_4x4x4 with four blocks (A[i][k] of block b in lane i+4b+16k, B[k][j] in lane
// j+4b+16k, D[i][j] in lane j+4b+16i), its four blocks spanning the 16 columns of the other tile,
// so that a 4-row tail costs a quarter of a 16-row tile and lands in the lane layout of a
// 16x16x4 result row 16+g.  A workgroup computes the output columns u3 < 16 of one output brick,
// or its last (up to) four columns u3 = 16 + j; 10 waves own two input slices v1 each.
//   mode 3, per slice: rows v2 < 16 by 16x16x4, rows 16..19 by 4x4x4, contraction over v3 in
//     five K-steps (v3 = 4g + s for s < 4 from four consecutive doubles, then v3 = 16 + g);
//   mode 2, straight from the mode-3 accumulators (register i holds v2 = 4i + g, the tail holds
//     v2 = 16 + g): rows u2 < 16 by 16x16x4, rows 16..19 by 4x4x4, again five K-steps;
//   mode 1 through an LDS transpose of the mode-2 result, rows u1 split the same way.
// The last-columns workgroup uses the 4x4x4 form only: in modes 3 and 2 its four blocks take
// the four groups v2 = 4b + i of rows 0..15 (block b's result in mode 2 is a partial sum over its
// group, the blocks summed across lanes at the end of a plane), rows 16..19 once more with one
// block live; in mode 1 the blocks take the output rows u1 = 4b + i.
// The FP32 class reads FP32 copies of the input bricks and runs every 16 x 16 tile on
// v_mfma_f32_16x16x4 (A and B as above, D[4g+i][n] in lane 16g+n, register i: the rows of a
// result register are the K slots of the next mode, a permutation that the staged operands
// follow), its 4-row tails on the FP64 4x4x4 form as in the FP64 class, and adds each mode-1
// result to an FP64 output accumulator; it adds to the output bricks that the FP64 launch wrote.
#include <algorithm>

#include "contract.h"

namespace mwns {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int WCW = 10;            // waves per workgroup
constexpr int WCT = 64 * WCW;
constexpr int WS3_V = 36;          // LDS stride of the staged mode-3 operand [L][v3][u3 of this half]
constexpr int WSA_V = 48;          // LDS stride of the staged mode-2 / mode-1 operands [L][v][u < 32]

template <int K>
struct Wide {
    static constexpr int D = 2 * K;
    static constexpr int TPW = (D + WCW - 1) / WCW;
    static constexpr int T2_V1 = D * 16 + 16;     // LDS stride of the mode-2 result [v1][u2][16]
    static constexpr int SM_T2 = D * T2_V1;
    static constexpr int SM_S3 = NMAX * D * WS3_V;
    static constexpr int SM_SA = NMAX * D * WSA_V;
    static constexpr int SMEM = SM_T2 + SM_S3 + 2 * SM_SA;
    static_assert(D > 16 && D <= 20, "two tiles per dimension with the fifth K-step covering 16..19");
};

// Masked super-block entry S^{m,L}[u][v] (rows: output u = su*K + a; columns: input v); zero
// outside the 2K extent and outside the fine-displacement mask [mlo, mhi].
template <int K>
__device__ inline double wsop(const double* __restrict__ Fm, int L, int mlo, int mhi, int u, int v) {
    if (u >= 2 * K || v >= 2 * K) return 0.0;
    const int su = u >= K, sv = v >= K;
    const int l = 2 * L + su - sv;
    if (l < mlo || l > mhi) return 0.0;
    return Fm[(l + LF) * K * K + (u - su * K) * K + (v - sv * K)];
}

__device__ inline void wlds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// The step list of job tp for the brick whose neighbour table is nb: the cells of the box whose
// input exists, in (L1, L2, L3) order, as (input index, q1 << 4 | q2 << 2 | q3).  Returns their
// number; starts with a barrier (the previous job's readers are done) and ends with one.
__device__ inline int wide_steps(const Tpl& tp, const int32_t* __restrict__ nb, int Lr, int2* steps, int* nsteps) {
    const int NL = 2 * Lr + 1;
    const int n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
    wlds_barrier();
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
        if (t == 0) *nsteps = __popcll(in);
    }
    wlds_barrier();
    return __builtin_amdgcn_readfirstlane(*nsteps);
}

// Stages term m of job tp (the coefficient c w_m folded into S1): S1, S2 as [L][v][u < 32], S3 as
// [L][v3][UW columns u3 = u0 + ul]; ends with a barrier.
template <int K, int UW>
__device__ inline void wide_stage(const LevelDesc& lv, const Tpl& tp, int m, int u0, double* S1s, double* S2s, double* S3s) {
    constexpr int D = 2 * K;
    const int n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
    const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
    const double cw = tp.dpart ? -lv.w[m] : lv.w[m];
    const int nA = (n1 + n2) * D * 32, nS3 = n3 * D * UW;
    for (int e = threadIdx.x; e < nA + nS3; e += WCT) {
        if (e < nA) {
            const int u = e & 31, v = (e >> 5) % D, sb = (e >> 5) / D;
            if (sb < n1) S1s[(sb * D + v) * WSA_V + u] = cw * wsop<K>(Fm, tp.lo[0] + sb, tp.mlo[0], tp.mhi[0], u, v);
            else {
                const int q = sb - n1;
                S2s[(q * D + v) * WSA_V + u] = wsop<K>(Fm, tp.lo[1] + q, tp.mlo[1], tp.mhi[1], u, v);
            }
        } else {
            const int e3 = e - nA;
            const int ul = e3 % UW, v = (e3 / UW) % D, q = (e3 / UW) / D;
            S3s[(q * D + v) * WS3_V + ul] = wsop<K>(Fm, tp.lo[2] + q, tp.mlo[2], tp.mhi[2], u0 + ul, v);
        }
    }
    wlds_barrier();
}

// Byte offsets of lane (g, r)'s loads of input slice v1 (element size ES): four values
// X[v1][v2][4g..4g+3] and one value X[v1][v2][16 + g], v2 = r for the 16-row tile (a = 0) and
// 16 + (r & 3) for the tail (a = 1, the A operand of the 4x4x4 form repeated over its blocks);
// invalid ones point past the buffer (the load returns 0).
template <int D, int ES>
__device__ inline void wide_offsets(int v1, int g, int r, uint32_t (&off4)[2], uint32_t (&off1)[2]) {
    for (int a = 0; a < 2; ++a) {
        const int v2 = a == 0 ? r : 16 + (r & 3);
        const bool ok = v1 < D && v2 < D;
        off4[a] = ok ? (uint32_t)(((v1 * D + v2) * D + 4 * g) * ES) : 0x40000000u;
        off1[a] = ok && 16 + g < D ? (uint32_t)(((v1 * D + v2) * D + 16 + g) * ES) : 0x40000000u;
    }
}

// The five values at (off4, off1) as doubles, from an FP64 (ES = 8) or FP32 (ES = 4) brick.
template <int ES>
__device__ inline void wide_load(__amdgpu_buffer_rsrc_t rs, uint32_t off4, uint32_t off1, double (&x)[5]) {
    if constexpr (ES == 8) {
        const dv2 x01 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, off4, 0, 0));
        const dv2 x23 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, off4 + 16, 0, 0));
        x[0] = x01.x;
        x[1] = x01.y;
        x[2] = x23.x;
        x[3] = x23.y;
        x[4] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off1, 0, 0));
    } else {
        const f4 v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, off4, 0, 0));
        for (int c = 0; c < 4; ++c) x[c] = (double)v[c];
        x[4] = (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off1, 0, 0));
    }
}

// One job of the FP64 class (both column parts) or the last-columns job of the FP32 class (whose
// arithmetic is the 4x4x4 FP64 form throughout, on FP32 inputs).
template <int K, bool TAIL, int PREC>
__device__ __forceinline__ void contract_brick_wide(const LevelDesc* __restrict__ levels, int2 job, double* smem,
                                                    int2* steps, int* nsteps) {
    static_assert(PREC == PREC_F64 || (PREC == PREC_F32 && TAIL), "the FP32 first-columns job is contract_brick_wide_f32");
    constexpr int ES = PREC == PREC_F64 ? 8 : 4;    // bytes per input element
    using W = Wide<K>;
    constexpr int D = W::D, TPW = W::TPW;
    constexpr bool FULL = (WCW * TPW == D);
    constexpr int64_t E = (int64_t)D * D * D;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const LevelDesc lv = levels[job.x];
    const int64_t b = job.y >> 1;
    const int c = TAIL ? 1 : 0;                     // output columns u3 = 16c + r (16 + (r & 3) for the tail)
    constexpr int UW = TAIL ? 4 : 16;               // staged columns of S3
    const int Lr = lv.Lr;
    const int NL = 2 * Lr + 1;
    const int32_t* nb = lv.nbr + b * NL * NL * NL;
    const int cmb = lv.cmask[b];
    double* T2s = smem;
    double* S3s = smem + W::SM_T2;
    double* S2s = S3s + W::SM_S3;
    double* S1s = S2s + W::SM_SA;
    uint32_t off4[TPW][2], off1[TPW][2];
    for (int t = 0; t < TPW; ++t) wide_offsets<D, ES>(wave * TPW + t, g, r, off4[t], off1[t]);
    // Y[t]: rows u1 = 4i + g; Yt[t]: row u1 = 16 + g (columns u3 = 16c + r, u2 = wave * TPW + t).
    // Tail: Y[t][0]: row u1 = 4(r >> 2) + g, Yt[t]: row u1 = 16 + g, columns u3 = 16 + (r & 3).
    d4 Y[TPW];
    double Yt[TPW];
    for (int t = 0; t < TPW; ++t) {
        Y[t] = (d4){0.0, 0.0, 0.0, 0.0};
        Yt[t] = 0.0;
    }
    for (int ti = 0; ti < lv.ntpl; ++ti) {
        const Tpl tp = lv.tpl[ti];
        if (tp.prec != PREC) continue;          // another class's launch runs this job
        if (tp.dpart && cmb == 0) continue;     // no internal child receives the down band
        const int ns = wide_steps(tp, nb, Lr, steps, nsteps);
        if (ns == 0) continue;
        const int total = __builtin_amdgcn_readfirstlane((tp.m2 - tp.m1 + 1) * ns);
        int m = tp.m1, si = 0;
        // T1[t] / T1t[t]: mode-3 result rows v2 = 4i + g / 16 + g; T2[t] / T2t[t]: mode-2 result
        // rows u2 = 4i + g / 16 + g; columns u3 = 16c + r throughout.
        // Tail: T1[t][0]: rows v2 = 4(r >> 2) + g, T1t[t]: rows v2 = 16 + g; T2u[t][q]: block
        // (r >> 2)'s partial sum of rows u2 = 4q + g; columns u3 = 16 + (r & 3).
        d4 T1[TPW], T2[TPW];
        double T1t[TPW], T2t[TPW], T2u[TPW][5];
        for (int t = 0; t < TPW; ++t) {
            T1[t] = T2[t] = (d4){0.0, 0.0, 0.0, 0.0};
            T1t[t] = T2t[t] = 0.0;
            for (int q = 0; q < 5; ++q) T2u[t][q] = 0.0;
        }
        for (int s = 0; s < total; ++s) {
            if (si == 0) wide_stage<K, UW>(lv, tp, m, 16 * c, S1s, S2s, S3s);
            const int2 st = steps[si];
            const int idx = __builtin_amdgcn_readfirstlane(st.x);
            const int cell = __builtin_amdgcn_readfirstlane(st.y);
            const int next = si + 1 < ns ? __builtin_amdgcn_readfirstlane(steps[si + 1].y) : -1;
            const int q1 = cell >> 4, q2 = (cell >> 2) & 3, q3 = cell & 3;
            const char* X = PREC == PREC_F64
                                 ? (const char*)(idx < lv.nreal ? lv.Xr + idx * E : lv.Xg + (idx - lv.nreal) * E)
                                 : (const char*)(idx < lv.nreal ? lv.Xr32 + idx * E : lv.Xg32 + (idx - lv.nreal) * E);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, (int)(E * ES), 0x00020000);
            // mode 3: T1 += X x_3 S3^{L3}
            if constexpr (TAIL) {
                double s3[5];
                for (int kk = 0; kk < 4; ++kk) s3[kk] = S3s[(q3 * D + 4 * g + kk) * WS3_V + (r & 3)];
                s3[4] = 16 + g < D ? S3s[(q3 * D + 16 + g) * WS3_V + (r & 3)] : 0.0;
                for (int t = 0; t < TPW; ++t) {
                    if (!FULL && wave * TPW + t >= D) break;
                    double x[2][5];     // both loads of the slice issued before the first use
                    for (int a = 0; a < 2; ++a) wide_load<ES>(rs, off4[t][a], off1[t][a], x[a]);
                    for (int a = 0; a < 2; ++a) {
                        double acc = a == 0 ? T1[t][0] : T1t[t];
                        for (int kk = 0; kk < 5; ++kk) acc = __builtin_amdgcn_mfma_f64_4x4x4f64(x[a][kk], s3[kk], acc, 0, 0, 0);
                        if (a == 0) T1[t][0] = acc;
                        else T1t[t] = acc;
                    }
                }
            } else {
                double s3[5];
                for (int kk = 0; kk < 4; ++kk) s3[kk] = S3s[(q3 * D + 4 * g + kk) * WS3_V + r];
                s3[4] = 16 + g < D ? S3s[(q3 * D + 16 + g) * WS3_V + r] : 0.0;
                for (int t = 0; t < TPW; ++t) {
                    if (!FULL && wave * TPW + t >= D) break;
                    double x[5], xt[5];
                    wide_load<ES>(rs, off4[t][0], off1[t][0], x);
                    wide_load<ES>(rs, off4[t][1], off1[t][1], xt);
                    d4 acc = T1[t];
                    for (int kk = 0; kk < 5; ++kk) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[kk], s3[kk], acc, 0, 0, 0);
                    T1[t] = acc;
                    double acct = T1t[t];
                    for (int kk = 0; kk < 5; ++kk) acct = __builtin_amdgcn_mfma_f64_4x4x4f64(xt[kk], s3[kk], acct, 0, 0, 0);
                    T1t[t] = acct;
                }
            }
            if (next < 0 || (next >> 2) != (cell >> 2)) {
                // end of an (L1, L2) row -- mode 2: T2 += S2^{L2} x_2 T1
                if constexpr (TAIL) {
                    // block b = r >> 2 contracts its own rows v2 = 4b + k of T1[t][0]; rows 16..19
                    // (T1t, the same in every block) go through block 0 only
                    double sa[5], sb[5];
                    for (int q = 0; q < 5; ++q) {
                        sa[q] = S2s[(q2 * D + 4 * (r >> 2) + g) * WSA_V + 4 * q + (r & 3)];
                        sb[q] = r < 4 && 16 + g < D ? S2s[(q2 * D + 16 + g) * WSA_V + 4 * q + (r & 3)] : 0.0;
                    }
                    for (int t = 0; t < TPW; ++t) {
                        if (!FULL && wave * TPW + t >= D) break;
                        for (int q = 0; q < 5; ++q) {
                            const double acc = __builtin_amdgcn_mfma_f64_4x4x4f64(sa[q], T1[t][0], T2u[t][q], 0, 0, 0);
                            T2u[t][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(sb[q], T1t[t], acc, 0, 0, 0);
                        }
                    }
                } else {
                double s2[5], s2t[5];
                for (int i = 0; i < 4; ++i) {
                    s2[i] = S2s[(q2 * D + 4 * i + g) * WSA_V + r];
                    s2t[i] = S2s[(q2 * D + 4 * i + g) * WSA_V + 16 + (r & 3)];
                }
                s2[4] = 16 + g < D ? S2s[(q2 * D + 16 + g) * WSA_V + r] : 0.0;
                s2t[4] = 16 + g < D ? S2s[(q2 * D + 16 + g) * WSA_V + 16 + (r & 3)] : 0.0;
                for (int t = 0; t < TPW; ++t) {
                    if (!FULL && wave * TPW + t >= D) break;
                    d4 acc = T2[t];
                    double acct = T2t[t];
                    for (int i = 0; i < 4; ++i) {
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s2[i], T1[t][i], acc, 0, 0, 0);
                        acct = __builtin_amdgcn_mfma_f64_4x4x4f64(s2t[i], T1[t][i], acct, 0, 0, 0);
                    }
                    T2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(s2[4], T1t[t], acc, 0, 0, 0);
                    T2t[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(s2t[4], T1t[t], acct, 0, 0, 0);
                }
                }
                for (int t = 0; t < TPW; ++t) {
                    T1[t] = (d4){0.0, 0.0, 0.0, 0.0};
                    T1t[t] = 0.0;
                }
            }
            if (next < 0 || (next >> 4) != (cell >> 4)) {
                // end of an L1 plane -- mode 1 through an LDS transpose: Y += S1^{L1} x_1 T2
                if constexpr (TAIL) {
                    // sum the four blocks' partial results (lanes r, r ^ 4, r ^ 8, r ^ 12), store
                    // T2[v1][u2 = 4q + g][16 + r] from lanes r < 4
                    for (int t = 0; t < TPW; ++t) {
                        const int v1 = wave * TPW + t;
                        if (!FULL && v1 >= D) break;
                        for (int q = 0; q < 5; ++q) {
                            double v = T2u[t][q];
                            v += __shfl_xor(v, 4);
                            v += __shfl_xor(v, 8);
                            if (r < 4 && 4 * q + g < D) T2s[v1 * W::T2_V1 + (4 * q + g) * 16 + r] = v;
                            T2u[t][q] = 0.0;
                        }
                    }
                    wlds_barrier();
                    for (int t = 0; t < TPW; ++t) {
                        const int u2 = wave * TPW + t;
                        if (!FULL && u2 >= D) break;
                        // B[k][j] = T2[v1][u2][16 + j], the same in every block; block b = r >> 2
                        // yields rows u1 = 4b + g, the second chain rows u1 = 16 + g
                        double bv[5];
                        for (int kk = 0; kk < 4; ++kk) bv[kk] = T2s[(4 * kk + g) * W::T2_V1 + u2 * 16 + (r & 3)];
                        bv[4] = 16 + g < D ? T2s[(16 + g) * W::T2_V1 + u2 * 16 + (r & 3)] : 0.0;
                        double acc = 0.0, acct = 0.0;
                        for (int kk = 0; kk < 4; ++kk) {
                            acc = __builtin_amdgcn_mfma_f64_4x4x4f64(S1s[(q1 * D + 4 * kk + g) * WSA_V + r], bv[kk], acc, 0, 0, 0);
                            acct = __builtin_amdgcn_mfma_f64_4x4x4f64(S1s[(q1 * D + 4 * kk + g) * WSA_V + 16 + (r & 3)], bv[kk], acct, 0, 0, 0);
                        }
                        acc = __builtin_amdgcn_mfma_f64_4x4x4f64(16 + g < D ? S1s[(q1 * D + 16 + g) * WSA_V + r] : 0.0, bv[4], acc, 0, 0, 0);
                        acct = __builtin_amdgcn_mfma_f64_4x4x4f64(16 + g < D ? S1s[(q1 * D + 16 + g) * WSA_V + 16 + (r & 3)] : 0.0,
                                                                  bv[4], acct, 0, 0, 0);
                        if (tp.dpart) {
                            // u3 = 16 + (r & 3) >= K: the z parity bit is set
                            const int u1 = 4 * (r >> 2) + g;
                            if ((cmb >> ((u1 >= K) + 2 * (u2 >= K) + 4)) & 1) Y[t][0] += acc;
                            if ((cmb >> (1 + 2 * (u2 >= K) + 4)) & 1) Yt[t] += acct;
                        } else {
                            Y[t][0] += acc;
                            Yt[t] += acct;
                        }
                    }
                    wlds_barrier();
                } else {
                for (int t = 0; t < TPW; ++t) {
                    const int v1 = wave * TPW + t;
                    if (!FULL && v1 >= D) break;
                    for (int i = 0; i < 4; ++i) T2s[v1 * W::T2_V1 + (4 * i + g) * 16 + r] = T2[t][i];
                    if (16 + g < D) T2s[v1 * W::T2_V1 + (16 + g) * 16 + r] = T2t[t];
                }
                wlds_barrier();
                for (int t = 0; t < TPW; ++t) {
                    const int u2 = wave * TPW + t;
                    if (!FULL && u2 >= D) break;
                    double bv[5];
                    for (int kk = 0; kk < 4; ++kk) bv[kk] = T2s[(4 * kk + g) * W::T2_V1 + u2 * 16 + r];
                    bv[4] = 16 + g < D ? T2s[(16 + g) * W::T2_V1 + u2 * 16 + r] : 0.0;
                    // the down band reaches only internal children: accumulate it apart, add it masked
                    d4 acc = tp.dpart ? (d4){0.0, 0.0, 0.0, 0.0} : Y[t];
                    double acct = tp.dpart ? 0.0 : Yt[t];
                    for (int kk = 0; kk < 4; ++kk) {
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(S1s[(q1 * D + 4 * kk + g) * WSA_V + r], bv[kk], acc, 0, 0, 0);
                        acct = __builtin_amdgcn_mfma_f64_4x4x4f64(S1s[(q1 * D + 4 * kk + g) * WSA_V + 16 + (r & 3)], bv[kk], acct, 0, 0, 0);
                    }
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(16 + g < D ? S1s[(q1 * D + 16 + g) * WSA_V + r] : 0.0, bv[4], acc, 0, 0, 0);
                    acct = __builtin_amdgcn_mfma_f64_4x4x4f64(16 + g < D ? S1s[(q1 * D + 16 + g) * WSA_V + 16 + (r & 3)] : 0.0,
                                                              bv[4], acct, 0, 0, 0);
                    if (tp.dpart) {
                        const int u3 = 16 * c + r;
                        for (int i = 0; i < 4; ++i) {
                            const int child = (4 * i + g >= K) + 2 * (u2 >= K) + 4 * (u3 >= K);
                            if ((cmb >> child) & 1) Y[t][i] += acc[i];
                        }
                        const int child = 1 + 2 * (u2 >= K) + 4 * (u3 >= K);   // u1 = 16 + g >= K
                        if ((cmb >> child) & 1) Yt[t] += acct;
                    } else {
                        Y[t] = acc;
                        Yt[t] = acct;
                    }
                }
                for (int t = 0; t < TPW; ++t) {
                    T2[t] = (d4){0.0, 0.0, 0.0, 0.0};
                    T2t[t] = 0.0;
                }
                wlds_barrier();
                }
            }
            if (++si == ns) {
                si = 0;
                ++m;
            }
        }
    }
    double* ob = lv.out + b * E;
    if constexpr (TAIL) {
        for (int t = 0; t < TPW; ++t) {
            const int u2 = wave * TPW + t;
            if (u2 >= D) break;
            const int u3 = 16 + (r & 3);
            if (u3 < D) {
                const int u1 = 4 * (r >> 2) + g;
                const bool ok = (lv.valid >> ((u1 >= K) + 2 * (u2 >= K) + 4)) & 1;
                double* o = ob + ((int64_t)u1 * D + u2) * D + u3;
                if (PREC == PREC_F64) *o = ok ? Y[t][0] : 0.0;
                else if (ok) *o += Y[t][0];
                if (r < 4 && 16 + g < D) {
                    const bool okt = (lv.valid >> (1 + 2 * (u2 >= K) + 4)) & 1;
                    double* ot = ob + ((int64_t)(16 + g) * D + u2) * D + u3;
                    if (PREC == PREC_F64) *ot = okt ? Yt[t] : 0.0;
                    else if (okt) *ot += Yt[t];
                }
            }
        }
        return;
    }
    const int u3 = 16 * c + r;
    for (int t = 0; t < TPW; ++t) {
        const int u2 = wave * TPW + t;
        if (u2 >= D || u3 >= D) break;
        for (int i = 0; i < 4; ++i) {
            const int u1 = 4 * i + g;
            const int child = (u1 >= K) + 2 * (u2 >= K) + 4 * (u3 >= K);
            ob[((int64_t)u1 * D + u2) * D + u3] = ((lv.valid >> child) & 1) ? Y[t][i] : 0.0;
        }
        const int u1 = 16 + g;
        if (u1 < D) {
            const int child = 1 + 2 * (u2 >= K) + 4 * (u3 >= K);
            ob[((int64_t)u1 * D + u2) * D + u3] = ((lv.valid >> child) & 1) ? Yt[t] : 0.0;
        }
    }
}

// The first-columns job (u3 < 16) of the FP32 class.  Mode products of the 16 x 16 tiles on
// v_mfma_f32_16x16x4 from FP32 operands (result register i holds rows 4g + i), the tails on the
// FP64 4x4x4 form; the plane results go to an FP64 accumulator Y (rows u1 = 4g + i) and Yt (row
// u1 = 16 + g), which are added to the output brick.
template <int K>
__device__ __forceinline__ void contract_brick_wide_f32(const LevelDesc* __restrict__ levels, int2 job, double* smem,
                                                        int2* steps, int* nsteps) {
    using W = Wide<K>;
    constexpr int D = W::D, TPW = W::TPW;
    constexpr bool FULL = (WCW * TPW == D);
    constexpr int64_t E = (int64_t)D * D * D;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const LevelDesc lv = levels[job.x];
    const int64_t b = job.y >> 1;
    const int Lr = lv.Lr;
    const int NL = 2 * Lr + 1;
    const int32_t* nb = lv.nbr + b * NL * NL * NL;
    const int cmb = lv.cmask[b];
    double* T2s = smem;
    double* S3s = smem + W::SM_T2;
    double* S2s = S3s + W::SM_S3;
    double* S1s = S2s + W::SM_SA;
    uint32_t off4[TPW][2], off1[TPW][2];
    for (int t = 0; t < TPW; ++t) wide_offsets<D, 4>(wave * TPW + t, g, r, off4[t], off1[t]);
    d4 Y[TPW];
    double Yt[TPW];
    for (int t = 0; t < TPW; ++t) {
        Y[t] = (d4){0.0, 0.0, 0.0, 0.0};
        Yt[t] = 0.0;
    }
    for (int ti = 0; ti < lv.ntpl; ++ti) {
        const Tpl tp = lv.tpl[ti];
        if (tp.prec != PREC_F32) continue;
        if (tp.dpart && cmb == 0) continue;
        const int ns = wide_steps(tp, nb, Lr, steps, nsteps);
        if (ns == 0) continue;
        const int total = __builtin_amdgcn_readfirstlane((tp.m2 - tp.m1 + 1) * ns);
        int m = tp.m1, si = 0;
        // T1[t] / T1t[t]: mode-3 result rows v2 = 4g + i / 16 + g; T2[t] / T2t[t]: mode-2 result
        // rows u2 = 4g + i / 16 + g; columns u3 = r
        f4 T1[TPW], T2[TPW];
        double T1t[TPW], T2t[TPW];
        for (int t = 0; t < TPW; ++t) {
            T1[t] = T2[t] = (f4){0.f, 0.f, 0.f, 0.f};
            T1t[t] = T2t[t] = 0.0;
        }
        for (int s = 0; s < total; ++s) {
            if (si == 0) wide_stage<K, 16>(lv, tp, m, 0, S1s, S2s, S3s);
            const int2 st = steps[si];
            const int idx = __builtin_amdgcn_readfirstlane(st.x);
            const int cell = __builtin_amdgcn_readfirstlane(st.y);
            const int next = si + 1 < ns ? __builtin_amdgcn_readfirstlane(steps[si + 1].y) : -1;
            const int q1 = cell >> 4, q2 = (cell >> 2) & 3, q3 = cell & 3;
            const float* X = idx < lv.nreal ? lv.Xr32 + idx * E : lv.Xg32 + (idx - lv.nreal) * E;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, (int)(E * 4), 0x00020000);
            // mode 3: T1 += X x_3 S3^{L3}; K slot g of step kk is v3 = 4g + kk (kk < 4), 16 + g
            {
                double s3[5];
                for (int kk = 0; kk < 4; ++kk) s3[kk] = S3s[(q3 * D + 4 * g + kk) * WS3_V + r];
                s3[4] = 16 + g < D ? S3s[(q3 * D + 16 + g) * WS3_V + r] : 0.0;
                double x[TPW][2][5];
                for (int t = 0; t < TPW; ++t)
                    for (int a = 0; a < 2; ++a) wide_load<4>(rs, off4[t][a], off1[t][a], x[t][a]);
                for (int t = 0; t < TPW; ++t) {
                    if (!FULL && wave * TPW + t >= D) break;
                    f4 acc = T1[t];
                    for (int kk = 0; kk < 5; ++kk)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)x[t][0][kk], (float)s3[kk], acc, 0, 0, 0);
                    T1[t] = acc;
                    double acct = T1t[t];
                    for (int kk = 0; kk < 5; ++kk) acct = __builtin_amdgcn_mfma_f64_4x4x4f64(x[t][1][kk], s3[kk], acct, 0, 0, 0);
                    T1t[t] = acct;
                }
            }
            if (next < 0 || (next >> 2) != (cell >> 2)) {
                // end of an (L1, L2) row -- mode 2: T2 += S2^{L2} x_2 T1; K slot g of step i is
                // v2 = 4g + i (the rows of T1 register i), then 16 + g
                float s2[5];
                double s2t[5];
                for (int i = 0; i < 4; ++i) {
                    s2[i] = (float)S2s[(q2 * D + 4 * g + i) * WSA_V + r];
                    s2t[i] = S2s[(q2 * D + 4 * g + i) * WSA_V + 16 + (r & 3)];
                }
                s2[4] = 16 + g < D ? (float)S2s[(q2 * D + 16 + g) * WSA_V + r] : 0.f;
                s2t[4] = 16 + g < D ? S2s[(q2 * D + 16 + g) * WSA_V + 16 + (r & 3)] : 0.0;
                for (int t = 0; t < TPW; ++t) {
                    if (!FULL && wave * TPW + t >= D) break;
                    f4 acc = T2[t];
                    double acct = T2t[t];
                    for (int i = 0; i < 4; ++i) {
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(s2[i], T1[t][i], acc, 0, 0, 0);
                        acct = __builtin_amdgcn_mfma_f64_4x4x4f64(s2t[i], (double)T1[t][i], acct, 0, 0, 0);
                    }
                    T2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(s2[4], (float)T1t[t], acc, 0, 0, 0);
                    T2t[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(s2t[4], T1t[t], acct, 0, 0, 0);
                }
                for (int t = 0; t < TPW; ++t) {
                    T1[t] = (f4){0.f, 0.f, 0.f, 0.f};
                    T1t[t] = 0.0;
                }
            }
            if (next < 0 || (next >> 4) != (cell >> 4)) {
                // end of an L1 plane -- mode 1 through the LDS transpose: Y += S1^{L1} x_1 T2
                for (int t = 0; t < TPW; ++t) {
                    const int v1 = wave * TPW + t;
                    if (!FULL && v1 >= D) break;
                    for (int i = 0; i < 4; ++i) T2s[v1 * W::T2_V1 + (4 * g + i) * 16 + r] = (double)T2[t][i];
                    if (16 + g < D) T2s[v1 * W::T2_V1 + (16 + g) * 16 + r] = T2t[t];
                }
                wlds_barrier();
                for (int t = 0; t < TPW; ++t) {
                    const int u2 = wave * TPW + t;
                    if (!FULL && u2 >= D) break;
                    double bv[5];
                    for (int kk = 0; kk < 4; ++kk) bv[kk] = T2s[(4 * kk + g) * W::T2_V1 + u2 * 16 + r];
                    bv[4] = 16 + g < D ? T2s[(16 + g) * W::T2_V1 + u2 * 16 + r] : 0.0;
                    f4 acc = {0.f, 0.f, 0.f, 0.f};
                    double acct = 0.0;
                    for (int kk = 0; kk < 4; ++kk) {
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)S1s[(q1 * D + 4 * kk + g) * WSA_V + r], (float)bv[kk], acc, 0, 0, 0);
                        acct = __builtin_amdgcn_mfma_f64_4x4x4f64(S1s[(q1 * D + 4 * kk + g) * WSA_V + 16 + (r & 3)], bv[kk], acct, 0, 0, 0);
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(16 + g < D ? (float)S1s[(q1 * D + 16 + g) * WSA_V + r] : 0.f,
                                                               (float)bv[4], acc, 0, 0, 0);
                    acct = __builtin_amdgcn_mfma_f64_4x4x4f64(16 + g < D ? S1s[(q1 * D + 16 + g) * WSA_V + 16 + (r & 3)] : 0.0,
                                                              bv[4], acct, 0, 0, 0);
                    for (int i = 0; i < 4; ++i) {
                        const int child = (4 * g + i >= K) + 2 * (u2 >= K) + 4 * (r >= K);
                        if (!tp.dpart || ((cmb >> child) & 1)) Y[t][i] += (double)acc[i];
                    }
                    const int childt = 1 + 2 * (u2 >= K) + 4 * (r >= K);   // u1 = 16 + g >= K
                    if (!tp.dpart || ((cmb >> childt) & 1)) Yt[t] += acct;
                }
                for (int t = 0; t < TPW; ++t) {
                    T2[t] = (f4){0.f, 0.f, 0.f, 0.f};
                    T2t[t] = 0.0;
                }
                wlds_barrier();
            }
            if (++si == ns) {
                si = 0;
                ++m;
            }
        }
    }
    double* ob = lv.out + b * E;
    for (int t = 0; t < TPW; ++t) {
        const int u2 = wave * TPW + t;
        if (u2 >= D) break;
        for (int i = 0; i < 4; ++i) {
            const int u1 = 4 * g + i;
            if ((lv.valid >> ((u1 >= K) + 2 * (u2 >= K) + 4 * (r >= K))) & 1) ob[((int64_t)u1 * D + u2) * D + r] += Y[t][i];
        }
        const int u1 = 16 + g;
        if (u1 < D && ((lv.valid >> (1 + 2 * (u2 >= K) + 4 * (r >= K))) & 1)) ob[((int64_t)u1 * D + u2) * D + r] += Yt[t];
    }
}

template <int K, int PREC>
__device__ __forceinline__ void wide_job(const LevelDesc* __restrict__ levels, int2 job, double* smem, int2* steps, int* nsteps) {
    if (job.y & 1) contract_brick_wide<K, true, PREC>(levels, job, smem, steps, nsteps);
    else if constexpr (PREC == PREC_F64) contract_brick_wide<K, false, PREC_F64>(levels, job, smem, steps, nsteps);
    else contract_brick_wide_f32<K>(levels, job, smem, steps, nsteps);
}

// order[] entries are (level descriptor, 2 * brick + column part).  queues: as the one-tile kernel.
template <int K, int PREC>
__global__ void __launch_bounds__(WCT) __attribute__((amdgpu_waves_per_eu(3, 3)))
ns_apply_wide_kernel(const LevelDesc* __restrict__ levels, const int2* __restrict__ order, int* __restrict__ queues) {
    __shared__ double smem[Wide<K>::SMEM];
    __shared__ int2 steps[NMAX * NMAX * NMAX];
    __shared__ int nsteps_s, pos_s;
    if (!queues) {
        wide_job<K, PREC>(levels, order[blockIdx.x], smem, steps, &nsteps_s);
        return;
    }
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
        wide_job<K, PREC>(levels, order[pos], smem, steps, &nsteps_s);
    }
}

// FP32 copy of nb bricks of D^3 doubles, in the same [brick][v1][v2][v3] order.
__global__ void convert_wide_kernel(int64_t n, const double* __restrict__ X, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)X[i];
}

template <int K, int PREC>
void launch_wide_k(hipStream_t st, int64_t nblocks, const LevelDesc* levels, const int2* order, int* queues) {
    ns_apply_wide_kernel<K, PREC><<<(unsigned)nblocks, WCT, 0, st>>>(levels, order, queues);
}

template <int K, int PREC>
int64_t resident_wide_k(int device) {
    int per_cu = 0, ncu = 0;
    MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ns_apply_wide_kernel<K, PREC>, WCT, 0));
    MWNS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    return (int64_t)std::max(1, per_cu) * ncu;
}

void check_wide(int k, int prec) {
    if (k != 9 && k != 10) fail(MWNS_EINVAL, "the two-tile contraction kernel takes 8 < k <= 10");
    if (prec != PREC_F64 && prec != PREC_F32) fail(MWNS_EINVAL, "the two-tile contraction kernel has the FP64 and FP32 classes");
}

}  // namespace

void launch_contract_wide(int k, int prec, hipStream_t st, int64_t nblocks, const LevelDesc* levels, const int2* order,
                          int* queues) {
    check_wide(k, prec);
    if (nblocks <= 0) return;
    if (k == 9) {
        if (prec == PREC_F64) launch_wide_k<9, PREC_F64>(st, nblocks, levels, order, queues);
        else launch_wide_k<9, PREC_F32>(st, nblocks, levels, order, queues);
    } else {
        if (prec == PREC_F64) launch_wide_k<10, PREC_F64>(st, nblocks, levels, order, queues);
        else launch_wide_k<10, PREC_F32>(st, nblocks, levels, order, queues);
    }
}

int64_t resident_blocks_wide(int k, int prec, int device) {
    check_wide(k, prec);
    if (k == 9) return prec == PREC_F64 ? resident_wide_k<9, PREC_F64>(device) : resident_wide_k<9, PREC_F32>(device);
    return prec == PREC_F64 ? resident_wide_k<10, PREC_F64>(device) : resident_wide_k<10, PREC_F32>(device);
}

void launch_convert_wide(int k, hipStream_t st, int64_t nb, const double* X, float* out) {
    check_wide(k, PREC_F64);
    const int64_t n = nb * 8 * (int64_t)k * k * k;
    if (n <= 0) return;
    convert_wide_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, X, out);
}

}  // namespace mwns
