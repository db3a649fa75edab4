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

// The FP32 class: the first-columns job (u3 < 16) or the last-columns job of one output brick.
template <int K>
__device__ __forceinline__ void wide_job_f32(const LevelDesc* __restrict__ levels, int2 job, double* smem, int2* steps,
                                             int* nsteps) {
    if (job.y & 1) contract_brick_wide<K, true, PREC_F32>(levels, job, smem, steps, nsteps);
    else contract_brick_wide_f32<K>(levels, job, smem, steps, nsteps);
}

// FP32 class: order[] entries are (level descriptor, 2 * brick + column part).  queues: as the
// one-tile kernel.
template <int K>
__global__ void __launch_bounds__(WCT) __attribute__((amdgpu_waves_per_eu(3, 3)))
ns_apply_wide_f32_kernel(const LevelDesc* __restrict__ levels, const int2* __restrict__ order, int* __restrict__ queues) {
    __shared__ double smem[Wide<K>::SMEM];
    __shared__ int2 steps[NMAX * NMAX * NMAX];
    __shared__ int nsteps_s, pos_s;
    if (!queues) {
        wide_job_f32<K>(levels, order[blockIdx.x], smem, steps, &nsteps_s);
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
        wide_job_f32<K>(levels, order[pos], smem, steps, &nsteps_s);
    }
}

// ---------------------------------------------------------------- FP64 class, whole brick
// One workgroup of four waves per output brick, two workgroups per CU (two waves per SIMD, so that
// one hides the other's loads and barriers).  A plane of cells (fixed L1) runs in five rounds; in
// round i wave w takes input slice v1 = w + 4i: every row (fixed L2) of the plane runs mode 3 over
// its cells and then mode 2, and the slice's mode-2 result goes to LDS.  After a barrier, each
// wave adds the round's four slices to its output rows u2 = w + 4q (q < 5) by one K step of mode 1,
// accumulating straight into the output registers.  The input slice of the next item (slice, cell)
// is loaded while the current one is computed.
// LDS holds the term's super-blocks S_d^{L} for the job's box, staged with the coefficient c w_m
// folded into mode 1, the fine-displacement mask applied, and zeros up to the padded extent
// DP = 20 (so k = 9 needs no bounds tests in the loops), plus two buffers of four exchanged slices.
// Tiles: 16 x 16 x 4 for rows and columns < 16, and the 4 x 4 x 4 four-block form for the rest:
//   row tail (rows 16..19, columns < 16): blocks = column groups; A replicated over the blocks;
//   column tail (rows < 16, columns 16..19): blocks = row groups; B replicated;
//   corner (rows and columns 16..19): both replicated (every block computes the same result).
// Lane (g, r) = (lane >> 4, lane & 15).  The K index of step s is 4g + s (s < 4) or 16 + g
// (s = 4) in mode 3, where the slice is loaded as four consecutive doubles per lane, and 4s + g in
// modes 2 and 1, where it is the row index of the previous mode's result registers (mode 1: the
// slot of the exchanged slice).
template <int K>
struct BrickShape {
    static constexpr int D = 2 * K;              // 18 or 20
    static constexpr int DP = 20;                // padded extent of staged blocks and exchanged slices
    static constexpr int BLK = DP * DP;
    static constexpr int SM_S = 3 * NMAX * BLK;  // staged super-blocks [d][L - lo_d][v][u]
    static constexpr int SM_X = 2 * 4 * BLK;     // exchange buffers [2][slot][u2][u3]
    static constexpr int SMEM = SM_S + SM_X;
    static_assert(D > 16 && D <= DP, "rows and columns 16..D-1 are the 4-row tails");
    static_assert(SMEM * 8 + 1024 <= 80 * 1024, "two workgroups per CU");
};

__device__ inline double mfma4(double a, double b, double c) { return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0); }
__device__ inline d4 mfma16(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Stages term m of job tp: for each mode d and L in [lo_d, hi_d], S_d^{L}[v][u] (u output, v input,
// u = su*K + a, v = sv*K + b) = F^{2L+su-sv}_{ab} when that fine displacement lies in the job's mask,
// else 0, and 0 for u or v >= 2K; block (d, L - lo_d) of Ss.  Mode 1 carries c w_m.
template <int K>
__device__ inline void brick_stage_mode(const double* __restrict__ Fm, int lo, int hi, int mlo, int mhi, double scale,
                                        double* __restrict__ Sd) {
    using B = BrickShape<K>;
    const int tot = (hi - lo + 1) * B::BLK;
    for (int e = threadIdx.x; e < tot; e += 256) {
        const int blk = e / B::BLK;
        const int rem = e - blk * B::BLK;
        const int v = rem / B::DP, u = rem - v * B::DP;
        double val = 0.0;
        if (u < 2 * K && v < 2 * K) {
            const int su = u >= K, sv = v >= K;
            const int l = 2 * (lo + blk) + su - sv;
            if (l >= mlo && l <= mhi) val = scale * Fm[(l + LF) * K * K + (u - su * K) * K + (v - sv * K)];
        }
        Sd[blk * B::BLK + v * B::DP + u] = val;
    }
}

template <int K>
__device__ inline void brick_stage(const LevelDesc& lv, const Tpl& tp, int m, double* __restrict__ Ss) {
    using B = BrickShape<K>;
    const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
    const double cw = tp.dpart ? -lv.w[m] : lv.w[m];
    brick_stage_mode<K>(Fm, tp.lo[0], tp.hi[0], tp.mlo[0], tp.mhi[0], cw, Ss);
    brick_stage_mode<K>(Fm, tp.lo[1], tp.hi[1], tp.mlo[1], tp.mhi[1], 1.0, Ss + NMAX * B::BLK);
    brick_stage_mode<K>(Fm, tp.lo[2], tp.hi[2], tp.mlo[2], tp.mhi[2], 1.0, Ss + 2 * NMAX * B::BLK);
}

// Lane constants of the input-slice loads: byte offsets within slice 0 of X[v1][v2][v3] of lane
// (g, r)'s four consecutive doubles of row r (of) and of tail row 16 + (r & 3) (ot), from column
// 4g, and of its single doubles in column 16 + g (of4, ot4); entries outside the brick get an
// offset past the buffer's record size, which reads as zero.
struct SliceOffsets {
    uint32_t of, ot, of4, ot4;
};
template <int D>
__device__ inline SliceOffsets slice_offsets(int g, int r) {
    const uint32_t BAD = 0x40000000u;
    const int rt = 16 + (r & 3);
    SliceOffsets o;
    o.of = (uint32_t)((r * D + 4 * g) * 8);
    o.ot = rt < D ? (uint32_t)((rt * D + 4 * g) * 8) : BAD;
    o.of4 = 16 + g < D ? (uint32_t)((r * D + 16 + g) * 8) : BAD;
    o.ot4 = rt < D && 16 + g < D ? (uint32_t)((rt * D + 16 + g) * 8) : BAD;
    return o;
}

// The ten doubles of lane (g, r) of input slice v1 of brick X: xf[s] = X[v1][r][v3] (rows < 16),
// xt[s] = X[v1][16 + (r & 3)][v3] (the tail rows, the same in every block), v3 = 4g + s or 16 + g.
template <int D>
__device__ inline void brick_slice_load(const double* __restrict__ X, int v1, const SliceOffsets& o, double (&xf)[5],
                                        double (&xt)[5]) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, D * D * D * 8, 0x00020000);
    const int so = v1 * D * D * 8;
    const dv2 a0 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, o.of, so, 0));
    const dv2 a1 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, o.of + 16, so, 0));
    const dv2 b0 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, o.ot, so, 0));
    const dv2 b1 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(rs, o.ot + 16, so, 0));
    xf[0] = a0.x; xf[1] = a0.y; xf[2] = a1.x; xf[3] = a1.y;
    xt[0] = b0.x; xt[1] = b0.y; xt[2] = b1.x; xt[3] = b1.y;
    xf[4] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, o.of4, so, 0));
    xt[4] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, o.ot4, so, 0));
}

// One job of the FP64 class for one output brick (see above); Y accumulates over the jobs.
// PF = 1 loads the input slice of the next item while the current one is computed, PF = 0 each
// slice when it is needed.  Down-band jobs whose brick has leaf children run mode 1 in two passes,
// one per half u1 < K, u1 >= K, each with the output columns of leaf children masked out of the
// exchanged slices.
template <int K, int PF>
__device__ __forceinline__ void brick_job(const LevelDesc& lv, const Tpl& tp, int ns, const int2* __restrict__ steps,
                                          double* __restrict__ smem, int wave, int g, int r, int cmb,
                                          d4 (&Yf)[5], double (&Yr)[5], double (&Yc)[5], double (&Yx)[5]) {
    using B = BrickShape<K>;
    constexpr int D = B::D, DP = B::DP, BLK = B::BLK;
    constexpr int64_t E = (int64_t)D * D * D;
    double* Ss = smem;
    double* XB = smem + B::SM_S;
    const int rt = 16 + (r & 3);
    const int nsl = (D - wave + 3) / 4;      // rounds with a slice for this wave (5; 4 for waves 2, 3 at k = 9)
    const bool split = tp.dpart && cmb != 0xff;
    const SliceOffsets so = slice_offsets<D>(g, r);
    // the step list in registers, lane c holding step c (read back with readlane, no LDS wait)
    const int lane = threadIdx.x & 63;
    const int2 stl = lane < ns ? steps[lane] : make_int2(0, 0);
    auto sx = [&](int c) { return __builtin_amdgcn_readlane(stl.x, c); };
    auto sy = [&](int c) { return __builtin_amdgcn_readlane(stl.y, c); };
    auto xload = [&](int c, int i, double (&xf)[5], double (&xt)[5]) {
        const int idx = sx(c);
        const double* X = idx < lv.nreal ? lv.Xr + (int64_t)idx * E : lv.Xg + (int64_t)(idx - lv.nreal) * E;
        brick_slice_load<D>(X, wave + 4 * i, so, xf, xt);
    };
    double nf[5], nt[5];
    if (PF) xload(0, 0, nf, nt);      // the job's first item
    int buf = 0;
    for (int m = tp.m1; m <= tp.m2; ++m) {
        if (m > tp.m1) wlds_barrier();      // the previous term's readers are done
        brick_stage<K>(lv, tp, m, Ss);
        wlds_barrier();
        for (int p0 = 0; p0 < ns;) {
            const int q1 = sy(p0) >> 4;
            int p1 = p0 + 1;
            while (p1 < ns && (sy(p1) >> 4) == q1) ++p1;
            const double* S1 = Ss + q1 * BLK;
            for (int i = 0; i < 5; ++i) {
                double* xo = XB + (buf * 4 + wave) * BLK;
                if (i < nsl) {
                    d4 T2f = (d4){0.0, 0.0, 0.0, 0.0};
                    double T2r = 0.0, T2c = 0.0, T2x = 0.0;
                    for (int r0 = p0; r0 < p1;) {
                        const int q12 = sy(r0) >> 2;
                        int r1 = r0 + 1;
                        while (r1 < p1 && (sy(r1) >> 2) == q12) ++r1;
                        d4 T1f = (d4){0.0, 0.0, 0.0, 0.0};
                        double T1r = 0.0, T1c = 0.0, T1x = 0.0;
                        for (int c = r0; c < r1; ++c) {
                            double xf[5], xt[5];
                            if (PF) {
#pragma unroll
                                for (int s = 0; s < 5; ++s) {
                                    xf[s] = nf[s];
                                    xt[s] = nt[s];
                                }
                                // the next item: the next cell of the plane, else the plane's first
                                // cell for the next round, else the next plane, else the first item
                                // again (the next term's, or an unused load after the last)
                                int cn = c + 1, in = i;
                                if (cn == p1) {
                                    if (i + 1 < nsl) {
                                        cn = p0;
                                        in = i + 1;
                                    } else {
                                        cn = p1 < ns ? p1 : 0;
                                        in = 0;
                                    }
                                }
                                xload(cn, in, nf, nt);
                            } else {
                                xload(c, i, xf, xt);
                            }
                            // mode 3: T1 += X x_3 S3 (B operands S3[u3][v3])
                            const double* S3 = Ss + (2 * NMAX + (sy(c) & 3)) * BLK;
#pragma unroll
                            for (int s = 0; s < 5; ++s) {
                                const int v3 = s < 4 ? 4 * g + s : 16 + g;
                                const double bs = S3[v3 * DP + r];
                                const double bt = S3[v3 * DP + rt];
                                T1f = mfma16(xf[s], bs, T1f);
                                T1r = mfma4(xt[s], bs, T1r);
                                T1c = mfma4(xf[s], bt, T1c);
                                T1x = mfma4(xt[s], bt, T1x);
                            }
                        }
                        // mode 2 at the end of the row: T2 += S2 x_2 T1 (A operands S2[u2][v2])
                        const double* S2 = Ss + (NMAX + (q12 & 3)) * BLK;
#pragma unroll
                        for (int s = 0; s < 5; ++s) {
                            const int v2 = 4 * s + g;
                            // rows 4s..4s+3 of T1, columns 16..19, sit in block s of the column tail
                            const double b1 = s < 4 ? T1f[s] : T1r;
                            const double bc = s < 4 ? __shfl(T1c, 16 * g + 4 * s + (r & 3)) : T1x;
                            const double as = S2[v2 * DP + r];
                            const double ar = S2[v2 * DP + rt];
                            T2f = mfma16(as, b1, T2f);
                            T2r = mfma4(ar, b1, T2r);
                            T2c = mfma4(as, bc, T2c);
                            T2x = mfma4(ar, bc, T2x);
                        }
                        r0 = r1;
                    }
                    // the slice's mode-2 result to its slot, [u2][u3]
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4) xo[(4 * c4 + g) * DP + r] = T2f[c4];
                    xo[(16 + g) * DP + r] = T2r;
                    xo[(4 * (r >> 2) + g) * DP + rt] = T2c;
                    xo[(16 + g) * DP + rt] = T2x;      // the same value from every block
                } else {
                    for (int e = lane; e < BLK; e += 64) xo[e] = 0.0;
                }
                wlds_barrier();
                // mode 1, K step i: Y += c w_m S1 x_1 T2 over the round's slices v1 = 4i + slot
                const double* xs = XB + buf * 4 * BLK + g * BLK;
                const double af = S1[(4 * i + g) * DP + r];
                const double ar = S1[(4 * i + g) * DP + rt];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const int u2 = wave + 4 * q;
                    if (u2 >= D) continue;
                    const double bf = xs[u2 * DP + r];
                    const double bt = xs[u2 * DP + rt];
                    if (!split) {
                        Yf[q] = mfma16(af, bf, Yf[q]);
                        Yr[q] = mfma4(ar, bf, Yr[q]);
                        Yc[q] = mfma4(af, bt, Yc[q]);
                        Yx[q] = mfma4(ar, bt, Yx[q]);
                        continue;
                    }
                    // child of output (u1, u2, u3) = (u1 >= K) + 2 (u2 >= K) + 4 (u3 >= K); u3 = rt >= K
                    const int c2 = 2 * (u2 >= K);
                    const int cf = c2 + 4 * (r >= K);
                    const double a0 = r < K ? af : 0.0;
                    const double a1 = r < K ? 0.0 : af;
                    Yf[q] = mfma16(a0, (cmb >> cf) & 1 ? bf : 0.0, Yf[q]);
                    Yc[q] = mfma4(a0, (cmb >> (c2 + 4)) & 1 ? bt : 0.0, Yc[q]);
                    const double bf1 = (cmb >> (1 + cf)) & 1 ? bf : 0.0;
                    const double bt1 = (cmb >> (1 + c2 + 4)) & 1 ? bt : 0.0;
                    Yf[q] = mfma16(a1, bf1, Yf[q]);
                    Yc[q] = mfma4(a1, bt1, Yc[q]);
                    Yr[q] = mfma4(ar, bf1, Yr[q]);
                    Yx[q] = mfma4(ar, bt1, Yx[q]);
                }
                buf ^= 1;
            }
            p0 = p1;
        }
    }
}

// Every FP64 job of one output brick, then the brick written (zero for children the level does
// not hold, i.e. the siblings of the root).
template <int K, int PF>
__device__ __forceinline__ void brick_contract(const LevelDesc* __restrict__ levels, int2 job, double* smem, int2* steps,
                                               int* nsteps) {
    using B = BrickShape<K>;
    constexpr int D = B::D;
    constexpr int64_t E = (int64_t)D * D * D;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const LevelDesc lv = levels[job.x];
    const int64_t b = job.y;
    const int Lr = lv.Lr;
    const int NL = 2 * Lr + 1;
    const int32_t* nb = lv.nbr + b * NL * NL * NL;
    const int cmb = lv.cmask[b];
    d4 Yf[5];
    double Yr[5], Yc[5], Yx[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        Yf[i] = (d4){0.0, 0.0, 0.0, 0.0};
        Yr[i] = Yc[i] = Yx[i] = 0.0;
    }
    for (int ti = 0; ti < lv.ntpl; ++ti) {
        const Tpl tp = lv.tpl[ti];
        if (tp.prec != PREC_F64) continue;      // another class's launch runs this job
        if (tp.dpart && cmb == 0) continue;     // no internal child receives the down band
        const int ns = wide_steps(tp, nb, Lr, steps, nsteps);
        if (ns == 0) continue;
        brick_job<K, PF>(lv, tp, ns, steps, smem, wave, g, r, cmb, Yf, Yr, Yc, Yx);
    }
    double* ob = lv.out + b * E;
    const int rt = 16 + (r & 3);
    auto put = [&](int u1, int u2, int u3, double v) {
        const int child = (u1 >= K) + 2 * (u2 >= K) + 4 * (u3 >= K);
        ob[((int64_t)u1 * D + u2) * D + u3] = ((lv.valid >> child) & 1) ? v : 0.0;
    };
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int u2 = wave + 4 * i;
        if (u2 >= D) continue;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) put(4 * c4 + g, u2, r, Yf[i][c4]);
        if (16 + g < D) put(16 + g, u2, r, Yr[i]);
        if (rt < D) put(4 * (r >> 2) + g, u2, rt, Yc[i]);
        if (16 + g < D && rt < D && (r >> 2) == 0) put(16 + g, u2, rt, Yx[i]);
    }
}

// order[] entries are (level descriptor, brick).  queues: as the one-tile kernel.
template <int K, int PF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
ns_apply_wide_kernel(const LevelDesc* __restrict__ levels, const int2* __restrict__ order, int* __restrict__ queues) {
    __shared__ double smem[BrickShape<K>::SMEM];
    __shared__ int2 steps[NMAX * NMAX * NMAX];
    __shared__ int nsteps_s, pos_s;
    if (!queues) {
        brick_contract<K, PF>(levels, order[blockIdx.x], smem, steps, &nsteps_s);
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
        brick_contract<K, PF>(levels, order[pos], smem, steps, &nsteps_s);
    }
}

// FP32 copy of nb bricks of D^3 doubles, in the same [brick][v1][v2][v3] order.
__global__ void convert_wide_kernel(int64_t n, const double* __restrict__ X, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)X[i];
}

// Variants of the FP64 kernel: 0 loads the next item's input slice while computing the current one
// (default), 1 loads each slice when it is needed.
constexpr int WIDE_VARIANTS = 2;
constexpr int wide_prefetch(int variant) { return variant == 1 ? 0 : 1; }

template <int K>
void launch_wide_k(int variant, int prec, hipStream_t st, int64_t nblocks, const LevelDesc* levels, const int2* order,
                   int* queues) {
    if (prec == PREC_F32) ns_apply_wide_f32_kernel<K><<<(unsigned)nblocks, WCT, 0, st>>>(levels, order, queues);
    else if (wide_prefetch(variant)) ns_apply_wide_kernel<K, 1><<<(unsigned)nblocks, 256, 0, st>>>(levels, order, queues);
    else ns_apply_wide_kernel<K, 0><<<(unsigned)nblocks, 256, 0, st>>>(levels, order, queues);
}

template <int K>
int64_t resident_wide_k(int variant, int prec, int device) {
    int per_cu = 0, ncu = 0;
    if (prec == PREC_F32)
        MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ns_apply_wide_f32_kernel<K>, WCT, 0));
    else if (wide_prefetch(variant))
        MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ns_apply_wide_kernel<K, 1>, 256, 0));
    else
        MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ns_apply_wide_kernel<K, 0>, 256, 0));
    MWNS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    return (int64_t)std::max(1, per_cu) * ncu;
}

void check_wide(int k, int prec) {
    if (k != 9 && k != 10) fail(MWNS_EINVAL, "the two-tile contraction kernels take 8 < k <= 10");
    if (prec != PREC_F64 && prec != PREC_F32) fail(MWNS_EINVAL, "the two-tile contraction kernels have the FP64 and FP32 classes");
}

}  // namespace

int num_wide_variants() { return WIDE_VARIANTS; }

void launch_contract_wide(int k, int variant, int prec, hipStream_t st, int64_t nblocks, const LevelDesc* levels,
                          const int2* order, int* queues) {
    check_wide(k, prec);
    if (nblocks <= 0) return;
    if (k == 9) launch_wide_k<9>(variant, prec, st, nblocks, levels, order, queues);
    else launch_wide_k<10>(variant, prec, st, nblocks, levels, order, queues);
}

int64_t resident_blocks_wide(int k, int variant, int prec, int device) {
    check_wide(k, prec);
    return k == 9 ? resident_wide_k<9>(variant, prec, device) : resident_wide_k<10>(variant, prec, device);
}

void launch_convert_wide(int k, hipStream_t st, int64_t nb, const double* X, float* out) {
    check_wide(k, PREC_F64);
    const int64_t n = nb * 8 * (int64_t)k * k * k;
    if (n <= 0) return;
    convert_wide_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, X, out);
}

}  // namespace mwns
