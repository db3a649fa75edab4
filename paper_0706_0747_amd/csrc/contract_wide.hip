// The contraction kernel of the apply for 8 < k <= 10 (2k = 18, 20): the FP64 class and the FP32
// class of the precision routing.
//
// Same method as contract.hip: sibling-group bricks, 2k x 2k super-blocks S^{j;m,L} per dimension,
// the nested-loop factorisation of Sec. 5 over boxes of coarse displacements, and the coefficient
// rule c_m = [m in R_j(L)] - [b internal][m in R_{j+1}(l)] of eq. apply_algo (whole band with +,
// down band with - at internal children).  Every dimension of the brick is split 16 + 4: the first
// 16 indices go through a 16x16x4 matrix-core product, the last (up to) four through the FP64
// 4x4x4 product with four blocks, its blocks spanning the 16 columns (or rows) of the other tile so
// that a 4-row tail costs a quarter of a 16-row tile and lands in the lane layout of a 16x16x4
// result.
//   v_mfma_f64_16x16x4: A[m][k] in lane m+16k, B[k][n] in lane n+16k, D[4i+g][n] in lane 16g+n,
//     register i;
//   v_mfma_f32_16x16x4: A and B as above, D[4g+i][n] in lane 16g+n, register i;
//   v_mfma_f64_4x4x4 (four blocks): A[i][k] of block b in lane i+4b+16k, B[k][j] in lane
//     j+4b+16k, D[i][j] in lane j+4b+16i.
// The FP32 class runs the 16 x 16 tiles in FP32 (inputs rounded to FP32 as they enter a product,
// the sums of modes 3 and 2 in FP32, each K step of mode 1 added to FP64 output accumulators) and
// the 4-row tails in FP64; it adds to the output bricks that the FP64 launch wrote.
#include <algorithm>

#include "contract.h"

namespace mwns {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

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

// ---------------------------------------------------------------- whole-brick kernel
// One workgroup per output brick: TG groups of four waves, each group on its own terms (TG = 1:
// two workgroups per CU; TG = 2: one, the groups on alternate terms of a job), so that a SIMD holds
// two waves and one hides the other's loads and barriers.  A plane of cells (fixed L1) runs in five
// rounds; in round i wave w of a group takes input slice v1 = w + 4i: every row (fixed L2) of the
// plane runs mode 3 over its cells and then mode 2, and the slice's mode-2 result goes to LDS.
// After a barrier, each wave adds the round's four slices to its output rows u2 = w + 4q (q < 5)
// by one K step of mode 1.  The input slice of the next item (slice, cell) is loaded while the
// current one is computed.
// LDS holds, per group, the term's super-blocks S_d^{L} for the job's box, staged with the
// coefficient c w_m folded into mode 1, the fine-displacement mask applied, and zeros up to the
// padded extent DP = 20 (so k = 9 needs no bounds tests in the loops), plus two buffers of four
// exchanged slices.
// Tiles: 16 x 16 x 4 for rows and columns < 16, and the 4 x 4 x 4 four-block form for the rest:
//   row tail (rows 16..19, columns < 16): blocks = column groups; A replicated over the blocks;
//   column tail (rows < 16, columns 16..19): blocks = row groups; B replicated;
//   corner (rows and columns 16..19): both replicated (every block computes the same result).
// Lane (g, r) = (lane >> 4, lane & 15).  The K index of step s is 4g + s (s < 4) or 16 + g
// (s = 4) in mode 3, where the slice is loaded as four consecutive doubles per lane; in mode 2 it
// is the row of the mode-3 result register s (Tile::row(s, g), 16 + g for s = 4), and in mode 1
// the slot of the exchanged slice.
template <int K>
struct BrickShape {
    static constexpr int D = 2 * K;              // 18 or 20
    static constexpr int DP = 20;                // padded extent of staged blocks and exchanged slices
    static constexpr int BLK = DP * DP;
    static constexpr int SM_S = 3 * NMAX * BLK;  // staged super-blocks [d][L - lo_d][v][u]
    static constexpr int SM_X = 2 * 4 * BLK;     // exchange buffers [2][slot][u2][u3]
    static constexpr int SMEM = SM_S + SM_X;     // per term group
    static constexpr int SMEM1 = SM_S + SM_X / 2;   // one exchange buffer: three workgroups per CU
    template <int NXB>
    static constexpr int smem() { return NXB == 2 ? SMEM : SMEM1; }
    static_assert(D > 16 && D <= DP, "rows and columns 16..D-1 are the 4-row tails");
    static_assert(SMEM * 8 + 1024 <= 80 * 1024, "one term group: two workgroups per CU");
    static_assert(2 * SMEM * 8 + 1024 <= 160 * 1024, "two term groups: one workgroup per CU");
    static_assert(4 * 35 * 64 <= 2 * SMEM, "the second group's accumulators fit the LDS of both");
    static_assert(3 * (SMEM1 * 8 + 1024) <= 160 * 1024, "one exchange buffer: three workgroups per CU");
};

__device__ inline double mfma4(double a, double b, double c) { return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0); }

// The 16 x 16 tiles of a precision class: operand type, accumulator, product, and the row of a
// result register (register i of lane group g).
template <int PREC>
struct Tile;
template <>
struct Tile<PREC_F64> {
    using T = double;
    using V = d4;
    static __device__ inline V mma(T a, T b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int i, int g) { return 4 * i + g; }
};
template <>
struct Tile<PREC_F32> {
    using T = float;
    using V = f4;
    static __device__ inline V mma(T a, T b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int i, int g) { return 4 * g + i; }
};

// Stages term m of job tp: for each mode d and L in [lo_d, hi_d], S_d^{L}[v][u] (u output, v input,
// u = su*K + a, v = sv*K + b) = F^{2L+su-sv}_{ab} when that fine displacement lies in the job's mask,
// else 0, and 0 for u or v >= 2K; block (d, L - lo_d) of Ss.  Mode 1 carries c w_m.  tid: the
// thread's index in its group of 256.
template <int K>
__device__ inline void brick_stage(const LevelDesc& lv, const Tpl& tp, int m, double* __restrict__ Ss, int tid) {
    using B = BrickShape<K>;
    constexpr int Q = (NMAX * B::BLK + 255) / 256;     // elements per thread and mode, at most
    const double* Fm = lv.Fj + (int64_t)m * NLF * K * K;
    const double cw = tp.dpart ? -lv.w[m] : lv.w[m];
    // every load of the three modes is issued before the first store (one memory latency per term)
    double val[3][Q];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int lo = __builtin_amdgcn_readfirstlane(tp.lo[d]), hi = __builtin_amdgcn_readfirstlane(tp.hi[d]);
        const int mlo = __builtin_amdgcn_readfirstlane(tp.mlo[d]), mhi = __builtin_amdgcn_readfirstlane(tp.mhi[d]);
        const int tot = (hi - lo + 1) * B::BLK;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q;
            const int blk = e / B::BLK;
            const int rem = e - blk * B::BLK;
            const int v = rem / B::DP, u = rem - v * B::DP;
            const int su = u >= K, sv = v >= K;
            const int l = 2 * (lo + blk) + su - sv;
            val[d][q] = (e < tot && u < 2 * K && v < 2 * K && l >= mlo && l <= mhi)
                            ? Fm[(l + LF) * K * K + (u - su * K) * K + (v - sv * K)] : 0.0;
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int tot = (__builtin_amdgcn_readfirstlane(tp.hi[d]) - __builtin_amdgcn_readfirstlane(tp.lo[d]) + 1) * B::BLK;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q;
            if (e < tot) Ss[d * NMAX * B::BLK + e] = d == 0 ? cw * val[d][q] : val[d][q];
        }
    }
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

// One job of precision class PREC for one output brick (see above); Y accumulates over the jobs,
// its 16 x 16 part Yf in the row order of the class's result registers.  PF = 1 loads the input
// slice of the next item while the current one is computed, PF = 0 each slice when it is needed.
// Down-band jobs whose brick has leaf children run mode 1 in two passes, one per half u1 < K,
// u1 >= K, each with the output columns of leaf children masked out of the exchanged slices.
template <int K, int PF, int TG, int PREC, int NXB>
__device__ __forceinline__ void brick_job(const LevelDesc& lv, const Tpl& tp, int ns, const int2* __restrict__ steps,
                                          double* __restrict__ smem, int h, int wave, int g, int r, int cmb,
                                          d4 (&Yf)[5], double (&Yr)[5], double (&Yc)[5], double (&Yx)[5]) {
    using B = BrickShape<K>;
    using Tl = Tile<PREC>;
    using T = typename Tl::T;
    using V = typename Tl::V;
    constexpr bool F32 = PREC == PREC_F32;
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
    // term group h takes the terms m1 + h, m1 + h + TG, ...; the groups pass the same barriers
    for (int mb = tp.m1; mb <= tp.m2; mb += TG) {
        const int m = mb + h;
        if (mb > tp.m1) wlds_barrier();      // the previous term's readers are done
        if (m <= tp.m2) brick_stage<K>(lv, tp, m, Ss, threadIdx.x & 255);
        wlds_barrier();
        if (m > tp.m2) {      // the last term of an odd count: this group only keeps the barriers
            for (int p0 = 0; p0 < ns;) {
                const int q1 = sy(p0) >> 4;
                while (++p0 < ns && (sy(p0) >> 4) == q1) {
                }
                for (int i = 0; i < 5; ++i) wlds_barrier();
            }
            break;
        }
        for (int p0 = 0; p0 < ns;) {
            const int q1 = sy(p0) >> 4;
            int p1 = p0 + 1;
            while (p1 < ns && (sy(p1) >> 4) == q1) ++p1;
            const double* S1 = Ss + q1 * BLK;
            for (int i = 0; i < 5; ++i) {
                double* xo = XB + (buf * 4 + wave) * BLK;
                if (i < nsl) {
                    V T2f = (V){0, 0, 0, 0};
                    double T2r = 0.0, T2c = 0.0, T2x = 0.0;
                    for (int r0 = p0; r0 < p1;) {
                        const int q12 = sy(r0) >> 2;
                        int r1 = r0 + 1;
                        while (r1 < p1 && (sy(r1) >> 2) == q12) ++r1;
                        V T1f = (V){0, 0, 0, 0};
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
                                T1f = Tl::mma((T)xf[s], (T)bs, T1f);
                                T1r = mfma4(xt[s], bs, T1r);
                                T1c = mfma4(xf[s], bt, T1c);
                                T1x = mfma4(xt[s], bt, T1x);
                            }
                        }
                        // mode 2 at the end of the row: T2 += S2 x_2 T1 (A operands S2[u2][v2]); the
                        // K index of step s < 4 is the row of the mode-3 result register s
                        const double* S2 = Ss + (NMAX + (q12 & 3)) * BLK;
#pragma unroll
                        for (int s = 0; s < 5; ++s) {
                            const int v2 = s < 4 ? Tl::row(s, g) : 16 + g;
                            const double b1 = s < 4 ? (double)T1f[s] : T1r;
                            // T1[v2][16 + (r & 3)] from the column tail, which holds
                            // T1[4 (r' >> 2) + g'][16 + (r' & 3)] in lane (g', r')
                            const int src = F32 ? 16 * s + 4 * g + (r & 3) : 16 * g + 4 * s + (r & 3);
                            const double bc = s < 4 ? __shfl(T1c, src) : T1x;
                            const double as = S2[v2 * DP + r];
                            const double ar = S2[v2 * DP + rt];
                            T2f = Tl::mma((T)as, (T)b1, T2f);
                            T2r = mfma4(ar, b1, T2r);
                            T2c = mfma4(as, bc, T2c);
                            T2x = mfma4(ar, bc, T2x);
                        }
                        r0 = r1;
                    }
                    // the slice's mode-2 result to its slot, [u2][u3]
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4) xo[Tl::row(c4, g) * DP + r] = (double)T2f[c4];
                    xo[(16 + g) * DP + r] = T2r;
                    xo[(4 * (r >> 2) + g) * DP + rt] = T2c;
                    xo[(16 + g) * DP + rt] = T2x;      // the same value from every block
                } else {
                    for (int e = lane; e < BLK; e += 64) xo[e] = 0.0;
                }
                wlds_barrier();
                // mode 1, K step i: Y += c w_m S1 x_1 T2 over the round's slices v1 = 4i + slot (FP32:
                // the 16 x 16 part of each step's product added to the FP64 accumulators)
                auto addf = [&](d4& y, V t) {
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4) y[c4] += (double)t[c4];
                };
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
                        if constexpr (F32) addf(Yf[q], Tl::mma((T)af, (T)bf, (V){0, 0, 0, 0}));
                        else Yf[q] = Tl::mma(af, bf, Yf[q]);
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
                    const double bf0 = (cmb >> cf) & 1 ? bf : 0.0;
                    const double bf1 = (cmb >> (1 + cf)) & 1 ? bf : 0.0;
                    const double bt1 = (cmb >> (1 + c2 + 4)) & 1 ? bt : 0.0;
                    if constexpr (F32) {
                        addf(Yf[q], Tl::mma((T)a1, (T)bf1, Tl::mma((T)a0, (T)bf0, (V){0, 0, 0, 0})));
                    } else {
                        Yf[q] = Tl::mma(a0, bf0, Yf[q]);
                        Yf[q] = Tl::mma(a1, bf1, Yf[q]);
                    }
                    Yc[q] = mfma4(a0, (cmb >> (c2 + 4)) & 1 ? bt : 0.0, Yc[q]);
                    Yc[q] = mfma4(a1, bt1, Yc[q]);
                    Yr[q] = mfma4(ar, bf1, Yr[q]);
                    Yx[q] = mfma4(ar, bt1, Yx[q]);
                }
                // two exchange buffers alternate; with one, the next round writes it only after every
                // wave's mode 1 has read it
                if (NXB == 2) buf ^= 1;
                else wlds_barrier();
            }
            p0 = p1;
        }
    }
}

// Every job of class PREC of one output brick, then the brick written (FP64: zero for children
// the level does not hold, i.e. the siblings of the root) or added to (FP32).
template <int K, int PF, int TG, int PREC, int NXB>
__device__ __forceinline__ void brick_contract(const LevelDesc* __restrict__ levels, int2 job, double* smem, int2* steps,
                                               int* nsteps) {
    using B = BrickShape<K>;
    using Tl = Tile<PREC>;
    constexpr int D = B::D;
    constexpr int64_t E = (int64_t)D * D * D;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = TG > 1 ? wid >> 2 : 0, wave = wid & 3;      // term group, wave within the group
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
        if (tp.prec != PREC) continue;          // another class's launch runs this job
        if (tp.dpart && cmb == 0) continue;     // no internal child receives the down band
        const int ns = wide_steps(tp, nb, Lr, steps, nsteps);
        if (ns == 0) continue;
        brick_job<K, PF, TG, PREC, NXB>(lv, tp, ns, steps, smem + h * B::template smem<NXB>(), h, wave, g, r, cmb, Yf, Yr,
                                        Yc, Yx);
    }
    if (TG > 1) {      // the second group's accumulators added to the first's, through LDS
        wlds_barrier();
        double* ys = smem + wave * 35 * 64 + lane;
        if (h == 1) {
#pragma unroll
            for (int i = 0; i < 5; ++i) {
#pragma unroll
                for (int c4 = 0; c4 < 4; ++c4) ys[(7 * i + c4) * 64] = Yf[i][c4];
                ys[(7 * i + 4) * 64] = Yr[i];
                ys[(7 * i + 5) * 64] = Yc[i];
                ys[(7 * i + 6) * 64] = Yx[i];
            }
        }
        wlds_barrier();
        if (h == 1) return;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) Yf[i][c4] += ys[(7 * i + c4) * 64];
            Yr[i] += ys[(7 * i + 4) * 64];
            Yc[i] += ys[(7 * i + 5) * 64];
            Yx[i] += ys[(7 * i + 6) * 64];
        }
    }
    double* ob = lv.out + b * E;
    const int rt = 16 + (r & 3);
    auto put = [&](int u1, int u2, int u3, double v) {
        const int child = (u1 >= K) + 2 * (u2 >= K) + 4 * (u3 >= K);
        double& o = ob[((int64_t)u1 * D + u2) * D + u3];
        if (PREC == PREC_F64) o = ((lv.valid >> child) & 1) ? v : 0.0;
        else if ((lv.valid >> child) & 1) o += v;
    };
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int u2 = wave + 4 * i;
        if (u2 >= D) continue;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) put(Tl::row(c4, g), u2, r, Yf[i][c4]);
        if (16 + g < D) put(16 + g, u2, r, Yr[i]);
        if (rt < D) put(4 * (r >> 2) + g, u2, rt, Yc[i]);
        if (16 + g < D && rt < D && (r >> 2) == 0) put(16 + g, u2, rt, Yx[i]);
    }
}

// order[] entries are (level descriptor, brick).  queues: as the one-tile kernel.  TG term groups
// of four waves: 256 TG threads, one workgroup per CU for TG = 2, two for TG = 1.
// NXB exchange buffers: 2, two waves per SIMD; 1 (one term group only), three.
template <int K, int PF, int TG, int PREC, int NXB>
__global__ void __launch_bounds__(256 * TG) __attribute__((amdgpu_waves_per_eu(NXB == 1 ? 3 : 2, NXB == 1 ? 3 : 2)))
ns_apply_wide_kernel(const LevelDesc* __restrict__ levels, const int2* __restrict__ order, int* __restrict__ queues) {
    static_assert(NXB == 2 || TG == 1, "one exchange buffer takes one term group");
    __shared__ double smem[TG * BrickShape<K>::template smem<NXB>()];
    __shared__ int2 steps[NMAX * NMAX * NMAX];
    __shared__ int nsteps_s, pos_s;
    if (!queues) {
        brick_contract<K, PF, TG, PREC, NXB>(levels, order[blockIdx.x], smem, steps, &nsteps_s);
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
        brick_contract<K, PF, TG, PREC, NXB>(levels, order[pos], smem, steps, &nsteps_s);
    }
}

// Variants: 0 (default) one term group of four waves, two workgroups per CU; 1 two term groups,
// one workgroup per CU; both load the next item's input slice while computing the current one.
// 2 as 0, loading each slice when it is needed.  3 as 2 with one exchange buffer (an extra barrier
// per round), which lets three workgroups share a CU (three waves per SIMD).
constexpr int WIDE_VARIANTS = 4;

template <int K, int PREC>
struct WideLaunch {
    static void run(int variant, hipStream_t st, int64_t nblocks, const LevelDesc* levels, const int2* order, int* queues) {
        if (variant == 1) ns_apply_wide_kernel<K, 1, 2, PREC, 2><<<(unsigned)nblocks, 512, 0, st>>>(levels, order, queues);
        else if (variant == 2) ns_apply_wide_kernel<K, 0, 1, PREC, 2><<<(unsigned)nblocks, 256, 0, st>>>(levels, order, queues);
        else if (variant == 3) ns_apply_wide_kernel<K, 0, 1, PREC, 1><<<(unsigned)nblocks, 256, 0, st>>>(levels, order, queues);
        else ns_apply_wide_kernel<K, 1, 1, PREC, 2><<<(unsigned)nblocks, 256, 0, st>>>(levels, order, queues);
    }
    static int per_cu(int variant) {
        int n = 0;
        if (variant == 1)
            MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ns_apply_wide_kernel<K, 1, 2, PREC, 2>, 512, 0));
        else if (variant == 2)
            MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ns_apply_wide_kernel<K, 0, 1, PREC, 2>, 256, 0));
        else if (variant == 3)
            MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ns_apply_wide_kernel<K, 0, 1, PREC, 1>, 256, 0));
        else
            MWNS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ns_apply_wide_kernel<K, 1, 1, PREC, 2>, 256, 0));
        return n;
    }
};

void check_wide(int k, int variant, int prec) {
    if (k != 9 && k != 10) fail(MWNS_EINVAL, "the whole-brick contraction kernel takes 8 < k <= 10");
    if (prec != PREC_F64 && prec != PREC_F32) fail(MWNS_EINVAL, "the whole-brick contraction kernel has the FP64 and FP32 classes");
    if (variant < 0 || variant >= WIDE_VARIANTS) fail(MWNS_EINVAL, "variant out of range");
}

}  // namespace

int num_wide_variants() { return WIDE_VARIANTS; }

void launch_contract_wide(int k, int variant, int prec, hipStream_t st, int64_t nblocks, const LevelDesc* levels,
                          const int2* order, int* queues) {
    check_wide(k, variant, prec);
    if (nblocks <= 0) return;
    if (k == 9) {
        if (prec == PREC_F64) WideLaunch<9, PREC_F64>::run(variant, st, nblocks, levels, order, queues);
        else WideLaunch<9, PREC_F32>::run(variant, st, nblocks, levels, order, queues);
    } else {
        if (prec == PREC_F64) WideLaunch<10, PREC_F64>::run(variant, st, nblocks, levels, order, queues);
        else WideLaunch<10, PREC_F32>::run(variant, st, nblocks, levels, order, queues);
    }
}

int64_t resident_blocks_wide(int k, int variant, int prec, int device) {
    check_wide(k, variant, prec);
    int per_cu = 0, ncu = 0;
    if (k == 9) per_cu = prec == PREC_F64 ? WideLaunch<9, PREC_F64>::per_cu(variant) : WideLaunch<9, PREC_F32>::per_cu(variant);
    else per_cu = prec == PREC_F64 ? WideLaunch<10, PREC_F64>::per_cu(variant) : WideLaunch<10, PREC_F32>::per_cu(variant);
    MWNS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    return (int64_t)std::max(1, per_cu) * ncu;
}

}  // namespace mwns
