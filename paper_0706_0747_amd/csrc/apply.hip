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

#include "contract.h"

namespace mwns {

struct LevelTab2 {
    int64_t node_off[MAXLEV + 2];
    int64_t brick_off[MAXLEV + 2];
    int depth;
};

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int AT = 256;            // threads per block of the transform kernels

// ---------------------------------------------------------------- closure
// The output levels of one apply's closure for one launch: level entry li takes the 256-thread
// blocks [bstart[li], bstart[li + 1]) (a block never spans two levels); its output bricks are
// the nout[li] parents pkeys[li] of level jm1[li] with band radius Lr[li], and it writes
// nbr[li] and miss[li] ([nout][NL^3] each); the fill maps the missing entries to the ng[li]
// sorted ghost keys gkeys[li].
struct ClosTab {
    int n = 0;
    int jm1[MAXLEV + 1], Lr[MAXLEV + 1];
    int64_t nout[MAXLEV + 1], ng[MAXLEV + 1];
    int64_t bstart[MAXLEV + 2];
    const uint64_t* pkeys[MAXLEV + 1];
    const uint64_t* gkeys[MAXLEV + 1];
    int32_t* nbr[MAXLEV + 1];
    uint64_t* miss[MAXLEV + 1];
};

__device__ inline int clos_entry(const ClosTab& ct) {
    int li = 0;
    while (li + 1 < ct.n && (int64_t)blockIdx.x >= ct.bstart[li + 1]) ++li;
    return li;
}

// For every output brick of level j (parent P at level j-1) and L in [-Lr,Lr]^3: index of the
// brick whose parent is P - L among the level's real bricks, -1 outside the cube, -2 when P - L is
// not an internal node (the key is written to miss[] for interpolation).
__global__ void closure_kernel(ClosTab ct) {
    const int li = clos_entry(ct);
    const int64_t nout = ct.nout[li];
    const int jm1 = ct.jm1[li], Lr = ct.Lr[li];
    const uint64_t* __restrict__ pkeys = ct.pkeys[li];
    int32_t* __restrict__ nbr = ct.nbr[li];
    uint64_t* __restrict__ miss = ct.miss[li];
    const int NL = 2 * Lr + 1, NL3 = NL * NL * NL;
    const int64_t idx = ((int64_t)blockIdx.x - ct.bstart[li]) * 256 + threadIdx.x;
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

// p[0..n) = v.
__global__ void fill_u64_kernel(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// The distinct missing keys (entries != ~0) of one apply's closure, appended to out in no
// particular order (a missing parent is reported once per neighbouring output box).  tab is an
// open-addressing set of cap entries (a power of two, at least twice n, all ~0 on entry); the
// first insertion of a key appends it.  No key equals ~0, and the set never fills, so every
// probe sequence ends at the key or at an empty slot.
__global__ void compact_distinct_kernel(int64_t n, const uint64_t* __restrict__ miss, uint64_t* __restrict__ tab,
                                        int64_t cap, uint64_t* __restrict__ out, unsigned int* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = miss[i];
    if (key == ~0ull) return;
    int64_t slot = (int64_t)((key * 0x9E3779B97F4A7C15ull) >> 20) & (cap - 1);
    for (int64_t probe = 0; probe < cap; ++probe) {
        const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long*>(tab + slot), ~0ull, key);
        if (prev == ~0ull) {
            out[atomicAdd(count, 1u)] = key;
            return;
        }
        if (prev == key) return;
        slot = (slot + 1) & (cap - 1);
    }
}

// The missing neighbours (nbr = -2) of every level point past the level's real bricks to its
// ghost bricks, in the order of the level's sorted ghost keys.
__global__ void closure_fill_kernel(ClosTab ct) {
    const int li = clos_entry(ct);
    const int NL = 2 * ct.Lr[li] + 1;
    const int64_t nreal = ct.nout[li];
    const int64_t idx = ((int64_t)blockIdx.x - ct.bstart[li]) * 256 + threadIdx.x;
    if (idx >= nreal * NL * NL * NL) return;
    int32_t* __restrict__ nbr = ct.nbr[li];
    if (nbr[idx] != -2) return;
    nbr[idx] = (int32_t)(nreal + find_sorted(ct.gkeys[li], ct.ng[li], ct.miss[li][idx]));
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

// The ghost bricks of every level of one apply, one block each: block b belongs to entry li with
// start[li] <= b < start[li + 1], parent level jm1[li], key keys[li][b - start[li]] and brick
// out[li] + (b - start[li]) (2k)^3.
struct GhostTab {
    int n = 0;
    int jm1[MAXLEV + 1];
    int64_t start[MAXLEV + 2];
    const uint64_t* keys[MAXLEV + 1];
    double* out[MAXLEV + 1];
};

// Ghost bricks: the children of a node Q of level j-1 that is not internal, interpolated from the
// deepest existing ancestor (a leaf) by repeated zero-detail reconstruction (Alg. 3 Step 2).
template <int K>
__global__ void __launch_bounds__(AT) ghost_kernel(GhostTab gt, const uint64_t* __restrict__ keys, int64_t nnodes,
                                                   LevelTab2 lt, const double* __restrict__ coef,
                                                   const double* __restrict__ Htg) {
    constexpr int P = 2 * K, K3 = K * K * K;
    __shared__ double Ht[2 * K * K];
    __shared__ double blk[K3], tmp1[K * P * P], tmp2[K * P * P];
    for (int e = threadIdx.x; e < 2 * K * K; e += AT) Ht[e] = Htg[e];
    __syncthreads();
    int li = 0;
    while (li + 1 < gt.n && (int64_t)blockIdx.x >= gt.start[li + 1]) ++li;
    const int64_t gi = (int64_t)blockIdx.x - gt.start[li];
    const int jm1 = gt.jm1[li];
    const uint64_t q = gt.keys[li][gi];
    int64_t l[3];
    key_coords(q, l);
    int i = jm1;
    int64_t node = -1;
    for (; i >= 0; --i) {
        node = find_sorted(keys, nnodes, make_key(i, l[0] >> (jm1 - i), l[1] >> (jm1 - i), l[2] >> (jm1 - i)));
        if (node >= 0) break;
    }
    double* go = gt.out[li] + gi * P * P * P;
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

// One level of the count (all levels go in one launch).
struct CountLevel {
    const uint64_t* pkeys;
    const uint8_t* cmask;
    const int32_t* Rj;
    const int32_t* Rj1;      // null when the operator has no row j+1
    int64_t first;           // first work item of the level: items are (brick, child, slab)
    int64_t nout;
    int j, valid;
};

// One thread per (output node, x-slab of the displacements): slab x in [-LP, LP] takes L_1 = x
// of the whole band and e_1 = x of the down band.
__global__ void count_kernel(const CountLevel* __restrict__ lv, int nlev, int64_t nitems,
                             unsigned long long* __restrict__ total) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nitems) return;
    int li = 0;
    while (li + 1 < nlev && lv[li + 1].first <= t) ++li;
    const CountLevel c = lv[li];
    const int64_t r = t - c.first;
    const int64_t b = r / (8 * NLP);
    const int child = (int)((r / NLP) % 8);
    const int x = (int)(r % NLP) - LP;
    if (!((c.valid >> child) & 1)) return;
    const int j = c.j;
    const int internal = (c.cmask[b] >> child) & 1;
    auto at = [](const int32_t* R, int x, int y, int z) {
        return R + (((x + LP) * NLP + (y + LP)) * NLP + (z + LP)) * 2;
    };
    long long cnt = 0;
    if (j == 0) {
        if (x != 0) return;
        const int32_t* w = at(c.Rj, 0, 0, 0);
        cnt = range_len(w);
        if (internal && c.Rj1) {
            const int32_t* d = at(c.Rj1, 0, 0, 0);
            const int ov = (range_len(w) && range_len(d)) ? max(0, min(w[1], d[1]) - max(w[0], d[0]) + 1) : 0;
            cnt += range_len(d) - 2 * ov;
        }
        atomicAdd(total, (unsigned long long)cnt);
        return;
    }
    int64_t p[3];
    key_coords(c.pkeys[b], p);
    const int64_t pside = (int64_t)1 << (j - 1), side = (int64_t)1 << j;
    if (p[0] - x >= 0 && p[0] - x < pside)
        for (int y = -LP; y <= LP; ++y)
            for (int z = -LP; z <= LP; ++z) {
                const int64_t q1 = p[1] - y, q2 = p[2] - z;
                if (q1 < 0 || q1 >= pside || q2 < 0 || q2 >= pside) continue;
                cnt += 8 * range_len(at(c.Rj, x, y, z));
            }
    if (internal && c.Rj1) {
        const int64_t o[3] = {2 * p[0] + (child & 1), 2 * p[1] + ((child >> 1) & 1), 2 * p[2] + (child >> 2)};
        const int e1 = x;
        const int64_t q0 = o[0] - e1;
        if (q0 >= 0 && q0 < side)
            for (int e2 = -LP; e2 <= LP; ++e2)
                for (int e3 = -LP; e3 <= LP; ++e3) {
                    const int64_t q[3] = {q0, o[1] - e2, o[2] - e3};
                    if (q[1] < 0 || q[1] >= side || q[2] < 0 || q[2] >= side) continue;
                    const int L[3] = {(int)((o[0] >> 1) - (q[0] >> 1)), (int)((o[1] >> 1) - (q[1] >> 1)),
                                      (int)((o[2] >> 1) - (q[2] >> 1))};
                    const int32_t* w = at(c.Rj, L[0], L[1], L[2]);   // |L_d| <= 2 here
                    const int32_t* d = at(c.Rj1, e1, e2, e3);
                    const int ov = (range_len(w) && range_len(d)) ? max(0, min(w[1], d[1]) - max(w[0], d[0]) + 1) : 0;
                    cnt += range_len(d) - 2 * ov;
                }
    }
    if (cnt) atomicAdd(total, (unsigned long long)cnt);
}

// Bricks of several levels for one launch of level_sumsq_kernel: entry i covers the blocks
// [start[i], start[i + 1]), bricks X[i] + (b - start[i]) 8k^3, and adds to *acc[i].
struct SumsqTab {
    int n = 0;
    int64_t start[2 * (MAXLEV + 1) + 1];
    const double* X[2 * (MAXLEV + 1)];
    double* acc[2 * (MAXLEV + 1)];
};

// Sum of squares of every brick element, one 256-thread block per brick, reduced in LDS and
// added to its entry's accumulator.
template <int K>
__global__ void __launch_bounds__(256) level_sumsq_kernel(SumsqTab tb) {
    constexpr int E = 8 * K * K * K;
    __shared__ double red[256];
    int i = 0;
    while (i + 1 < tb.n && (int64_t)blockIdx.x >= tb.start[i + 1]) ++i;
    const double* x = tb.X[i] + ((int64_t)blockIdx.x - tb.start[i]) * E;
    double s = 0.0;
    for (int e = threadIdx.x; e < E; e += 256) s += x[e] * x[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(tb.acc[i], red[0]);
}

template <int K>
struct LevelSumsqLaunch {
    static void run(hipStream_t st, int64_t nb, const SumsqTab& tb) {
        level_sumsq_kernel<K><<<(unsigned)nb, 256, 0, st>>>(tb);
    }
};

template <int K>
struct GhostLaunch {
    static void run(hipStream_t st, int64_t ng, const GhostTab& gt, const uint64_t* keys, int64_t nn,
                    const LevelTab2& lt, const double* coef, const double* Ht) {
        ghost_kernel<K><<<(unsigned)ng, AT, 0, st>>>(gt, keys, nn, lt, coef, Ht);
    }
};
template <int K>
struct AssembleLaunch {
    static void run(hipStream_t st, int64_t nb, int j, const int64_t* pb, const int* pc, int64_t off, const double* Ht,
                    double* coef) {
        assemble_kernel<K><<<(unsigned)nb, AT, 0, st>>>(j, pb, pc, off, Ht, coef);
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
// operand errors a (matrix) and b (input) and an FP32 accumulation over at most n = max(16, 2k)
// * NMAX products computes (|S1| (x) |S2| (x) |S3|) |X| up to the factor ((1 + a + b + n u32)^3 - 1).
// (The FP32 class of the whole-brick kernel, orders above KNARROW, runs its 4-row tails in FP64 and
// adds each K step of mode 1 in FP64, which the factor covers.)
constexpr double U32 = 0x1p-24, UBF = 0x1p-8, USPLIT = 0x1p-16;
constexpr double cube_minus_one(double d) { return (1.0 + d) * (1.0 + d) * (1.0 + d) - 1.0; }
struct Gammas {
    double g[NPREC];
};
Gammas class_gammas(int k) {
    const double nacc = std::max(16.0, 2.0 * k) * NMAX * U32;
    return Gammas{{0.0, cube_minus_one(2.0 * U32 + nacc), cube_minus_one(2.0 * (USPLIT + U32) + nacc),
                   cube_minus_one(UBF + USPLIT + 2.0 * U32 + nacc)}};
}
// Relative time per unit of work, for the routing objective only.
constexpr double COST[NPREC] = {1.0, 0.6, 0.3, 0.2};

struct RouteItem {
    int j, t, m, cls;
    double beta, work;
    bool pin;      // kept in FP64 whatever the budget
};

// Chooses a class for every (level, job, term) minimising the modelled time subject to
// sum gamma_class * beta <= tol (Lagrangian relaxation, bisection on the multiplier); beta bounds
// the item's contribution over its whole level, and the rounding error of a class is at most gamma
// times the same sum with every block replaced by its entrywise absolute value.  Two bounds of it:
//   |w_m| prod_d sum_{L_d} ||S_d^{m,L_d}||_F ||X_level||  (each input brick feeds one output brick
//   per displacement), and
//   |w_m| prod_d || sum_{L_d} |S_d^{m,L_d}| ||_2 ||X_level||  (the box is a product set, and a block
//   convolution with nonnegative blocks B_L has norm at most || sum_L B_L ||_2).
// beta is the smaller.  Returns the bound reached.
constexpr double MIN_CLASS_SHARE = 0.1;

double route(std::vector<RouteItem>& items, double tol, int allowed, int k) {
    const Gammas gm = class_gammas(k);
    const double* GAMMA = gm.g;
    auto eval = [&](double lam, bool commit) {
        double err = 0.0;
        for (RouteItem& it : items) {
            int best = PREC_F64;
            double bv = it.work * COST[PREC_F64];
            for (int p = 1; p < NPREC && !it.pin; ++p) {
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
    if (eval(std::pow(10.0, lo), false) <= tol) {
        eval(std::pow(10.0, lo), true);
    } else {
        for (int it = 0; it < 100; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (eval(std::pow(10.0, mid), false) <= tol) hi = mid;
            else lo = mid;
        }
        eval(std::pow(10.0, hi), true);
    }
    // A reduced class with less than MIN_CLASS_SHARE of the work is not used: its launch revisits
    // every output brick and input neighbourhood it touches, which costs more than the little work
    // it takes off FP64.  Moving items to FP64 only lowers the error.
    double total = 0.0, share[NPREC] = {0.0, 0.0, 0.0, 0.0};
    for (const RouteItem& it : items) {
        total += it.work;
        share[it.cls] += it.work;
    }
    double err = 0.0;
    for (RouteItem& it : items) {
        if (it.cls != PREC_F64 && share[it.cls] < MIN_CLASS_SHARE * total) it.cls = PREC_F64;
        err += GAMMA[it.cls] * it.beta;
    }
    return err;
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

namespace {

__global__ void zero_ints_kernel(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// A device pointer into an arena (owned elsewhere).
template <class T>
struct DevView {
    T* p = nullptr;
};

// Small host arrays of one phase gathered into one device block with a single copy (each
// separate hipMemcpyAsync from pageable memory costs tens of microseconds).  Views receive their
// device addresses at commit; the host copy stays alive with the arena.
struct UploadArena {
    std::vector<char> host;
    std::vector<std::pair<size_t, void**>> fix;
    DevArray<char> dev;
    template <class T>
    void add(const T* data, size_t n, DevView<T>& view) {
        const size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + n * sizeof(T));
        if (n) std::memcpy(host.data() + off, data, n * sizeof(T));
        fix.push_back({off, reinterpret_cast<void**>(&view.p)});
    }
    void commit(mwns_ctx* ctx) {
        if (host.empty()) return;
        dev.reset(ctx, host.size());
        dev.upload(host.data(), host.size(), ctx->stream);
        for (auto& f : fix) *f.second = dev.p + f.first;
        fix.clear();
    }
};

struct LevelWork {
    std::vector<Tpl> tpl;
    std::vector<uint8_t> cm;
    std::vector<uint64_t> pk;
    int Lr = 0;
    int64_t nout = 0, nghost = 0, miss_off = 0;
    int valid = 0xff;
    DevArray<int32_t> nbr;
    DevView<uint8_t> cmask;
    DevView<Tpl> dtpl;
    DevView<double> ghosts;         // this level's part of TreeApply::ghost_store
    DevView<uint64_t> pkeys, gkeys;
    DevArray<u4> xr32, xg32, xrb, xgb;     // reduced-precision copies of the inputs (routed applies)
    DevView<int64_t> apb;                  // assembly: parent's brick of every brick of the level
    DevView<int> apc;                      //           parent's child slot in that brick
};

// One (operator, input tree) pair of an apply and everything its device work needs.
struct TreeApply {
    const mwns_op* op = nullptr;
    const mwns_tree* f = nullptr;
    std::unique_ptr<mwns_tree> out;
    int k = 0, depth = 0;
    std::vector<LevelWork> W;
    DevView<double> dHt;
    UploadArena setup_arena, ghost_arena, desc_arena;
    DevArray<double> ghost_store;    // the ghost bricks of all levels, level by level
    LevelTab2 lt{};
    int64_t miss_base = 0, miss_total = 0, total_ghosts = 0, jobs = 0;
    double err_bound = 0.0, flops = 0.0, class_flops[NPREC] = {0.0, 0.0, 0.0, 0.0};
    double own_flops = 0.0, mfma_flops = 0.0;
    size_t desc_base = 0;
};

// Validation, output skeleton, jobs of every level (whole band from plan row j, down band from
// row j+1), child masks, parent keys, neighbour-table storage and assembly maps.
void setup(mwns_ctx* ctx, TreeApply& a, const mwns_op* op, const mwns_tree* f) {
    if (!op || !f) fail(MWNS_EINVAL, "NULL operator or tree");
    if (op->ctx != ctx || f->ctx != ctx) fail(MWNS_EINVAL, "operator or tree belongs to another context");
    if (op->k != f->k) fail(MWNS_EINVAL, "operator and tree have different k");
    if (op->max_level < f->depth) fail(MWNS_EINVAL, "operator max_level is below the tree depth");
    a.op = op;
    a.f = f;
    const int k = a.k = f->k;
    const int64_t E = brick_elems(k);
    hipStream_t st = ctx->stream;
    a.out.reset(new mwns_tree);
    mwns_tree* out = a.out.get();
    out->ctx = ctx;
    out->hold.set(ctx);
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
    a.lt = level_tab2(f);
    {
        std::vector<double> H(2 * k * k), Ht(2 * k * k);
        two_scale_filters(k, H.data(), H.data() + k * k);
        for (int s = 0; s < 2; ++s)
            for (int x = 0; x < k; ++x)
                for (int c = 0; c < k; ++c) Ht[s * k * k + c * k + x] = H[s * k * k + x * k + c];
        a.setup_arena.add(Ht.data(), Ht.size(), a.dHt);
    }
    const int depth = a.depth = f->depth;
    const int64_t planrow = (int64_t)NLP3 * 2;
    a.W.clear();
    a.W.resize(depth + 1);
    a.miss_total = 0;
    for (int j = 0; j <= depth; ++j) {
        LevelWork& lw = a.W[j];
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
                for (int x = t.lo[d]; x <= t.hi[d]; x += NMAX) {
                    cuts[d][nc[d]][0] = x;
                    cuts[d][nc[d]][1] = std::min(t.hi[d], x + NMAX - 1);
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
        a.setup_arena.add(lw.cm.data(), lw.nout, lw.cmask);
        lw.nbr.reset(ctx, (size_t)lw.nout * NL3);
        if (j > 0) {
            lw.pk.resize(lw.nout);
            for (int64_t b = 0; b < lw.nout; ++b) lw.pk[b] = f->keys[f->brick_parent[L.brick_off + b]];
            a.setup_arena.add(lw.pk.data(), lw.nout, lw.pkeys);
            std::vector<int64_t> pb(lw.nout);
            std::vector<int> pc(lw.nout);
            for (int64_t b = 0; b < lw.nout; ++b) node_brick(f, f->brick_parent[L.brick_off + b], &pb[b], &pc[b]);
            a.setup_arena.add(pb.data(), pb.size(), lw.apb);
            a.setup_arena.add(pc.data(), pc.size(), lw.apc);
        }
        if (lw.tpl.empty()) continue;
        if (j == 0) {
            std::vector<int32_t> nb(NL3, -1);
            nb[(Lr * NL + Lr) * NL + Lr] = 0;
            lw.nbr.upload(nb.data(), NL3, st);
            continue;
        }
        lw.miss_off = a.miss_total;
        a.miss_total += lw.nout * NL3;
    }
    a.setup_arena.commit(ctx);
}

// Neighbour closure kernels of every level; missing parents' keys go to miss[miss_base + ...].
// The table of the closure launches of one apply: the output levels j >= 1 with work (with_ghosts:
// only those that have ghosts).
ClosTab closure_table(const TreeApply& a, uint64_t* miss, bool with_ghosts) {
    ClosTab ct;
    int64_t blocks = 0;
    for (int j = 1; j <= a.depth; ++j) {
        const LevelWork& lw = a.W[j];
        if (lw.tpl.empty() || (with_ghosts && !lw.nghost)) continue;
        const int NL = 2 * lw.Lr + 1;
        ct.jm1[ct.n] = j - 1;
        ct.Lr[ct.n] = lw.Lr;
        ct.nout[ct.n] = lw.nout;
        ct.ng[ct.n] = lw.nghost;
        ct.bstart[ct.n] = blocks;
        ct.pkeys[ct.n] = lw.pkeys.p;
        ct.gkeys[ct.n] = lw.gkeys.p;
        ct.nbr[ct.n] = lw.nbr.p;
        ct.miss[ct.n] = miss + a.miss_base + lw.miss_off;
        ++ct.n;
        blocks += (lw.nout * NL * NL * NL + 255) / 256;
    }
    ct.bstart[ct.n] = blocks;
    return ct;
}

void launch_closure(mwns_ctx* ctx, TreeApply& a, uint64_t* miss) {
    const ClosTab ct = closure_table(a, miss, false);
    if (ct.bstart[ct.n] == 0) return;
    closure_kernel<<<(unsigned)ct.bstart[ct.n], 256, 0, ctx->stream>>>(ct);
    MWNS_HIP(hipGetLastError());
}

// Sorts the keys and drops any repeats.  An LSD radix sort over only the bytes in which the keys
// differ (level bits and the Morton bits of the deepest level): a few passes over data that stays
// in cache.
void sort_unique_keys(std::vector<uint64_t>& keys) {
    const size_t n = keys.size();
    if (n < 2) return;
    uint64_t diff = 0;
    for (const uint64_t key : keys) diff |= key ^ keys[0];
    std::vector<uint64_t> tmp(n);
    uint64_t* src = keys.data();
    uint64_t* dst = tmp.data();
    for (int sh = 0; sh < 64; sh += 8) {
        if (((diff >> sh) & 0xff) == 0) continue;
        size_t pos[256] = {};
        for (size_t i = 0; i < n; ++i) ++pos[(src[i] >> sh) & 0xff];
        size_t s = 0;
        for (size_t& p : pos) {
            const size_t c = p;
            p = s;
            s += c;
        }
        for (size_t i = 0; i < n; ++i) dst[pos[(src[i] >> sh) & 0xff]++] = src[i];
        std::swap(src, dst);
    }
    if (src != keys.data()) keys.swap(tmp);
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
}

// The distinct missing keys of every level become its ghost bricks (Alg. 3 Step 2): their
// indices complete the neighbour tables and their storage is allocated.
void discover_ghosts(mwns_ctx* ctx, TreeApply& a, std::vector<uint64_t>& keys, uint64_t* dmiss) {
    a.total_ghosts = 0;
    // a missing parent key of level j-1 belongs to the closure of output level j
    sort_unique_keys(keys);
    size_t pos = 0;
    for (int j = 1; j <= a.depth; ++j) {
        LevelWork& lw = a.W[j];
        const size_t b0 = pos;
        while (pos < keys.size() && key_level(keys[pos]) == j - 1) ++pos;
        if (lw.tpl.empty()) continue;
        lw.nghost = (int64_t)(pos - b0);
        a.total_ghosts += lw.nghost;
        if (lw.nghost) a.ghost_arena.add(keys.data() + b0, lw.nghost, lw.gkeys);
    }
    a.ghost_arena.commit(ctx);
    a.ghost_store.reset(ctx, (size_t)a.total_ghosts * brick_elems(a.k));
    size_t goff = 0;
    for (int j = 1; j <= a.depth; ++j) {
        LevelWork& lw = a.W[j];
        lw.ghosts.p = nullptr;
        if (lw.tpl.empty() || !lw.nghost) continue;
        lw.ghosts.p = a.ghost_store.p + goff;
        goff += (size_t)lw.nghost * brick_elems(a.k);
    }
    const ClosTab ct = closure_table(a, dmiss, true);
    if (ct.bstart[ct.n]) {
        closure_fill_kernel<<<(unsigned)ct.bstart[ct.n], 256, 0, ctx->stream>>>(ct);
        MWNS_HIP(hipGetLastError());
    }
}

// Ghost values: interpolation from the deepest existing ancestor (depends on f's coefficients).
// All levels in one launch: the ghosts of different levels are independent.
void launch_ghosts(mwns_ctx* ctx, TreeApply& a) {
    GhostTab gt;
    int64_t total = 0;
    for (int j = 1; j <= a.depth; ++j) {
        const LevelWork& lw = a.W[j];
        if (lw.tpl.empty() || !lw.nghost) continue;
        gt.jm1[gt.n] = j - 1;
        gt.start[gt.n] = total;
        gt.keys[gt.n] = lw.gkeys.p;
        gt.out[gt.n] = lw.ghosts.p;
        ++gt.n;
        total += lw.nghost;
    }
    if (!total) return;
    gt.start[gt.n] = total;
    dispatch_k<GhostLaunch>(a.k, ctx->stream, total, gt, a.f->dkeys.p, a.f->nnodes, a.lt, a.f->coef.p, a.dHt.p);
    MWNS_HIP(hipGetLastError());
}

// Routed apply: the sum of squares of every level's inputs (real and ghost) into lsq[0..depth].
void launch_level_norms(mwns_ctx* ctx, TreeApply& a, double* lsq) {
    const int64_t E = brick_elems(a.k);
    SumsqTab tb;
    int64_t total = 0;
    auto add = [&](int64_t nb, const double* X, double* acc) {
        if (nb <= 0) return;
        tb.start[tb.n] = total;
        tb.X[tb.n] = X;
        tb.acc[tb.n] = acc;
        ++tb.n;
        total += nb;
    };
    for (int j = 0; j <= a.depth; ++j) {
        const LevelWork& lw = a.W[j];
        if (lw.tpl.empty()) continue;
        add(lw.nout, a.f->coef.p + a.f->lev[j].brick_off * E, lsq + j);
        add(lw.nghost, lw.ghosts.p, lsq + j);
    }
    if (!total) return;
    tb.start[tb.n] = total;
    dispatch_k<LevelSumsqLaunch>(a.k, ctx->stream, total, tb);
    MWNS_HIP(hipGetLastError());
}

// Upper bound of || B ||_2 for B = sum_{L=lo..hi} |S^{j;m,L}|, the entrywise absolute values of the
// super-blocks masked to fine displacements [mlo, mhi] (2k x 2k).  For the nonnegative C = B^T B,
// rho(C) <= max_i (C v)_i / v_i for every positive v (Collatz-Wielandt); v after a few power steps
// from the ones vector makes the bound tight.  Cached in the operator.
double abs_box_norm(const mwns_op* op, int j, int m, int lo, int hi, int mlo, int mhi) {
    const std::array<int, 6> key{j, m, lo, hi, mlo, mhi};
    const auto it = op->absnorm.find(key);
    if (it != op->absnorm.end()) return it->second;
    const int k = op->k, D = 2 * k;
    const double* Fm = op->Fh.data() + ((size_t)j * op->M + m) * NLF * k * k;
    std::vector<double> B((size_t)D * D, 0.0), C((size_t)D * D, 0.0), v(D, 1.0), cv(D);
    for (int L = lo; L <= hi; ++L)
        for (int su = 0; su < 2; ++su)
            for (int sv = 0; sv < 2; ++sv) {
                const int l = 2 * L + su - sv;
                if (l < mlo || l > mhi || l < -LF || l > LF) continue;
                for (int a = 0; a < k; ++a)
                    for (int b = 0; b < k; ++b) B[(su * k + a) * D + sv * k + b] += std::fabs(Fm[((l + LF) * k + a) * k + b]);
            }
    for (int p = 0; p < D; ++p)
        for (int q = 0; q < D; ++q) {
            double c = 0.0;
            for (int r = 0; r < D; ++r) c += B[r * D + p] * B[r * D + q];
            C[p * D + q] = c;
        }
    auto apply_c = [&]() {
        for (int p = 0; p < D; ++p) {
            double c = 0.0;
            for (int q = 0; q < D; ++q) c += C[p * D + q] * v[q];
            cv[p] = c;
        }
    };
    for (int iter = 0; iter < 30; ++iter) {
        apply_c();
        const double mx = *std::max_element(cv.begin(), cv.end());
        if (!(mx > 0.0)) break;
        for (int p = 0; p < D; ++p) v[p] = std::max(cv[p] / mx, 1e-30);     // stays positive
    }
    apply_c();
    double rho = 0.0;
    for (int p = 0; p < D; ++p) rho = std::max(rho, cv[p] / v[p]);
    const double bound = std::sqrt(rho) * (1.0 + 1e-12);     // margin for the rounding of this estimate
    op->absnorm.emplace(key, bound);
    return bound;
}

// Routed apply: classes of every (level, job, term) from the level norms, jobs split into runs of
// one class, reduced-precision input copies allocated.
void route_tree(mwns_ctx* ctx, TreeApply& a, const double* lsq, const mwns_mixed_opts& opts) {
    const mwns_op* op = a.op;
    std::vector<RouteItem> items;
    const int M = op->M;
    if (op->Fh.empty()) {
        op->Fh.resize(op->F.n);
        MWNS_HIP(hipMemcpy(op->Fh.data(), op->F.p, op->F.n * sizeof(double), hipMemcpyDeviceToHost));
    }
    for (int j = 0; j <= a.depth; ++j) {
        const LevelWork& lw = a.W[j];
        const double xn = std::sqrt(lsq[j]);
        int64_t ninternal = 0;
        for (int64_t b = 0; b < lw.nout; ++b) ninternal += lw.cm[b] != 0;
        for (int t = 0; t < (int)lw.tpl.size(); ++t) {
            const Tpl& tp = lw.tpl[t];
            const double nb = tp.dpart ? (double)ninternal : (double)lw.nout;
            const double n1 = tp.hi[0] - tp.lo[0] + 1, n2 = tp.hi[1] - tp.lo[1] + 1, n3 = tp.hi[2] - tp.lo[2] + 1;
            for (int m = tp.m1; m <= tp.m2; ++m) {
                const double* fr = op->fro.data() + ((int64_t)j * M + m) * NLF;
                // two bounds of the job's contribution; the smaller one is used
                double bfro = 1.0, babs = 1.0;
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int L = tp.lo[d]; L <= tp.hi[d]; ++L) {
                        double s2 = 0.0;
                        for (int su = 0; su < 2; ++su)
                            for (int sv = 0; sv < 2; ++sv) {
                                const int l = 2 * L + su - sv;
                                if (l >= tp.mlo[d] && l <= tp.mhi[d]) s2 += fr[l + LF] * fr[l + LF];
                            }
                        s += std::sqrt(s2);
                    }
                    bfro *= s;
                    babs *= abs_box_norm(op, j, m, tp.lo[d], tp.hi[d], tp.mlo[d], tp.mhi[d]);
                }
                const double beta = std::fabs(op->w[m]) * xn * std::min(bfro, babs);
                // near-diagonal narrow Gaussians stay in FP64: the job's box holds the zero
                // displacement and the term's width in level-j box units, 2^j / sqrt(tau_m), is at
                // most 1/(2k), below the resolution of the degree k-1 polynomials of a box
                // (tau_m >= 4 k^2 4^j): its blocks act on the box itself almost alone
                const bool diag = tp.lo[0] <= 0 && tp.hi[0] >= 0 && tp.lo[1] <= 0 && tp.hi[1] >= 0 && tp.lo[2] <= 0 && tp.hi[2] >= 0;
                const bool pin = diag && op->tau[m] >= 4.0 * a.k * a.k * std::ldexp(1.0, 2 * j);
                items.push_back(RouteItem{j, t, m, PREC_F64, beta, nb * (n1 * n2 * n3 + n1 * n2 + n1), pin});
            }
        }
    }
    // (the whole-brick kernel, orders above KNARROW, has the FP32 class only: the callers reject
    // the BF16 bits there)
    a.err_bound = route(items, opts.tol, opts.classes, a.k);
    size_t pos = 0;
    for (int j = 0; j <= a.depth; ++j) {
        LevelWork& lw = a.W[j];
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
        // 16-byte units per brick of the one-tile kernel's copies (padded rows); the whole-brick
        // kernel (orders above KNARROW) rounds its FP64 inputs to FP32 as they enter a product
        const int64_t D = 2 * a.k;
        const int64_t units = 4 * D * D;
        if (a.k > KNARROW) need32 = needbf = false;
        if (need32) {
            lw.xr32.reset(ctx, (size_t)lw.nout * units);
            if (lw.nghost) lw.xg32.reset(ctx, (size_t)lw.nghost * units);
        }
        if (needbf) {
            lw.xrb.reset(ctx, (size_t)lw.nout * units);
            if (lw.nghost) lw.xgb.reset(ctx, (size_t)lw.nghost * units);
        }
    }
}

// Routed apply: fill the reduced-precision input copies.
void launch_convert_inputs(mwns_ctx* ctx, TreeApply& a) {
    const int64_t E = brick_elems(a.k);
    ConvTab tb;
    for (int j = 0; j <= a.depth; ++j) {
        LevelWork& lw = a.W[j];
        const double* xr = a.f->coef.p + a.f->lev[j].brick_off * E;
        if (lw.xr32.p) tb.add(a.k, lw.nout, xr, lw.xr32.p, false);
        if (lw.xg32.p) tb.add(a.k, lw.nghost, lw.ghosts.p, lw.xg32.p, false);
        if (lw.xrb.p) tb.add(a.k, lw.nout, xr, lw.xrb.p, true);
        if (lw.xgb.p) tb.add(a.k, lw.nghost, lw.ghosts.p, lw.xgb.p, true);
    }
    if (tb.n) launch_convert(a.k, ctx->stream, tb);   // the one-tile kernel's copies, one launch
    MWNS_HIP(hipGetLastError());
}

// Level descriptors of the contraction kernel (appended to descs) and, per precision class, the
// cost of every output brick with jobs of that class (for the launch orders): entries are
// (cost, (descriptor index, brick)).  The FP64 list holds every brick, since its launch writes
// every output brick.
void build_descs(mwns_ctx* ctx, TreeApply& a, std::vector<LevelDesc>& descs,
                 std::vector<std::pair<double, int2>> (&cost)[NPREC]) {
    const int k = a.k;
    const int64_t E = brick_elems(k);
    for (int j = 0; j <= a.depth; ++j)
        if (!a.W[j].tpl.empty()) a.desc_arena.add(a.W[j].tpl.data(), a.W[j].tpl.size(), a.W[j].dtpl);
    a.desc_arena.commit(ctx);
    a.desc_base = descs.size();
    a.jobs = 0;
    a.flops = 0.0;
    for (int p = 0; p < NPREC; ++p) a.class_flops[p] = 0.0;
    a.own_flops = 0.0;
    a.mfma_flops = 0.0;
    // FP64 matrix-core flops issued per (brick, term) and unit of `steps`: the one-tile kernel runs
    // four 16x16x4 products (2048 flops each) per slice and step on its 2k real slices; the brick
    // kernel (orders above KNARROW) per slice five 16x16x4 and fifteen 4x4x4 (512 flops) products
    // in modes 3 and 2, and the same per output row u2 in mode 1, except that mode 1 of a down-band
    // job at a brick with leaf children runs two passes: per row and K step two 16x16x4 and four
    // 4x4x4 products instead of one and three.  Its FP32 class runs the 4x4x4 products (the tails)
    // in FP64 and the 16x16x4 ones in FP32.
    const double D2 = 2.0 * k;
    const double tile16 = k > KNARROW ? 5.0 * 2048.0 * D2 : 4.0 * 2048.0 * D2;
    const double tails = k > KNARROW ? 15.0 * 512.0 * D2 : 0.0;
    const double tile16_split = 5.0 * 2.0 * 2048.0 * D2, tails_split = 5.0 * 4.0 * 512.0 * D2;
    for (int j = 0; j <= a.depth; ++j) {
        LevelWork& lw = a.W[j];
        LevelDesc d{};
        d.out = a.out->coef.p + a.f->lev[j].brick_off * E;
        const int di = (int)descs.size();
        if (lw.tpl.empty()) {
            descs.push_back(d);
            continue;
        }

        d.Xr = a.f->coef.p + a.f->lev[j].brick_off * E;
        d.Xg = lw.ghosts.p;
        d.Xr32 = reinterpret_cast<const float*>(lw.xr32.p);
        d.Xg32 = reinterpret_cast<const float*>(lw.xg32.p);
        d.Xrb = lw.xrb.p;
        d.Xgb = lw.xgb.p;
        d.nbr = lw.nbr.p;
        d.cmask = lw.cmask.p;
        d.tpl = lw.dtpl.p;
        d.Fj = a.op->F.p + (int64_t)j * a.op->M * NLF * k * k;
        d.w = a.op->dw.p;
        d.nreal = lw.nout;
        d.Lr = lw.Lr;
        d.valid = lw.valid;
        d.ntpl = (int)lw.tpl.size();
        descs.push_back(d);
        // down-band jobs whose terms all lie in the whole band's range R_j(L) at every coarse L of
        // their box: at internal children they cancel whole-band terms (net coefficient 0)
        std::vector<char> nested(lw.tpl.size(), 0);
        const int32_t* row = a.op->plan.data() + (int64_t)j * NLP3 * 2;
        for (size_t ti = 0; ti < lw.tpl.size(); ++ti) {
            const Tpl& t = lw.tpl[ti];
            if (!t.dpart) continue;
            bool in = true;
            for (int x = t.lo[0]; x <= t.hi[0] && in; ++x)
                for (int y = t.lo[1]; y <= t.hi[1] && in; ++y)
                    for (int z = t.lo[2]; z <= t.hi[2] && in; ++z) {
                        if (std::abs(x) > LP || std::abs(y) > LP || std::abs(z) > LP) { in = false; break; }
                        const int32_t* r = row + (((x + LP) * NLP + (y + LP)) * NLP + (z + LP)) * 2;
                        in = r[0] <= t.m1 && t.m2 <= r[1];
                    }
            nested[ti] = in;
        }
        // Whole-band pairs with net coefficient 0: at an internal child s, the pair (L, input child
        // s', term m) with m in R_{j+1}(2L + s - s') is cancelled by the down band.  ov[t] holds, per
        // coarse L of whole-band job t's box and per fine offset delta = s - s' in {-1,0,1}^3, how
        // many of the job's terms lie in R_{j+1}(2L + delta); ovsum[t] the sums over the box.
        const bool has_down = j > 0 && j < a.depth && j + 1 <= a.op->max_level;
        const int32_t* rown = has_down ? a.op->plan.data() + (int64_t)(j + 1) * NLP3 * 2 : nullptr;
        std::vector<std::vector<int>> ov(lw.tpl.size());
        std::vector<std::array<double, 27>> ovsum(lw.tpl.size());
        for (size_t ti = 0; ti < lw.tpl.size() && has_down; ++ti) {
            const Tpl& t = lw.tpl[ti];
            ovsum[ti].fill(0.0);
            if (t.dpart) continue;
            const int n1 = t.hi[0] - t.lo[0] + 1, n2 = t.hi[1] - t.lo[1] + 1, n3 = t.hi[2] - t.lo[2] + 1;
            ov[ti].assign((size_t)n1 * n2 * n3 * 27, 0);
            for (int x = 0; x < n1; ++x)
                for (int y = 0; y < n2; ++y)
                    for (int z = 0; z < n3; ++z)
                        for (int dl = 0; dl < 27; ++dl) {
                            const int l0 = 2 * (t.lo[0] + x) + dl / 9 - 1, l1 = 2 * (t.lo[1] + y) + (dl / 3) % 3 - 1;
                            const int l2 = 2 * (t.lo[2] + z) + dl % 3 - 1;
                            if (std::abs(l0) > LP || std::abs(l1) > LP || std::abs(l2) > LP) continue;
                            const int32_t* r = rown + (((l0 + LP) * NLP + (l1 + LP)) * NLP + (l2 + LP)) * 2;
                            const int o = std::max(0, std::min(r[1], t.m2) - std::max(r[0], t.m1) + 1);
                            ov[ti][((size_t)(x * n2 + y) * n3 + z) * 27 + dl] = o;
                            ovsum[ti][dl] += o;
                        }
        }
        const int64_t pside = j > 0 ? ((int64_t)1 << (j - 1)) : 1;
        for (int64_t b = 0; b < lw.nout; ++b) {
            int64_t pp[3] = {0, 0, 0};
            if (j > 0) key_coords(lw.pk[b], pp);
            double c[NPREC] = {0.0, 0.0, 0.0, 0.0};
            // cnt[delta]: pairs (internal child s, input child s') with s - s' = delta (child bit d = s_d)
            double cnt[27];
            const int cmb = lw.cm[b];
            if (has_down && cmb != 0)
                for (int dl = 0; dl < 27; ++dl) {
                    const int dd[3] = {dl / 9 - 1, (dl / 3) % 3 - 1, dl % 3 - 1};
                    int n = 0;
                    for (int s = 0; s < 8; ++s) {
                        if (!(cmb >> s & 1)) continue;
                        bool ok = true;
                        for (int e = 0; e < 3; ++e) {
                            const int sp = ((s >> e) & 1) - dd[e];
                            ok = ok && sp >= 0 && sp <= 1;
                        }
                        n += ok;
                    }
                    cnt[dl] = n;
                }
            for (size_t ti = 0; ti < lw.tpl.size(); ++ti) {
                const Tpl& t = lw.tpl[ti];
                if (t.dpart && lw.cm[b] == 0) continue;
                double nin[3];     // displacements L of the box with P - L inside the cube
                for (int dd = 0; dd < 3; ++dd)
                    nin[dd] = (double)std::max<int64_t>(
                        0, std::min<int64_t>(t.hi[dd], pp[dd]) - std::max<int64_t>(t.lo[dd], pp[dd] - pside + 1) + 1);
                if (nin[0] * nin[1] * nin[2] == 0) continue;     // the box lies outside the cube
                const double nt = t.m2 - t.m1 + 1;
                const double steps = nin[0] * nin[1] * nin[2] + nin[0] * nin[1] + nin[0];
                c[t.prec] += nt * steps;
                a.jobs += (int64_t)nt;
                const double fl = nt * 2.0 * D2 * D2 * D2 * D2 * steps;
                a.flops += fl;
                a.class_flops[t.prec] += fl;
                if (!nested[ti]) {
                    double own = fl;
                    if (has_down && cmb != 0 && !t.dpart) {
                        // share of the job's (child, L, s', m) pairs whose net coefficient is 0
                        const int n1 = t.hi[0] - t.lo[0] + 1, n2 = t.hi[1] - t.lo[1] + 1, n3 = t.hi[2] - t.lo[2] + 1;
                        double canc = 0.0;
                        if (nin[0] == n1 && nin[1] == n2 && nin[2] == n3) {
                            for (int dl = 0; dl < 27; ++dl) canc += ovsum[ti][dl] * cnt[dl];
                        } else {
                            for (int x = 0; x < n1; ++x)
                                for (int y = 0; y < n2; ++y)
                                    for (int z = 0; z < n3; ++z) {
                                        const int64_t L[3] = {t.lo[0] + x, t.lo[1] + y, t.lo[2] + z};
                                        bool in = true;
                                        for (int e = 0; e < 3; ++e) in = in && pp[e] - L[e] >= 0 && pp[e] - L[e] < pside;
                                        if (!in) continue;
                                        const int* o = ov[ti].data() + ((size_t)(x * n2 + y) * n3 + z) * 27;
                                        for (int dl = 0; dl < 27; ++dl) canc += o[dl] * cnt[dl];
                                    }
                        }
                        own *= 1.0 - canc / (64.0 * nt * nin[0] * nin[1] * nin[2]);
                    }
                    a.own_flops += own;
                }
                if (t.prec == PREC_F64 || (k > KNARROW && t.prec == PREC_F32)) {
                    const double f16 = t.prec == PREC_F64 ? 1.0 : 0.0;
                    if (k > KNARROW && t.dpart && lw.cm[b] != 0xff)
                        a.mfma_flops += nt * ((f16 * tile16 + tails) * (steps - nin[0]) + (f16 * tile16_split + tails_split) * nin[0]);
                    else
                        a.mfma_flops += nt * (f16 * tile16 + tails) * steps;
                }
            }
            for (int p = 0; p < NPREC; ++p)
                if (p == PREC_F64 || c[p] > 0.0) cost[p].push_back({c[p], make_int2(di, (int)b)});
        }
    }
}

// Outputs of levels without jobs are zero (a kernel, so that the sequence can be captured).
void launch_zero_outputs(mwns_ctx* ctx, TreeApply& a) {
    const int64_t E = brick_elems(a.k);
    for (int j = 0; j <= a.depth; ++j) {
        const LevelWork& lw = a.W[j];
        if (!lw.tpl.empty() || lw.nout == 0) continue;
        const int64_t n = lw.nout * E;
        fill_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(a.out->coef.p + a.f->lev[j].brick_off * E, n, 0.0);
    }
    MWNS_HIP(hipGetLastError());
}

// Assembly (eq. g_assemble), level by level.
void launch_assembly(mwns_ctx* ctx, TreeApply& a) {
    for (int j = 1; j <= a.depth; ++j) {
        const mwns_level& L = a.f->lev[j];
        dispatch_k<AssembleLaunch>(a.k, ctx->stream, L.nbricks, j, a.W[j].apb.p, a.W[j].apc.p, L.brick_off, a.dHt.p,
                                   a.out->coef.p);
        MWNS_HIP(hipGetLastError());
    }
}

// Launch order.  Workgroups are dealt round-robin to the 8 XCDs, each with its own L2, and the
// input sibling groups of neighbouring output bricks overlap: so (tree, level) groups go costliest
// per brick first, each group is cut into 8 contiguous Morton ranges of equal length, and XCD x
// takes range x of every group.  For the one-workgroup-per-brick launch the ranges are
// interleaved (position 8i + x holds the i-th brick of range x); for the persistent launch they
// are concatenated into 8 queues (queue x = every group's range x, costliest group first).
void make_order(const std::vector<std::pair<double, int2>>& cost, bool persistent, std::vector<int2>& order,
                std::vector<int>& queues) {
    std::vector<std::pair<size_t, size_t>> groups;   // [begin, end) of each descriptor's bricks in cost
    std::vector<double> per;                         // cost per brick of each group
    for (size_t pos = 0; pos < cost.size();) {
        size_t e = pos;
        double c = 0.0;
        while (e < cost.size() && cost[e].second.x == cost[pos].second.x) c += cost[e++].first;
        groups.push_back({pos, e});
        per.push_back(c / (double)(e - pos));
        pos = e;
    }
    std::vector<size_t> gi(groups.size());
    for (size_t i = 0; i < gi.size(); ++i) gi[i] = i;
    std::stable_sort(gi.begin(), gi.end(), [&](size_t x, size_t y) { return per[x] > per[y]; });
    order.clear();
    order.reserve(cost.size());
    queues.assign(QUEUE_INTS, 0);
    if (!persistent) {
        for (size_t g : gi) {
            const size_t b0 = groups[g].first, n = groups[g].second - b0;
            const size_t step = (n + NXCD - 1) / NXCD;
            for (size_t i = 0; i < step; ++i)
                for (int x = 0; x < NXCD; ++x)
                    if (x * step + i < n) order.push_back(cost[b0 + x * step + i].second);
        }
        return;
    }
    for (int x = 0; x < NXCD; ++x) {
        queues[NXCD + x] = (int)order.size();
        for (size_t g : gi) {
            const size_t b0 = groups[g].first, n = groups[g].second - b0;
            const size_t step = (n + NXCD - 1) / NXCD;
            for (size_t i = x * step; i < std::min(n, (x + 1) * step); ++i) order.push_back(cost[b0 + i].second);
        }
        queues[2 * NXCD + x] = (int)order.size();
    }
}

// Device contraction count and ||g|| of one apply into s (synchronises).
void collect_stats(mwns_ctx* ctx, TreeApply& a, int mode, mwns_apply_stats& s) {
    s.brick_jobs += a.jobs;
    s.ghost_bricks += a.total_ghosts;
    s.useful_flops += a.flops;
    s.own_flops += a.own_flops;
    s.f64_mfma_flops += a.mfma_flops;
    s.err_bound = std::max(s.err_bound, a.err_bound);
    for (int p = 0; p < NPREC; ++p) s.class_flops[p] += a.class_flops[p];
    if (mode & MWNS_TIMES_ONLY) {
        s.contractions = -1;
        return;
    }
    hipStream_t st = ctx->stream;
    const int64_t planrow = (int64_t)NLP3 * 2;
    const int64_t E = brick_elems(a.k);
    DevArray<unsigned long long> tot(ctx, 1);
    DevArray<double> gsq(ctx, 1);
    fill_kernel<<<1, 64, 0, st>>>(gsq.p, 1, 0.0);
    zero_ints_kernel<<<1, 64, 0, st>>>(reinterpret_cast<int*>(tot.p), 2);
    DevArray<int32_t> dplan(ctx, a.op->plan.size());
    dplan.upload(a.op->plan.data(), a.op->plan.size(), st);
    std::vector<CountLevel> cl;
    int64_t nitems = 0;
    for (int j = 0; j <= a.depth; ++j) {
        const LevelWork& lw = a.W[j];
        CountLevel c{};
        c.pkeys = lw.pkeys.p;
        c.cmask = lw.cmask.p;
        c.Rj = dplan.p + (int64_t)j * planrow;
        c.Rj1 = (j + 1 <= a.op->max_level) ? dplan.p + (int64_t)(j + 1) * planrow : nullptr;
        c.first = nitems;
        c.nout = lw.nout;
        c.j = j;
        c.valid = lw.valid;
        cl.push_back(c);
        nitems += lw.nout * 8 * NLP;
    }
    DevArray<CountLevel> dcl(ctx, cl.size());
    dcl.upload(cl.data(), cl.size(), st);
    count_kernel<<<(unsigned)((nitems + 255) / 256), 256, 0, st>>>(dcl.p, (int)cl.size(), nitems, tot.p);
    // ||g||_2: the leaves' scaling functions are orthonormal with disjoint supports
    if (!(mode & MWNS_NO_ASSEMBLY))
        for (int j = 0; j <= a.depth; ++j)
            dispatch_k<LeafsqLaunch>(a.k, st, a.f->lev[j].nbricks, a.f->lev[j].node_off, j == 0 ? 1 : 8, a.f->dleaf.p,
                                     a.out->coef.p + a.f->lev[j].brick_off * E, gsq.p);
    MWNS_HIP(hipGetLastError());
    unsigned long long c = 0;
    double g2 = 0.0;
    tot.download(&c, 1, st);
    gsq.download(&g2, 1, st);
    MWNS_HIP(hipStreamSynchronize(st));
    s.contractions += (int64_t)c;
    s.g_norm = std::sqrt(s.g_norm * s.g_norm + g2);
}

// Everything before the value phase: structure, closure (one host round trip for the whole
// batch), ghost discovery and, for routed applies, the level norms and classes (a second round
// trip).  Ghost values and converted inputs are computed here too when `values` is set.
void prepare(mwns_ctx* ctx, std::vector<std::unique_ptr<TreeApply>>& trees, const mwns_op* const* ops,
             const mwns_tree* const* fs, const mwns_mixed_opts* mixed, bool values, DevArray<uint64_t>& miss) {
    hipStream_t st = ctx->stream;
    const int n = (int)trees.size();
    int64_t miss_total = 0;
    for (int i = 0; i < n; ++i) {
        setup(ctx, *trees[i], ops[i], fs[i]);
        trees[i]->miss_base = miss_total;
        miss_total += trees[i]->miss_total;
    }
    miss.reset(ctx, std::max<int64_t>(1, miss_total));
    for (auto& a : trees) launch_closure(ctx, *a, miss.p);
    // only the distinct missing keys travel to the host: compact them per tree on the device
    const int nt = (int)trees.size();
    DevArray<uint64_t> comp(ctx, std::max<int64_t>(1, miss_total));
    DevArray<unsigned int> cnt(ctx, nt);
    zero_ints_kernel<<<(nt + 63) / 64, 64, 0, st>>>(reinterpret_cast<int*>(cnt.p), nt);
    std::vector<int64_t> cap(nt, 0), tab_off(nt + 1, 0);
    for (int i = 0; i < nt; ++i) {
        if (trees[i]->miss_total) {
            int64_t c = 1;
            while (c < 2 * trees[i]->miss_total) c <<= 1;
            cap[i] = c;
        }
        tab_off[i + 1] = tab_off[i] + cap[i];
    }
    DevArray<uint64_t> tab(ctx, std::max<int64_t>(1, tab_off[nt]));
    if (tab_off[nt])
        fill_u64_kernel<<<(unsigned)((tab_off[nt] + 255) / 256), 256, 0, st>>>(tab.p, tab_off[nt], ~0ull);
    for (int i = 0; i < nt; ++i) {
        const TreeApply& a = *trees[i];
        if (a.miss_total)
            compact_distinct_kernel<<<(unsigned)((a.miss_total + 255) / 256), 256, 0, st>>>(
                a.miss_total, miss.p + a.miss_base, tab.p + tab_off[i], cap[i], comp.p + a.miss_base, cnt.p + i);
    }
    MWNS_HIP(hipGetLastError());
    std::vector<unsigned int> hc(nt);
    cnt.download(hc.data(), nt, st);
    MWNS_HIP(hipStreamSynchronize(st));
    std::vector<std::vector<uint64_t>> keys(nt);
    size_t nkeys = 0;
    for (int i = 0; i < nt; ++i) nkeys += hc[i];
    uint64_t* pin = static_cast<uint64_t*>(pinned_staging(ctx, std::max<size_t>(1, nkeys) * sizeof(uint64_t)));
    size_t off = 0;
    for (int i = 0; i < nt; off += hc[i], ++i)
        if (hc[i]) MWNS_HIP(hipMemcpyAsync(pin + off, comp.p + trees[i]->miss_base, hc[i] * sizeof(uint64_t),
                                          hipMemcpyDeviceToHost, st));
    MWNS_HIP(hipStreamSynchronize(st));
    off = 0;
    for (int i = 0; i < nt; off += hc[i], ++i) keys[i].assign(pin + off, pin + off + hc[i]);
    for (int i = 0; i < nt; ++i) discover_ghosts(ctx, *trees[i], keys[i], miss.p);
    if (mixed) {
        // routing needs the ghosts' values for the level norms
        size_t nl = 0;
        for (auto& a : trees) nl += a->depth + 1;
        DevArray<double> lsq(ctx, nl);
        fill_kernel<<<(unsigned)((nl + 63) / 64), 64, 0, st>>>(lsq.p, (int64_t)nl, 0.0);
        size_t off = 0;
        for (auto& a : trees) {
            launch_ghosts(ctx, *a);
            launch_level_norms(ctx, *a, lsq.p + off);
            off += a->depth + 1;
        }
        std::vector<double> hl(nl);
        lsq.download(hl.data(), nl, st);
        MWNS_HIP(hipStreamSynchronize(st));
        off = 0;
        for (int i = 0; i < n; ++i) {
            route_tree(ctx, *trees[i], hl.data() + off, mixed[i]);
            off += trees[i]->depth + 1;
        }
        if (values)
            for (auto& a : trees) launch_convert_inputs(ctx, *a);
    } else if (values) {
        for (auto& a : trees) launch_ghosts(ctx, *a);
    }
}

// Descriptors and launch orders of a batch, one contraction launch per basis order k.
struct Launches {
    std::vector<LevelDesc> descs;
    DevArray<LevelDesc> ddesc;
    struct Group {
        int k = 0, variant = 0, prec = PREC_F64;
        int64_t nblocks = 0;
        std::vector<int2> order;
        std::vector<int> queue_init;
        DevArray<int2> dorder;
        DevArray<int> dqueue;
    };
    std::vector<Group> groups;
};

void build_launches(mwns_ctx* ctx, std::vector<std::unique_ptr<TreeApply>>& trees, bool persistent, Launches& Lz) {
    std::vector<int> ks;
    for (auto& a : trees)
        if (std::find(ks.begin(), ks.end(), a->k) == ks.end()) ks.push_back(a->k);
    std::vector<std::array<std::vector<std::pair<double, int2>>, NPREC>> costs(ks.size());
    for (auto& a : trees) {
        const size_t gi = std::find(ks.begin(), ks.end(), a->k) - ks.begin();
        std::vector<std::pair<double, int2>> c[NPREC];
        build_descs(ctx, *a, Lz.descs, c);
        for (int p = 0; p < NPREC; ++p) costs[gi][p].insert(costs[gi][p].end(), c[p].begin(), c[p].end());
    }
    Lz.ddesc.reset(ctx, std::max<size_t>(1, Lz.descs.size()));
    Lz.ddesc.upload(Lz.descs.data(), Lz.descs.size(), ctx->stream);
    Lz.groups.clear();
    for (size_t gi = 0; gi < ks.size(); ++gi)
        for (int p = 0; p < NPREC; ++p) {     // FP64 first: its launch writes every output brick
            if (costs[gi][p].empty()) continue;
            Lz.groups.emplace_back();
            auto& g = Lz.groups.back();
            g.k = ks[gi];
            g.prec = p;
            g.variant = variant_for(ctx, g.k);
            make_order(costs[gi][p], persistent, g.order, g.queue_init);
            g.dorder.reset(ctx, std::max<size_t>(1, g.order.size()));
            g.dorder.upload(g.order.data(), g.order.size(), ctx->stream);
            if (persistent) {
                g.dqueue.reset(ctx, QUEUE_INTS);
                g.dqueue.upload(g.queue_init.data(), QUEUE_INTS, ctx->stream);
                const int64_t res = g.k > KNARROW ? resident_blocks_wide(g.k, g.variant, g.prec, ctx->device)
                                                  : resident_blocks(g.k, g.variant, g.prec, ctx->device);
                g.nblocks = std::min<int64_t>((int64_t)g.order.size(), res);
            } else {
                g.nblocks = (int64_t)g.order.size();
            }
        }
}

void launch_contractions(mwns_ctx* ctx, Launches& Lz) {
    for (auto& g : Lz.groups) {
        if (g.order.empty()) continue;
        if (g.dqueue.p) zero_ints_kernel<<<1, 64, 0, ctx->stream>>>(g.dqueue.p, NXCD);
        if (g.k > KNARROW)
            launch_contract_wide(g.k, g.variant, g.prec, ctx->stream, g.nblocks, Lz.ddesc.p, g.dorder.p, g.dqueue.p);
        else
            launch_contract(g.k, g.variant, g.prec, g.prec != PREC_F64, ctx->stream, g.nblocks, Lz.ddesc.p, g.dorder.p,
                            g.dqueue.p);
        MWNS_HIP(hipGetLastError());
    }
}

// Batched apply of n (operator, tree) pairs; mixed: NULL (FP64) or n routing options.
void apply_batch(mwns_ctx* ctx, int n, const mwns_op* const* ops, const mwns_tree* const* fs,
                 const mwns_mixed_opts* mixed, int mode, bool persistent, mwns_tree** gs, mwns_apply_stats* stats) {
    if (!ctx || !ops || !fs || !gs || n < 1) fail(MWNS_EINVAL, "NULL argument or empty batch");
    hipStream_t st = ctx->stream;
    std::vector<std::unique_ptr<TreeApply>> trees;
    for (int i = 0; i < n; ++i) trees.emplace_back(new TreeApply);
    Timer tclos(st), tcon(st), tasm(st);
    tclos.start();
    DevArray<uint64_t> miss;     // read by the closure kernels until the stream passes them
    prepare(ctx, trees, ops, fs, mixed, true, miss);
    Launches Lz;
    build_launches(ctx, trees, persistent, Lz);
    for (auto& a : trees) launch_zero_outputs(ctx, *a);
    tclos.stop();
    tcon.start();
    launch_contractions(ctx, Lz);
    tcon.stop();
    tasm.start();
    if (!(mode & MWNS_NO_ASSEMBLY))
        for (auto& a : trees) launch_assembly(ctx, *a);
    tasm.stop();
    if (stats) {
        mwns_apply_stats s{};
        for (auto& a : trees) collect_stats(ctx, *a, mode, s);
        s.ms_closure = tclos.ms();
        s.ms_contract = tcon.ms();
        s.ms_assemble = tasm.ms();
        *stats = s;
    } else {
        MWNS_HIP(hipStreamSynchronize(st));
    }
    for (int i = 0; i < n; ++i) gs[i] = trees[i]->out.release();
}

}  // namespace

// A reusable apply: structure, closure, ghost keys, routing and buffers fixed at creation; the
// value phase (ghost values, input copies, contractions, assembly) captured once as a hipGraph.
struct mwns_plan {
    mwns::CtxHold hold;
    mwns_ctx* ctx = nullptr;
    int mode = 0;
    std::vector<std::unique_ptr<TreeApply>> trees;
    Launches launches;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~mwns_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

void record_values(mwns_plan* pl, hipStream_t st) {
    mwns_ctx tmp = *pl->ctx;      // the same device and allocator, launches on st
    tmp.stream = st;
    for (auto& a : pl->trees) {
        launch_ghosts(&tmp, *a);
        launch_convert_inputs(&tmp, *a);
        launch_zero_outputs(&tmp, *a);
    }
    launch_contractions(&tmp, pl->launches);
    if (!(pl->mode & MWNS_NO_ASSEMBLY))
        for (auto& a : pl->trees) launch_assembly(&tmp, *a);
}

}  // namespace

extern "C" mwns_status mwns_apply(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, int mode, mwns_tree** g,
                                  mwns_apply_stats* stats) {
    MWNS_GUARD_BEGIN
    if ((mode & 0xff) != MWNS_F64 || (mode & ~(0xff | MWNS_NO_ASSEMBLY | MWNS_TIMES_ONLY))) fail(MWNS_EINVAL, "unsupported mode");
    if (!ctx || !op || !f || !g) fail(MWNS_EINVAL, "NULL argument");
    apply_batch(ctx, 1, &op, &f, nullptr, mode, false, g, stats);
    return MWNS_OK;
    MWNS_GUARD_END
}

namespace {
void check_mixed(const mwns_mixed_opts* opts, const mwns_tree* f) {
    if (!(opts->tol >= 0.0) || !std::isfinite(opts->tol)) fail(MWNS_EINVAL, "tol must be finite and >= 0");
    if (opts->classes & ~(MWNS_CLASS_F32 | MWNS_CLASS_BF16C | MWNS_CLASS_BF16)) fail(MWNS_EINVAL, "unknown precision class");
    if (f && f->k > KNARROW && (opts->classes & (MWNS_CLASS_BF16C | MWNS_CLASS_BF16)))
        fail(MWNS_EINVAL, "the BF16 classes are not available for k > " + std::to_string(KNARROW) + " (k = " +
                              std::to_string(f->k) + "): allow MWNS_CLASS_F32 only");
}
}  // namespace

extern "C" mwns_status mwns_apply_mixed(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, const mwns_mixed_opts* opts,
                                        int flags, mwns_tree** g, mwns_apply_stats* stats) {
    MWNS_GUARD_BEGIN
    if (!opts) fail(MWNS_EINVAL, "opts is NULL");
    if (flags & ~(MWNS_NO_ASSEMBLY | MWNS_TIMES_ONLY)) fail(MWNS_EINVAL, "unsupported flags");
    if (!ctx || !op || !f || !g) fail(MWNS_EINVAL, "NULL argument");
    check_mixed(opts, f);
    apply_batch(ctx, 1, &op, &f, opts, flags, false, g, stats);
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_apply_batch(mwns_ctx* ctx, int n, const mwns_op* const* ops, const mwns_tree* const* fs,
                                        const mwns_mixed_opts* mixed, int flags, mwns_tree** gs, mwns_apply_stats* stats) {
    MWNS_GUARD_BEGIN
    if (flags & ~(MWNS_NO_ASSEMBLY | MWNS_TIMES_ONLY)) fail(MWNS_EINVAL, "unsupported flags");
    if (mixed)
        for (int i = 0; i < n; ++i) check_mixed(mixed + i, fs ? fs[i] : nullptr);
    if (gs)
        for (int i = 0; i < n; ++i) gs[i] = nullptr;
    apply_batch(ctx, n, ops, fs, mixed, flags, true, gs, stats);
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_plan_create(mwns_ctx* ctx, int n, const mwns_op* const* ops, const mwns_tree* const* fs,
                                        const mwns_mixed_opts* mixed, int flags, mwns_plan** out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !ops || !fs || !out || n < 1) fail(MWNS_EINVAL, "NULL argument or empty batch");
    if (flags & ~MWNS_NO_ASSEMBLY) fail(MWNS_EINVAL, "unsupported flags");
    if (mixed)
        for (int i = 0; i < n; ++i) check_mixed(mixed + i, fs[i]);
    std::unique_ptr<mwns_plan> pl(new mwns_plan);
    pl->ctx = ctx;
    pl->hold.set(ctx);
    pl->mode = flags;
    for (int i = 0; i < n; ++i) pl->trees.emplace_back(new TreeApply);
    {
        DevArray<uint64_t> miss;
        prepare(ctx, pl->trees, ops, fs, mixed, false, miss);
        build_launches(ctx, pl->trees, true, pl->launches);
        MWNS_HIP(hipStreamSynchronize(ctx->stream));
    }
    // capture the value phase on a private stream (default priority) and instantiate it
    hipStream_t cap;
    MWNS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        try {
            record_values(pl.get(), cap);
        } catch (...) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(cap, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
            (void)hipStreamDestroy(cap);
            throw;
        }
        e = hipStreamEndCapture(cap, &pl->graph);
    }
    (void)hipStreamDestroy(cap);
    check_hip(e, "capturing the apply graph");
    MWNS_HIP(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0));
    *out = pl.release();
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_plan_execute(mwns_plan* pl) {
    MWNS_GUARD_BEGIN
    if (!pl) fail(MWNS_EINVAL, "plan is NULL");
    MWNS_HIP(hipGraphLaunch(pl->exec, pl->ctx->stream));
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_plan_output(const mwns_plan* pl, int i, const mwns_tree** g) {
    MWNS_GUARD_BEGIN
    if (!pl || !g) fail(MWNS_EINVAL, "NULL argument");
    if (i < 0 || i >= (int)pl->trees.size()) fail(MWNS_EINVAL, "output index out of range");
    *g = pl->trees[i]->out.get();
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" mwns_status mwns_plan_stats(const mwns_plan* pl, mwns_apply_stats* stats) {
    MWNS_GUARD_BEGIN
    if (!pl || !stats) fail(MWNS_EINVAL, "NULL argument");
    mwns_apply_stats s{};
    for (auto& a : pl->trees) collect_stats(pl->ctx, *a, pl->mode, s);
    *stats = s;
    return MWNS_OK;
    MWNS_GUARD_END
}

extern "C" void mwns_plan_destroy(mwns_plan* pl) { delete pl; }

extern "C" mwns_status mwns_tune_apply(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, int reps, int* best,
                                       double* times_ms) {
    MWNS_GUARD_BEGIN
    if (!ctx || !op || !f || !best) fail(MWNS_EINVAL, "NULL argument");
    if (reps < 1) fail(MWNS_EINVAL, "reps must be >= 1");
    std::vector<std::unique_ptr<TreeApply>> trees;
    trees.emplace_back(new TreeApply);
    DevArray<uint64_t> miss;
    prepare(ctx, trees, &op, &f, nullptr, true, miss);
    Launches Lz;
    build_launches(ctx, trees, false, Lz);
    launch_zero_outputs(ctx, *trees[0]);
    const int nv = f->k > KNARROW ? num_wide_variants() : num_variants();
    std::vector<double> t(nv, 0.0);
    Timer tm(ctx->stream);
    for (int v = 0; v < nv; ++v) {
        for (auto& g : Lz.groups) g.variant = v;
        launch_contractions(ctx, Lz);     // warm-up
        tm.start();
        for (int r = 0; r < reps; ++r) launch_contractions(ctx, Lz);
        tm.stop();
        t[v] = tm.ms() / reps;
    }
    int b = 0;
    for (int v = 1; v < nv; ++v)
        if (t[v] < t[b]) b = v;
    ctx->variant[f->k] = b;
    *best = b;
    if (times_ms) std::copy(t.begin(), t.end(), times_ms);
    return MWNS_OK;
    MWNS_GUARD_END
}
