// Operator construction: the 1-D blocks F^{j;m,l} (eq. KernelFactor) and the screening plan
// (Sec. 4) on the device.
//
// F^{j;m,l}_ab = 2^-j int_{-1}^{1} exp(-beta (x+l)^2) Phi_ab(x) dx, beta = tau_m / 4^j.  On [0,1],
// Phi^+_ab = sum_{n<2k} C_abn phi_n (App. A.4: Phi^+ is a polynomial of degree <= 2k-1), and
// Phi^-_ab(-x) = (-1)^{a+b} Phi^+_ab(x) (Prop. 1, item 2) folds [-1,0] onto [0,1], so
//   F^{j;m,l}_ab = 2^-j sum_n C_abn (I_n(l) + (-1)^{a+b} I_n(-l)),
//   I_n(l) = int_0^1 exp(-beta (x+l)^2) phi_n(x) dx,
// which needs 2k Gaussian moments per (j, m, l) instead of k^2 integrals.  The moments use a
// composite 24-point Gauss-Legendre rule on panels graded around the point of [0,1] nearest to the
// Gaussian centre -l (widths 2^q / sqrt(beta)), plus a uniform split of [0,1] in eighths.
//
// Screening: for scale j >= 1, term m and coarse |L| = 0..3 the kernels form the 2k x 2k
// super-blocks S = [[F^{2L}, F^{2L-1}], [F^{2L+1}, F^{2L}]] and U = [H0 H1]^T F^{j-1;L} [H0 H1] and
// their Frobenius norms N_F, N_upF, N_dif (eq. BlockNorms); the plan kernel combines them into the
// 3-D estimate (eq. NormEstimateUsing1DBlocks) for each of the 20 classes of sorted |L| and keeps
// the term range left after discarding the longest prefix and suffix whose cumulative weighted
// estimate stays <= theta/2 (empty if the total is <= theta), theta = eps sum_m w_m ||F^{0;m,0}||_F^3.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "mwns_internal.h"

namespace mwns {
namespace {

constexpr int NGL = 24;          // points per panel
constexpr int MAXBRK = 40;       // panel end points per integral
constexpr int MOMW = 64;         // threads per moment block

// One block per (j, m, l).  The panel end points are the distinct values among 0, 1, the eighths
// and p -+ s 2^q inside (0, 1); every candidate is placed by its rank, then repeats are dropped.
template <int K>
__global__ void __launch_bounds__(MOMW) moments_kernel(int M, const double* __restrict__ tau,
                                                       const double* __restrict__ glx, const double* __restrict__ glw,
                                                       double* __restrict__ mom /* [nlev][M][NLF][2k] */) {
    constexpr int K2 = 2 * K;
    constexpr int NCAND = 9 + 20;     // 0, 1, i/8 (i = 1..7), p - s 2^q and p + s 2^q (q = -3..6)
    static_assert(NCAND <= MOMW && NCAND <= MAXBRK, "one candidate per thread");
    const int blk = blockIdx.x;
    const int li = blk % NLF;
    const int m = (blk / NLF) % M;
    const int j = blk / (NLF * M);
    const int tid = threadIdx.x;
    const double l = (double)(li - LF);
    const double beta = tau[m] * ldexp(1.0, -2 * j);
    __shared__ double cand[NCAND];    // -1 marks a candidate outside (0, 1)
    __shared__ double srt[NCAND];
    __shared__ double brk[MAXBRK];
    __shared__ int nbrk;
    __shared__ double part[MOMW][K2];
    if (tid < NCAND) {
        double v;
        if (tid == 0) v = 0.0;
        else if (tid == 1) v = 1.0;
        else if (tid < 9) v = (tid - 1) / 8.0;
        else {
            const double c = -l;
            const double p = c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
            const double sc = 1.0 / sqrt(beta);
            const double d = sc * ldexp(1.0, (tid - 9) / 2 - 3);
            v = (tid - 9) % 2 == 0 ? p - d : p + d;
            if (!(v > 0.0 && v < 1.0)) v = -1.0;
        }
        cand[tid] = v;
    }
    __syncthreads();
    if (tid < NCAND && cand[tid] >= 0.0) {
        const double v = cand[tid];
        int rank = 0;
        for (int u = 0; u < NCAND; ++u) {
            const double w = cand[u];
            rank += (w >= 0.0) && (w < v || (w == v && u < tid));
        }
        srt[rank] = v;
    }
    __syncthreads();
    if (tid == 0) {
        int nv = 0;
        for (int u = 0; u < NCAND; ++u) nv += cand[u] >= 0.0;
        int n = 0;
        for (int a = 0; a < nv; ++a)
            if (n == 0 || srt[a] > brk[n - 1]) brk[n++] = srt[a];
        nbrk = n;
    }
    __syncthreads();
    double acc[K2];
#pragma unroll
    for (int n = 0; n < K2; ++n) acc[n] = 0.0;
    const int npts = (nbrk - 1) * NGL;
    for (int pt = tid; pt < npts; pt += MOMW) {
        const int pan = pt / NGL, g = pt % NGL;
        const double a = brk[pan], b = brk[pan + 1];
        const double x = a + (b - a) * glx[g];
        const double wt = (b - a) * glw[g] * exp(-beta * (x + l) * (x + l));
        // phi_n(x) = sqrt(2n+1) P_n(2x-1) by the three-term recurrence
        const double t = 2.0 * x - 1.0;
        double p0 = 1.0, p1 = t;
        acc[0] += wt;
        if (K2 > 1) acc[1] += wt * t * 1.7320508075688772;
#pragma unroll
        for (int n = 2; n < K2; ++n) {
            double p2 = ((2 * n - 1) * t * p1 - (n - 1) * p0) / n;
            acc[n] += wt * p2 * sqrt(2.0 * n + 1.0);
            p0 = p1;
            p1 = p2;
        }
    }
#pragma unroll
    for (int n = 0; n < K2; ++n) part[tid][n] = acc[n];
    __syncthreads();
    if (tid < K2) {
        double s = 0.0;
        for (int r = 0; r < MOMW; ++r) s += part[r][tid];
        mom[(int64_t)blk * K2 + tid] = s;
    }
}

template <int K>
void launch_moments(int nlev, int M, const double* tau, const double* gx, const double* gw, double* mom, hipStream_t st) {
    moments_kernel<K><<<nlev * M * NLF, MOMW, 0, st>>>(M, tau, gx, gw, mom);
}

__global__ void combine_kernel(int k, int M, int nlev, const double* __restrict__ C, const double* __restrict__ mom,
                               double* __restrict__ F /* [nlev][M][NLF][k][k] */) {
    const int64_t total = (int64_t)nlev * M * NLF * k * k;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int b = idx % k;
    const int a = (idx / k) % k;
    const int li = (idx / (k * k)) % NLF;
    const int64_t jm = idx / ((int64_t)k * k * NLF);   // j * M + m
    const int j = (int)(jm / M);
    const int K2 = 2 * k;
    const double* mp = mom + (jm * NLF + li) * K2;
    const double* mm = mom + (jm * NLF + (2 * LF - li)) * K2;   // I_n(-l)
    const double sg = ((a + b) & 1) ? -1.0 : 1.0;
    const double* c = C + (a * k + b) * K2;
    double s = 0.0;
    for (int n = 0; n < K2; ++n) s += c[n] * (mp[n] + sg * mm[n]);
    F[idx] = ldexp(s, -j);
}

// Frobenius norms of the super-blocks for scales 1..nlev-1, |L| = 0..LP: one 64-lane block per
// (j, m, L), lane e owns entries e, e+64, .. of each of the four k x k sub-blocks; U is formed as
// H^{so T} (F^{j-1;m,L} H^{si}).  Block 0 of the grid also writes nf0[m] = ||F^{0;m,0}||_F.
__global__ void __launch_bounds__(64) norms_kernel(int k, int M, int nlev, const double* __restrict__ F,
                                                   const double* __restrict__ H, double* __restrict__ norms,
                                                   double* __restrict__ nf0) {
    const int kk = k * k;
    const int nL = LP + 1;
    const int lane = threadIdx.x;
    __shared__ double Hs[2 * KMAX * KMAX], Fc[KMAX * KMAX], T[2][KMAX * KMAX], red[3][64];
    if (blockIdx.x == (unsigned)((nlev - 1) * M * nL)) {    // the extra last block: nf0
        for (int m = lane; m < M; m += 64) {
            const double* f = F + ((int64_t)m * NLF + LF) * kk;
            double s = 0.0;
            for (int i = 0; i < kk; ++i) s += f[i] * f[i];
            nf0[m] = sqrt(s);
        }
        return;
    }
    const int L = blockIdx.x % nL;
    const int m = (blockIdx.x / nL) % M;
    const int j = 1 + blockIdx.x / (nL * M);
    const double* Fj = F + ((int64_t)j * M + m) * NLF * kk;
    const double* Fcg = F + ((int64_t)(j - 1) * M + m) * NLF * kk + (L + LF) * kk;
    for (int e = lane; e < 2 * kk; e += 64) Hs[e] = H[e];
    for (int e = lane; e < kk; e += 64) Fc[e] = Fcg[e];
    __syncthreads();
    // lane owns the entries (a, b) = divmod(e, k) for e = lane, lane + 64, ... (one entry for k <= 8)
    for (int e = lane; e < kk; e += 64) {
        const int a = e / k, b = e % k;
        for (int si = 0; si < 2; ++si) {            // T[si][a][b] = sum_q F[a][q] H^si[q][b]
            double t = 0.0;
            for (int q = 0; q < k; ++q) t += Fc[a * k + q] * Hs[si * kk + q * k + b];
            T[si][a * k + b] = t;
        }
    }
    __syncthreads();
    double sF = 0.0, sU = 0.0, sD = 0.0;
    for (int e = lane; e < kk; e += 64) {
        const int a = e / k, b = e % k;
        for (int so = 0; so < 2; ++so)
            for (int si = 0; si < 2; ++si) {
                double u = 0.0;                     // (H^so^T F^{j-1;L} H^si)_ab
                for (int p = 0; p < k; ++p) u += Hs[so * kk + p * k + a] * T[si][p * k + b];
                const double f = Fj[(2 * L + so - si + LF) * kk + a * k + b];
                sF += f * f;
                sU += u * u;
                sD += (f - u) * (f - u);
            }
    }
    red[0][lane] = sF;
    red[1][lane] = sU;
    red[2][lane] = sD;
    __syncthreads();
    if (lane < 3) {
        double s = 0.0;
        for (int i = 0; i < 64; ++i) s += red[lane][i];
        norms[(((int64_t)j * M + m) * nL + L) * 3 + lane] = sqrt(s);
    }
}

// Frobenius norm of every block F^{j;m,l}, one thread per (j, m, l); used to bound the rounding
// error of reduced-precision contractions.
__global__ void fro_kernel(int k, int64_t n, const double* __restrict__ F, double* __restrict__ fro) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* f = F + i * k * k;
    double s = 0.0;
    for (int e = 0; e < k * k; ++e) s += f[e] * f[e];
    fro[i] = sqrt(s);
}

// One thread per (scale j >= 1, canonical class (c0 <= c1 <= c2)): term range.
// One wave per (level j >= 1, class of sorted |L|): the lanes evaluate the weighted estimates of 64
// terms at a time into LDS and lane 0 forms the prefix and suffix sums in term order.
__global__ void __launch_bounds__(64) plan_kernel(int M, double eps, const double* __restrict__ w,
                                                  const double* __restrict__ norms, const double* __restrict__ nf0,
                                                  int32_t* __restrict__ ranges /* [nlev][20][2] */) {
    const int idx = blockIdx.x;
    const int lane = threadIdx.x;
    const int cls = idx % 20;
    const int j = 1 + idx / 20;
    int c[3] = {0, 0, 0}, cnt = 0;
    for (int a = 0; a <= LP; ++a)
        for (int b = a; b <= LP; ++b)
            for (int d = b; d <= LP; ++d) {
                if (cnt == cls) { c[0] = a; c[1] = b; c[2] = d; }
                ++cnt;
            }
    double theta = 0.0;
    for (int m = 0; m < M; ++m) theta += w[m] * nf0[m] * nf0[m] * nf0[m];
    theta *= eps;
    const int nL = LP + 1;
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    auto e_of = [&](int m) {
        const double* nb = norms + ((int64_t)j * M + m) * nL * 3;
        double tot = 0.0;
        for (int q = 0; q < 6; ++q) {
            const double* P = nb + c[perm[q][0]] * 3;
            const double* Q = nb + c[perm[q][1]] * 3;
            const double* R = nb + c[perm[q][2]] * 3;
            // N_dif N_F N_F + N_upF N_dif N_F + N_upF N_upF N_dif
            tot += P[2] * Q[0] * R[0] + P[1] * Q[2] * R[0] + P[1] * Q[1] * R[2];
        }
        return w[m] * (tot / 6.0);
    };
    __shared__ double est[64];
    __shared__ int flag;
    double total = 0.0;
    int m1 = -1;
    for (int m0 = 0; m0 < M; m0 += 64) {
        if (m0 + lane < M) est[lane] = e_of(m0 + lane);
        __syncthreads();
        if (lane == 0)
            for (int u = 0; u < min(64, M - m0); ++u) {
                total += est[u];
                if (m1 < 0 && total > 0.5 * theta) m1 = m0 + u;
            }
        __syncthreads();
    }
    int32_t* out = ranges + (int64_t)idx * 2;
    if (lane == 0) flag = total <= theta;
    __syncthreads();
    if (flag) {
        if (lane == 0) { out[0] = 0; out[1] = -1; }
        return;
    }
    double suf = 0.0;
    int m2 = M - 1;
    for (int m0 = ((M - 1) / 64) * 64; m0 >= 0; m0 -= 64) {
        if (m0 + lane < M) est[lane] = e_of(m0 + lane);
        __syncthreads();
        if (lane == 0) {
            flag = 0;
            for (int u = min(64, M - m0) - 1; u >= 0; --u) {
                suf += est[u];
                if (suf > 0.5 * theta) { m2 = m0 + u; flag = 1; break; }
            }
        }
        __syncthreads();
        if (flag) break;
    }
    if (lane == 0) {
        out[0] = m1;
        out[1] = m2;
    }
}

int class_index(int a, int b, int c) {   // a <= b <= c
    int cnt = 0;
    for (int x = 0; x <= LP; ++x)
        for (int y = x; y <= LP; ++y)
            for (int z = y; z <= LP; ++z) {
                if (x == a && y == b && z == c) return cnt;
                ++cnt;
            }
    return -1;
}

}  // namespace
}  // namespace mwns

using namespace mwns;

extern "C" {

mwns_status mwns_op_create(mwns_ctx* ctx, int k, int M, const double* tau, const double* w, double eps, int max_level,
                           const mwns_op_opts* opts, mwns_op** out) {
    MWNS_GUARD_BEGIN
    if (!ctx || !out || !tau || !w) fail(MWNS_EINVAL, "NULL argument");
    if (k < 1 || k > KMAX) fail(MWNS_EINVAL, "k must be in [1, " + std::to_string(KMAX) + "]");
    if (M < 1 || max_level < 0 || max_level > MAXLEV || !(eps > 0.0)) fail(MWNS_EINVAL, "M, max_level or eps out of range");
    for (int m = 0; m < M; ++m)
        if (!(tau[m] > 0.0) || !(w[m] >= 0.0) || !std::isfinite(tau[m]) || !std::isfinite(w[m]))
            fail(MWNS_EINVAL, "tau must be > 0 and w >= 0, finite");
    std::unique_ptr<mwns_op> op(new mwns_op);
    op->ctx = ctx;
    op->hold.set(ctx);
    op->k = k;
    op->M = M;
    op->max_level = max_level;
    op->eps = eps;
    op->group = opts ? (opts->group_regions != 0) : 1;
    op->tau.assign(tau, tau + M);
    op->w.assign(w, w + M);
    const int nlev = max_level + 1;
    const int K2 = 2 * k;
    hipStream_t st = ctx->stream;
    // tables
    std::vector<double> C(k * k * K2);
    crosscorr_plus_coeffs(k, C.data());
    Quad gl = gauss_legendre01(NGL);
    DevArray<double> dC(ctx, C.size()), dtau(ctx, M), dgx(ctx, NGL), dgw(ctx, NGL);
    dC.upload(C.data(), C.size(), st);
    dtau.upload(tau, M, st);
    dgx.upload(gl.x.data(), NGL, st);
    dgw.upload(gl.w.data(), NGL, st);
    op->dw.reset(ctx, M);
    op->dw.upload(w, M, st);
    DevArray<double> mom(ctx, (size_t)nlev * M * NLF * K2);
    op->F.reset(ctx, (size_t)nlev * M * NLF * k * k);
    switch (k) {
        case 1: launch_moments<1>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 2: launch_moments<2>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 3: launch_moments<3>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 4: launch_moments<4>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 5: launch_moments<5>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 6: launch_moments<6>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 7: launch_moments<7>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 8: launch_moments<8>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 9: launch_moments<9>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        case 10: launch_moments<10>(nlev, M, dtau.p, dgx.p, dgw.p, mom.p, st); break;
        default: fail(MWNS_EINVAL, "unsupported k");
    }
    MWNS_HIP(hipGetLastError());
    const int64_t nF = (int64_t)nlev * M * NLF * k * k;
    combine_kernel<<<(unsigned)((nF + 255) / 256), 256, 0, st>>>(k, M, nlev, dC.p, mom.p, op->F.p);
    MWNS_HIP(hipGetLastError());
    // screening
    DevArray<double> dH = upload_filters(ctx, k);
    const int nL = LP + 1;
    DevArray<double> norms(ctx, (size_t)nlev * M * nL * 3), nf0(ctx, M);
    norms_kernel<<<(nlev - 1) * M * nL + 1, 64, 0, st>>>(k, M, nlev, op->F.p, dH.p, norms.p, nf0.p);
    MWNS_HIP(hipGetLastError());
    // the plan's ranges, the terms' norms and the blocks' Frobenius norms come down together
    // through the context's pinned staging block, behind one synchronisation
    std::vector<int32_t> ranges(std::max(1, (nlev - 1) * 20) * 2);
    const int64_t nb = (int64_t)nlev * M * NLF;
    const size_t b_rng = (ranges.size() * sizeof(int32_t) + 7) & ~(size_t)7;
    char* pin = static_cast<char*>(pinned_staging(ctx, b_rng + (size_t)(M + nb) * sizeof(double)));
    double* pin_nf0 = reinterpret_cast<double*>(pin + b_rng);
    double* pin_fro = pin_nf0 + M;
    DevArray<int32_t> dr(ctx, ranges.size());
    if (nlev > 1) {
        plan_kernel<<<(nlev - 1) * 20, 64, 0, st>>>(M, eps, op->dw.p, norms.p, nf0.p, dr.p);
        MWNS_HIP(hipGetLastError());
        MWNS_HIP(hipMemcpyAsync(pin, dr.p, ranges.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    MWNS_HIP(hipMemcpyAsync(pin_nf0, nf0.p, M * sizeof(double), hipMemcpyDeviceToHost, st));
    DevArray<double> dfro(ctx, nb);
    fro_kernel<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(k, nb, op->F.p, dfro.p);
    MWNS_HIP(hipGetLastError());
    MWNS_HIP(hipMemcpyAsync(pin_fro, dfro.p, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    MWNS_HIP(hipStreamSynchronize(st));
    if (nlev > 1) std::memcpy(ranges.data(), pin, ranges.size() * sizeof(int32_t));
    // band overflow: a term kept at the edge of the band (max |L_d| = LP) means that the
    // displacements beyond it, which the plan cannot hold, would still contribute
    if (!(opts && opts->allow_band_overflow))
        for (int j = 1; j < nlev; ++j)
            for (int a = 0; a <= LP; ++a)
                for (int b = a; b <= LP; ++b)
                    for (int c = b; c <= LP; ++c) {
                        if (c < LP) continue;
                        const int32_t* r = ranges.data() + (size_t)(j - 1) * 40 + class_index(a, b, c) * 2;
                        if (r[1] >= r[0])
                            fail(MWNS_ERANGE, "band overflow: level " + std::to_string(j) + " keeps terms " +
                                                  std::to_string(r[0]) + ".." + std::to_string(r[1]) + " at |L| = (" +
                                                  std::to_string(a) + "," + std::to_string(b) + "," + std::to_string(c) +
                                                  "), the edge of the band |L_d| <= 3");
                    }
    std::vector<double> hnf0(pin_nf0, pin_nf0 + M);
    op->fro.assign(pin_fro, pin_fro + nb);
    double theta = 0.0;
    for (int m = 0; m < M; ++m) theta += w[m] * hnf0[m] * hnf0[m] * hnf0[m];
    op->theta = theta * eps;
    // expand to [nlev][7][7][7][2] (grouping: hull of the ranges of Core / Boundary-1/2/3)
    op->plan.assign((size_t)nlev * NLP3 * 2, 0);
    for (size_t i = 1; i < op->plan.size(); i += 2) op->plan[i] = -1;
    const int root = ((LP * NLP) + LP) * NLP + LP;
    op->plan[root * 2] = 0;
    op->plan[root * 2 + 1] = M - 1;
    for (int j = 1; j < nlev; ++j) {
        const int32_t* rj = ranges.data() + (size_t)(j - 1) * 40;
        int hull[4][2];
        for (int g = 0; g < 4; ++g) { hull[g][0] = M; hull[g][1] = -1; }
        for (int a = 0; a <= LP; ++a)
            for (int b = a; b <= LP; ++b)
                for (int c = b; c <= LP; ++c) {
                    int ci = class_index(a, b, c);
                    int g = (a > 1) + (b > 1) + (c > 1);
                    if (rj[ci * 2 + 1] >= rj[ci * 2]) {
                        hull[g][0] = std::min(hull[g][0], rj[ci * 2]);
                        hull[g][1] = std::max(hull[g][1], rj[ci * 2 + 1]);
                    }
                }
        for (int x = -LP; x <= LP; ++x)
            for (int y = -LP; y <= LP; ++y)
                for (int z = -LP; z <= LP; ++z) {
                    int s[3] = {std::abs(x), std::abs(y), std::abs(z)};
                    std::sort(s, s + 3);
                    int ci = class_index(s[0], s[1], s[2]);
                    int g = (s[0] > 1) + (s[1] > 1) + (s[2] > 1);
                    int m1 = rj[ci * 2], m2 = rj[ci * 2 + 1];
                    if (op->group) {
                        if (hull[g][1] >= hull[g][0]) { m1 = hull[g][0]; m2 = hull[g][1]; }
                        else { m1 = 0; m2 = -1; }
                    }
                    size_t o = (((size_t)j * NLP3) + ((x + LP) * NLP + (y + LP)) * NLP + (z + LP)) * 2;
                    op->plan[o] = m1;
                    op->plan[o + 1] = m2;
                }
    }
    *out = op.release();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_op_plan_export(const mwns_op* op, int32_t* plan, size_t* count) {
    MWNS_GUARD_BEGIN
    if (!op || !count) fail(MWNS_EINVAL, "NULL argument");
    if (!plan) { *count = op->plan.size(); return MWNS_OK; }
    if (*count < op->plan.size()) {
        *count = op->plan.size();
        fail(MWNS_ERANGE, "plan buffer too small");
    }
    std::copy(op->plan.begin(), op->plan.end(), plan);
    *count = op->plan.size();
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_op_plan_import(mwns_op* op, const int32_t* plan, size_t count) {
    MWNS_GUARD_BEGIN
    if (!op || !plan) fail(MWNS_EINVAL, "NULL argument");
    if (count != op->plan.size()) fail(MWNS_EINVAL, "plan size mismatch");
    for (size_t i = 0; i < count; i += 2) {
        int32_t a = plan[i], b = plan[i + 1];
        if (b >= a && (a < 0 || b >= op->M)) fail(MWNS_EINVAL, "plan range outside [0, M)");
    }
    op->plan.assign(plan, plan + count);
    return MWNS_OK;
    MWNS_GUARD_END
}

mwns_status mwns_op_tables_export(mwns_ctx* ctx, const mwns_op* op, double* F, size_t* count) {
    MWNS_GUARD_BEGIN
    if (!ctx || !op || !count) fail(MWNS_EINVAL, "NULL argument");
    const size_t n = op->F.n;
    if (!F) { *count = n; return MWNS_OK; }
    if (*count < n) {
        *count = n;
        fail(MWNS_ERANGE, "table buffer too small");
    }
    op->F.download(F, n, ctx->stream);
    MWNS_HIP(hipStreamSynchronize(ctx->stream));
    *count = n;
    return MWNS_OK;
    MWNS_GUARD_END
}

double mwns_op_threshold(const mwns_op* op) { return op ? op->theta : 0.0; }

void mwns_op_destroy(mwns_op* op) { delete op; }

}  // extern "C"
