/*
 * CPU oracle core (TEST INFRASTRUCTURE ONLY; never linked into the product).
 *
 * Plain, unblocked C for the two heavy oracle steps:
 *   - one level of the adaptive projection of a Gaussian-sum source   (Alg. 1, App. A.1 eq. fvals2coefs)
 *   - the modified ns-form apply per output node                       (eq. apply_algo, Alg. 3 Steps 1-3)
 *   - the banded difference form, used only to cross-check the above   (eqs. g_scales_band, sep_apply)
 * Keys: level << 57 | morton(lx, ly, lz), x in bit 0 of each bit triple; the tree is an array
 * of nodes sorted by key.  Coefficient blocks are [a][b][c] (a: x degree, b: y, c: z; c fastest).
 * Operator tables: F[j][m][l+7][a][b] with l = l_out - l_in and row a = output degree
 * (eq. KernelFactor).  Plan: R[j][L1+3][L2+3][L3+3][2] = inclusive term range, empty if m2 < m1.
 * All loops run in a fixed order; OpenMP only splits independent output nodes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LMAXF 7
#define NLF (2 * LMAXF + 1)
#define LMAXP 3
#define NLP (2 * LMAXP + 1)

/* ---------------------------------------------------------------- keys */
static uint64_t spread3(uint64_t v) {
    uint64_t r = 0;
    for (int i = 0; i < 19; ++i) r |= ((v >> i) & 1ull) << (3 * i);
    return r;
}
static uint64_t compact3(uint64_t v) {
    uint64_t r = 0;
    for (int i = 0; i < 19; ++i) r |= ((v >> (3 * i)) & 1ull) << i;
    return r;
}
static uint64_t make_key(int j, int64_t x, int64_t y, int64_t z) {
    return ((uint64_t)j << 57) | spread3((uint64_t)x) | (spread3((uint64_t)y) << 1) | (spread3((uint64_t)z) << 2);
}
static void decode_key(uint64_t key, int* j, int64_t* l) {
    uint64_t m = key & ((1ull << 57) - 1);
    *j = (int)(key >> 57);
    l[0] = (int64_t)compact3(m);
    l[1] = (int64_t)compact3(m >> 1);
    l[2] = (int64_t)compact3(m >> 2);
}
static int64_t find_key(int64_t n, const uint64_t* keys, uint64_t key) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == key) return mid;
        if (keys[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------- Legendre scaling fns */
/* phi_a(x) = sqrt(2a+1) P_a(2x-1) on [0,1] (App. A.1, eq. scalingFNC) */
static void phi_all(int k, double x, double* out) {
    double t = 2.0 * x - 1.0, p0 = 1.0, p1 = t;
    out[0] = 1.0;
    if (k > 1) out[1] = t;
    for (int a = 1; a + 1 < k; ++a) {
        double p2 = ((2 * a + 1) * t * p1 - a * p0) / (a + 1);
        out[a + 1] = p2;
        p0 = p1; p1 = p2;
    }
    for (int a = 0; a < k; ++a) out[a] *= sqrt(2.0 * a + 1.0);
}

/* y += s * (A1 (x) A2 (x) A3) x : mode products over the three indices of a k^3 block;
 * A_d is k x k with A_d[out][in]. */
static void apply3(int k, const double* A1, const double* A2, const double* A3, const double* x,
                   double s, double* y, double* t1, double* t2) {
    for (int c1 = 0; c1 < k; ++c1)
        for (int c2 = 0; c2 < k; ++c2)
            for (int a3 = 0; a3 < k; ++a3) {
                double acc = 0.0;
                for (int c3 = 0; c3 < k; ++c3) acc += A3[a3 * k + c3] * x[(c1 * k + c2) * k + c3];
                t1[(c1 * k + c2) * k + a3] = acc;
            }
    for (int c1 = 0; c1 < k; ++c1)
        for (int a2 = 0; a2 < k; ++a2)
            for (int a3 = 0; a3 < k; ++a3) {
                double acc = 0.0;
                for (int c2 = 0; c2 < k; ++c2) acc += A2[a2 * k + c2] * t1[(c1 * k + c2) * k + a3];
                t2[(c1 * k + a2) * k + a3] = acc;
            }
    for (int a1 = 0; a1 < k; ++a1)
        for (int a2 = 0; a2 < k; ++a2)
            for (int a3 = 0; a3 < k; ++a3) {
                double acc = 0.0;
                for (int c1 = 0; c1 < k; ++c1) acc += A1[a1 * k + c1] * t2[(c1 * k + a2) * k + a3];
                y[(a1 * k + a2) * k + a3] += s * acc;
            }
}

static void transpose(int k, const double* a, double* at) {
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) at[j * k + i] = a[i * k + j];
}

/* ------------------------------------------- Alg. 1: one level of boxes */
static double source_value(int nsrc, const double* xyz, const double* ex, const double* cf,
                           double x, double y, double z) {
    double f = 0.0;
    for (int i = 0; i < nsrc; ++i) {
        double dx = x - xyz[3 * i], dy = y - xyz[3 * i + 1], dz = z - xyz[3 * i + 2];
        f += cf[i] * exp(-ex[i] * (dx * dx + dy * dy + dz * dz));
    }
    return f;
}

/* For each candidate box at level j (keys[b]):
 *   s_out[b]  = its coefficients from the source values at its k^3 Gauss-Legendre nodes (eq. fvals2coefs, 3-D)
 *   err_out[b]= max over the 8 children and their k^3 nodes of |f - f~|, f~ interpolated from s (Alg. 1)
 *   refine[b] = (j < jmax) && err_out[b] > thr
 * gx, gw: k-point Gauss-Legendre nodes/weights on [0,1].  cf already contains the normalisation. */
int orc_project_level(int k, int j, int jmax, int64_t nbox, const uint64_t* keys,
                      int nsrc, const double* xyz, const double* ex, const double* cf, double thr,
                      const double* gx, const double* gw, double* s_out, uint8_t* refine, double* err_out) {
    const int k3 = k * k * k;
    double* P = (double*)malloc(sizeof(double) * k * k);        /* P[i][a]  = phi_a(x_i) w_i */
    double* Q = (double*)malloc(sizeof(double) * 2 * k * k);    /* Q[s][i][a] = phi_a((s + x_i)/2) */
    for (int i = 0; i < k; ++i) {
        double v[64];
        phi_all(k, gx[i], v);
        for (int a = 0; a < k; ++a) P[i * k + a] = v[a] * gw[i];
        for (int s = 0; s < 2; ++s) {
            phi_all(k, 0.5 * (s + gx[i]), v);
            for (int a = 0; a < k; ++a) Q[(s * k + i) * k + a] = v[a];
        }
    }
    double* Pt = (double*)malloc(sizeof(double) * k * k);       /* Pt[a][i] */
    transpose(k, P, Pt);
    const double h = ldexp(1.0, -j);
    const double norm_c = pow(2.0, -1.5 * j);   /* 2^{-3j/2} in eq. fvals2coefs (3-D) */
    const double norm_i = pow(2.0, 1.5 * j);    /* 2^{3j/2} in eq. func_interp (3-D)  */
#pragma omp parallel
    {
        double* fv = (double*)malloc(sizeof(double) * k3);
        double* t1 = (double*)malloc(sizeof(double) * k3);
        double* t2 = (double*)malloc(sizeof(double) * k3);
#pragma omp for schedule(dynamic, 4)
        for (int64_t b = 0; b < nbox; ++b) {
            int jj; int64_t l[3];
            decode_key(keys[b], &jj, l);
            /* source values at the box's own nodes */
            for (int i1 = 0; i1 < k; ++i1)
                for (int i2 = 0; i2 < k; ++i2)
                    for (int i3 = 0; i3 < k; ++i3)
                        fv[(i1 * k + i2) * k + i3] = source_value(nsrc, xyz, ex, cf,
                            h * (l[0] + gx[i1]), h * (l[1] + gx[i2]), h * (l[2] + gx[i3]));
            /* s_abc = 2^{-3j/2} sum_i f(x_i) phi_a(x_i1) w_i1 phi_b(x_i2) w_i2 phi_c(x_i3) w_i3 */
            double* s = s_out + b * k3;
            memset(s, 0, sizeof(double) * k3);
            apply3(k, Pt, Pt, Pt, fv, norm_c, s, t1, t2);
            /* interpolate to every child's nodes and compare with direct values */
            double emax = 0.0;
            if (j < jmax) {
                double* ft = (double*)malloc(sizeof(double) * k3);
                for (int sg = 0; sg < 8; ++sg) {
                    int sx = sg & 1, sy = (sg >> 1) & 1, sz = (sg >> 2) & 1;
                    memset(ft, 0, sizeof(double) * k3);
                    apply3(k, Q + sx * k * k, Q + sy * k * k, Q + sz * k * k, s, norm_i, ft, t1, t2);
                    const double hc = 0.5 * h;
                    for (int i1 = 0; i1 < k; ++i1)
                        for (int i2 = 0; i2 < k; ++i2)
                            for (int i3 = 0; i3 < k; ++i3) {
                                double fx = source_value(nsrc, xyz, ex, cf,
                                    hc * (2 * l[0] + sx + gx[i1]), hc * (2 * l[1] + sy + gx[i2]),
                                    hc * (2 * l[2] + sz + gx[i3]));
                                double e = fabs(fx - ft[(i1 * k + i2) * k + i3]);
                                if (e > emax) emax = e;
                            }
                }
                free(ft);
            }
            err_out[b] = emax;
            refine[b] = (uint8_t)((j < jmax) && (emax > thr));
        }
        free(fv); free(t1); free(t2);
    }
    free(P); free(Q); free(Pt);
    return 0;
}

/* -------------------------------------------------------- input boxes */
/* f_{(j,l)} from the redundant tree, or, when the box is not a node, by zero-detail upsampling
 * from its deepest existing ancestor (Alg. 3 Step 2; eq. recon_even/odd with d = 0).
 * Returns 0 on success, -1 if the box is outside [0,2^j)^3, -2 on a malformed tree. */
static int input_block(int k, int64_t N, const uint64_t* keys, const uint8_t* leaf, const double* coef,
                       const double* H0, const double* H1, int j, const int64_t* l,
                       double* out, double* tmp, double* t1, double* t2) {
    const int k3 = k * k * k;
    int64_t side = (int64_t)1 << j;
    for (int d = 0; d < 3; ++d) if (l[d] < 0 || l[d] >= side) return -1;
    int64_t idx = find_key(N, keys, make_key(j, l[0], l[1], l[2]));
    if (idx >= 0) { memcpy(out, coef + idx * k3, sizeof(double) * k3); return 0; }
    int i = j - 1;
    for (; i >= 0; --i) {
        idx = find_key(N, keys, make_key(i, l[0] >> (j - i), l[1] >> (j - i), l[2] >> (j - i)));
        if (idx >= 0) break;
    }
    if (i < 0 || !leaf[idx]) return -2;
    double H0t[400], H1t[400];
    transpose(k, H0, H0t);
    transpose(k, H1, H1t);
    memcpy(out, coef + idx * k3, sizeof(double) * k3);
    for (int t = i + 1; t <= j; ++t) {
        const double* A[3];
        for (int d = 0; d < 3; ++d) A[d] = ((l[d] >> (j - t)) & 1) ? H1t : H0t;
        memset(tmp, 0, sizeof(double) * k3);
        apply3(k, A[0], A[1], A[2], out, 1.0, tmp, t1, t2);
        memcpy(out, tmp, sizeof(double) * k3);
    }
    return 0;
}

static const int32_t* plan_at(const int32_t* R, int nlevR, int j, const int64_t* L) {
    if (j >= nlevR) return NULL;
    for (int d = 0; d < 3; ++d) if (L[d] < -LMAXP || L[d] > LMAXP) return NULL;
    return R + ((((int64_t)j * NLP + (L[0] + LMAXP)) * NLP + (L[1] + LMAXP)) * NLP + (L[2] + LMAXP)) * 2;
}

/* ---------------------------------------------- modified ns-form apply */
/* ghat for each requested output node (eq. apply_algo, Alg. 3 Steps 1-3).  For output node b at
 * level j and input b' = b - ell (inside the unit cube) with coarse displacement
 * L = (b >> 1) - (b' >> 1), term m carries the coefficient
 *     c_m = [m in R_j(L)] - [b internal] [m in R_{j+1}(ell)]
 * (whole band at leaves; the band of scale j minus the down-sampled band of scale j+1 at
 * internal nodes).  R_j is empty beyond |L_d| <= 3 and for j beyond the plan; at the root
 * L = 0 and R_0(0) holds every term.  Contributions are summed with ell lexicographic
 * (ell_1 slowest) and m ascending. */
int orc_apply_modified(int k, int64_t N, const uint64_t* keys, const uint8_t* leaf, const double* coef,
                       int M, const double* w, int nlevF, const double* F, int nlevR, const int32_t* R,
                       const double* H0, const double* H1, int64_t nout, const int64_t* out_idx,
                       double* ghat) {
    const int k3 = k * k * k, kk = k * k;
    int status = 0;
#pragma omp parallel
    {
        double* x = (double*)malloc(sizeof(double) * k3);
        double* tmp = (double*)malloc(sizeof(double) * k3);
        double* t1 = (double*)malloc(sizeof(double) * k3);
        double* t2 = (double*)malloc(sizeof(double) * k3);
        int* cm = (int*)malloc(sizeof(int) * M);
#pragma omp for schedule(dynamic, 1)
        for (int64_t o = 0; o < nout; ++o) {
            int64_t b = out_idx[o];
            int j; int64_t l[3];
            decode_key(keys[b], &j, l);
            double* y = ghat + o * k3;
            memset(y, 0, sizeof(double) * k3);
            if (j >= nlevF) { status = -3; continue; }
            for (int e1 = -LMAXF; e1 <= LMAXF; ++e1)
                for (int e2 = -LMAXF; e2 <= LMAXF; ++e2)
                    for (int e3 = -LMAXF; e3 <= LMAXF; ++e3) {
                        int64_t ell[3] = {e1, e2, e3};
                        int64_t lp[3] = {l[0] - e1, l[1] - e2, l[2] - e3};
                        int64_t side = (int64_t)1 << j;
                        if (lp[0] < 0 || lp[0] >= side || lp[1] < 0 || lp[1] >= side || lp[2] < 0 || lp[2] >= side)
                            continue;
                        int64_t L[3];
                        for (int d = 0; d < 3; ++d) L[d] = (l[d] >> 1) - (lp[d] >> 1);
                        const int32_t* wr = plan_at(R, nlevR, j, L);
                        const int32_t* dr = leaf[b] ? NULL : plan_at(R, nlevR, j + 1, ell);
                        int any = 0;
                        for (int m = 0; m < M; ++m) {
                            int c = 0;
                            if (wr && m >= wr[0] && m <= wr[1]) c += 1;
                            if (dr && m >= dr[0] && m <= dr[1]) c -= 1;
                            cm[m] = c;
                            any |= c;
                        }
                        if (!any) continue;
                        int st = input_block(k, N, keys, leaf, coef, H0, H1, j, lp, x, tmp, t1, t2);
                        if (st == -2) { status = -2; continue; }
                        for (int m = 0; m < M; ++m) {
                            if (!cm[m]) continue;
                            const double* Fj = F + ((int64_t)j * M + m) * NLF * kk;
                            apply3(k, Fj + (e1 + LMAXF) * kk, Fj + (e2 + LMAXF) * kk, Fj + (e3 + LMAXF) * kk,
                                   x, cm[m] * w[m], y, t1, t2);
                        }
                    }
        }
        free(x); free(tmp); free(t1); free(t2); free(cm);
    }
    return status;
}

/* --------------------------------------------- banded difference form */
/* ghat^D for each requested node: at level j >= 1, for every in-domain input b - ell with coarse
 * L and m in R_j(L):  w_m (F1 (x) F2 (x) F3 - G1 (x) G2 (x) G3) f_{b-ell},
 * G_d = H^{s_d}^T F^{j-1;m,L_d} H^{s'_d} with s = output parity, s' = input parity (the upsampled
 * coarse block, eq. sep_apply); at the root every term of T_0 (eq. g_scales_band). */
int orc_apply_difference(int k, int64_t N, const uint64_t* keys, const uint8_t* leaf, const double* coef,
                         int M, const double* w, int nlevF, const double* F, int nlevR, const int32_t* R,
                         const double* H0, const double* H1, int64_t nout, const int64_t* out_idx,
                         double* ghat) {
    const int k3 = k * k * k, kk = k * k;
    int status = 0;
#pragma omp parallel
    {
        double* x = (double*)malloc(sizeof(double) * k3);
        double* tmp = (double*)malloc(sizeof(double) * k3);
        double* t1 = (double*)malloc(sizeof(double) * k3);
        double* t2 = (double*)malloc(sizeof(double) * k3);
        double G[3][400], T[400];
        const double* Hs[2] = {H0, H1};
#pragma omp for schedule(dynamic, 1)
        for (int64_t o = 0; o < nout; ++o) {
            int64_t b = out_idx[o];
            int j; int64_t l[3];
            decode_key(keys[b], &j, l);
            double* y = ghat + o * k3;
            memset(y, 0, sizeof(double) * k3);
            if (j >= nlevF) { status = -3; continue; }
            if (j == 0) {
                const double* F0 = F;
                for (int m = 0; m < M; ++m)
                    apply3(k, F0 + (m * NLF + LMAXF) * kk, F0 + (m * NLF + LMAXF) * kk, F0 + (m * NLF + LMAXF) * kk,
                           coef + b * k3, w[m], y, t1, t2);
                continue;
            }
            for (int e1 = -LMAXF; e1 <= LMAXF; ++e1)
                for (int e2 = -LMAXF; e2 <= LMAXF; ++e2)
                    for (int e3 = -LMAXF; e3 <= LMAXF; ++e3) {
                        int64_t lp[3] = {l[0] - e1, l[1] - e2, l[2] - e3};
                        int64_t side = (int64_t)1 << j;
                        if (lp[0] < 0 || lp[0] >= side || lp[1] < 0 || lp[1] >= side || lp[2] < 0 || lp[2] >= side)
                            continue;
                        int64_t L[3];
                        for (int d = 0; d < 3; ++d) L[d] = (l[d] >> 1) - (lp[d] >> 1);
                        const int32_t* wr = plan_at(R, nlevR, j, L);
                        if (!wr || wr[1] < wr[0]) continue;
                        int st = input_block(k, N, keys, leaf, coef, H0, H1, j, lp, x, tmp, t1, t2);
                        if (st == -2) { status = -2; continue; }
                        for (int m = wr[0]; m <= wr[1]; ++m) {
                            const double* Fj = F + ((int64_t)j * M + m) * NLF * kk;
                            const double* Fc = F + ((int64_t)(j - 1) * M + m) * NLF * kk;
                            apply3(k, Fj + (e1 + LMAXF) * kk, Fj + (e2 + LMAXF) * kk, Fj + (e3 + LMAXF) * kk,
                                   x, w[m], y, t1, t2);
                            for (int d = 0; d < 3; ++d) {
                                const double* Hs_out = Hs[l[d] & 1];
                                const double* Hs_in = Hs[lp[d] & 1];
                                const double* Fl = Fc + (L[d] + LMAXF) * kk;
                                /* T = F^{j-1} H^{s'} ; G = H^{s}^T T */
                                for (int a = 0; a < k; ++a)
                                    for (int c = 0; c < k; ++c) {
                                        double acc = 0.0;
                                        for (int q = 0; q < k; ++q) acc += Fl[a * k + q] * Hs_in[q * k + c];
                                        T[a * k + c] = acc;
                                    }
                                for (int a = 0; a < k; ++a)
                                    for (int c = 0; c < k; ++c) {
                                        double acc = 0.0;
                                        for (int q = 0; q < k; ++q) acc += Hs_out[q * k + a] * T[q * k + c];
                                        G[d][a * k + c] = acc;
                                    }
                            }
                            apply3(k, G[0], G[1], G[2], x, -w[m], y, t1, t2);
                        }
                    }
        }
        free(x); free(tmp); free(t1); free(t2);
    }
    return status;
}
