/* The oracle's plain-C core run under AddressSanitizer and UndefinedBehaviorSanitizer: reads one
 * case written by the Python side (a redundant tree, operator tables, a plan, filters and a
 * projection level), runs the three entry points and writes their outputs for comparison with
 * the regular build.  Binary layout of the input file (native endianness): int32 k, nlevF,
 * nlevR, M, int64 N, nout, nbox, nsrc, j; then keys[N] u64, leaf[N] u8, coef[N k^3] f64,
 * w[M], F[nlevF M 15 k k], R[nlevR 7 7 7 2] i32, H0[k k], H1[k k], out_idx[nout] i64,
 * boxes[nbox] u64, xyz[3 nsrc], ex[nsrc], cf[nsrc], thr, gx[k], gw[k]. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_project_level(int k, int j, int jmax, int64_t nbox, const uint64_t* keys, int nsrc, const double* xyz,
                      const double* ex, const double* cf, double thr, const double* gx, const double* gw,
                      double* s_out, uint8_t* refine, double* err_out);
int orc_apply_modified(int k, int64_t N, const uint64_t* keys, const uint8_t* leaf, const double* coef, int M,
                       const double* w, int nlevF, const double* F, int nlevR, const int32_t* R, const double* H0,
                       const double* H1, int64_t nout, const int64_t* out_idx, double* ghat);
int orc_apply_difference(int k, int64_t N, const uint64_t* keys, const uint8_t* leaf, const double* coef, int M,
                         const double* w, int nlevF, const double* F, int nlevR, const int32_t* R, const double* H0,
                         const double* H1, int64_t nout, const int64_t* out_idx, double* ghat);

static void* take(FILE* f, size_t n) {
    void* p = malloc(n ? n : 1);
    if (!p || fread(p, 1, n, f) != n) { fprintf(stderr, "short input\n"); exit(2); }
    return p;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t* hi = take(f, 4 * sizeof(int32_t));
    int64_t* hl = take(f, 5 * sizeof(int64_t));
    const int k = hi[0], nlevF = hi[1], nlevR = hi[2], M = hi[3];
    const int64_t N = hl[0], nout = hl[1], nbox = hl[2], nsrc = hl[3], j = hl[4];
    const size_t k3 = (size_t)k * k * k;
    uint64_t* keys = take(f, N * 8);
    uint8_t* leaf = take(f, N);
    double* coef = take(f, N * k3 * 8);
    double* w = take(f, M * 8);
    double* F = take(f, (size_t)nlevF * M * 15 * k * k * 8);
    int32_t* R = take(f, (size_t)nlevR * 343 * 2 * 4);
    double* H0 = take(f, k * k * 8);
    double* H1 = take(f, k * k * 8);
    int64_t* out_idx = take(f, nout * 8);
    uint64_t* boxes = take(f, nbox * 8);
    double* xyz = take(f, 3 * nsrc * 8);
    double* ex = take(f, nsrc * 8);
    double* cf = take(f, nsrc * 8);
    double* thr = take(f, 8);
    double* gx = take(f, k * 8);
    double* gw = take(f, k * 8);
    fclose(f);
    double* g1 = calloc(nout * k3, 8);
    double* g2 = calloc(nout * k3, 8);
    double* s = calloc(nbox * k3, 8);
    uint8_t* ref = calloc(nbox, 1);
    double* err = calloc(nbox, 8);
    int st = orc_apply_modified(k, N, keys, leaf, coef, M, w, nlevF, F, nlevR, R, H0, H1, nout, out_idx, g1);
    st |= orc_apply_difference(k, N, keys, leaf, coef, M, w, nlevF, F, nlevR, R, H0, H1, nout, out_idx, g2);
    st |= orc_project_level(k, (int)j, 19, nbox, boxes, (int)nsrc, xyz, ex, cf, *thr, gx, gw, s, ref, err);
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(g1, 8, nout * k3, o);
    fwrite(g2, 8, nout * k3, o);
    fwrite(s, 8, nbox * k3, o);
    fwrite(ref, 1, nbox, o);
    fwrite(err, 8, nbox, o);
    fclose(o);
    free(hi); free(hl); free(keys); free(leaf); free(coef); free(w); free(F); free(R); free(H0); free(H1);
    free(out_idx); free(boxes); free(xyz); free(ex); free(cf); free(thr); free(gx); free(gw);
    free(g1); free(g2); free(s); free(ref); free(err);
    return st ? 1 : 0;
}
