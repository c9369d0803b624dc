/*
 * Driver that runs the FP64 oracle (oracle/tnrd_oracle.c, linked in) on one
 * case read from a file, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Test infrastructure only.
 *
 * usage: oracle_sanitize <case file> <output file>
 * case file: int32 reaction, ks, N, H, W, T, Nk, Nrbf; float64 mu0, step,
 *   sigma, cproj; float64 f[N][H][W], filters[T][Nk][ks][ks],
 *   rbf_w[T][Nk][Nrbf], lam[T], gT[N][H][W].
 * output: float64 uT, states[T+1], utilde[T] (forward), dK, dW, dlam, g0, gf
 *   (backward), then K u and K^T v of image 0 with filter 0 of stage 0 for
 *   u = f[0] and v = gT[0], in that order.
 */
#include <stdio.h>
#include <stdlib.h>

void oracle_forward_ex(const double *f, int N, int H, int W, int T, int Nk, int ks, int Nrbf,
                       double mu0, double step, double sigma, const double *filters,
                       const double *rbf_w, const double *lam, int reaction, double cproj,
                       double *uT, double *states, double *utilde, int nthreads);
void oracle_backward_ex(const double *f, int N, int H, int W, int T, int Nk, int ks, int Nrbf,
                        double mu0, double step, double sigma, const double *filters,
                        const double *rbf_w, const double *lam, int reaction, double cproj,
                        const double *states, const double *gT, double *dK, double *dW,
                        double *dlam, double *g0, double *gf, int nthreads);
void oracle_conv(const double *u, int H, int W, const double *k, int ks, double *z);
void oracle_conv_adj(const double *v, int H, int W, const double *k, int ks, double *x);

static double *take(FILE *fp, size_t n)
{
    double *p = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (!p || fread(p, sizeof(double), n, fp) != n) {
        fprintf(stderr, "short case file\n");
        exit(2);
    }
    return p;
}

static void put(FILE *fp, const double *p, size_t n)
{
    if (fwrite(p, sizeof(double), n, fp) != n) {
        fprintf(stderr, "write failed\n");
        exit(2);
    }
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s case out\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int h[8];
    double c[4];
    if (fread(h, sizeof(int), 8, in) != 8 || fread(c, sizeof(double), 4, in) != 4) return 2;
    const int reaction = h[0], ks = h[1], N = h[2], H = h[3], W = h[4], T = h[5], Nk = h[6],
              Nrbf = h[7];
    const size_t n = (size_t)N * H * W, kk = (size_t)ks * ks;
    double *f = take(in, n), *filt = take(in, (size_t)T * Nk * kk);
    double *rbfw = take(in, (size_t)T * Nk * Nrbf), *lam = take(in, (size_t)T), *gT = take(in, n);
    fclose(in);

    /* exact-size outputs, so that any access past an array's end is caught */
    double *uT = malloc(sizeof(double) * n), *states = malloc(sizeof(double) * (T + 1) * n);
    double *utilde = malloc(sizeof(double) * T * n);
    oracle_forward_ex(f, N, H, W, T, Nk, ks, Nrbf, c[0], c[1], c[2], filt, rbfw, lam, reaction,
                      c[3], uT, states, utilde, 1);
    double *dK = malloc(sizeof(double) * T * Nk * kk), *dW = malloc(sizeof(double) * T * Nk * Nrbf);
    double *dlam = malloc(sizeof(double) * T), *g0 = malloc(sizeof(double) * n);
    double *gf = malloc(sizeof(double) * n);
    oracle_backward_ex(f, N, H, W, T, Nk, ks, Nrbf, c[0], c[1], c[2], filt, rbfw, lam, reaction,
                       c[3], states, gT, dK, dW, dlam, g0, gf, 1);
    const size_t n1 = (size_t)H * W;
    double *z = malloc(sizeof(double) * n1), *x = malloc(sizeof(double) * n1);
    oracle_conv(f, H, W, filt, ks, z);
    oracle_conv_adj(gT, H, W, filt, ks, x);

    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    put(out, uT, n);
    put(out, states, (T + 1) * n);
    put(out, utilde, T * n);
    put(out, dK, T * Nk * kk);
    put(out, dW, T * Nk * Nrbf);
    put(out, dlam, T);
    put(out, g0, n);
    put(out, gf, n);
    put(out, z, n1);
    put(out, x, n1);
    fclose(out);
    free(f); free(filt); free(rbfw); free(lam); free(gT); free(uT); free(states); free(utilde);
    free(dK); free(dW); free(dlam); free(g0); free(gf); free(z); free(x);
    return 0;
}
