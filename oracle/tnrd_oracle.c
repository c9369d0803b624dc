/*
 * FP64 CPU oracle for the trained reaction-diffusion despeckling filter
 * (Feng & Chen, "Speckle Reduction with Trained Nonlinear Diffusion Filtering").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  It shares no code, header,
 * table or constant with the HIP library; the product path never calls it.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.
 *
 * Every routine follows the paper's definitions in the order the paper states
 * them, in double precision, with no blocking, fusion or reordering:
 *
 *   stage (Sec. 3.1, eq. diffusionprocessfinal):
 *     z_i = k_i * u_{t-1}                 true 2-D convolution (Sec. 2.2.1, eq. diffusion)
 *     v_i = phi_i(z_i)                    influence function, Gaussian RBF sum
 *     x   = sum_i K_i^T v_i               back-projection, exact adjoint of K_i
 *     ut  = u_{t-1} - x
 *     u_t = prox(ut) = (ut + sqrt(ut^2 + 8(1+2l)l f^2)) / (2(1+2l))   (eq. subproblemGIdiv)
 *
 *   gradients (Sec. 3.2, eqs. derv1, derv1-1, derv2, derv4): see oracle_backward.
 *
 *   projected variant (Sec. 3.1, eq. diffusion_backP), the paper's comparison model:
 *     ut  = u_{t-1} - ( x + (l / u_{t-1}) (1 - f^2 / u_{t-1}^2) )
 *     u_t = max(ut, c)
 *
 *   quadratic data term (Sec. 2.2.1, eq. diffusion with G = 0, D = l/2 ||u - f||^2,
 *   psi = l (u - f): the Gaussian-denoising reaction of the TNRD framework):
 *     u_t = u_{t-1} - ( x + l (u_{t-1} - f) )
 *
 * Readings of points the paper leaves open, each with its reason:
 *   - u_0 = f (the paper leaves the initial state I_0 open);
 *   - K_i is a true convolution: the kernel is flipped (the paper defines k*u as
 *     2-D convolution and bar k as k rotated by 180 degrees);
 *   - the image is extended by half-sample symmetric reflection
 *     (-1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2) and K_i^T is the exact adjoint of
 *     "extend, then convolve", i.e. the full correlation folded back through the
 *     same reflection (the paper asks for K^T "with careful boundary handling");
 *   - phi_i(z) = sum_j w_ij exp(-(z - mu_j)^2 / (2 sigma^2)), mu_j = mu0 + j*step
 *     (the paper leaves the influence function's form open);
 *   - all RBF terms are summed (no window).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Half-sample symmetric reflection of index q into [0, n).  Valid for
 * -n <= q < 2n, which covers every use below (|overhang| <= r < n). */
int oracle_reflect(int q, int n)
{
    if (q < 0) return -q - 1;
    if (q >= n) return 2 * n - 1 - q;
    return q;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* z = K u: z[p] = sum_{a,b} k[a,b] * ubar[p - (a-r, b-r)], ubar the reflected
 * extension of u.  k is ks x ks row-major, ks odd. */
void oracle_conv(const double *u, int H, int W, const double *k, int ks, double *z)
{
    int r = ks / 2;
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int a = 0; a < ks; ++a) {
                for (int b = 0; b < ks; ++b) {
                    int yy = oracle_reflect(y - (a - r), H);
                    int xx = oracle_reflect(x - (b - r), W);
                    acc += k[a * ks + b] * u[(size_t)yy * W + xx];
                }
            }
            z[(size_t)y * W + x] = acc;
        }
    }
}

/* All padded positions q in [-r, n-1+r] with oracle_reflect(q, n) == p.  The
 * reflection maps q to one of p, -p-1 or 2n-1-p, so those are the only
 * candidates; each is kept if it lies in the padded range and reflects onto p. */
static int preimages(int p, int n, int r, int *out)
{
    int cand[3] = { p, -p - 1, 2 * n - 1 - p };
    int m = 0;
    for (int c = 0; c < 3; ++c) {
        int q = cand[c];
        if (q < -r || q >= n + r) continue;
        if (oracle_reflect(q, n) != p) continue;
        int dup = 0;
        for (int d = 0; d < m; ++d) dup |= (out[d] == q);
        if (!dup) out[m++] = q;
    }
    return m;
}

/* x = K^T v, the exact adjoint of oracle_conv.
 * Step 1: on the padded domain q in [-r, H-1+r] x [-r, W-1+r],
 *         X[q] = sum_{a,b} k[a,b] * v[q + (a-r, b-r)], v taken as 0 outside the image.
 * Step 2: fold, x[p] = sum over the padded q with R(q) = p of X[q]. */
void oracle_conv_adj(const double *v, int H, int W, const double *k, int ks, double *x)
{
    int r = ks / 2;
    int Hp = H + 2 * r, Wp = W + 2 * r;
    double *X = (double *)malloc(sizeof(double) * (size_t)Hp * Wp);
    #pragma omp parallel for schedule(static)
    for (int qy = -r; qy < H + r; ++qy) {
        for (int qx = -r; qx < W + r; ++qx) {
            double acc = 0.0;
            for (int a = 0; a < ks; ++a) {
                for (int b = 0; b < ks; ++b) {
                    int py = qy + (a - r), px = qx + (b - r);
                    if (py < 0 || py >= H || px < 0 || px >= W) continue;
                    acc += k[a * ks + b] * v[(size_t)py * W + px];
                }
            }
            X[(size_t)(qy + r) * Wp + (qx + r)] = acc;
        }
    }
    /* fold: gather, for every image pixel, the padded positions that reflect onto it */
    #pragma omp parallel for schedule(static)
    for (int py = 0; py < H; ++py) {
        int qys[3], nqy = preimages(py, H, r, qys);
        for (int px = 0; px < W; ++px) {
            int qxs[3], nqx = preimages(px, W, r, qxs);
            double acc = 0.0;
            for (int iy = 0; iy < nqy; ++iy)
                for (int ix = 0; ix < nqx; ++ix)
                    acc += X[(size_t)(qys[iy] + r) * Wp + (qxs[ix] + r)];
            x[(size_t)py * W + px] = acc;
        }
    }
    free(X);
}

/* j-th Gaussian RBF G_j(z) = exp(-(z - mu_j)^2 / (2 sigma^2)). */
double oracle_rbf(double z, int j, double mu0, double step, double sigma)
{
    double d = z - (mu0 + j * step);
    return exp(-(d * d) / (2.0 * sigma * sigma));
}

/* phi(z) = sum_j w_j G_j(z), all nrbf terms. */
double oracle_phi(double z, const double *w, int nrbf, double mu0, double step, double sigma)
{
    double acc = 0.0;
    for (int j = 0; j < nrbf; ++j)
        acc += w[j] * oracle_rbf(z, j, mu0, step, sigma);
    return acc;
}

/* phi'(z) = sum_j w_j * (-(z - mu_j) / sigma^2) * G_j(z). */
double oracle_dphi(double z, const double *w, int nrbf, double mu0, double step, double sigma)
{
    double acc = 0.0;
    for (int j = 0; j < nrbf; ++j) {
        double d = z - (mu0 + j * step);
        acc += w[j] * (-d / (sigma * sigma)) * oracle_rbf(z, j, mu0, step, sigma);
    }
    return acc;
}

/* Closed-form proximal map of lambda <u^2 - 2 f^2 log u, 1> (eq. subproblemGIdiv). */
double oracle_prox(double ut, double f, double lam)
{
    double c = 1.0 + 2.0 * lam;
    double s = sqrt(ut * ut + 8.0 * c * lam * f * f);
    return (ut + s) / (2.0 * c);
}

/* Derivatives of the prox: y = du/d(ut) (eq. derv2) and xl = du/dlambda
 * (eq. derv4), exactly as printed.  Degenerate s = 0 (only when lambda*f = 0
 * and ut = 0): ut/s := 0 and xl := 0. */
void oracle_prox_grad(double ut, double f, double lam, double *y, double *xl)
{
    double c = 1.0 + 2.0 * lam;
    double s = sqrt(ut * ut + 8.0 * c * lam * f * f);
    if (s == 0.0) {
        *y = 0.5 / c;
        *xl = 0.0;
        return;
    }
    *y = (1.0 + ut / s) / (2.0 * c);
    *xl = (2.0 * f * f + 8.0 * lam * f * f) / (c * s) - (ut + s) / (c * c);
}

/* Full derivative of the prox output with respect to f (f enters only
 * through s): du/df = 4 lambda f / s, s = sqrt(ut^2 + 8(1+2l) l f^2). */
double oracle_prox_df(double ut, double f, double lam)
{
    double c = 1.0 + 2.0 * lam;
    double s = sqrt(ut * ut + 8.0 * c * lam * f * f);
    if (s == 0.0) return 0.0;
    return 4.0 * lam * f / s;
}

/* Reaction of the projected variant (eq. diffusion_backP), exactly as printed:
 * psi(u) = (lambda / u) (1 - f^2 / u^2). */
double oracle_psi(double u, double f, double lam)
{
    return lam / u * (1.0 - f * f / (u * u));
}

/* Its partial derivatives: d psi / du = lambda (3 f^2 / u^4 - 1 / u^2),
 * d psi / d lambda = (1 / u) (1 - f^2 / u^2), d psi / df = -2 lambda f / u^3. */
double oracle_psi_du(double u, double f, double lam)
{
    return lam * (3.0 * f * f / (u * u * u * u) - 1.0 / (u * u));
}
double oracle_psi_dlam(double u, double f)
{
    return (1.0 / u) * (1.0 - f * f / (u * u));
}
double oracle_psi_df(double u, double f, double lam)
{
    return -2.0 * lam * f / (u * u * u);
}

/* Pointer helpers for the parameter layout
 *   filters [T][Nk][ks][ks], rbf_w [T][Nk][Nrbf], lambda [T]. */
static const double *filt(const double *filters, int t, int i, int Nk, int ks)
{
    return filters + ((size_t)t * Nk + i) * ks * ks;
}
static const double *rbfw(const double *w, int t, int i, int Nk, int Nrbf)
{
    return w + ((size_t)t * Nk + i) * Nrbf;
}

/* Reaction of a stage: 0 = proximal step of eq. diffusionprocessfinal,
 * 1 = gradient step and projection max(., c) of eq. diffusion_backP,
 * 2 = gradient step on the quadratic data term (l/2) ||u - f||^2. */
enum { REACT_PROX = 0, REACT_PROJECTED = 1, REACT_L2 = 2 };

/* One stage on one image: computes ut (length H*W) and u_next from u_prev. */
static void stage_forward(const double *u_prev, const double *f, int H, int W, int t,
                          int Nk, int ks, int Nrbf, double mu0, double step, double sigma,
                          const double *filters, const double *rbf_w, const double *lam,
                          int reaction, double cproj, double *ut, double *u_next)
{
    size_t n = (size_t)H * W;
    double *z = (double *)malloc(sizeof(double) * n);
    double *v = (double *)malloc(sizeof(double) * n);
    double *xi = (double *)malloc(sizeof(double) * n);
    double *x = (double *)calloc(n, sizeof(double));
    for (int i = 0; i < Nk; ++i) {
        const double *k = filt(filters, t, i, Nk, ks);
        const double *w = rbfw(rbf_w, t, i, Nk, Nrbf);
        oracle_conv(u_prev, H, W, k, ks, z);                       /* z_i = K_i u */
        #pragma omp parallel for schedule(static)
        for (long p = 0; p < (long)n; ++p)
            v[p] = oracle_phi(z[p], w, Nrbf, mu0, step, sigma);   /* v_i = phi_i(z_i) */
        oracle_conv_adj(v, H, W, k, ks, xi);                        /* K_i^T v_i */
        for (size_t p = 0; p < n; ++p) x[p] += xi[p];
    }
    for (size_t p = 0; p < n; ++p) {
        if (reaction == REACT_PROJECTED) {
            ut[p] = u_prev[p] - (x[p] + oracle_psi(u_prev[p], f[p], lam[t]));
            u_next[p] = ut[p] > cproj ? ut[p] : cproj;
        } else if (reaction == REACT_L2) {
            ut[p] = u_prev[p] - (x[p] + lam[t] * (u_prev[p] - f[p]));
            u_next[p] = ut[p];
        } else {
            ut[p] = u_prev[p] - x[p];
            u_next[p] = oracle_prox(ut[p], f[p], lam[t]);
        }
    }
    free(z); free(v); free(xi); free(x);
}

/* Stage t alone (0-based) on N images: u_next = stage_t(u_prev) with data f,
 * and the pre-reaction values ut.  The same routine the forward chains; it lets
 * a caller start a stage from states of its own. */
void oracle_stage_ex(const double *u_prev, const double *f, int N, int H, int W, int t,
                     int Nk, int ks, int Nrbf, double mu0, double step, double sigma,
                     const double *filters, const double *rbf_w, const double *lam,
                     int reaction, double cproj, double *ut, double *u_next, int nthreads)
{
    set_threads(nthreads);
    size_t n = (size_t)H * W;
    for (int img = 0; img < N; ++img)
        stage_forward(u_prev + (size_t)img * n, f + (size_t)img * n, H, W, t, Nk, ks, Nrbf,
                      mu0, step, sigma, filters, rbf_w, lam, reaction, cproj,
                      ut + (size_t)img * n, u_next + (size_t)img * n);
}

/* Forward pass of the T-stage filter over N images of H x W.
 *   uT      [N][H][W]               output u_T
 *   states  [T+1][N][H][W] or NULL  u_0 .. u_T
 *   utilde  [T][N][H][W] or NULL    ut_1 .. ut_T (pre-prox values)
 */
void oracle_forward_ex(const double *f, int N, int H, int W, int T, int Nk, int ks, int Nrbf,
                       double mu0, double step, double sigma,
                       const double *filters, const double *rbf_w, const double *lam,
                       int reaction, double cproj,
                       double *uT, double *states, double *utilde, int nthreads)
{
    set_threads(nthreads);
    size_t n = (size_t)H * W;
    double *ua = (double *)malloc(sizeof(double) * n);
    double *ub = (double *)malloc(sizeof(double) * n);
    double *ut = (double *)malloc(sizeof(double) * n);
    for (int img = 0; img < N; ++img) {
        const double *fi = f + (size_t)img * n;
        memcpy(ua, fi, sizeof(double) * n);                        /* u_0 = f */
        if (states) memcpy(states + (size_t)img * n, ua, sizeof(double) * n);
        for (int t = 0; t < T; ++t) {
            stage_forward(ua, fi, H, W, t, Nk, ks, Nrbf, mu0, step, sigma,
                          filters, rbf_w, lam, reaction, cproj, ut, ub);
            if (states) memcpy(states + ((size_t)(t + 1) * N + img) * n, ub, sizeof(double) * n);
            if (utilde) memcpy(utilde + ((size_t)t * N + img) * n, ut, sizeof(double) * n);
            double *tmp = ua; ua = ub; ub = tmp;
        }
        memcpy(uT + (size_t)img * n, ua, sizeof(double) * n);
    }
    free(ua); free(ub); free(ut);
}

/* The proximal model (eq. diffusionprocessfinal). */
void oracle_forward(const double *f, int N, int H, int W, int T, int Nk, int ks, int Nrbf,
                    double mu0, double step, double sigma,
                    const double *filters, const double *rbf_w, const double *lam,
                    double *uT, double *states, double *utilde, int nthreads)
{
    oracle_forward_ex(f, N, H, W, T, Nk, ks, Nrbf, mu0, step, sigma, filters, rbf_w, lam,
                      REACT_PROX, 0.0, uT, states, utilde, nthreads);
}

/* Backward pass (Sec. 3.2).  Given gT = dl/du_T and the forward states
 * u_0..u_T ([T+1][N][H][W]), accumulates over all images:
 *   dK   [T][Nk][ks][ks]  dl/dk_i^t
 *   dW   [T][Nk][Nrbf]    dl/dw_ij^t
 *   dlam [T]              dl/dlambda^t
 *   g0   [N][H][W] or NULL  dl/du_0 (through the diffusion chain only; u_0 = f
 *                           also enters the prox, which is not included here)
 *   gf   [N][H][W] or NULL  dl/df in full: g0 plus, at every stage, g_t times the
 *                           explicit derivative of u_t with respect to f
 *                           (prox: 4 lambda f / s; projected: m . (-d psi / df))
 *
 * Per stage t = T..1, with g = dl/du_t:
 *   ut  = u_{t-1} - sum_i K_i^T phi_i(K_i u_{t-1})   (recomputed)
 *   y   = du_t/d ut (eq. derv2),  xl = du_t/d lambda^t (eq. derv4)
 *   dlam^t = <g, xl>
 *   e   = y . g                                       (dl/d ut)
 *   a_i = K_i e
 *   dW_ij  = - sum_p a_i[p] G_j(z_i[p])
 *   dK_i[a,b] = - sum_p ( v_i[p] ebar[p-(a-r,b-r)] + phi_i'(z_i[p]) a_i[p] ubar[p-(a-r,b-r)] )
 *   g  <- e - sum_i K_i^T( phi_i'(z_i) . a_i )        (eq. derv1-1 transposed)
 * The k and phi parts follow from differentiating -<e, K_i^T phi_i(K_i u)>,
 * which the paper defers to the original TNRD derivation.
 *
 * Projected variant (eq. diffusion_backP): the projection's derivative is
 * m = 1 where ut > c and 0 elsewhere, e = m . g, dlam^t = -<e, d psi / d lambda>,
 * and the reaction adds -(d psi / du)(u_{t-1}) . e to g_{t-1}.
 * Quadratic data term: e = g, dlam^t = -<e, u_{t-1} - f>, the reaction adds
 * -lambda e to g_{t-1}, and u_t depends on f explicitly through +lambda f.
 */
void oracle_backward_ex(const double *f, int N, int H, int W, int T, int Nk, int ks, int Nrbf,
                        double mu0, double step, double sigma,
                        const double *filters, const double *rbf_w, const double *lam,
                        int reaction, double cproj,
                        const double *states, const double *gT,
                        double *dK, double *dW, double *dlam, double *g0, double *gf, int nthreads)
{
    set_threads(nthreads);
    size_t n = (size_t)H * W;
    int r = ks / 2, kk = ks * ks;
    memset(dK, 0, sizeof(double) * (size_t)T * Nk * kk);
    memset(dW, 0, sizeof(double) * (size_t)T * Nk * Nrbf);
    memset(dlam, 0, sizeof(double) * (size_t)T);

    double *g = (double *)malloc(sizeof(double) * n);
    double *e = (double *)malloc(sizeof(double) * n);
    double *ut = (double *)malloc(sizeof(double) * n);
    double *unext = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *v = (double *)malloc(sizeof(double) * n);
    double *a = (double *)malloc(sizeof(double) * n);
    double *dp = (double *)malloc(sizeof(double) * n);
    double *xi = (double *)malloc(sizeof(double) * n);
    double *gacc = (double *)malloc(sizeof(double) * n);
    double *fexp = (double *)malloc(sizeof(double) * n);

    for (int img = 0; img < N; ++img) {
        const double *fi = f + (size_t)img * n;
        memcpy(g, gT + (size_t)img * n, sizeof(double) * n);
        memset(fexp, 0, sizeof(double) * n);
        for (int t = T - 1; t >= 0; --t) {
            const double *uprev = states + ((size_t)t * N + img) * n;
            /* recompute ut_t from u_{t-1} exactly as the forward does */
            stage_forward(uprev, fi, H, W, t, Nk, ks, Nrbf, mu0, step, sigma,
                          filters, rbf_w, lam, reaction, cproj, ut, unext);
            double dl = 0.0;
            if (reaction == REACT_PROJECTED) {
                /* projection backward: e = m g with m = [ut > c] */
                for (size_t p = 0; p < n; ++p) {
                    e[p] = ut[p] > cproj ? g[p] : 0.0;
                    dl -= e[p] * oracle_psi_dlam(uprev[p], fi[p]);
                    fexp[p] -= e[p] * oracle_psi_df(uprev[p], fi[p], lam[t]);
                }
            } else if (reaction == REACT_L2) {
                for (size_t p = 0; p < n; ++p) {
                    e[p] = g[p];
                    dl -= e[p] * (uprev[p] - fi[p]);
                    fexp[p] += e[p] * lam[t];
                }
            } else {
                /* prox backward */
                for (size_t p = 0; p < n; ++p) {
                    double y, xl;
                    oracle_prox_grad(ut[p], fi[p], lam[t], &y, &xl);
                    dl += g[p] * xl;
                    e[p] = y * g[p];
                    fexp[p] += g[p] * oracle_prox_df(ut[p], fi[p], lam[t]);
                }
            }
            dlam[t] += dl;
            memset(gacc, 0, sizeof(double) * n);
            for (int i = 0; i < Nk; ++i) {
                const double *k = filt(filters, t, i, Nk, ks);
                const double *w = rbfw(rbf_w, t, i, Nk, Nrbf);
                double *dk = dK + ((size_t)t * Nk + i) * kk;
                double *dw = dW + ((size_t)t * Nk + i) * Nrbf;
                oracle_conv(uprev, H, W, k, ks, z);   /* z_i = K_i u_{t-1} */
                oracle_conv(e, H, W, k, ks, a);       /* a_i = K_i e */
                #pragma omp parallel for schedule(static)
                for (long p = 0; p < (long)n; ++p) {
                    v[p] = oracle_phi(z[p], w, Nrbf, mu0, step, sigma);
                    dp[p] = oracle_dphi(z[p], w, Nrbf, mu0, step, sigma);
                }
                /* dW_ij = - sum_p a_i[p] G_j(z_i[p]) */
                #pragma omp parallel for schedule(static)
                for (int j = 0; j < Nrbf; ++j) {
                    double acc = 0.0;
                    for (size_t p = 0; p < n; ++p)
                        acc += a[p] * oracle_rbf(z[p], j, mu0, step, sigma);
                    dw[j] -= acc;
                }
                /* dK_i[a,b] = - sum_p ( v[p] ebar[p-d] + phi'(z[p]) a[p] ubar[p-d] ) */
                #pragma omp parallel for schedule(static)
                for (int tap = 0; tap < kk; ++tap) {
                    int ta = tap / ks, tb = tap % ks;
                    double acc = 0.0;
                    for (int py = 0; py < H; ++py) {
                        for (int px = 0; px < W; ++px) {
                            int yy = oracle_reflect(py - (ta - r), H);
                            int xx = oracle_reflect(px - (tb - r), W);
                            size_t p = (size_t)py * W + px, q = (size_t)yy * W + xx;
                            acc += v[p] * e[q] + dp[p] * a[p] * uprev[q];
                        }
                    }
                    dk[tap] -= acc;
                }
                /* K_i^T (phi_i'(z_i) . a_i) */
                for (size_t p = 0; p < n; ++p) dp[p] *= a[p];
                oracle_conv_adj(dp, H, W, k, ks, xi);
                for (size_t p = 0; p < n; ++p) gacc[p] += xi[p];
            }
            for (size_t p = 0; p < n; ++p) {
                g[p] = e[p] - gacc[p];
                if (reaction == REACT_PROJECTED) g[p] -= oracle_psi_du(uprev[p], fi[p], lam[t]) * e[p];
                if (reaction == REACT_L2) g[p] -= lam[t] * e[p];
            }
        }
        if (g0) memcpy(g0 + (size_t)img * n, g, sizeof(double) * n);
        if (gf)
            for (size_t p = 0; p < n; ++p) gf[(size_t)img * n + p] = g[p] + fexp[p];  /* u_0 = f */
    }
    free(g); free(e); free(ut); free(unext); free(z); free(v); free(a);
    free(dp); free(xi); free(gacc); free(fexp);
}

/* The proximal model (eq. diffusionprocessfinal), without dl/df. */
void oracle_backward(const double *f, int N, int H, int W, int T, int Nk, int ks, int Nrbf,
                     double mu0, double step, double sigma,
                     const double *filters, const double *rbf_w, const double *lam,
                     const double *states, const double *gT,
                     double *dK, double *dW, double *dlam, double *g0, int nthreads)
{
    oracle_backward_ex(f, N, H, W, T, Nk, ks, Nrbf, mu0, step, sigma, filters, rbf_w, lam,
                       REACT_PROX, 0.0, states, gT, dK, dW, dlam, g0, NULL, nthreads);
}
