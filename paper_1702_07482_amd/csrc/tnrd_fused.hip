// Host side of the fused stage kernel: influence-form constants, tile and
// form selection, configuration checks.  The kernels are instantiated in
// tnrd_fused_{fwd,mixed,bwd,batched}.hip.
#include <string.h>

#include <atomic>

#include "tnrd_fused_tile.hpp"

namespace tnrd {

// Monomial coefficients M[k][m] (k = 0..7) of the degree-7 interpolant at the
// Chebyshev points of [-1/2, 1/2] of exp(-rho (d - m)^2 / 2) (deriv = false)
// or of its derivative -rho (d - m) exp(-rho (d - m)^2 / 2) (deriv = true), in FP64.
static void poly_gauss_coeffs(double rho, bool deriv, double M[POLY_NC][POLY_MW + 1])
{
    const double pi = 3.14159265358979323846;
    double x[POLY_NC];
    for (int n = 0; n < POLY_NC; ++n) x[n] = 0.5 * cos((2 * n + 1) * pi / (2 * POLY_NC));
    for (int m = 0; m <= POLY_MW; ++m) {
        // Vandermonde system V c = g, Gaussian elimination with partial pivoting
        double A[POLY_NC][POLY_NC + 1];
        for (int n = 0; n < POLY_NC; ++n) {
            double p = 1.0;
            for (int k = 0; k < POLY_NC; ++k) {
                A[n][k] = p;
                p *= x[n];
            }
            const double g = exp(-rho * (x[n] - m) * (x[n] - m) / 2.0);
            A[n][POLY_NC] = deriv ? -rho * (x[n] - m) * g : g;
        }
        for (int col = 0; col < POLY_NC; ++col) {
            int piv = col;
            for (int r = col + 1; r < POLY_NC; ++r)
                if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
            if (piv != col)
                for (int k = 0; k <= POLY_NC; ++k) {
                    double t = A[col][k];
                    A[col][k] = A[piv][k];
                    A[piv][k] = t;
                }
            for (int r = 0; r < POLY_NC; ++r) {
                if (r == col) continue;
                const double fct = A[r][col] / A[col][col];
                for (int k = col; k <= POLY_NC; ++k) A[r][k] -= fct * A[col][k];
            }
        }
        for (int k = 0; k < POLY_NC; ++k) M[k][m] = A[k][POLY_NC] / A[k][k];
    }
}

// Monomial coefficients P[k][m + POLY_MW] (k = 0..3, |m| <= POLY_MW) of the
// cubic interpolant at the Chebyshev points of e in [0, 1] of
// g(x) = exp(-rho x^2 / 2) (deriv = false) or -rho x exp(-rho x^2 / 2)
// (deriv = true) at x = (e - 1/2) / 2 + off - m: the Gaussian of centre j0 + m
// seen from the half interval centred at j0 + off (off = -1/4 or +1/4), whose
// points are j0 + off + (e - 1/2) / 2, in FP64.
static void poly3_gauss_coeffs(double rho, bool deriv, double off, double P[POLY3_NC][POLY3_NM])
{
    const double pi = 3.14159265358979323846;
    double e[POLY3_NC];
    for (int n = 0; n < POLY3_NC; ++n) e[n] = 0.5 + 0.5 * cos((2 * n + 1) * pi / (2 * POLY3_NC));
    for (int mi = 0; mi < POLY3_NM; ++mi) {
        const double m = mi - POLY_MW;
        double A[POLY3_NC][POLY3_NC + 1];
        for (int n = 0; n < POLY3_NC; ++n) {
            double p = 1.0;
            for (int k = 0; k < POLY3_NC; ++k) {
                A[n][k] = p;
                p *= e[n];
            }
            const double x = 0.5 * (e[n] - 0.5) + off - m;
            const double g = exp(-rho * x * x / 2.0);
            A[n][POLY3_NC] = deriv ? -rho * x * g : g;
        }
        for (int col = 0; col < POLY3_NC; ++col) {
            int piv = col;
            for (int r = col + 1; r < POLY3_NC; ++r)
                if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
            if (piv != col)
                for (int k = 0; k <= POLY3_NC; ++k) {
                    double t = A[col][k];
                    A[col][k] = A[piv][k];
                    A[piv][k] = t;
                }
            for (int r = 0; r < POLY3_NC; ++r) {
                if (r == col) continue;
                const double fct = A[r][col] / A[col][col];
                for (int k = col; k <= POLY3_NC; ++k) A[r][k] -= fct * A[col][k];
            }
        }
        for (int k = 0; k < POLY3_NC; ++k) P[k][mi] = A[k][POLY3_NC] / A[k][k];
    }
}

static FusedRbf make_fused_rbf_uncached(const RbfGrid &grid);

// The constants depend on the grid only; the two 8 x 8 solves per centre
// offset are done once per grid and thread, not once per stage launch.
FusedRbf make_fused_rbf(const RbfGrid &grid)
{
    static thread_local bool have = false;
    static thread_local float key[4];
    static thread_local int key_n = 0;
    static thread_local FusedRbf last;
    if (!have || key[0] != grid.mu0 || key[1] != grid.step || key[2] != grid.neg_half_inv_var ||
        key[3] != grid.inv_step || key_n != grid.nrbf) {
        last = make_fused_rbf_uncached(grid);
        key[0] = grid.mu0;
        key[1] = grid.step;
        key[2] = grid.neg_half_inv_var;
        key[3] = grid.inv_step;
        key_n = grid.nrbf;
        have = true;
    }
    return last;
}

static FusedRbf make_fused_rbf_uncached(const RbfGrid &grid)
{
    FusedRbf rb;
    const double step = grid.step;
    const double sigma = 1.0 / sqrt(-2.0 * (double)grid.neg_half_inv_var);
    const double rho = (step / sigma) * (step / sigma);
    rb.mu0_over_step = (float)(grid.mu0 / step);
    rb.inv_step = (float)(1.0 / step);
    rb.rho_log2e = (float)(rho * 1.4426950408889634);
    rb.jmax = (float)(grid.nrbf - 1 + RBF_WIN);
    rb.rho_over_step = (float)(rho / step);
    for (int n = 0; n < RBF_TERMS; ++n) {
        double m = n - RBF_WIN;
        rb.c[n] = (float)exp(-rho * m * m / 2.0);
    }
    double M[POLY_NC][POLY_MW + 1], Md[POLY_NC][POLY_MW + 1];
    poly_gauss_coeffs(rho, false, M);
    poly_gauss_coeffs(rho, true, Md);
    for (int k = 0; k < POLY_NC; ++k)
        for (int m = 0; m <= POLY_MW; ++m) {
            rb.pm[k][m] = (float)M[k][m];
            rb.pmd[k][m] = (float)Md[k][m];
        }
    for (int h = 0; h < 2; ++h) {
        double P[POLY3_NC][POLY3_NM], Pd[POLY3_NC][POLY3_NM];
        poly3_gauss_coeffs(rho, false, h ? 0.25 : -0.25, P);
        poly3_gauss_coeffs(rho, true, h ? 0.25 : -0.25, Pd);
        for (int k = 0; k < POLY3_NC; ++k)
            for (int m = 0; m < POLY3_NM; ++m) {
                rb.p3[h][k][m] = (float)P[k][m];
                rb.p3d[h][k][m] = (float)Pd[k][m];
            }
    }
    return rb;
}

// The polynomial form is used with the automatic window only, i.e. for
// rho = (step / sigma)^2 in [0.914, 1.365), where the interpolation error summed
// over all centres stays below 8e-7 of the largest weight for phi (2.5e-7 at
// rho = 1) and below 1e-6 of it for d phi / ds (1.8e-7 at rho = 1).
bool poly_form_ok(const RbfGrid &grid, int automatic_window)
{
    if (!automatic_window || grid.window != RBF_WIN || grid.nrbf > POLY_NRBF_MAX) return false;
    const double sigma = 1.0 / sqrt(-2.0 * (double)grid.neg_half_inv_var);
    const double rho = ((double)grid.step / sigma) * ((double)grid.step / sigma);
    return rho > 0.0 && rho < 1.4;
}

static bool lds_fits(int ks, int nk, int nrbf, int th, int tw, int nb, int nw, int mode, int rbfm)
{
    const int nmb = (nk + 15) / 16 <= 2 ? 2 : 3;
    FusedLds L = fused_lds(ks, nmb, nb, th, tw, nrbf, nw, mode, rbfm);
    return (size_t)L.total * sizeof(float) <= 160 * 1024;
}

// Compute units of the current device (cached per device; concurrent first
// calls from several threads store the same value).
static int device_cus()
{
    static std::atomic<int> cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

struct TilePlan {
    int th, tw, nb, nw, rbfm;
    bool ok;
};

// Tile, wave count and influence form of one stage launch.  A requested tile
// is taken as given (clamped to the image).  Otherwise the tile minimises the
// modelled time: the kernel holds one workgroup per compute unit (its LDS
// footprint), so a launch of n tiles runs in ceil(n / CUs) rounds, each as
// long as one tile.  A tile's Th rows (every mode works on the tile's own
// pixels) go to its waves in rounds, so a wave runs ceil(rows / waves) rows of
// nb 16-pixel blocks, plus a fixed cost (prologue, output passes) worth about
// 2 such blocks.  Among tiles of equal modelled time the one with the fewest
// rows wins (its output passes and prologue are the shortest), then the one
// with fewer tiles.  Tile widths are those whose rows fill their blocks
// exactly (16 nb).  Tiles are at least 2R on each side, so a padded position
// lies in the rings of at most two tiles per axis.
static TilePlan plan_tile(int ks, int nk, int nrbf, int N, int H, int W, int req_h, int req_w,
                          int waves, int mode, bool poly)
{
    const int R = ks / 2;
    const bool xf = mode == MODE_FWD;
    const int tmin = 2 * R;  // smallest tile side
    TilePlan p;
    p.nw = waves == 4 ? 4 : 8;
    p.ok = false;
    auto form = [&](int th, int tw, int nb) {
        if (poly && lds_fits(ks, nk, nrbf, th, tw, nb, p.nw, mode, RBF_POLY))
            return (int)RBF_POLY;
        if (lds_fits(ks, nk, nrbf, th, tw, nb, p.nw, mode, RBF_HORNER)) return (int)RBF_HORNER;
        return -1;
    };
    if (req_h > 0 || req_w > 0) {
        p.tw = req_w > 0 ? req_w : 32;
        p.th = req_h > 0 ? req_h : 32;
        if (p.tw > W) p.tw = W;
        if (p.th > H) p.th = H;
        p.nb = (p.tw + 15) / 16;
        if (p.nb < 2) p.nb = 2;
        p.rbfm = p.nb <= 4 ? form(p.th, p.tw, p.nb) : -1;
        p.ok = p.nb <= 4 && p.th >= tmin && p.tw >= tmin && p.rbfm >= 0;
        return p;
    }
    const long cus = device_cus();
    double best = 0.0;
    // heights: forward from 2R (its LDS holds taller tiles), input-gradient mode 8..96
    const int th_lo = xf ? tmin : 8, th_hi = xf ? 160 : 96;
    // the polynomial form wherever a tile fits it (the Gaussian form's extra
    // exponentials cost far more than a slightly worse tile)
    bool poly_fits = false;
    for (int nb = 2; nb <= 4 && poly; ++nb)
        poly_fits = poly_fits || form(th_lo > H ? H : th_lo, 16 * nb > W ? W : 16 * nb, nb) == RBF_POLY;
    for (int nb = 2; nb <= 4; ++nb) {
        int tw = 16 * nb;
        if (tw > W) tw = W;
        for (int th = th_lo; th <= th_hi; ++th) {
            const int t = th > H ? H : th;
            const int rbfm = form(t, tw, nb);
            if (rbfm < 0 || (poly_fits && rbfm != RBF_POLY)) continue;
            const long tiles = (long)N * ((H + t - 1) / t) * ((W + tw - 1) / tw);
            const long rounds = (tiles + cus - 1) / cus;
            // per wave: ceil(rows / waves) rows of nb blocks (the rows go to the
            // waves in rounds); a block of the Gaussian form costs about 1.3 blocks
            // of the polynomial form
            const int rows = t < H ? t : H;
            const double blk = (rbfm == RBF_HORNER ? 1.3 : 1.0) * ((rows + p.nw - 1) / p.nw) * nb;
            const double cost = (double)rounds * (blk + 2) + 1e-4 * rows * nb + 1e-9 * (double)tiles;
            if (!p.ok || cost < best) {
                best = cost;
                p.th = t;
                p.tw = tw;
                p.nb = nb;
                p.rbfm = rbfm;
                p.ok = true;
            }
            if (th >= H) break;
        }
    }
    return p;
}

// plan_tile scans a few hundred candidate tiles; every stage of a call asks the
// same question, so the answers are kept per thread (the last few shapes).
static TilePlan plan_tile_cached(int ks, int nk, int nrbf, int N, int H, int W, int req_h, int req_w,
                                 int waves, int mode, bool poly)
{
    struct Entry {
        int key[12];
        TilePlan plan;
    };
    constexpr int SLOTS = 8;
    static thread_local Entry cache[SLOTS];
    static thread_local int used = 0, next = 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const int key[12] = {ks, nk, nrbf, N, H, W, req_h, req_w, waves, mode, poly ? 1 : 0, dev};
    for (int i = 0; i < used; ++i)
        if (memcmp(cache[i].key, key, sizeof(key)) == 0) return cache[i].plan;
    const TilePlan p = plan_tile(ks, nk, nrbf, N, H, W, req_h, req_w, waves, mode, poly);
    memcpy(cache[next].key, key, sizeof(key));
    cache[next].plan = p;
    next = (next + 1) % SLOTS;
    if (used < SLOTS) ++used;
    return p;
}

template <int MODE>
static hipError_t fused_dispatch(const StageArgs &s, hipStream_t stream)
{
    const bool poly = s.poly && poly_form_ok(s.grid, 1);
    const TilePlan p = plan_tile_cached(s.ks, s.Nk, s.grid.nrbf, s.N, s.H, s.W, s.tile_h, s.tile_w,
                                        s.waves, MODE, poly);
    if (!p.ok) return hipErrorInvalidValue;
    // BF16 operands read the cubic half-interval table (fused_prep_form)
    const int rbfm = p.rbfm == RBF_POLY && (fused_prep_form(s) & 2) ? RBF_POLY3 : p.rbfm;
    if (MODE == MODE_BWD_INPUT) return fused_launch_bwd(s, p.th, p.tw, p.nb, p.nw, rbfm, stream);
    if (s.prec == PREC_BF16 || s.prec == PREC_F16)
        return fused_launch_fwd_mixed(s, p.th, p.tw, p.nb, p.nw, rbfm, stream);
    return fused_launch_fwd_f32(s, p.th, p.tw, p.nb, p.nw, p.rbfm, stream);
}

// Whether a requested tile and wave count can run (an automatic tile always
// can).
bool fused_config_ok(int ks, int nk, int nrbf, int H, int W, int tile_h, int tile_w, int waves,
                     int mode)
{
    return plan_tile(ks, nk, nrbf, 1, H, W, tile_h, tile_w, waves, mode, false).ok;
}

bool fused_supported(int ks, int nk, int nrbf, int window, int prec)
{
    if (prec != PREC_F32 && !(ks == 7 && (prec == PREC_BF16 || prec == PREC_F16))) return false;
    if (ks != 5 && ks != 7) return false;
    if (nk < 1 || nk > 48) return false;
    if (window != RBF_WIN) return false;
    if (nrbf < 1 || nrbf > 200) return false;
    return true;
}

size_t fused_scratch_floats(int, int, int, int, int) { return 0; }

bool fused_uses_prep(const StageArgs &s)
{
    return s.poly && poly_form_ok(s.grid, 1);
}

hipError_t fused_stage(const StageArgs &s, hipStream_t stream)
{
    return fused_dispatch<MODE_FWD>(s, stream);
}

hipError_t fused_finish(const StageArgs &s, hipStream_t stream)
{
    const bool poly = s.poly && poly_form_ok(s.grid, 1);
    const TilePlan p = plan_tile_cached(s.ks, s.Nk, s.grid.nrbf, s.N, s.H, s.W, s.tile_h, s.tile_w,
                                        s.waves, MODE_FWD, poly);
    if (!p.ok) return hipErrorInvalidValue;
    return fused_launch_final(s, p.th, p.tw, stream);
}

hipError_t fused_grad_finish(const StageArgs &s, hipStream_t stream)
{
    const bool poly = s.poly && poly_form_ok(s.grid, 1);
    const TilePlan p = plan_tile_cached(s.ks, s.Nk, s.grid.nrbf, s.N, s.H, s.W, s.tile_h, s.tile_w,
                                        s.waves, MODE_BWD_INPUT, poly);
    if (!p.ok) return hipErrorInvalidValue;
    return fused_launch_grad_finish(s, p.th, p.tw, stream);
}

size_t fused_slab_floats(int ks, int nk, int nrbf, int N, int H, int W, int tile_h, int tile_w,
                         int waves, bool poly, int mode)
{
    const TilePlan p = plan_tile_cached(ks, nk, nrbf, N, H, W, tile_h, tile_w, waves, mode, poly);
    if (!p.ok) return 0;
    const int R = ks / 2;
    const size_t tiles = (size_t)N * ((H + p.th - 1) / p.th) * ((W + p.tw - 1) / p.tw);
    return tiles * (size_t)(p.th + 2 * R) * (p.tw + 2 * R);
}

hipError_t fused_stage_input_grad(const StageArgs &s, hipStream_t stream)
{
    return fused_dispatch<MODE_BWD_INPUT>(s, stream);
}
// Blocks per row of a batched (forward, exchange form) tile of width tw.
static int batched_blocks(int tw) { return tw <= 32 ? 2 : (tw + 15) / 16; }

bool batched_config_ok(int ks, int nk, int nrbf, int th, int tw, int nw)
{
    const int R = ks / 2;
    const int nb = batched_blocks(tw);
    if (nb > 4 || th < 2 * R || tw < 2 * R) return false;  // a ring reaches one tile at most
    return lds_fits(ks, nk, nrbf, th, tw, nb, nw == 4 ? 4 : 8, MODE_FWD, RBF_HORNER);
}
hipError_t batched_launch(const BatchArgs &a, int ks, int nw, hipStream_t stream)
{
    const int nb = batched_blocks(a.Tw);
    const int rbfm = a.poly && lds_fits(ks, a.Nk, a.Nrbf, a.Th, a.Tw, nb, nw, MODE_FWD, RBF_POLY)
                         ? RBF_POLY
                         : RBF_HORNER;
    if (rbfm == RBF_POLY) {
        hipError_t e = batched_prep(a, ks, a.n_models, stream);
        if (e != hipSuccess) return e;
    }
    return batched_launch_impl(a, ks, nb, nw, rbfm, stream);
}

}  // namespace tnrd
