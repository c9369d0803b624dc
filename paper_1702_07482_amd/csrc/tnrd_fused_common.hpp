// Definitions shared by the fused forward/input-gradient kernel and the
// parameter-gradient kernels: MFMA vector type, RBF Horner constants, tap
// geometry.
#pragma once

#include <hip/hip_runtime.h>

#include "tnrd_device.hpp"

namespace tnrd {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short short4v __attribute__((ext_vector_type(4)));
typedef _Float16 half4v __attribute__((ext_vector_type(4)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef int int2v __attribute__((ext_vector_type(2)));
typedef int int4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// Operand types of the 16x16x16 MFMAs used by the mixed-precision path
// (v_mfma_f32_16x16x16_{bf16,f16}): lane l holds A[l % 16][4 (l / 16) + i]
// and B[4 (l / 16) + i][l % 16], i = 0..3; D is laid out as for 16x16x4 f32.
// Conversions round to nearest even.  The BF16 cvt4 converts four values as
// two packed pairs joined as 32-bit words: converting element by element into
// the operand vector compiled to one conversion per value plus a repacking
// permute per pair (FP16 pairs them either way).
enum Prec { PREC_F32 = 0, PREC_BF16 = 1, PREC_F16 = 2 };
template <int P> struct Mix;
template <> struct Mix<PREC_BF16> {
    typedef short4v V;
    static __device__ __forceinline__ short cvt(float x) { return __builtin_bit_cast(short, (__bf16)x); }
    static __device__ __forceinline__ V cvt4(floatx4 x)
    {
        const int lo = __builtin_bit_cast(int, __builtin_convertvector(float2v{x[0], x[1]}, bf16x2v));
        const int hi = __builtin_bit_cast(int, __builtin_convertvector(float2v{x[2], x[3]}, bf16x2v));
        return __builtin_bit_cast(V, int2v{lo, hi});
    }
    static __device__ __forceinline__ floatx4 mfma(V a, V b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    // the four values of an operand back in FP32 (exact)
    static __device__ __forceinline__ floatx4 widen4(V v)
    {
        floatx4 r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = __builtin_bit_cast(float, (int)((unsigned)(unsigned short)v[i] << 16));
        return r;
    }
};
template <> struct Mix<PREC_F16> {
    typedef half4v V;
    static __device__ __forceinline__ _Float16 cvt(float x) { return (_Float16)x; }
    static __device__ __forceinline__ V cvt4(floatx4 x)  // element-wise compiles well for FP16
    {
        return V{(_Float16)x[0], (_Float16)x[1], (_Float16)x[2], (_Float16)x[3]};
    }
    static __device__ __forceinline__ floatx4 mfma(V a, V b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ floatx4 widen4(V v)
    {
        return floatx4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    }
};
template <> struct Mix<PREC_F32> {  // placeholder so templates instantiate; never used
    typedef short4v V;
    static __device__ __forceinline__ short cvt(float) { return 0; }
    static __device__ __forceinline__ V cvt4(floatx4) { return V{0, 0, 0, 0}; }
    static __device__ __forceinline__ floatx4 mfma(V, V, floatx4 c) { return c; }
    static __device__ __forceinline__ floatx4 widen4(V) { return floatx4{0.f, 0.f, 0.f, 0.f}; }
};

constexpr int RBF_WIN = 5;                // Horner window half-width (11 centres)
constexpr int RBF_TERMS = 2 * RBF_WIN + 1;

// Piecewise polynomial form of the influence function (forward only).  On the
// unit interval of s = (z - mu0) / step around centre j0 (|s - j0| <= 1/2),
// phi is replaced by its degree-7 interpolant at the Chebyshev points of that
// interval.  The interpolant is linear in the weights:
//   phi(j0 + d) ~ sum_k c_k d^k,  c_k = sum_{|m| <= POLY_MW} M[k][|m|] sgn(m)^k w_{j0+m},
// where M[k][m] are the monomial coefficients of the interpolant of the single
// Gaussian exp(-rho (d - m)^2 / 2) (rho = (step/sigma)^2), so the table of c_k
// is built from the weights once per call (k_prep_stage).  Intervals run
// over j0 = -W .. Nrbf-1+W (W = RBF_WIN) with one zero interval at each end;
// beyond them phi is taken as 0, the same cut as the window of the Gaussian
// form.  Centres farther than POLY_MW spacings from the interval contribute
// below exp(-rho 6.5^2 / 2) of their weight and are left out.  The input-
// gradient mode, which needs phi', uses the interpolant of d phi / ds built the
// same way from the derivatives -rho (d - m) exp(-rho (d - m)^2 / 2) (Md[k][m],
// odd in m: c_k = sum Md[k][|m|] sgn(m)^(k+1) w_{j0+m}).
constexpr int POLY_DEG = 7;
constexpr int POLY_NC = POLY_DEG + 1;     // coefficients per interval
constexpr int POLY_MW = RBF_WIN + 1;      // centres on each side of j0 in the fit

__host__ __device__ inline int poly_intervals(int nrbf) { return nrbf + 2 * RBF_WIN + 2; }
// The table is laid out for at most POLY_NRBF_MAX centres (intervals past a
// smaller model's last one are zero), so its geometry is known at compile
// time and the kernel's table reads take immediate offsets.  Rows are padded
// to 4 mod 16 floats per filter, so the four filters a register quad's lane
// groups read start in distinct banks.
constexpr int POLY_NRBF_MAX = 63;
constexpr int POLY_NI = POLY_NRBF_MAX + 2 * RBF_WIN + 2;  // intervals per filter
constexpr int POLY_TFP = POLY_NC * POLY_NI + ((4 - POLY_NC * POLY_NI % 16) + 16) % 16;
// Interval coordinate given to masked-off pixels: an integer far beyond every
// table, so it clamps to the zero interval at the top end with d = 0.
constexpr float POLY_OFF_MASKED = 1048576.f;

// Cubic half-interval form (BF16 operands only): each unit interval's table row
// of 8 floats holds instead two cubics, one per half.  Half h (0: s below the
// centre j0, 1: above) is [j0 - 1/2 + h/2, j0 + h/2); with e = 2 (s - its left
// end) in [0, 1), phi ~ sum_{k<4} c_k e^k, the degree-3 interpolant at the
// Chebyshev points of e, c_k = sum_{|m| <= POLY_MW} P3[h][k][m + POLY_MW] w_{j0+m}
// (P3d for d phi / ds).  Summed over the centres its error stays below 2.6e-4
// (phi) and 6.7e-4 (d phi / ds) of the largest weight for rho < 1.4, a tenth of
// the BF16 rounding (2^-8) that the influence values get for the K^T GEMM.
constexpr int POLY3_NC = 4;
constexpr int POLY3_NM = 2 * POLY_MW + 1;

// Prepared-block form bits (beside bit 0, d phi / ds, and bit 1, the cubic
// half-interval table): the operand part holds the mixed kernels' filter
// operands converted to BF16 or FP16 instead of the FP32 kernels' ones.
constexpr int PREP_MIXED_BF16 = 8;
constexpr int PREP_MIXED_F16 = 16;

// Influence evaluation of the fused stage kernel.
enum RbfMethod { RBF_HORNER = 0, RBF_POLY = 1, RBF_POLY3 = 2 };

// Constants of the windowed Horner evaluation of phi.
//   s = (z - mu0) / step = j0 + d, j0 the nearest centre, |d| <= 1/2,
//   G_{j0+m}(z) = exp(-rho (d - m)^2 / 2), rho = (step / sigma)^2
//              = exp(-rho d^2 / 2) * q^m * exp(-rho m^2 / 2),  q = exp(rho d)
//   phi(z) = exp(-rho d^2 / 2 - rho W d) * sum_{n=0}^{2W} w_{j0-W+n} c_n q^n,
//   c_n = exp(-rho (n - W)^2 / 2).
struct FusedRbf {
    float mu0_over_step;  // mu0 / step
    float inv_step;       // 1 / step
    float rho_log2e;      // rho * log2(e)
    float jmax;           // Nrbf - 1 + W (largest clamped centre index)
    float rho_over_step;  // rho / step (chain factor of d phi / dz)
    float c[RBF_TERMS];
    float pm[POLY_NC][POLY_MW + 1];   // M[k][m] of the polynomial form of phi
    float pmd[POLY_NC][POLY_MW + 1];  // the same for d phi / ds (input-gradient mode)
    float p3[2][POLY3_NC][POLY3_NM];  // P3[h][k][m + POLY_MW] of the cubic half-interval form
    float p3d[2][POLY3_NC][POLY3_NM]; // the same for d phi / ds
};

// Forward stage in exchange form.  A tile computes z, phi and K^T v from its
// own pixels only; K^T spreads them over the tile plus an R ring, so each tile
// writes the diffusion force it contributes to those padded positions into a
// slab of its own:
//   slab_tau[dy][dx] = sum over own sources p of sum_i sum_(a,b) with
//                      p - (a - R, b - R) = (ty0 - R + dy, tx0 - R + dx)
//                      of k_i[a][b] v_i[p],
// dy < Th + 2R, dx < Tw + 2R (row pitch sw = Tw + 2R, sl = (Th + 2R) sw
// floats per slab, slabs tile-major).  The force at padded position q is the
// sum of the slabs of the tiles whose ring covers q, and the force at pixel p
// the sum over the padded positions that reflect onto p (the exact adjoint's
// fold).  The reaction of stage t is applied where u_t is next needed: in the
// prologue of stage t + 1 (over its u tile, own pixels written back) or by
// the final reaction kernel after the last stage.  Every tile then works on
// its own pixels only, with no recomputed halo of z and phi.
struct XTiles {
    int H, W;      // image
    int Th, Tw;    // tile (>= 2R each, so a padded position lies in the rings of at most 2 x 2 tiles)
    int nx, ny;    // tiles per row and per column
    int sw, sl;    // slab row pitch and floats per slab
};

// Tile of workgroup b in a 1-D grid of n tile workgroups.  The dispatcher deals
// consecutive workgroups to the eight XCDs in turn (b on XCD b mod 8), each XCD with
// its own L2; XCD x takes the contiguous run of tiles from x q + min(x, r) on
// (q = n / 8, r = n mod 8), so that a tile's neighbours, whose slabs and halo
// rows it reads, mostly run on its XCD.  A bijection of [0, n).
__host__ __device__ inline int xcd_tile_order(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

__host__ __device__ inline XTiles make_xtiles(int H, int W, int th, int tw, int R)
{
    XTiles x;
    x.H = H;
    x.W = W;
    x.Th = th;
    x.Tw = tw;
    x.nx = (W + tw - 1) / tw;
    x.ny = (H + th - 1) / th;
    x.sw = tw + 2 * R;
    x.sl = (th + 2 * R) * x.sw;
    return x;
}

// The slab entry of tile (ty, tx) at padded position (qy, qx) sits at
//   (ty nx + tx) sl + (qy - ty Th + R) sw + (qx - tx Tw + R)
//   = [ty nx sl + (qy - ty Th + R) sw] + [tx sl + (qx - tx Tw + R)],
// a row term plus a column term.  AxisTerms holds, for one axis of a pixel,
// the terms of its padded images (the pixel itself and, within R of the
// border, its mirror position, whose force the exact adjoint folds onto it)
// and of the one or two tiles whose ring covers each image.  A missing second
// tile repeats the first one's term (its load is masked), so every force sum
// issues the same loads in the same order.
struct AxisTerms {
    int t[2][2];   // [image][covering tile] term
    bool two[2];   // [image] a second covering tile exists
    bool mir;      // the mirror image exists
};

// Terms of pixel coordinate p (0 <= p < n) along an axis of tiles of size ts,
// nt of them; tile-index stride `ts_stride` (row axis: nx sl; column axis:
// sl) and coordinate stride `c_stride` (row axis: sw; column axis: 1).
template <int R>
__host__ __device__ __forceinline__ AxisTerms axis_terms(int p, int n, int ts, int nt, int ts_stride,
                                                         int c_stride)
{
    AxisTerms a;
    const int m = p < R ? -p - 1 : (p >= n - R ? 2 * n - 1 - p : p);
    a.mir = m != p;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int q = k == 0 ? p : m;
        const int tc = min(max(q, 0) / ts, nt - 1);
        const bool lo = tc > 0 && q < tc * ts + R;            // tile tc - 1 covers q
        const bool hi = tc + 1 < nt && q >= (tc + 1) * ts - R;  // tile tc + 1 covers q
        const int t0 = lo ? tc - 1 : tc, t1 = hi ? tc + 1 : tc;
        a.t[k][0] = t0 * ts_stride + (q - t0 * ts + R) * c_stride;
        a.t[k][1] = t1 * ts_stride + (q - t1 * ts + R) * c_stride;
        a.two[k] = t1 != t0;
    }
    return a;
}

template <int R>
__host__ __device__ __forceinline__ AxisTerms row_terms(const XTiles &g, int y)
{
    return axis_terms<R>(y, g.H, g.Th, g.ny, g.nx * g.sl, g.sw);
}

template <int R>
__host__ __device__ __forceinline__ AxisTerms col_terms(const XTiles &g, int x)
{
    return axis_terms<R>(x, g.W, g.Tw, g.nx, g.sl, 1);
}

// Force at the padded position given by row image iy and column image ix:
// the covering tiles' entries added in a fixed order.
__device__ __forceinline__ float xpad_terms(const float *__restrict__ xs, const AxisTerms &Y, int iy,
                                            const AxisTerms &X, int ix)
{
    const float v00 = xs[Y.t[iy][0] + X.t[ix][0]], v01 = xs[Y.t[iy][0] + X.t[ix][1]];
    const float v10 = xs[Y.t[iy][1] + X.t[ix][0]], v11 = xs[Y.t[iy][1] + X.t[ix][1]];
    float s = v00;
    s += X.two[ix] ? v01 : 0.f;
    s += Y.two[iy] ? v10 : 0.f;
    s += (Y.two[iy] && X.two[ix]) ? v11 : 0.f;
    return s;
}

// Diffusion force x[p] = sum_i K_i^T v_i at the pixel whose row and column
// terms are Y and X: the padded force at p plus, within R of the border, at
// its mirror positions.  Every caller (stage prologues, final reaction) forms
// the same bits.
__device__ __forceinline__ float force_at(const float *__restrict__ xs, const AxisTerms &Y,
                                          const AxisTerms &X)
{
    float s = xpad_terms(xs, Y, 0, X, 0);
    if (X.mir) s += xpad_terms(xs, Y, 0, X, 1);
    if (Y.mir) {
        s += xpad_terms(xs, Y, 1, X, 0);
        if (X.mir) s += xpad_terms(xs, Y, 1, X, 1);
    }
    return s;
}

template <int R>
__device__ __forceinline__ float pixel_force(const float *__restrict__ xs, const XTiles &g, int y, int x)
{
    return force_at(xs, row_terms<R>(g, y), col_terms<R>(g, x));
}

// Kernel arguments of one stage (forward or input-gradient mode).
struct FusedIO {
    const float *u_prev;  // forward: the stage input u_{t-1}, or with `pend` the state
                          // u_{t-2} its pending reaction starts from; input gradient: u_{t-1}
    const float *f;
    float *out;           // input gradient: g_{t-1}
    const float *u_cur;   // input gradient: u_t
    const float *g_cur;   // input gradient: g_t = dl/du_t
    float *za;            // input gradient, optional: z = K u and a = K e at the tile's own
                          // pixels, layout of za_index() (BF16 words with BF16 operands)
    int react;            // tnrd_reaction of the stage
    float proj_c;         // projected reaction: threshold c
    const float *prep;    // polynomial form: the stage's prepared table (and FP32 operands),
                          // k_prep_stage layout
    // forward (exchange form)
    const float *x_prev;  // pend: the previous stage's slabs (this image's first)
    float *x_out;         // this stage's slabs (this image's first)
    float *u_keep;        // pend: the tile's own pixels of u_{t-1} after the pending reaction
    const float *lam_prev;  // pend: lambda of the previous stage
    int pend;             // the previous stage's reaction is still to be applied
    int keep_table;       // polynomial form: the workgroup's LDS already holds this stage's
                          // table (a persistent workgroup's previous item), no copy
    XTiles xt;            // this image's tiling
};

// Export of z = K u and a = K e for the parameter-gradient kernels: per pixel
// 8 ceil(Nk / 4) floats, filters in quads, each quad's four z followed by its
// four a, so a lane holding four consecutive filters writes two 16-byte words.
__host__ __device__ inline int za_stride(int nk) { return 8 * ((nk + 3) / 4); }
__host__ __device__ inline size_t za_index(size_t pix, int nk, int f)  // z; a at + 4
{
    return pix * za_stride(nk) + 8 * (f >> 2) + (f & 3);
}
// With BF16 operands the export holds BF16 words (rounded to nearest even) at
// the same positions counted in 2-byte words: z and a as the BF16 filter-bank
// GEMMs produce them, in half the bytes.  Every other precision exports FP32
// (FP16's exponent range would not hold z).
__host__ __device__ inline bool za_is_bf16(int prec) { return prec == PREC_BF16; }
__device__ __forceinline__ float za_value(float x) { return x; }
__device__ __forceinline__ float za_value(unsigned short h)
{
    return __builtin_bit_cast(float, (unsigned)h << 16);
}

enum FusedMode { MODE_FWD = 0, MODE_BWD_INPUT = 1 };

FusedRbf make_fused_rbf(const RbfGrid &grid);

template <int KS>
struct Geo {
    static constexpr int R = KS / 2;
    static constexpr int KK = KS * KS;
    static constexpr int KS1 = (KK + 3) / 4;                         // GEMM1 k-steps
    static constexpr int MB2 = (KK % 16 <= 1) ? KK / 16 : (KK + 15) / 16;  // GEMM2 slot blocks
    static constexpr int VTAP = (KK > 16 * MB2) ? 1 : 0;             // leftover tap on the VALU
};

// Tap-slot geometry of the fused stage's K^T GEMM: accumulator register
// R' = 4 mb2 + r holds tap column b = R' / HB and, in lane group g, tap row
// a = 4 (R' % HB) + g, so that one register is one x-shift for all its lanes.
template <int KS>
struct Geo2 {
    static constexpr int HB = (KS + 3) / 4;            // registers per tap column
    static constexpr int NREG = KS * HB;               // registers that carry taps
    static constexpr int MB2 = (NREG + 3) / 4;         // 16-slot MFMA blocks
};

// Row shift of a DPP row (16 lanes): lane i of the result holds lane i + n of
// v (row_shl) or lane i - n (row_shr); lanes whose source is outside the row
// read 0.
template <int CTRL>
__device__ __forceinline__ float dpp_zero(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float row_shl(float v, int n)
{
    switch (n) {
    case 1: return dpp_zero<0x101>(v);
    case 2: return dpp_zero<0x102>(v);
    case 3: return dpp_zero<0x103>(v);
    case 4: return dpp_zero<0x104>(v);
    case 5: return dpp_zero<0x105>(v);
    case 6: return dpp_zero<0x106>(v);
    case 7: return dpp_zero<0x107>(v);
    case 8: return dpp_zero<0x108>(v);
    case 9: return dpp_zero<0x109>(v);
    case 10: return dpp_zero<0x10A>(v);
    case 11: return dpp_zero<0x10B>(v);
    case 12: return dpp_zero<0x10C>(v);
    case 13: return dpp_zero<0x10D>(v);
    case 14: return dpp_zero<0x10E>(v);
    case 15: return dpp_zero<0x10F>(v);
    default: return v;
    }
}

__device__ __forceinline__ float row_shr(float v, int n)
{
    switch (n) {
    case 1: return dpp_zero<0x111>(v);
    case 2: return dpp_zero<0x112>(v);
    case 3: return dpp_zero<0x113>(v);
    case 4: return dpp_zero<0x114>(v);
    case 5: return dpp_zero<0x115>(v);
    case 6: return dpp_zero<0x116>(v);
    case 7: return dpp_zero<0x117>(v);
    case 8: return dpp_zero<0x118>(v);
    case 9: return dpp_zero<0x119>(v);
    case 10: return dpp_zero<0x11A>(v);
    case 11: return dpp_zero<0x11B>(v);
    case 12: return dpp_zero<0x11C>(v);
    case 13: return dpp_zero<0x11D>(v);
    case 14: return dpp_zero<0x11E>(v);
    case 15: return dpp_zero<0x11F>(v);
    default: return v;
    }
}

}  // namespace tnrd
