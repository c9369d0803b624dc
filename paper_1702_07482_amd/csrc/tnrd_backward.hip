// Backward pass of the T-stage filter (gradients for training, Sec. 3.2).
//
// Per stage t (from T down to 1), with g = dl/du_t and the states u_{t-1}, u_t:
//
//   y   = du_t/d(ut_t) = u_t^2 / ((1+2l) u_t^2 + 2 l f^2)        (eq. derv2 via the prox output)
//   x_l = du_t/dl      = 2 (f^2 - u_t^2) / s,  s = (1+2l) u_t + 2 l f^2 / u_t   (eq. derv4)
//   e   = y g
//   z_i = K_i u_{t-1},  a_i = K_i e
//   dl^t   = sum_p g x_l
//   dW_ij  = - sum_p a_i G_j(z_i)
//   dK_i   = - sum_p ( phi_i(z_i) ebar[p - d] + phi_i'(z_i) a_i ubar[p - d] )   (d = tap offset)
//   g_{t-1} = e - sum_i K_i^T (phi_i'(z_i) a_i)                  (transposed eq. derv1-1)
//
// Three kernels per stage, then one deterministic reduction:
//   k_fused_stage<.., MODE_BWD_INPUT>  the force sum_i K_i^T(phi_i'(z_i) a_i) of
//                  each tile's own pixels into its slab (tnrd_fused_tile.hpp), then
//                  k_grad_finish forms g_{t-1} from the slabs; with FP32 or BF16
//                  operands the first also stores z and a of every pixel
//                  (za_index layout; BF16 words with BF16 operands)
//   k_bwd_params   dK and dl partial sums per tile, from the stored z, a (FP32,
//                  BF16), or computing and storing them itself (FP16, and the
//                  first stage when dl/du_0 is not asked for)
//   k_bwd_dw       dW partial sums from the stored z, a
//   k_reduce_partials  fixed-order sums of the partials into the outputs (one launch)
//
// In k_bwd_params lane (g, j) holds, for register r, pixel 4g + r of a 16-pixel
// block and filter j of a 16-filter block: that register is exactly the B
// operand of the dK^T GEMM (rows = taps, k = pixels) for k-step r if k-row g
// of that step is pixel 4g + r, so v and phi'a go from the influence function
// straight into the weight-gradient contraction without passing through LDS.
// When it computes z and a itself, the filter-bank GEMM runs transposed
// (rows = 16 pixels, columns = 16 filters) to leave them in that layout.
// With BF16/FP16 operands (the mixed-precision backward), the dK contraction
// runs on v_mfma_f32_16x16x16_{bf16,f16} with FP32 accumulation (k = the
// block's 16 pixels in one step, whose B operand is the block's v or phi'a
// quad, pixels 4g .. 4g+3 of filter j, converted once), and ubar enters the
// second dK term as a BF16/FP16 pair ubar = hi + lo (two MFMAs).  With FP16, e
// enters scaled by a per-tile power of two (max |e| -> 2^10, FP16's normal
// range) that is undone in FP32 on dK and on the exported a.  With BF16, z and a are
// the input-gradient kernel's (its BF16 GEMMs; z is then where the BF16
// forward evaluated phi), loaded from its BF16 export.  With FP16, and at a
// first stage without dl/du_0, k_bwd_params computes them: a = K e on the
// 16x16x16 instruction (the transposed bank, k = 16 taps per step), and z = K u
// on the same BF16 instruction with BF16 operands, or on the FP32 instruction
// with FP16 operands, since u carries a large mean that 11 mantissa bits of u
// or of k would move z by several units.  The influence function and dlambda
// stay FP32.
//
// k_bwd_dw scatters a_i G_j(z_i) into per-wave histograms, each lane working
// on one filter and owning its column (a filter has several lanes, each with a
// share of the pixels), so no two lanes ever update the same word and no
// atomics are needed.
#include <limits.h>
#include <math.h>

#include <type_traits>
#include <vector>

#include "tnrd.h"
#include "tnrd_api_internal.hpp"
#include "tnrd_device.hpp"
#include "tnrd_fused_common.hpp"
#include "tnrd_internal.hpp"

namespace tnrd {

constexpr int BP_TH_MIN = 16;  // k_bwd_params tile height range (the workspace is sized
constexpr int BP_TH_MAX = 64;  // for the smallest, i.e. the most tiles)
constexpr int BP_NBW = 2;   // 16-pixel blocks per tile row (tile width 32)
constexpr int BP_NW = 4;    // waves per workgroup
constexpr int DW_U = 16;    // k_bwd_dw pixels per wave step
constexpr int ZA_PAD = 128; // slack after the z/a export: a filter block past Nk read at the
                            // last pixel stays inside the buffer (32 NMB - 1 < ZA_PAD words)

struct BwdParamsIO {
    const float *u_prev;  // u_{t-1}
    const float *u_cur;   // u_t
    const float *f;
    const float *g_cur;   // dl/du_t
    float *za;            // z = K u_{t-1} and a = K e per pixel (za_index layout)
    float *dk_part;       // [tiles][Nk*KK]
    float *dl_part;       // [tiles]
    float *gf;            // nullable [N*H*W]: dl/df, this stage's explicit term added
    int gf_first;         // nonzero: write gf instead of adding to it
    int react;            // tnrd_reaction
    float proj_c;         // projected reaction: threshold c
};

struct BpLds {
    int ldw, tile_size, u_off, e_off, t_off, t_pitch, red_off, red_size, dl_off, mb_off, total;
};

// mixed: room for the BF16/FP16 filter operands of a = K e, [nb][k-step][lane]
// (8 bytes each)
__host__ __device__ inline BpLds bp_lds(int ks, int nmb, int th, int tw, int nrbf, int nw,
                                        bool mixed = false)
{
    const int R = ks / 2;
    BpLds l;
    l.ldw = tw + 2 * R + 1;
    l.tile_size = (th + 2 * R) * l.ldw;
    l.u_off = 0;
    l.e_off = l.tile_size;
    l.t_pitch = nrbf + 4 * RBF_WIN + 1;  // weight positions per filter (zero padded by 2W)
    l.t_off = 2 * l.tile_size;
    l.red_off = l.t_off + 16 * nmb * l.t_pitch;
    l.red_size = 16 * nmb * ks * ks;
    l.dl_off = l.red_off + l.red_size;
    l.mb_off = (l.dl_off + nw + 1) & ~1;
    l.total = l.mb_off + (mixed ? nmb * ((ks * ks + 15) / 16) * 64 * 2 : 0);
    return l;
}

// Horner evaluation of phi(z) and phi'(z) from the LDS weight table: the
// weights of a block of 16 filters are position-major, [position][16]; col
// points at the lane's filter in position 0.  Lanes of one read hold 16
// different filters (distinct banks whatever their positions, up to a multiple
// of 16) and four pixels each.
__device__ __forceinline__ void rbf_phi_dphi_horner(float z, const float *__restrict__ col,
                                                    const FusedRbf &rb, float &phi, float &dphi)
{
    float s = fmaf(z, rb.inv_step, -rb.mu0_over_step);
    float jr = fminf(fmaxf(rintf(s), -(float)RBF_WIN), rb.jmax);
    float d = s - jr;
    const float *w = col + ((int)jr + RBF_WIN) * 16;
    float q = __builtin_amdgcn_exp2f(rb.rho_log2e * d);
    float E = __builtin_amdgcn_exp2f(-rb.rho_log2e * d * fmaf(0.5f, d, (float)RBF_WIN));
    float acc = w[16 * 2 * RBF_WIN] * rb.c[2 * RBF_WIN];
    float accd = 0.f;
#pragma unroll
    for (int n = 2 * RBF_WIN - 1; n >= 0; --n) {
        accd = fmaf(accd, q, acc);
        acc = fmaf(acc, q, w[16 * n] * rb.c[n]);
    }
    const bool in = fabsf(d) <= 0.5f;
    phi = in ? E * acc : 0.f;
    dphi = in ? rb.rho_over_step * E * fmaf(q, accd, -(d + (float)RBF_WIN) * acc) : 0.f;
}

// The variant loading z and a is held to 128 registers (4 waves per SIMD when
// the LDS allows it); it loads each block's z and a right before using them.
// The one computing them is held to 256 (2 waves per SIMD); it reads a filter
// block's GEMM operands from the LDS copy of the bank when it starts the block.
template <int KS, int NMB, int NBW, int NW, bool LOADZA, int PREC>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(LOADZA ? 3 : 2, 8)))
k_bwd_params(
    BwdParamsIO io, int H, int W, int Th, int tiles_x, int tiles_per_img,
    const float *__restrict__ filt, int Nk, const float *__restrict__ rbfw, int Nrbf, FusedRbf rb,
    const float *__restrict__ lam_t)
{
    using G = Geo<KS>;
    constexpr int R = G::R, KK = G::KK, KS1 = G::KS1, MB2 = G::MB2;
    constexpr int THREADS = 64 * NW;
    constexpr int Tw = 16 * NBW;
    constexpr bool MIXED = PREC != PREC_F32;
    static_assert(!(LOADZA && PREC == PREC_F16), "FP16 operands: z and a are computed here");
    using MX = Mix<PREC>;
    typedef typename MX::V MV;
    constexpr int KSH = (KK + 15) / 16;  // mixed: transposed filter-bank k-steps of 16 taps

    extern __shared__ float lds[];
    const BpLds L = bp_lds(KS, NMB, Th, Tw, Nrbf, NW, MIXED && !LOADZA);
    float *su = lds + L.u_off;
    float *se = lds + L.e_off;
    float *stab = lds + L.t_off;
    float *red = lds + L.red_off;
    float *sdl = lds + L.dl_off;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int bid = xcd_tile_order((int)blockIdx.x, (int)gridDim.x);  // tile and partial slot
    const int img = bid / tiles_per_img;
    const int trem = bid - img * tiles_per_img;
    const int ty = trem / tiles_x, tx = trem - ty * tiles_x;
    const int ty0 = ty * Th, tx0 = tx * Tw;
    const size_t plane = (size_t)H * W;
    const float lam = lam_t[0];
    const float c1 = 1.f + 2.f * lam, c2 = 2.f * lam;

    // ---- prologue: filters (via red; not needed when z and a are loaded),
    // u_{t-1} and e tiles with an R ring, weight table
    if (!LOADZA) {
        const int nf = Nk * KK;
        for (int base = 0; base < nf; base += 8 * THREADS) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = filt[min(base + k * THREADS + tid, nf - 1)];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (base + k * THREADS + tid < nf) red[base + k * THREADS + tid] = v[k];
        }
    }
    float dl_acc = 0.f;
    float emax = 0.f;  // mixed: largest |e| of the tile
    {
        const float *un = io.u_prev + img * plane;
        const float *uc = io.u_cur + img * plane;
        const float *fn = io.f + img * plane;
        const float *gn = io.g_cur + img * plane;
        const int luh = Th + 2 * R, luw = Tw + 2 * R;
        const int n = luh * luw;
        for (int base = 0; base < n; base += 4 * THREADS) {
            float uu[4], uv[4], ff[4], gg[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int i = min(base + k * THREADS + tid, n - 1);
                int ly = i / luw, lx = i - ly * luw;
                int yy = reflect_clamp(ty0 - R + ly, H), xx = reflect_clamp(tx0 - R + lx, W);
                size_t q = (size_t)yy * W + xx;
                uu[k] = un[q];
                uv[k] = uc[q];
                ff[k] = fn[q];
                gg[k] = gn[q];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int i = base + k * THREADS + tid;
                if (i < n) {
                    int ly = i / luw, lx = i - ly * luw;
                    float u2 = uv[k] * uv[k], f2 = ff[k] * ff[k];
                    float den = fmaf(c1, u2, c2 * f2);  // u s
                    su[ly * L.ldw + lx] = uu[k];
                    const bool proj = io.react == 1, quad = io.react == 2;
                    // e = y g: prox y = u_t^2 / (u_t s); projected y = [u_t > c]; quadratic y = 1
                    const float ev = proj ? (uv[k] > io.proj_c ? gg[k] : 0.f)
                                     : quad ? gg[k] : u2 / den * gg[k];
                    se[ly * L.ldw + lx] = ev;
                    emax = fmaxf(emax, fabsf(ev));
                    int yi = ty0 - R + ly, xi = tx0 - R + lx;
                    bool own = ly >= R && ly < R + Th && lx >= R && lx < R + Tw && yi < H && xi < W;
                    if (own) {
                        // dl/dlambda over the tile's own pixels: prox g 2 (f - u)(f + u) / s (the
                        // factored difference keeps its precision when u ~ f); projected
                        // -e (d psi/dl)(u_{t-1}); quadratic -e (u_{t-1} - f)
                        dl_acc = proj   ? fmaf(-ev, proj_psi_dlam(uu[k], ff[k]), dl_acc)
                                 : quad ? fmaf(-ev, uu[k] - ff[k], dl_acc)
                                        : fmaf(gg[k], 2.f * (ff[k] - uv[k]) * (ff[k] + uv[k]) * uv[k] / den, dl_acc);
                        if (io.gf) {
                            // explicit f-dependence of u_t: prox du/df = 4 l f / s = 4 l f u / (u s);
                            // projected -e (d psi/df)(u_{t-1}); quadratic l e
                            const float fx = proj   ? -ev * proj_psi_df(uu[k], ff[k], lam)
                                             : quad ? lam * ev
                                                    : gg[k] * (4.f * lam * ff[k] * uv[k] / den);
                            float *gp = io.gf + img * plane + (size_t)yi * W + xi;
                            *gp = io.gf_first ? fx : *gp + fx;
                        }
                    }
                }
            }
        }
    }
    {
        const int n = 16 * NMB * L.t_pitch;
        const int nw = Nk * Nrbf;
        for (int base = 0; base < n; base += 8 * THREADS) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                int i = base + k * THREADS + tid;
                // table word i = (nb t_pitch + position) 16 + filter-in-block
                const int blk = i / (16 * L.t_pitch), rem = i - blk * 16 * L.t_pitch;
                const int pos = rem >> 4, fi = 16 * blk + (rem & 15), jj = pos - 2 * RBF_WIN;
                float w = rbfw[min(max(fi * Nrbf + jj, 0), nw - 1)];
                v[k] = (fi < Nk && jj >= 0 && jj < Nrbf) ? w : 0.f;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (base + k * THREADS + tid < n) stab[base + k * THREADS + tid] = v[k];
        }
    }
    // FP16 operands: e is scaled by 2^(10 - ilogb(max |e|)) before its conversion
    // (FP16's normal range is 2^-14 .. 65504; |K e| <= 7 max|e| for unit-norm 7x7
    // filters).  BF16 has FP32's exponent range and needs no scale.
    constexpr bool ESCALE = PREC == PREC_F16;
    float escale = 1.f, einv = 1.f;
    if (ESCALE) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) emax = fmaxf(emax, __shfl_xor(emax, o));
        if (lane == 0) sdl[wave] = emax;
    }
    __syncthreads();
    if (ESCALE) {
        float mx = 0.f;
        for (int w = 0; w < NW; ++w) mx = fmaxf(mx, sdl[w]);
        if (mx > 0.f && isfinite(mx)) {
            const int ex = ilogbf(mx);
            escale = ldexpf(1.f, 10 - ex);
            einv = ldexpf(1.f, ex - 10);
        }
        __syncthreads();  // sdl is read again for dlambda at the end
    }

    // filter bank as the B operand of the transposed GEMM: B[k=g][n=j] = k_{16 nb + j}[tap 4 s + g]
    // (block nb read from the staged bank in red when it is used)
    auto load_bf = [&](int nb, float *bf) {
#pragma unroll
        for (int s = 0; s < KS1; ++s) {
            const int fi = 16 * nb + j, t = 4 * s + g;
            bf[s] = (fi < Nk && t < KK) ? red[fi * KK + t] : 0.f;
        }
    };
    int off1[KS1];
#pragma unroll
    for (int s = 0; s < KS1; ++s) {
        int t = 4 * s + g;
        off1[s] = t < KK ? (t / KS) * L.ldw + (t % KS) : 0;
    }
    // dK^T GEMM rows: tap 16 mt + j
    int offt[MB2];
    bool tapok[MB2];
#pragma unroll
    for (int mt = 0; mt < MB2; ++mt) {
        int t = 16 * mt + j;
        tapok[mt] = t < KK;
        offt[mt] = t < KK ? (t / KS) * L.ldw + (t % KS) : 0;
    }
    const int offv = ((KK - 1) / KS) * L.ldw + (KK - 1) % KS;  // leftover tap (VALU)

    floatx4 dkt[MB2][NMB];
#pragma unroll
    for (int mt = 0; mt < MB2; ++mt)
#pragma unroll
        for (int nb = 0; nb < NMB; ++nb) dkt[mt][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    float acc48[NMB];
#pragma unroll
    for (int nb = 0; nb < NMB; ++nb) acc48[nb] = 0.f;

    // dK^T GEMM of one filter block nb of a 16-pixel block: k-step r, k-row g =
    // pixel 4 g + r; vz = v = phi(z), vh = phi'(z) a of those pixels
    auto dk_block = [&](int y, int cb, int nb, const floatx4 &vz, const floatx4 &vh) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = 16 * cb + 4 * g + r;
            const int b2 = (y + 2 * R) * L.ldw + x + 2 * R;
#pragma unroll
            for (int mt = 0; mt < MB2; ++mt) {
                float ae = tapok[mt] ? se[b2 - offt[mt]] : 0.f;
                float au = tapok[mt] ? su[b2 - offt[mt]] : 0.f;
                dkt[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ae, vz[r], dkt[mt][nb], 0, 0, 0);
                dkt[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(au, vh[r], dkt[mt][nb], 0, 0, 0);
            }
            if (G::VTAP) {
                float ev = se[b2 - offv], uvv = su[b2 - offv];
                acc48[nb] = fmaf(vz[r], ev, fmaf(vh[r], uvv, acc48[nb]));
            }
        }
    };

    if constexpr (LOADZA) {
        // z and a exported by the input-gradient kernel, pixel 4 g + r of the
        // block and filter 16 nb + j per lane, loaded at the start of the block
        // (the other waves of the SIMD cover the wait)
        const int ylim = min(Th, H - ty0);
        const int nrows = ylim > wave ? (ylim - wave + NW - 1) / NW : 0;
        const int nblk = nrows * NBW;
        const int zst = za_stride(Nk);
        // filter 16 nb + j of pixel p sits at p zst + 32 nb + 8 (j >> 2) + (j & 3) (z; a four
        // words on): one address per pixel, the filter blocks at immediate offsets.  The
        // address of a pixel past the image row or of a row past the tile is clamped into
        // the image (its values are dropped); a filter block past Nk may read into the next
        // pixel, and the export buffer carries ZA_PAD floats of slack for the last one.
        // FP32 words, or BF16 words with BF16 operands
        using ZT = typename std::conditional<MIXED, unsigned short, float>::type;
        const ZT *zaimg = reinterpret_cast<const ZT *>(io.za) + img * plane * zst + 8 * (j >> 2) + (j & 3);
        ZT zn[NMB][4], an[NMB][4];
        // raw values; the mask of a pixel past the image row or a filter past Nk
        // is applied when the block is used
        auto load = [&](int b) {
            const int y = wave + NW * (b / NBW), cb = b % NBW;
            const int yy = b < nblk ? ty0 + y : ty0;
            const ZT *rowp = zaimg + (size_t)yy * W * zst;
            const int xb = tx0 + 16 * cb + 4 * g;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const ZT *pp = rowp + (size_t)(min(xb + r, W - 1) * zst);
#pragma unroll
                for (int nb = 0; nb < NMB; ++nb) {
                    zn[nb][r] = pp[32 * nb];
                    an[nb][r] = pp[32 * nb + 4];
                }
            }
        };
        // one block ahead: the loads of block b + 1 are in flight while block b
        // is computed (a block past the end loads clamped in-image addresses)
        if (nblk > 0) load(0);
#pragma unroll 1
        for (int b = 0; b < nblk; ++b) {
            float zc[NMB][4], ac[NMB][4];
            const int xb = tx0 + 16 * (b % NBW) + 4 * g;
#pragma unroll
            for (int nb = 0; nb < NMB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool ok = xb + r < W && 16 * nb + j < Nk;
                    zc[nb][r] = ok ? za_value(zn[nb][r]) : 0.f;
                    ac[nb][r] = ok ? escale * za_value(an[nb][r]) : 0.f;
                }
            load(b + 1);
            const int y = wave + NW * (b / NBW), cb = b % NBW;
            if constexpr (MIXED) {
                // BF16: the dK contraction on the 16x16x16 instruction, as in the
                // computing variant below (A = scaled ebar, and ubar as hi + lo)
                MV de[MB2], duh[MB2], dul[MB2];
#pragma unroll
                for (int mt = 0; mt < MB2; ++mt) {
                    floatx4 xe, xu, xl;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int b2 = (y + 2 * R) * L.ldw + 16 * cb + 4 * g + i + 2 * R;
                        xe[i] = tapok[mt] ? escale * se[b2 - offt[mt]] : 0.f;
                        xu[i] = tapok[mt] ? su[b2 - offt[mt]] : 0.f;
                    }
                    de[mt] = MX::cvt4(xe);
                    duh[mt] = MX::cvt4(xu);
                    const floatx4 hi = MX::widen4(duh[mt]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) xl[i] = xu[i] - hi[i];
                    dul[mt] = MX::cvt4(xl);
                }
#pragma unroll
                for (int nb = 0; nb < NMB; ++nb) {
                    const float *row = stab + nb * 16 * L.t_pitch + j;
                    floatx4 vz, vh;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bool valid = tx0 + 16 * cb + 4 * g + r < W;
                        float ph, dph;
                        rbf_phi_dphi_horner(zc[nb][r], row, rb, ph, dph);
                        vz[r] = valid ? ph : 0.f;
                        vh[r] = valid ? dph * ac[nb][r] : 0.f;
                    }
                    const MV vb = MX::cvt4(vz), hb = MX::cvt4(vh);
#pragma unroll
                    for (int mt = 0; mt < MB2; ++mt) {
                        dkt[mt][nb] = MX::mfma(de[mt], vb, dkt[mt][nb]);
                        dkt[mt][nb] = MX::mfma(duh[mt], hb, dkt[mt][nb]);
                        dkt[mt][nb] = MX::mfma(dul[mt], hb, dkt[mt][nb]);
                    }
                    if (G::VTAP) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int b2 = (y + 2 * R) * L.ldw + 16 * cb + 4 * g + r + 2 * R;
                            const float ev = escale * se[b2 - offv], uvv = su[b2 - offv];
                            acc48[nb] = fmaf(vz[r], ev, fmaf(vh[r], uvv, acc48[nb]));
                        }
                    }
                }
            } else {
#pragma unroll
                for (int nb = 0; nb < NMB; ++nb) {
                    const float *row = stab + nb * 16 * L.t_pitch + j;
                    floatx4 vz, vh;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bool valid = tx0 + 16 * cb + 4 * g + r < W;
                        float ph, dph;
                        rbf_phi_dphi_horner(zc[nb][r], row, rb, ph, dph);
                        vz[r] = valid ? ph : 0.f;
                        vh[r] = valid ? dph * ac[nb][r] : 0.f;
                    }
                    dk_block(y, cb, nb, vz, vh);
                }
            }
        }
    }
    if constexpr (MIXED && !LOADZA) {
        // transposed filter bank of a = K e as the B operand, converted once into
        // LDS, [nb][s][lane]: lane (g, j) holds taps 16 s + 4 g + i (i = 0..3) of
        // filter 16 nb + j
        MV *smb = reinterpret_cast<MV *>(lds + L.mb_off);
        for (int q = tid; q < NMB * KSH * 64; q += THREADS) {
            const int ql = q & 63, qs = (q >> 6) % KSH, qn = (q >> 6) / KSH;
            const int qg = ql >> 4, qj = ql & 15;
            floatx4 x;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int fi = 16 * qn + qj, t = 16 * qs + 4 * qg + i;
                x[i] = (fi < Nk && t < KK) ? red[fi * KK + t] : 0.f;
            }
            smb[q] = MX::cvt4(x);
        }
        __syncthreads();
        int offm[KSH][4];
#pragma unroll
        for (int s = 0; s < KSH; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int t = 16 * s + 4 * g + i;
                offm[s][i] = t < KK ? (t / KS) * L.ldw + (t % KS) : 0;
            }
        for (int y = wave; y < Th; y += NW) {
            const int yi = ty0 + y;
            if (yi >= H) break;
#pragma unroll 1
            for (int cb = 0; cb < NBW; ++cb) {
                // A operands of K u (FP16 operands: FP32, 4 taps per k-step; BF16:
                // BF16, 16 taps per k-step, as the input-gradient kernel's z of the
                // other stages) and of K e (scaled, 16 taps per k-step) at pixel j
                const float *ubase = su + (y + 2 * R) * L.ldw + 16 * cb + j + 2 * R;
                const float *ebase = se + (y + 2 * R) * L.ldw + 16 * cb + j + 2 * R;
                constexpr bool ZB = PREC == PREC_BF16;
                float bu[ZB ? 1 : KS1];
                if constexpr (!ZB) {
#pragma unroll
                    for (int s = 0; s < KS1; ++s) bu[s] = ubase[-off1[s]];
                }
                MV ae[KSH], au[ZB ? KSH : 1];
#pragma unroll
                for (int s = 0; s < KSH; ++s) {
                    floatx4 xe, xu;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        xe[i] = escale * ebase[-offm[s][i]];
                        if constexpr (ZB) xu[i] = ubase[-offm[s][i]];
                    }
                    ae[s] = MX::cvt4(xe);
                    if constexpr (ZB) au[s] = MX::cvt4(xu);
                }
                // A operands of the dK contraction: rows = taps 16 mt + j, k = the
                // block's pixels 4 g + i: scaled ebar, and ubar as hi + lo
                MV de[MB2], duh[MB2], dul[MB2];
#pragma unroll
                for (int mt = 0; mt < MB2; ++mt) {
                    floatx4 xe, xu, xl;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int b2 = (y + 2 * R) * L.ldw + 16 * cb + 4 * g + i + 2 * R;
                        xe[i] = tapok[mt] ? escale * se[b2 - offt[mt]] : 0.f;
                        xu[i] = tapok[mt] ? su[b2 - offt[mt]] : 0.f;
                    }
                    de[mt] = MX::cvt4(xe);
                    duh[mt] = MX::cvt4(xu);
                    const floatx4 hi = MX::widen4(duh[mt]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) xl[i] = xu[i] - hi[i];
                    dul[mt] = MX::cvt4(xl);
                }
#pragma unroll
                for (int nb = 0; nb < NMB; ++nb) {
                    floatx4 accz = floatx4{0.f, 0.f, 0.f, 0.f}, acca = floatx4{0.f, 0.f, 0.f, 0.f};
                    if constexpr (!ZB) {
                        float bf[KS1];
                        load_bf(nb, bf);
#pragma unroll
                        for (int s = 0; s < KS1; ++s)
                            accz = __builtin_amdgcn_mfma_f32_16x16x4f32(bu[s], bf[s], accz, 0, 0, 0);
                    }
#pragma unroll
                    for (int s = 0; s < KSH; ++s) {
                        const MV kb = smb[(nb * KSH + s) * 64 + lane];
                        if constexpr (ZB) accz = MX::mfma(au[s], kb, accz);
                        acca = MX::mfma(ae[s], kb, acca);
                    }
                    // influence, export (a unscaled), and the dK operands v, h (scaled) in place
                    const float *row = stab + nb * 16 * L.t_pitch + j;
                    const int fi = 16 * nb + j;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int x = 16 * cb + 4 * g + r, xi = tx0 + x;
                        const bool valid = xi < W;
                        const float z = accz[r], a = acca[r];
                        float ph, dph;
                        rbf_phi_dphi_horner(z, row, rb, ph, dph);
                        if (valid && fi < Nk) {
                            const size_t zi = za_index(img * plane + (size_t)yi * W + xi, Nk, fi);
                            if constexpr (PREC == PREC_BF16) {
                                unsigned short *zq = reinterpret_cast<unsigned short *>(io.za);
                                zq[zi] = (unsigned short)MX::cvt(z);
                                zq[zi + 4] = (unsigned short)MX::cvt(a * einv);
                            } else {
                                io.za[zi] = z;
                                io.za[zi + 4] = a * einv;
                            }
                        }
                        accz[r] = valid ? ph : 0.f;
                        acca[r] = valid ? dph * a : 0.f;
                    }
                    const MV vb = MX::cvt4(accz), hb = MX::cvt4(acca);
#pragma unroll
                    for (int mt = 0; mt < MB2; ++mt) {
                        dkt[mt][nb] = MX::mfma(de[mt], vb, dkt[mt][nb]);
                        dkt[mt][nb] = MX::mfma(duh[mt], hb, dkt[mt][nb]);
                        dkt[mt][nb] = MX::mfma(dul[mt], hb, dkt[mt][nb]);
                    }
                    if (G::VTAP) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int b2 = (y + 2 * R) * L.ldw + 16 * cb + 4 * g + r + 2 * R;
                            const float ev = escale * se[b2 - offv], uvv = su[b2 - offv];
                            acc48[nb] = fmaf(accz[r], ev, fmaf(acca[r], uvv, acc48[nb]));
                        }
                    }
                }
            }
        }
    }
    if constexpr (MIXED) {
        // back to the gradient's own scale
#pragma unroll
        for (int nb = 0; nb < NMB; ++nb) {
            acc48[nb] *= einv;
#pragma unroll
            for (int mt = 0; mt < MB2; ++mt) dkt[mt][nb] *= einv;
        }
    }
    for (int y = wave; !LOADZA && !MIXED && y < Th; y += NW) {
        const int yi = ty0 + y;
        if (yi >= H) break;
#pragma unroll 1
        for (int cb = 0; cb < NBW; ++cb) {
            // transposed GEMM1: rows = pixels j of the block, columns = filters;
            // its B operands (u and e at every tap) are read once per block
            const float *ubase = su + (y + 2 * R) * L.ldw + 16 * cb + j + 2 * R;
            const float *ebase = se + (y + 2 * R) * L.ldw + 16 * cb + j + 2 * R;
            float bu[KS1], be[KS1];
#pragma unroll
            for (int s = 0; s < KS1; ++s) {
                bu[s] = ubase[-off1[s]];
                be[s] = ebase[-off1[s]];
            }
            // one filter block at a time keeps 8 response registers live
#pragma unroll
            for (int nb = 0; nb < NMB; ++nb) {
                floatx4 accz = floatx4{0.f, 0.f, 0.f, 0.f}, acca = floatx4{0.f, 0.f, 0.f, 0.f};
                float bf[KS1];
                load_bf(nb, bf);
#pragma unroll
                for (int s = 0; s < KS1; ++s) {
                    accz = __builtin_amdgcn_mfma_f32_16x16x4f32(bu[s], bf[s], accz, 0, 0, 0);
                    acca = __builtin_amdgcn_mfma_f32_16x16x4f32(be[s], bf[s], acca, 0, 0, 0);
                }
                // influence, export, and the two dK operands (v, h) in place
                const float *row = stab + nb * 16 * L.t_pitch + j;
                const int fi = 16 * nb + j;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int x = 16 * cb + 4 * g + r, xi = tx0 + x;
                    const bool valid = xi < W;
                    float z = accz[r], a = acca[r];
                    float ph, dph;
                    rbf_phi_dphi_horner(z, row, rb, ph, dph);
                    if (valid && fi < Nk) {
                        size_t pix = img * plane + (size_t)yi * W + xi;
                        io.za[za_index(pix, Nk, fi)] = z;
                        io.za[za_index(pix, Nk, fi) + 4] = a;
                    }
                    accz[r] = valid ? ph : 0.f;
                    acca[r] = valid ? dph * a : 0.f;
                }
                dk_block(y, cb, nb, accz, acca);
            }
        }
    }

    // ---- tile reduction of dK (waves in order) and dl
    if (G::VTAP) {
#pragma unroll
        for (int nb = 0; nb < NMB; ++nb) {
            acc48[nb] += __shfl_xor(acc48[nb], 16);
            acc48[nb] += __shfl_xor(acc48[nb], 32);
        }
    }
    __syncthreads();  // red (filter staging) is free again
    for (int w = 0; w < NW; ++w) {
        if (wave == w) {
#pragma unroll
            for (int mt = 0; mt < MB2; ++mt)
#pragma unroll
                for (int nb = 0; nb < NMB; ++nb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        int t = 16 * mt + 4 * g + r, fi = 16 * nb + j;
                        if (t < KK && !(G::VTAP && t == KK - 1)) {
                            float *dst = red + fi * KK + t;
                            *dst = (w == 0 ? 0.f : *dst) + dkt[mt][nb][r];
                        }
                    }
            if (G::VTAP && g == 0) {
#pragma unroll
                for (int nb = 0; nb < NMB; ++nb) {
                    float *dst = red + (16 * nb + j) * KK + KK - 1;
                    *dst = (w == 0 ? 0.f : *dst) + acc48[nb];
                }
            }
        }
        __syncthreads();
    }
    // dl: wave sums, then the waves in order
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dl_acc += __shfl_xor(dl_acc, o);
    if (lane == 0) sdl[wave] = dl_acc;
    __syncthreads();
    float *dkp = io.dk_part + (size_t)bid * Nk * KK;
    for (int i = tid; i < Nk * KK; i += THREADS) dkp[i] = red[i];
    if (tid == 0) {
        float sum = 0.f;
        for (int w = 0; w < NW; ++w) sum += sdl[w];
        io.dl_part[bid] = sum;
    }
}

// k_bwd_dw histograms are bin-major, [bin][64 lanes]: bin b of the lane's
// filter at word (b + 2W) * 64 + lane.  Every lane of a wave owns a bank of its
// own, so the 64 lanes of an update never conflict whatever bins their z
// values fall in (a filter-major layout, [filter][bins], puts lanes whose
// bins differ by a multiple of the bank count on one bank).  Updates are
// plain read-modify-writes: the LDS float atomic add measured over ten times
// slower for this pattern.
__host__ __device__ inline int dw_bins(int nrbf) { return nrbf + 4 * RBF_WIN; }
__host__ __device__ inline size_t dw_wave_bytes(int nrbf) { return (size_t)dw_bins(nrbf) * 64 * sizeof(float); }

// dW partial sums: each wave its own histogram, each lane one filter and a share
// of the workgroup's pixels.  ZT: the export's words (float, or BF16 bits).
template <int NW, typename ZT>
__global__ void __launch_bounds__(64 * NW) k_bwd_dw(
    const ZT *__restrict__ za, long long P, long long per_wg,
    int Nk, int Nrbf, FusedRbf rb, float *__restrict__ dw_part)
{
    extern __shared__ float lds[];
    const int hsize = dw_bins(Nrbf) * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < NW * hsize; i += 64 * NW) lds[i] = 0.f;
    __syncthreads();
    float *hist = lds + wave * hsize + 2 * RBF_WIN * 64 + lane;
    const long long p0 = (long long)blockIdx.x * per_wg;
    const long long p1 = min(P, p0 + per_wg);
    // slot sl = 64 wave + lane bins filter sl mod Nk for every ns-th pixel of
    // [p0, p1) from p0 + sl / Nk on, ns being the number of slots of that
    // filter (every lane works, whatever Nk; the final sum adds a filter's slots)
    const int sl = 64 * wave + lane;
    const int fi = sl % Nk, sub = sl / Nk;
    const int ns = (64 * NW - 1 - fi) / Nk + 1;
    const int npix = (int)(p1 - p0);  // per_wg < 2^30 (host check)
    const int steps = npix > 0 ? (npix + 64 * NW / Nk - 1) / (64 * NW / Nk) : 0;
    if (steps > 0) {
        // DW_U pixels per step; the z and a of the next step are loaded while
        // this step's are binned.  Both loads always run (a pixel past p1 reads
        // pixel p0 instead), and its a is replaced by 0, so it adds 0.
        constexpr int U = DW_U;
        ZT zn[U], an[U];
        const ZT *zl = za + za_index((size_t)p0, Nk, fi);
        const unsigned zst = (unsigned)za_stride(Nk);
        // raw words; a pixel past p1 is masked when its step is binned
        auto load = [&](int kb) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int pl = sub + ns * (kb + u);
                const ZT *qp = zl + (size_t)((unsigned)(pl < npix ? pl : 0) * zst);
                zn[u] = qp[0];
                an[u] = qp[4];
            }
        };
        load(0);
        for (int kb = 0; kb < steps; kb += U) {
            float zc[U], ac[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                zc[u] = za_value(zn[u]);
                ac[u] = sub + ns * (kb + u) < npix ? za_value(an[u]) : 0.f;
            }
            load(kb + U);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float z = zc[u];
                float s = fmaf(z, rb.inv_step, -rb.mu0_over_step);
                float jr = fminf(fmaxf(rintf(s), -(float)RBF_WIN), rb.jmax);
                float d = s - jr;
                // beyond every centre by more than W spacings: nothing to add
                const float a = fabsf(d) <= 0.5f ? ac[u] : 0.f;
                // G_{jr+m} = E q^(m+W) c_m,  E = exp(-rho d (d/2 + W)),  q = exp(rho d):
                // one product chain from the lowest bin up, two exponentials
                const float E = __builtin_amdgcn_exp2f(-rb.rho_log2e * d * fmaf(0.5f, d, (float)RBF_WIN));
                const float q = __builtin_amdgcn_exp2f(rb.rho_log2e * d);
                float *hrow = hist + (int)jr * 64;
                // the pixel's 2W + 1 bins are read together (one wait for all of them)
                // while its Gaussians are formed, then written back
                float hv[2 * RBF_WIN + 1];
#pragma unroll
                for (int m = -RBF_WIN; m <= RBF_WIN; ++m) hv[m + RBF_WIN] = hrow[64 * m];
                __builtin_amdgcn_sched_barrier(0);
                float gm = a * E;
#pragma unroll
                for (int k = 0; k <= 2 * RBF_WIN; ++k) {
                    hv[k] = fmaf(gm, rb.c[k], hv[k]);
                    if (k < 2 * RBF_WIN) gm *= q;
                }
#pragma unroll
                for (int m = -RBF_WIN; m <= RBF_WIN; ++m) hrow[64 * m] = hv[m + RBF_WIN];
            }
        }
    }
    __syncthreads();
    float *dst = dw_part + (size_t)blockIdx.x * Nk * Nrbf;
    for (int i = tid; i < Nk * Nrbf; i += 64 * NW) {
        const int f = i / Nrbf, jj = i - f * Nrbf;
        float sum = 0.f;
        for (int s2 = f; s2 < 64 * NW; s2 += Nk) sum += lds[(s2 >> 6) * hsize + (jj + 2 * RBF_WIN) * 64 + (s2 & 63)];
        dst[i] = sum;
    }
}

// Fixed-order sums of partials, several outputs per launch:
// out[e] = scale * sum_k part[k * nelem + e] for each job.  A block owns 16
// consecutive elements of one job; its 16 rows of threads sum interleaved
// subsets of k (row r takes k = r, r + 16, ...) and the 16 row sums are then
// added in row order, so the result does not depend on scheduling.
constexpr int RED_E = 16, RED_R = 16, RED_JOBS = 3;
struct RedJob {
    const float *part;
    float *out;
    int nparts, nelem;
    float scale;
    int block0;  // first block of this job
};
struct RedJobs {
    RedJob j[RED_JOBS];
    int n;
};

__global__ void __launch_bounds__(RED_E * RED_R) k_reduce_partials(RedJobs jobs)
{
    __shared__ float rows[RED_R][RED_E];
    int q = 0;
    for (int k = 1; k < jobs.n; ++k)
        if ((int)blockIdx.x >= jobs.j[k].block0) q = k;
    const RedJob jb = jobs.j[q];
    const int te = threadIdx.x % RED_E, tr = threadIdx.x / RED_E;
    const int e = ((int)blockIdx.x - jb.block0) * RED_E + te;
    const float *part = jb.part;
    const int nparts = jb.nparts, nelem = jb.nelem;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (e < nelem) {
        int k = tr;
        for (; k + 3 * RED_R < nparts; k += 4 * RED_R) {
            s0 += part[(size_t)k * nelem + e];
            s1 += part[(size_t)(k + RED_R) * nelem + e];
            s2 += part[(size_t)(k + 2 * RED_R) * nelem + e];
            s3 += part[(size_t)(k + 3 * RED_R) * nelem + e];
        }
        for (; k < nparts; k += RED_R) s0 += part[(size_t)k * nelem + e];
    }
    rows[tr][te] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (tr == 0 && e < nelem) {
        float s = 0.f;
        for (int r = 0; r < RED_R; ++r) s += rows[r][te];
        jb.out[e] = jb.scale * s;
    }
}

// acc += x elementwise (dl/df = explicit terms + dl/du_0).
__global__ void __launch_bounds__(256) k_add_plane(float *__restrict__ acc, const float *__restrict__ x,
                                                   size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) acc[i] += x[i];
}

// p[0 .. n) = 0 (a kernel, not a memset, so that a captured graph replays it correctly)
__global__ void __launch_bounds__(256) k_zero(float *__restrict__ p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------------ host side
namespace {

struct BwdGeom {
    int th;                        // k_bwd_params tile height
    int tiles_x, tiles_y, tiles;   // k_bwd_params tiles (per image) and total
    int dw_grid;
    long long dw_per_wg;
    size_t img;                    // N*H*W
};

// k_bwd_params tiles of th rows (and 16 BP_NBW columns); the dW grid.
BwdGeom bwd_geom(int N, int H, int W, int th)
{
    BwdGeom gm;
    const int tw = 16 * BP_NBW;
    gm.th = th;
    gm.tiles_x = (W + tw - 1) / tw;
    gm.tiles_y = (H + th - 1) / th;
    gm.tiles = gm.tiles_x * gm.tiles_y * N;
    gm.img = (size_t)N * H * W;
    long long P = (long long)gm.img;
    // at most 256 workgroups: k_bwd_dw holds one per compute unit (its LDS
    // histograms), and a longer workgroup pays the zeroing and the final
    // reduction of its histograms once
    long long grid = (P + 255) / 256;
    if (grid > 256) grid = 256;
    if (grid < 1) grid = 1;
    gm.dw_per_wg = (P + grid - 1) / grid;
    if (gm.dw_per_wg < 1) gm.dw_per_wg = 1;  // no pixels: an empty dW grid
    gm.dw_grid = (int)((P + gm.dw_per_wg - 1) / gm.dw_per_wg);
    return gm;
}

// The k_bwd_params instance for a filter size, filter-block count, variant
// (loadza: z and a loaded from the export; else computed) and operand precision.
template <int KS, int NMB>
static const void *bp_kernel_t(bool loadza, int prec)
{
    if (loadza && KS == 7 && prec == PREC_BF16) return (const void *)k_bwd_params<7, NMB, BP_NBW, BP_NW, true, PREC_BF16>;
    if (loadza) return (const void *)k_bwd_params<KS, NMB, BP_NBW, BP_NW, true, PREC_F32>;
    if (KS == 7 && prec == PREC_BF16) return (const void *)k_bwd_params<7, NMB, BP_NBW, BP_NW, false, PREC_BF16>;
    if (KS == 7 && prec == PREC_F16) return (const void *)k_bwd_params<7, NMB, BP_NBW, BP_NW, false, PREC_F16>;
    return (const void *)k_bwd_params<KS, NMB, BP_NBW, BP_NW, false, PREC_F32>;
}

static const void *bp_kernel(int ks, int nmb, bool loadza, int prec)
{
    if (ks == 7) return nmb == 2 ? bp_kernel_t<7, 2>(loadza, prec) : bp_kernel_t<7, 3>(loadza, prec);
    return nmb == 2 ? bp_kernel_t<5, 2>(loadza, prec) : bp_kernel_t<5, 3>(loadza, prec);
}

// Workgroups per compute unit that the k_bwd_params tile plan assumes for one
// kernel instance (bp_kernel) and tile height th: the runtime's occupancy for
// its register footprint and the LDS of that tile, but at least 2 (with a
// single resident workgroup the taller tiles of a 1-per-CU plan ran slower
// than the 2-per-CU plan's); cached per thread.
static int bp_per_cu(int ks, int nk, int nrbf, bool loadza, int prec, int th)
{
    const int nmb = (nk + 15) / 16 <= 2 ? 2 : 3;
    int dev = 0;
    (void)hipGetDevice(&dev);
    static thread_local int key[5][5] = {{-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1},
                                         {-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}};
    static thread_local int cached[5][BP_TH_MAX + 1];
    const int v = loadza ? (prec == PREC_BF16 ? 4 : 3) : (prec >= 0 && prec <= 2 ? prec : 0);
    th = th < BP_TH_MIN ? BP_TH_MIN : (th > BP_TH_MAX ? BP_TH_MAX : th);
    if (!(key[v][0] == ks && key[v][1] == nmb && key[v][2] == nrbf && key[v][3] == dev && key[v][4] == prec)) {
        for (int i = 0; i <= BP_TH_MAX; ++i) cached[v][i] = 0;
        key[v][0] = ks;
        key[v][1] = nmb;
        key[v][2] = nrbf;
        key[v][3] = dev;
        key[v][4] = prec;
    }
    if (cached[v][th] > 0) return cached[v][th];
    const BpLds L = bp_lds(ks, nmb, th, 16 * BP_NBW, nrbf, BP_NW, !loadza && prec != PREC_F32);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bp_kernel(ks, nmb, loadza, prec), 64 * BP_NW,
                                                     (size_t)L.total * sizeof(float)) != hipSuccess ||
        n < 2)
        n = 2;
    (void)hipGetLastError();
    cached[v][th] = n;
    return n;
}

// Tile height of k_bwd_params: with p(th) workgroups resident per compute unit,
// n tiles run in ceil(n / (p CUs)) rounds of th rows of BP_NBW blocks each (plus
// a fixed cost of ~4 blocks).
int bwd_tile_h(int N, int H, int W, int ks, int nk, int nrbf, bool loadza, int prec)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    int best_th = BP_TH_MIN;
    double best = 0.0;
    for (int th = BP_TH_MIN; th <= BP_TH_MAX; ++th) {
        const long slots = (long)bp_per_cu(ks, nk, nrbf, loadza, prec, th) * cus;
        const long tiles = (long)N * ((H + th - 1) / th) * ((W + 16 * BP_NBW - 1) / (16 * BP_NBW));
        const long rounds = (tiles + slots - 1) / slots;
        const double cost = (double)rounds * (th * BP_NBW + 4) + 1e-6 * th;
        if (th == BP_TH_MIN || cost < best) {
            best = cost;
            best_th = th;
        }
        if (th >= H) break;
    }
    return best_th;
}

constexpr size_t AL = 256;
size_t al(size_t x) { return (x + AL - 1) / AL * AL; }

struct BwdWs {
    float *g[2], *za, *dk_part, *dl_part, *dw_part, *seg;
    float *prep_b;  // prepared blocks of the input-gradient stages (d phi / ds tables)
    float *prep_f;  // prepared blocks of the recomputed forward stages (phi tables)
    float *slab[2]; // exchange buffers of the recomputed forward stages
    float *slab_b;  // the input-gradient kernel's slabs
    size_t bytes;
};

// prep: floats of T stages' prepared blocks (0: the kernels build them);
// slab: floats of one set of the forward's slabs; slab_b: of the input-gradient kernel's
BwdWs bwd_ws_layout(char *base, int N, int H, int W, const tnrd_model *m, int s, size_t prep,
                    size_t slab, size_t slab_b)
{
    BwdGeom gm = bwd_geom(N, H, W, BP_TH_MIN);  // the most tiles any launch uses
    const size_t kk = (size_t)m->ksize * m->ksize;
    BwdWs w;
    size_t off = AL;  // flags
    auto take = [&](size_t floats) {
        float *p = base ? (float *)(base + off) : nullptr;
        off += al(floats * sizeof(float));
        return p;
    };
    w.g[0] = take(gm.img);
    w.g[1] = take(gm.img);
    w.za = take(gm.img * za_stride(m->Nk) + ZA_PAD);
    w.dk_part = take((size_t)gm.tiles * m->Nk * kk);
    w.dl_part = take((size_t)gm.tiles);
    w.dw_part = take((size_t)gm.dw_grid * m->Nk * m->Nrbf);
    w.seg = s > 1 ? take(gm.img * (size_t)(s + 1)) : nullptr;
    w.prep_b = prep ? take(prep) : nullptr;
    w.prep_f = prep && s > 1 ? take(prep) : nullptr;
    w.slab[0] = s > 1 ? take(slab) : nullptr;
    w.slab[1] = s > 1 ? take(slab) : nullptr;
    w.slab_b = take(slab_b);
    w.bytes = off;
    return w;
}

template <int KS, int NMB, bool LOADZA, int PREC>
hipError_t launch_bwd_params(const BwdParamsIO &io, const BwdGeom &gm, int H, int W, const float *filt,
                             int Nk, const float *rbfw, const RbfGrid &grid, const float *lam,
                             hipStream_t stream)
{
    BpLds L = bp_lds(KS, NMB, gm.th, 16 * BP_NBW, grid.nrbf, BP_NW, PREC != PREC_F32 && !LOADZA);
    size_t lds_bytes = (size_t)L.total * sizeof(float);
    raise_lds_limit((const void *)k_bwd_params<KS, NMB, BP_NBW, BP_NW, LOADZA, PREC>);
    const int per_img = gm.tiles_x * gm.tiles_y;
    FusedRbf rb = make_fused_rbf(grid);
    hipLaunchKernelGGL((k_bwd_params<KS, NMB, BP_NBW, BP_NW, LOADZA, PREC>), dim3(gm.tiles),
                       dim3(64 * BP_NW), lds_bytes, stream, io, H, W, gm.th, gm.tiles_x, per_img, filt, Nk,
                       rbfw, grid.nrbf, rb, lam);
    return hipGetLastError();
}

template <int KS, int NMB>
hipError_t launch_bwd_params_mode(bool loadza, int prec, const BwdParamsIO &io, const BwdGeom &gm, int H,
                                  int W, const float *filt, int Nk, const float *rbfw,
                                  const RbfGrid &grid, const float *lam, hipStream_t stream)
{
    if (loadza && KS == 7 && prec == PREC_BF16)
        return launch_bwd_params<7, NMB, true, PREC_BF16>(io, gm, H, W, filt, Nk, rbfw, grid, lam, stream);
    if (loadza) return launch_bwd_params<KS, NMB, true, PREC_F32>(io, gm, H, W, filt, Nk, rbfw, grid, lam, stream);
    if (KS == 7 && prec == PREC_BF16)
        return launch_bwd_params<7, NMB, false, PREC_BF16>(io, gm, H, W, filt, Nk, rbfw, grid, lam, stream);
    if (KS == 7 && prec == PREC_F16)
        return launch_bwd_params<7, NMB, false, PREC_F16>(io, gm, H, W, filt, Nk, rbfw, grid, lam, stream);
    return launch_bwd_params<KS, NMB, false, PREC_F32>(io, gm, H, W, filt, Nk, rbfw, grid, lam, stream);
}

// Parameter-gradient partials of one stage.  loadza: z = K u and a = K e come
// from the input-gradient kernel's export (FP32 or BF16 operands, the export's
// words); otherwise they are computed here, with the operand precision prec,
// and exported for k_bwd_dw.
hipError_t bwd_params(bool loadza, int prec, const BwdParamsIO &io, const BwdGeom &gm, int H, int W,
                      int ks, const float *filt, int Nk, const float *rbfw, const RbfGrid &grid,
                      const float *lam, hipStream_t stream)
{
    const int nmb = (Nk + 15) / 16;
    if (prec != PREC_F32 && (ks != 7 || (loadza && prec != PREC_BF16))) return hipErrorInvalidValue;
    if (ks == 7)
        return nmb <= 2 ? launch_bwd_params_mode<7, 2>(loadza, prec, io, gm, H, W, filt, Nk, rbfw, grid, lam, stream)
                        : launch_bwd_params_mode<7, 3>(loadza, prec, io, gm, H, W, filt, Nk, rbfw, grid, lam, stream);
    if (ks == 5)
        return nmb <= 2 ? launch_bwd_params_mode<5, 2>(loadza, prec, io, gm, H, W, filt, Nk, rbfw, grid, lam, stream)
                        : launch_bwd_params_mode<5, 3>(loadza, prec, io, gm, H, W, filt, Nk, rbfw, grid, lam, stream);
    return hipErrorInvalidValue;
}

template <int NW, typename ZT>
hipError_t launch_bwd_dw(const ZT *za, const BwdGeom &gm, int Nk,
                         const RbfGrid &grid, float *dw_part, hipStream_t stream)
{
    const size_t lds_bytes = NW * dw_wave_bytes(grid.nrbf);
    raise_lds_limit((const void *)k_bwd_dw<NW, ZT>);
    // the kernel indexes a workgroup's pixels with 32-bit offsets and gives
    // every filter at least one of its 64 NW lanes
    if (gm.dw_per_wg >= (1LL << 30) || (long long)gm.dw_per_wg * za_stride(Nk) >= (1LL << 32) ||
        Nk < 1 || Nk > 64 * NW)
        return hipErrorInvalidValue;
    FusedRbf rb = make_fused_rbf(grid);
    hipLaunchKernelGGL((k_bwd_dw<NW, ZT>), dim3(gm.dw_grid), dim3(64 * NW), lds_bytes, stream,
                       za, (long long)gm.img, gm.dw_per_wg, Nk, grid.nrbf, rb, dw_part);
    return hipGetLastError();
}

// As many waves (histograms) per workgroup as fit the LDS: 7 for 63 RBFs.
template <typename ZT>
hipError_t bwd_dw_t(const ZT *za, const BwdGeom &gm, int Nk, const RbfGrid &grid, float *dw_part,
                    hipStream_t stream)
{
    const size_t per_wave = dw_wave_bytes(grid.nrbf), cap = 160 * 1024;
    if (7 * per_wave <= cap) return launch_bwd_dw<7>(za, gm, Nk, grid, dw_part, stream);
    if (4 * per_wave <= cap) return launch_bwd_dw<4>(za, gm, Nk, grid, dw_part, stream);
    if (2 * per_wave <= cap) return launch_bwd_dw<2>(za, gm, Nk, grid, dw_part, stream);
    return launch_bwd_dw<1>(za, gm, Nk, grid, dw_part, stream);
}

// za: the export in the words of operand precision prec (za_is_bf16)
hipError_t bwd_dw(const float *za, int prec, const BwdGeom &gm, int Nk, const RbfGrid &grid,
                  float *dw_part, hipStream_t stream)
{
    if (za_is_bf16(prec))
        return bwd_dw_t(reinterpret_cast<const unsigned short *>(za), gm, Nk, grid, dw_part, stream);
    return bwd_dw_t(za, gm, Nk, grid, dw_part, stream);
}

// acc += x over n floats.
hipError_t zero_floats(float *p, size_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t add_plane(float *acc, const float *x, size_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_plane, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, acc, x, n);
    return hipGetLastError();
}

// One launch for the (up to RED_JOBS) reductions of a stage.
hipError_t reduce_partials(const RedJob *jobs, int n, hipStream_t stream)
{
    RedJobs J;
    J.n = n;
    int blocks = 0;
    for (int k = 0; k < n; ++k) {
        J.j[k] = jobs[k];
        J.j[k].block0 = blocks;
        blocks += (jobs[k].nelem + RED_E - 1) / RED_E;
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3(blocks), dim3(RED_E * RED_R), 0, stream, J);
    return hipGetLastError();
}

bool bwd_lds_ok(const tnrd_model *m)
{
    const int nmb = (m->Nk + 15) / 16 <= 2 ? 2 : 3;
    BpLds L = bp_lds(m->ksize, nmb, BP_TH_MAX, 16 * BP_NBW, m->Nrbf, BP_NW, true);
    return (size_t)L.total * sizeof(float) <= 160 * 1024 && dw_wave_bytes(m->Nrbf) <= 160 * 1024 &&
           m->Nk <= 64;
}

}  // namespace

// Floats of the input-gradient kernel's slabs (its own tiling, automatic tiles).
size_t bwd_slab_floats(int N, int H, int W, const tnrd_model *m, const tnrd_opts &o, int window)
{
    const bool poly = o.rbf_window < 0 && poly_form_ok(make_grid(m, window), 1);
    return fused_slab_floats(m->ksize, m->Nk, m->Nrbf, N, H, W, 0, 0, 0, poly, MODE_BWD_INPUT);
}

size_t backward_ws_bytes(int N, int H, int W, const tnrd_model *m, const tnrd_opts &o, int window)
{
    if (!fused_supported(m->ksize, m->Nk, m->Nrbf, window, o.prec) || !bwd_lds_ok(m)) return 0;
    const int s = o.recompute_every < 1 ? 1 : o.recompute_every;
    return bwd_ws_layout(nullptr, N, H, W, m, s,
                         prep_region_floats(m, o, TNRD_IMPL_FUSED, window, m->T),
                         slab_region_floats(N, H, W, m, o, TNRD_IMPL_FUSED, window),
                         bwd_slab_floats(N, H, W, m, o, window)).bytes;
}

}  // namespace tnrd

using namespace tnrd;

extern "C" int tnrd_backward(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                             const float *states, const float *grad_uT, float *grad_filters,
                             float *grad_rbf_w, float *grad_lambda, float *grad_u0, float *grad_f,
                             const tnrd_opts *o, void *ws, size_t ws_bytes, void *stream_)
{
    tnrd_opts oo;
    resolve_opts(o, &oo);
    int st = check_image_args(f, N, H, W, L, m, grad_uT);
    if (st != TNRD_OK) return st;
    if (!states || !grad_filters || !grad_rbf_w || !grad_lambda) return TNRD_ERR_ARG;
    if (grad_f && grad_f == grad_u0) return TNRD_ERR_ARG;
    if (oo.prec < TNRD_PREC_FP32 || oo.prec > TNRD_PREC_FP16) return TNRD_ERR_ARG;
    const int window = rbf_window_for(m, oo.rbf_window);
    if (!fused_supported(m->ksize, m->Nk, m->Nrbf, window, oo.prec) || !bwd_lds_ok(m))
        return TNRD_ERR_UNSUPPORTED;
    // the input-gradient kernel uses its own tile; the forward tile options
    // only steer the recomputation of checkpointed states
    if (!fused_config_ok(m->ksize, m->Nk, m->Nrbf, H, W, 0, 0, 0, 1))
        return TNRD_ERR_UNSUPPORTED;
    const int T = m->T;
    const int s = oo.recompute_every < 1 ? 1 : oo.recompute_every;
    const size_t prep = prep_region_floats(m, oo, TNRD_IMPL_FUSED, window, T);
    const size_t slab = slab_region_floats(N, H, W, m, oo, TNRD_IMPL_FUSED, window);
    const size_t slab_b = bwd_slab_floats(N, H, W, m, oo, window);
    const size_t need = bwd_ws_layout(nullptr, N, H, W, m, s, prep, slab, slab_b).bytes;
    if (N > 0 && (!ws || ws_bytes < need)) return TNRD_ERR_WORKSPACE;
    hipStream_t stream = (hipStream_t)stream_;
    const size_t kk = (size_t)m->ksize * m->ksize;
    if (N == 0) {
        // empty batch: every gradient is zero
        if (zero_floats(grad_filters, (size_t)T * m->Nk * kk, stream) != hipSuccess ||
            zero_floats(grad_rbf_w, (size_t)T * m->Nk * m->Nrbf, stream) != hipSuccess ||
            zero_floats(grad_lambda, (size_t)T, stream) != hipSuccess)
            return TNRD_ERR_HIP;
        return TNRD_OK;
    }
    BwdWs w = bwd_ws_layout((char *)ws, N, H, W, m, s, prep, slab, slab_b);
    // the two variants of k_bwd_params hold different numbers of workgroups per
    // compute unit, so each gets its own tile height (gm: loading z and a)
    // B2 geometries: loading the export (FP32 or BF16 operands), and computing z and a
    const int prec_load = oo.prec == TNRD_PREC_BF16 ? TNRD_PREC_BF16 : TNRD_PREC_FP32;
    BwdGeom gm = bwd_geom(N, H, W, bwd_tile_h(N, H, W, m->ksize, m->Nk, m->Nrbf, true, prec_load));
    const BwdGeom gm_own =
        bwd_geom(N, H, W, bwd_tile_h(N, H, W, m->ksize, m->Nk, m->Nrbf, false, oo.prec));
    const size_t img = gm.img;
    if (oo.validate) {
        st = run_domain_check(f, img, (int *)ws, stream, oo.prec);
        if (st != TNRD_OK) return st;
    }

    // u_t for every t of the current checkpoint segment: stored states, or
    // recomputed from the segment's first checkpoint into w.seg.
    const int nck = tnrd_num_checkpoints(T, s);
    std::vector<const float *> ut(T + 1, nullptr);
    StageArgs ia;  // input-gradient stage arguments
    ia.N = N;
    ia.H = H;
    ia.W = W;
    ia.ks = m->ksize;
    ia.Nk = m->Nk;
    ia.f = f;
    ia.grid = make_grid(m, window);
    ia.scratch = nullptr;
    ia.prec = oo.prec;
    ia.tile_h = 0;
    ia.tile_w = 0;
    ia.waves = 0;
    ia.poly = oo.rbf_window < 0;
    ia.react = m->reaction;
    ia.proj_c = m->proj_c;
    // the input-gradient stages' d phi / ds tables and filter operands, all stages at once
    const bool use_prep = fused_uses_prep(ia);
    const size_t prep_sf = use_prep ? fused_prep_floats(m->ksize, m->Nk, m->Nrbf) : 0;
    if (use_prep && fused_prep(m->filters, m->rbf_w, T, m->ksize, m->Nk, ia.grid, 1 | fused_prep_form(ia),
                               w.prep_b, stream) !=
                        hipSuccess)
        return TNRD_ERR_HIP;

    const float *g_cur = grad_uT;
    int ping = 0;
    int seg_hi = T;  // segment [seg_lo, seg_hi]
    while (seg_hi > 0) {
        const int seg_lo = ((seg_hi - 1) / s) * s;
        // states of the segment
        ut[seg_lo] = states + (size_t)(seg_lo / s) * img;
        ut[seg_hi] = states + (size_t)(seg_hi == T ? nck - 1 : seg_hi / s) * img;
        if (seg_hi - seg_lo > 1) {
            // recompute u_{seg_lo+1} .. u_{seg_hi-1} with the forward kernel
            std::vector<float *> dst(seg_hi - seg_lo - 1);
            for (int t = seg_lo + 1; t < seg_hi; ++t) {
                dst[t - seg_lo - 1] = w.seg + (size_t)(t - seg_lo) * img;
                ut[t] = dst[t - seg_lo - 1];
            }
            st = run_stages(f, N, H, W, m, oo, TNRD_IMPL_FUSED, window, seg_lo, seg_hi - 1,
                            ut[seg_lo], dst.data(), nullptr, w.prep_f, w.slab, stream);
            if (st != TNRD_OK) return st;
        }
        for (int t = seg_hi; t > seg_lo; --t) {
            const int ts = t - 1;  // 0-based stage index
            const float *filt = m->filters + (size_t)ts * m->Nk * kk;
            const float *rbfw = m->rbf_w + (size_t)ts * m->Nk * m->Nrbf;
            const float *lam = m->lambda + ts;
            BwdParamsIO io{};
            io.u_prev = ut[t - 1];
            io.u_cur = ut[t];
            io.f = f;
            io.g_cur = g_cur;
            io.za = w.za;
            io.gf = grad_f;
            io.gf_first = t == T;
            io.react = m->reaction;
            io.proj_c = m->proj_c;
            io.dk_part = w.dk_part;
            io.dl_part = w.dl_part;
            // The input-gradient kernel (FP32 or BF16 operands) computes z = K u
            // and a = K e at every pixel anyway and exports them, so it runs first
            // and the parameter-gradient kernels load them instead of recomputing.
            const bool need_g = t > 1 || grad_u0 || grad_f;
            const bool loadza = need_g && (oo.prec == TNRD_PREC_FP32 || oo.prec == TNRD_PREC_BF16) &&
                                (long long)H * W <= INT_MAX;
            float *g_next = (t == 1 && grad_u0) ? grad_u0 : w.g[ping];
            if (need_g) {
                // the input-gradient kernel leaves the force of e in its slabs; the
                // finisher forms g_{t-1} from them
                ia.u_prev = ut[t - 1];
                ia.u_cur = ut[t];
                ia.g_cur = g_cur;
                ia.u_next = nullptr;
                ia.x_out = w.slab_b;
                ia.filt = filt;
                ia.rbfw = rbfw;
                ia.lam = lam;
                ia.za = loadza ? w.za : nullptr;
                ia.prep = use_prep ? w.prep_b + (size_t)ts * prep_sf : nullptr;
                if (fused_stage_input_grad(ia, stream) != hipSuccess) return TNRD_ERR_HIP;
                StageArgs fa = ia;
                fa.x_prev = w.slab_b;
                fa.u_next = g_next;
                if (fused_grad_finish(fa, stream) != hipSuccess) return TNRD_ERR_HIP;
            }
            const BwdGeom &gp = loadza ? gm : gm_own;
            if (bwd_params(loadza, oo.prec, io, gp, H, W, m->ksize, filt, m->Nk,
                           rbfw, ia.grid, lam, stream) !=
                hipSuccess)
                return TNRD_ERR_HIP;
            if (bwd_dw(w.za, oo.prec, gm, m->Nk, ia.grid, w.dw_part, stream) != hipSuccess)
                return TNRD_ERR_HIP;
            const RedJob jobs[RED_JOBS] = {
                {w.dk_part, grad_filters + (size_t)ts * m->Nk * kk, gp.tiles, (int)(m->Nk * kk), -1.f, 0},
                {w.dw_part, grad_rbf_w + (size_t)ts * m->Nk * m->Nrbf, gm.dw_grid, m->Nk * m->Nrbf, -1.f, 0},
                {w.dl_part, grad_lambda + ts, gp.tiles, 1, 1.f, 0}};
            if (reduce_partials(jobs, RED_JOBS, stream) != hipSuccess) return TNRD_ERR_HIP;
            if (need_g) {
                g_cur = g_next;
                ping ^= 1;
            }
        }
        seg_hi = seg_lo;
    }
    // dl/df = the stages' explicit terms (accumulated by k_bwd_params) + dl/du_0 (u_0 = f)
    if (grad_f && add_plane(grad_f, g_cur, img, stream) != hipSuccess) return TNRD_ERR_HIP;
    return TNRD_OK;
}
