// Fused forward stage: one kernel per stage computes, for a tile of output
// pixels,
//
//   z_i = K_i u        filter bank as an implicit GEMM on MFMA (v_mfma_f32_16x16x4_f32)
//   v_i = phi_i(z_i)   Gaussian-RBF influence, windowed, on the vector ALUs
//   Y   = K^T-GEMM     [taps x pixels] = [taps x filters] . [filters x pixels] on MFMA
//   x   = col2im(Y)    shift-add of the tap columns (plus the reflected-border fold)
//   u'  = prox(u - x)
//
// without writing the Nk response maps anywhere but registers and LDS.
//
// Tile geometry (R = (KS-1)/2): the workgroup owns an output tile of Th x Tw
// pixels.  K^T needs v on the tile plus an R ring ("E region", Eh x Ew), and
// z on E needs u on the tile plus a 2R ring (the u tile staged in LDS).  Each
// wave takes whole E rows; a row is cut into NB blocks of 16 pixels, the N
// dimension of every MFMA.  Pixels of a block that fall outside the image (or
// beyond Ew) carry v = 0.
//
// GEMM layouts for v_mfma_f32_16x16x4_f32 (lane l, g = l / 16, j = l % 16):
//   A operand  A[j][g]   (row j, k = g)
//   B operand  B[g][j]
//   D          D[4g + r][j] in accumulator register r
// GEMM1: rows = filters (16 per m-block), k = taps (4 per k-step), cols = pixels.
//   D gives lane l the responses of pixel j for filters 16 mb + 4 g + r.
// GEMM2: rows = tap slots, k = filters, cols = pixels.  Its B operand for k-step
//   (mb, r) is exactly GEMM1's D register r of m-block mb if k-row g of that
//   step is taken to be filter 16 mb + 4 g + r, so the responses never move.
//   Tap slot L (0..16*MB2-1) holds tap (a, b) = (L % KS, L / KS), arranged so
//   that the four lane groups of one D register hold four different a.
//
// col2im: lane (g, j) of D register r of slot block mb2 holds Y for source
// pixel (e, c) and tap (a, b); it belongs to output (e - a, c - b) in tile
// coordinates.  Each wave writes the Y of its E row into a private scratch
// Ys[c][slot] (plain 16-byte stores of the four D registers), then reduces
// the row along x into P[e][a][qx + 2R] = sum_b Ys[qx + b][slot(a, b)] with
// plain loads and stores: every P entry is written once, by the wave that
// owns E row e, so the result is deterministic and no LDS atomics are needed.
// After a barrier, X(y, x) = sum_a P[y + a][a][x + 2R].
//
// The border fold (K^T is the exact adjoint of "reflect, then convolve"): an
// output pixel within R of the image border also receives X at its mirror
// position in the padded ring, which the tile's P already holds.
#include "tnrd_device.hpp"
#include "tnrd_fused_common.hpp"
#include "tnrd_internal.hpp"

namespace tnrd {

struct FusedLds {
    int ldw;      // u tile row pitch
    int u_off, u_size;
    int e_off;    // input-gradient mode: e tile, same shape as the u tile
    int t_off, t_pitch;   // RBF table
    int p_off, pw, p_size;
    int y_off, yp, y_size;  // per-wave Y scratch: [16 nb][yp] floats per wave
    int red_off;            // 8 floats for workgroup reductions
    int total;
};

__host__ __device__ inline int fused_yp(int ks)
{
    const int kk = ks * ks;
    const int mb2 = (kk % 16 <= 1) ? kk / 16 : (kk + 15) / 16;
    return 16 * mb2 + 4;  // slots of the MFMA blocks + one for the leftover tap, 16 B aligned
}

__host__ __device__ inline FusedLds fused_lds(int ks, int nmb, int nb, int th, int tw, int nrbf,
                                              int nw, int mode = MODE_FWD)
{
    const int R = ks / 2;
    FusedLds l;
    const int luh = th + 4 * R;
    l.ldw = tw + 4 * R + 1;
    l.u_off = 0;
    l.u_size = luh * l.ldw;
    l.e_off = l.u_off + l.u_size;
    l.t_pitch = nrbf + 4 * RBF_WIN + 1;
    l.t_off = l.e_off + (mode == MODE_BWD_INPUT ? l.u_size : 0);
    const int eh = th + 2 * R;
    l.pw = 16 * nb + 2 * R;
    l.p_off = l.t_off + 16 * nmb * l.t_pitch;
    l.p_size = eh * ks * l.pw;
    if (l.p_size < 16 * nmb * ks * ks) l.p_size = 16 * nmb * ks * ks;  // also stages the filters
    l.yp = fused_yp(ks);
    l.y_off = (l.p_off + l.p_size + 3) & ~3;
    l.y_size = nw * 16 * nb * l.yp;
    l.red_off = l.y_off + l.y_size;
    l.total = l.red_off + 8;
    return l;
}

// One output tile of one stage.  The pointers in `io` are those of the tile's
// image ([H][W] planes); (ty0, tx0) is the tile's origin.  The caller's
// workgroup runs it with 64 * NW threads and the dynamic LDS of fused_lds().
template <int KS, int NMB, int NB, int NW, int MODE, int PREC = PREC_F32>
__device__ __forceinline__ void fused_tile(
    const FusedIO &io, int H, int W, int Th, int Tw, int ty0, int tx0,
    const float *__restrict__ filt, int Nk, const float *__restrict__ rbfw, int Nrbf,
    const FusedRbf &rb, const float *__restrict__ lam_t, float *lds)
{
    constexpr bool BWD = MODE == MODE_BWD_INPUT;
    const float *__restrict__ u_prev = io.u_prev;
    const float *__restrict__ f = io.f;
    using G = Geo<KS>;
    constexpr int R = G::R, KK = G::KK, KS1 = G::KS1, MB2 = G::MB2;
    constexpr int KS2 = 4 * NMB;  // GEMM2 k-steps (4 filters each)
    constexpr int FUSED_THREADS = 64 * NW;
    constexpr int FUSED_WAVES = NW;

    const FusedLds L = fused_lds(KS, NMB, NB, Th, Tw, Nrbf, NW, MODE);
    float *su = lds + L.u_off;
    float *se = lds + L.e_off;
    float *stab = lds + L.t_off;
    float *sp = lds + L.p_off;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;

    const float *un = u_prev;

    const int Eh = Th + 2 * R, Ew = Tw + 2 * R;
    const int luh = Th + 4 * R, luw = Tw + 4 * R;

    // ---- prologue: every global load of a thread is issued before the first
    // use, so the workgroup pays one memory latency, not one per element.
    // (1) the stage's filters, staged through the P area of LDS
    {
        const int nf = Nk * KK;
        float *sf = sp;
        for (int base = 0; base < nf; base += 8 * FUSED_THREADS) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = filt[min(base + k * FUSED_THREADS + tid, nf - 1)];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (base + k * FUSED_THREADS + tid < nf) sf[base + k * FUSED_THREADS + tid] = v[k];
        }
    }
    // (2) the u tile (rows ty0-2R .. ty0+Th+2R-1), reflected at the border
    {
        const int n = luh * luw;
        for (int base = 0; base < n; base += 8 * FUSED_THREADS) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                int i = min(base + k * FUSED_THREADS + tid, n - 1);
                int ly = i / luw, lx = i - ly * luw;
                int yy = reflect_clamp(ty0 - 2 * R + ly, H), xx = reflect_clamp(tx0 - 2 * R + lx, W);
                v[k] = un[(size_t)yy * W + xx];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                int i = base + k * FUSED_THREADS + tid;
                if (i < n) {
                    int ly = i / luw, lx = i - ly * luw;
                    su[ly * L.ldw + lx] = v[k];
                }
            }
        }
    }
    // (2b) input-gradient mode: e = y * g_t over the same region, where
    // y = du_t/d(ut_t) = u_t^2 / ((1+2l) u_t^2 + 2 l f^2) is the prox derivative
    // written with the prox output (equal to the closed form of eq. derv2).
    float emax = 0.f;  // largest |e| of the tile (input-gradient mode)
    if (BWD) {
        const float lam0 = lam_t[0];
        const float c1 = 1.f + 2.f * lam0, c2 = 2.f * lam0;
        const float *ucn = io.u_cur;
        const float *gcn = io.g_cur;
        const float *fcn = f;
        const int n = luh * luw;
        for (int base = 0; base < n; base += 4 * FUSED_THREADS) {
            float uu[4], ff[4], gg[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int i = min(base + k * FUSED_THREADS + tid, n - 1);
                int ly = i / luw, lx = i - ly * luw;
                int yy = reflect_clamp(ty0 - 2 * R + ly, H), xx = reflect_clamp(tx0 - 2 * R + lx, W);
                size_t q = (size_t)yy * W + xx;
                uu[k] = ucn[q];
                ff[k] = fcn[q];
                gg[k] = gcn[q];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int i = base + k * FUSED_THREADS + tid;
                if (i < n) {
                    int ly = i / luw, lx = i - ly * luw;
                    float u2 = uu[k] * uu[k];
                    float y = u2 / fmaf(c1, u2, c2 * ff[k] * ff[k]);
                    float ev = y * gg[k];
                    se[ly * L.ldw + lx] = ev;
                    emax = fmaxf(emax, fabsf(ev));
                }
            }
        }
    }
    // (3) RBF weight table, zero padded by 2W on both sides of every row
    {
        const int n = 16 * NMB * L.t_pitch;
        const int nw = Nk * Nrbf;
        for (int base = 0; base < n; base += 8 * FUSED_THREADS) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                int i = base + k * FUSED_THREADS + tid;
                int fi = i / L.t_pitch, jj = i - fi * L.t_pitch - 2 * RBF_WIN;
                int src = min(max(fi * Nrbf + jj, 0), nw - 1);
                float w = rbfw[src];
                v[k] = (fi < Nk && jj >= 0 && jj < Nrbf) ? w : 0.f;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (base + k * FUSED_THREADS + tid < n) stab[base + k * FUSED_THREADS + tid] = v[k];
        }
    }
    __syncthreads();

    // Mixed-precision input gradient: e, a = K e and phi' a go through BF16/FP16
    // operands with a power-of-two tile scale that puts max|e| at 2^10 (FP16's
    // normal range starts at 2^-14 and ends below 2^16; |K e| <= 7 max|e| for
    // unit-norm 7x7 filters), undone in FP32 when g_{t-1} is formed.
    float escale = 1.f, einv = 1.f;
    if (BWD && PREC != PREC_F32) {
        float wmax = emax;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) wmax = fmaxf(wmax, __shfl_xor(wmax, o));
        float *red = lds + L.red_off;
        if (lane == 0) red[wave] = wmax;
        __syncthreads();
        float m = 0.f;
        for (int w = 0; w < FUSED_WAVES; ++w) m = fmaxf(m, red[w]);
        if (m > 0.f && isfinite(m)) {
            int ex = ilogbf(m);
            escale = ldexpf(1.f, 10 - ex);
            einv = ldexpf(1.f, ex - 10);
        }
    }

    // ---- filter operands in registers (from the staged copy)
    const float *sf = sp;
    float a1[NMB][KS1];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
        for (int s = 0; s < KS1; ++s) {
            int fi = 16 * mb + j, t = 4 * s + g;
            a1[mb][s] = (fi < Nk && t < KK) ? sf[fi * KK + t] : 0.f;
        }
    float a2[MB2][KS2];
#pragma unroll
    for (int mb2 = 0; mb2 < MB2; ++mb2)
#pragma unroll
        for (int s = 0; s < KS2; ++s) {
            int fi = 16 * (s >> 2) + 4 * g + (s & 3);
            int Ls = 16 * mb2 + 4 * (j & 3) + (j >> 2);  // slot of A row j
            int ta = Ls % KS, tb = Ls / KS;
            a2[mb2][s] = (fi < Nk && Ls < KK) ? sf[fi * KK + ta * KS + tb] : 0.f;
        }
    float av[NMB][4];  // leftover tap (KS-1, KS-1) when 16*MB2 == KK-1
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int fi = 16 * mb + 4 * g + r;
            av[mb][r] = (G::VTAP && fi < Nk) ? sf[fi * KK + KK - 1] : 0.f;
        }

    // mixed precision: 16-wide k-steps, operands converted once to BF16/FP16
    using MX = Mix<PREC>;
    typedef typename MX::V MV;
    constexpr bool MIXED = PREC != PREC_F32;
    constexpr int KSH = (KK + 15) / 16;  // GEMM1 k-steps of 16 taps
    MV a1m[NMB][MIXED ? KSH : 1];
    MV a2m[MB2][MIXED ? NMB : 1];
    int offm[MIXED ? KSH : 1][4];
    if (MIXED) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int s = 0; s < KSH; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int fi = 16 * mb + j, t = 16 * s + 4 * g + i;
                    a1m[mb][s][i] = MX::cvt((fi < Nk && t < KK) ? sf[fi * KK + t] : 0.f);
                }
#pragma unroll
        for (int mb2 = 0; mb2 < MB2; ++mb2)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int fi = 16 * mb + 4 * g + i;
                    int Ls = 16 * mb2 + 4 * (j & 3) + (j >> 2);
                    int ta = Ls % KS, tb = Ls / KS;
                    a2m[mb2][mb][i] = MX::cvt((fi < Nk && Ls < KK) ? sf[fi * KK + ta * KS + tb] : 0.f);
                }
    }
    __syncthreads();  // the staged filters in the P area are consumed

    // GEMM1 B-operand offsets: tap t = 4 s + g -> (a, b) = (t / KS, t % KS)
    int off1[KS1];
#pragma unroll
    for (int s = 0; s < KS1; ++s) {
        int t = 4 * s + g;
        off1[s] = t < KK ? (t / KS) * L.ldw + (t % KS) : 0;
    }
    if (MIXED) {
#pragma unroll
        for (int s = 0; s < KSH; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int t = 16 * s + 4 * g + i;
                offm[s][i] = t < KK ? (t / KS) * L.ldw + (t % KS) : 0;
            }
    }
    __syncthreads();

    const float lam = lam_t[0];
    float *ys = lds + L.y_off + wave * (16 * NB * L.yp);
    for (int e = wave; e < Eh; e += FUSED_WAVES) {
        const int yi = ty0 - R + e;
        if (yi < 0 || yi >= H) continue;  // rows outside the image contribute v = 0 (never read)
#pragma unroll 1
        for (int cb = 0; cb < NB; ++cb) {
            const int c = 16 * cb + j;
            const int xi = tx0 - R + c;
            const bool valid = (c < Ew) && (xi >= 0) && (xi < W);
            const int cc = c < Ew ? c : Ew - 1;
            const float *ub = su + (e + 2 * R) * L.ldw + cc + 2 * R;
            const float *eb = se + (e + 2 * R) * L.ldw + cc + 2 * R;

            // GEMM1: z = K u  (and a = K e in input-gradient mode)
            floatx4 acc1[NMB], acca[NMB];
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) {
                acc1[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
                acca[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
            if (MIXED) {
#pragma unroll
                for (int s = 0; s < KSH; ++s) {
                    MV bu, be;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        bu[i] = MX::cvt(ub[-offm[s][i]]);
                        be[i] = MX::cvt(BWD ? escale * eb[-offm[s][i]] : 0.f);
                    }
#pragma unroll
                    for (int mb = 0; mb < NMB; ++mb) {
                        acc1[mb] = MX::mfma(a1m[mb][s], bu, acc1[mb]);
                        if (BWD) acca[mb] = MX::mfma(a1m[mb][s], be, acca[mb]);
                    }
                }
            } else {
#pragma unroll
                for (int s = 0; s < KS1; ++s) {
                    float bv = ub[-off1[s]];
                    float be = BWD ? eb[-off1[s]] : 0.f;
#pragma unroll
                    for (int mb = 0; mb < NMB; ++mb) {
                        acc1[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[mb][s], bv, acc1[mb], 0, 0, 0);
                        if (BWD)
                            acca[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[mb][s], be, acca[mb], 0, 0, 0);
                    }
                }
            }

            // influence: v = phi(z), lane-local (pixel j, filters 16 mb + 4 g + r)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float z = acc1[mb][r];
                    float s = fmaf(z, rb.inv_step, -rb.mu0_over_step);
                    float jr = fminf(fmaxf(rintf(s), -(float)RBF_WIN), rb.jmax);
                    float d = s - jr;
                    const float *w = stab + (16 * mb + 4 * g + r) * L.t_pitch + (int)jr + RBF_WIN;
                    float q = __builtin_amdgcn_exp2f(rb.rho_log2e * d);
                    float E = __builtin_amdgcn_exp2f(-rb.rho_log2e * d * fmaf(0.5f, d, (float)RBF_WIN));
                    float acc = w[2 * RBF_WIN] * rb.c[2 * RBF_WIN];
                    float accd = 0.f;  // derivative of the Horner polynomial
#pragma unroll
                    for (int n = 2 * RBF_WIN - 1; n >= 0; --n) {
                        if (BWD) accd = fmaf(accd, q, acc);
                        acc = fmaf(acc, q, w[n] * rb.c[n]);
                    }
                    float v;
                    if (BWD) {
                        // phi'(z) = (rho/step) E (q P'(q) - (d + W) P(q)), times a
                        float dphi = rb.rho_over_step * E * fmaf(q, accd, -(d + (float)RBF_WIN) * acc);
                        v = dphi * acca[mb][r];
                    } else {
                        v = E * acc;
                    }
                    acc1[mb][r] = (valid && fabsf(d) <= 0.5f) ? v : 0.f;
                }

            // GEMM2: Y = K^T-slots . v
            floatx4 acc2[MB2];
#pragma unroll
            for (int mb2 = 0; mb2 < MB2; ++mb2) acc2[mb2] = floatx4{0.f, 0.f, 0.f, 0.f};
            if (MIXED) {
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb) {
                    MV vb;  // filters 16 mb + 4 g + i of pixel j: GEMM1's register quad
#pragma unroll
                    for (int i = 0; i < 4; ++i) vb[i] = MX::cvt(acc1[mb][i]);
#pragma unroll
                    for (int mb2 = 0; mb2 < MB2; ++mb2) acc2[mb2] = MX::mfma(a2m[mb2][mb], vb, acc2[mb2]);
                }
            } else {
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int mb2 = 0; mb2 < MB2; ++mb2)
                            acc2[mb2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[mb2][4 * mb + r],
                                                                             acc1[mb][r], acc2[mb2], 0, 0, 0);
            }

            // Y of this block into the wave's scratch: slots 16 mb2 + 4 g + r
            float *yb = ys + c * L.yp;
#pragma unroll
            for (int mb2 = 0; mb2 < MB2; ++mb2)
                *reinterpret_cast<floatx4 *>(yb + 16 * mb2 + 4 * g) = acc2[mb2];
            if (G::VTAP) {
                float part = 0.f;
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) part = fmaf(av[mb][r], acc1[mb][r], part);
                part += __shfl_xor(part, 16);
                part += __shfl_xor(part, 32);
                if (g == 0) yb[16 * MB2] = part;
            }
        }
        // x-direction col2im of the row: P[e][a][qx + 2R] = sum_b Ys[qx + b][slot(a, b)]
        float *prow = sp + e * KS * L.pw;
        for (int o = lane; o < KS * L.pw; o += 64) {
            const int a = o / L.pw, colp = o - a * L.pw;
            const int qx = colp - 2 * R;
            float acc = 0.f;
#pragma unroll
            for (int b = 0; b < KS; ++b) {
                const int c = qx + b;
                const int Lt = a + KS * b;  // slot order of tap (a, b)
                const int slot = Lt < 16 * MB2 ? 16 * (Lt >> 4) + 4 * (Lt & 3) + ((Lt & 15) >> 2)
                                               : 16 * MB2;
                if (c >= 0 && c < 16 * NB) acc += ys[c * L.yp + slot];
            }
            prow[o] = acc;
        }
    }
    __syncthreads();

    // ---- gather X, fold the border ring, prox, store
    const float *fn = f;
    float *uo = io.out;
    for (int i = tid; i < Th * Tw; i += FUSED_THREADS) {
        const int y = i / Tw, x = i - (i / Tw) * Tw;
        const int yi = ty0 + y, xi = tx0 + x;
        if (yi >= H || xi >= W) continue;
        int qy[2] = {y, 0}, qx[2] = {x, 0};
        int nqy = 1, nqx = 1;
        if (yi < R) qy[nqy++] = -yi - 1 - ty0;
        else if (yi >= H - R) qy[nqy++] = 2 * H - 1 - yi - ty0;
        if (xi < R) qx[nqx++] = -xi - 1 - tx0;
        else if (xi >= W - R) qx[nqx++] = 2 * W - 1 - xi - tx0;
        float xs = 0.f;
        for (int iy = 0; iy < nqy; ++iy)
            for (int ix = 0; ix < nqx; ++ix) {
                const int col = qx[ix] + 2 * R;
#pragma unroll
                for (int a = 0; a < KS; ++a) {
                    const int e = qy[iy] + a;
                    const int ye = ty0 - R + e;
                    if (e >= 0 && e < Eh && ye >= 0 && ye < H) xs += sp[(e * KS + a) * L.pw + col];
                }
            }
        const size_t p = (size_t)yi * W + xi;
        if (BWD) {
            // g_{t-1} = e - sum_i K_i^T (phi_i'(z_i) a_i)  (transposed eq. derv1-1)
            uo[p] = se[(y + 2 * R) * L.ldw + x + 2 * R] - xs * einv;
        } else {
            const float uv = su[(y + 2 * R) * L.ldw + x + 2 * R];
            uo[p] = prox(uv - xs, fn[p], lam);
        }
    }
    __syncthreads();  // LDS is free for the workgroup's next tile
}

template <int KS, int NMB, int NB, int NW, int MODE, int PREC>
__global__ void __launch_bounds__(64 * NW) k_fused_stage(
    FusedIO io, int H, int W, int Th, int Tw, int tiles_x, int tiles_per_img,
    const float *__restrict__ filt, int Nk, const float *__restrict__ rbfw, int Nrbf,
    FusedRbf rb, const float *__restrict__ lam_t)
{
    extern __shared__ float lds[];
    const int img = blockIdx.x / tiles_per_img;
    const int trem = blockIdx.x - img * tiles_per_img;
    const int ty = trem / tiles_x, tx = trem - ty * tiles_x;
    const size_t plane = (size_t)H * W;
    FusedIO ii;
    ii.u_prev = io.u_prev + img * plane;
    ii.f = io.f + img * plane;
    ii.out = io.out + img * plane;
    ii.u_cur = io.u_cur ? io.u_cur + img * plane : nullptr;
    ii.g_cur = io.g_cur ? io.g_cur + img * plane : nullptr;
    fused_tile<KS, NMB, NB, NW, MODE, PREC>(ii, H, W, Th, Tw, ty * Th, tx * Tw, filt, Nk, rbfw, Nrbf,
                                            rb, lam_t, lds);
}

// ------------------------------------------------------------------ batched
// One launch per stage covers the tiles of every image of an uneven batch:
// workgroup b takes the b-th (image, tile) item of the stage and runs the
// fused stage on it with that image's model (chosen by its look number).
// Stages are ordered by the kernel boundaries, so no workgroup ever waits on
// another.  Ping-pong: stage t writes u_out if T-1-t is even, else the
// image's scratch plane, and reads the other (stage 0 reads f).
template <int KS, int NMB, int NB, int NW>
__global__ void __launch_bounds__(64 * NW) k_batched_stage(BatchArgs a, int t)
{
    extern __shared__ float lds[];
    constexpr int KK = KS * KS;
    const BatchItem it = a.items[blockIdx.x];
    const BatchImage im = a.imgs[it.image];
    const int ty = it.tile / im.tiles_x, tx = it.tile - ty * im.tiles_x;
    const bool to_out = ((a.T - 1 - t) & 1) == 0;
    FusedIO io;
    io.f = im.f;
    io.u_prev = t == 0 ? im.f : (to_out ? im.u_tmp : im.u_out);
    io.out = to_out ? im.u_out : im.u_tmp;
    io.u_cur = nullptr;
    io.g_cur = nullptr;
    const BatchModel md = a.models[im.model];
    fused_tile<KS, NMB, NB, NW, MODE_FWD>(io, im.H, im.W, a.Th, a.Tw, ty * a.Th, tx * a.Tw,
                                          md.filt + (size_t)t * a.Nk * KK, a.Nk,
                                          md.rbfw + (size_t)t * a.Nk * a.Nrbf, a.Nrbf, a.rb,
                                          md.lam + t, lds);
}

// ------------------------------------------------------------------ host side
FusedRbf make_fused_rbf(const RbfGrid &grid)
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
    return rb;
}

template <int KS, int NMB, int NB, int NW, int MODE, int PREC>
static hipError_t launch_fused(const StageArgs &s, int th, int tw, hipStream_t stream)
{
    FusedLds L = fused_lds(KS, NMB, NB, th, tw, s.grid.nrbf, NW, MODE);
    size_t lds_bytes = (size_t)L.total * sizeof(float);
    static bool attr_set = false;
    if (!attr_set) {
        // raise the dynamic LDS limit to the CU's 160 KB; a failure here shows
        // up as a launch error below, so the status is cleared
        (void)hipFuncSetAttribute((const void *)k_fused_stage<KS, NMB, NB, NW, MODE, PREC>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipGetLastError();
        attr_set = true;
    }
    if (lds_bytes > 160 * 1024) return hipErrorInvalidValue;
    FusedRbf rb = make_fused_rbf(s.grid);
    FusedIO io;
    io.u_prev = s.u_prev;
    io.f = s.f;
    io.out = s.u_next;
    io.u_cur = s.u_cur;
    io.g_cur = s.g_cur;
    const int tiles_x = (s.W + tw - 1) / tw, tiles_y = (s.H + th - 1) / th;
    const int tiles = tiles_x * tiles_y;
    dim3 grid(tiles * s.N);
    hipLaunchKernelGGL((k_fused_stage<KS, NMB, NB, NW, MODE, PREC>), grid, dim3(64 * NW), lds_bytes,
                       stream, io, s.H, s.W, th, tw, tiles_x, tiles, s.filt, s.Nk, s.rbfw,
                       s.grid.nrbf, rb, s.lam);
    return hipGetLastError();
}

// Tile used when the caller does not pick one: 32 x 32 output pixels for the
// forward (three 16-pixel blocks per E row for 7x7 filters), 32 x 26 for the
// input-gradient mode (two blocks per E row, which leaves LDS room for the e
// tile), clamped to the image.
static void fused_tile(int ks, int H, int W, int req_h, int req_w, int mode, int &th, int &tw,
                       int &nb)
{
    const int R = ks / 2;
    tw = req_w > 0 ? req_w : (mode == MODE_FWD ? 32 : 32 - 2 * R);
    th = req_h > 0 ? req_h : 32;
    if (tw > W) tw = W;
    if (th > H) th = H;
    nb = (tw + 2 * R + 15) / 16;
}

template <int KS, int NMB, int NW, int MODE, int PREC>
static hipError_t fused_nb(const StageArgs &s, int th, int tw, int nb, hipStream_t stream)
{
    switch (nb) {
    case 2: return launch_fused<KS, NMB, 2, NW, MODE, PREC>(s, th, tw, stream);
    case 3: return launch_fused<KS, NMB, 3, NW, MODE, PREC>(s, th, tw, stream);
    case 4: return launch_fused<KS, NMB, 4, NW, MODE, PREC>(s, th, tw, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int KS, int NMB, int MODE, int PREC>
static hipError_t fused_nw(const StageArgs &s, int th, int tw, int nb, int nw, hipStream_t stream)
{
    if (nw == 4) return fused_nb<KS, NMB, 4, MODE, PREC>(s, th, tw, nb, stream);
    return fused_nb<KS, NMB, 8, MODE, PREC>(s, th, tw, nb, stream);
}

template <int MODE>
static hipError_t fused_dispatch(const StageArgs &s, hipStream_t stream)
{
    int th, tw, nb;
    fused_tile(s.ks, s.H, s.W, s.tile_h, s.tile_w, MODE, th, tw, nb);
    if (nb < 2) nb = 2;
    if (nb > 4) return hipErrorInvalidValue;
    const int nw = s.waves == 4 ? 4 : 8;
    const int nmb = (s.Nk + 15) / 16;
    if (s.prec == PREC_BF16 || s.prec == PREC_F16) {
        // mixed-precision filter bank: 7x7 filters only
        if (s.ks != 7) return hipErrorInvalidValue;
        if (s.prec == PREC_BF16)
            return nmb <= 2 ? fused_nw<7, 2, MODE, PREC_BF16>(s, th, tw, nb, nw, stream)
                            : fused_nw<7, 3, MODE, PREC_BF16>(s, th, tw, nb, nw, stream);
        return nmb <= 2 ? fused_nw<7, 2, MODE, PREC_F16>(s, th, tw, nb, nw, stream)
                        : fused_nw<7, 3, MODE, PREC_F16>(s, th, tw, nb, nw, stream);
    }
    if (s.ks == 7) {
        if (nmb <= 2) return fused_nw<7, 2, MODE, PREC_F32>(s, th, tw, nb, nw, stream);
        return fused_nw<7, 3, MODE, PREC_F32>(s, th, tw, nb, nw, stream);
    }
    if (s.ks == 5) {
        if (nmb <= 2) return fused_nw<5, 2, MODE, PREC_F32>(s, th, tw, nb, nw, stream);
        return fused_nw<5, 3, MODE, PREC_F32>(s, th, tw, nb, nw, stream);
    }
    return hipErrorInvalidValue;
}

bool fused_config_ok(int ks, int nk, int nrbf, int H, int W, int tile_h, int tile_w, int waves,
                     int mode)
{
    int th, tw, nb;
    fused_tile(ks, H, W, tile_h, tile_w, mode, th, tw, nb);
    if (nb < 2) nb = 2;
    if (nb > 4 || th < ks / 2 || tw < ks / 2) return false;
    const int nw = waves == 4 ? 4 : 8;
    const int nmb = (nk + 15) / 16;
    FusedLds L = fused_lds(ks, nmb <= 2 ? 2 : 3, nb, th, tw, nrbf, nw, mode);
    return (size_t)L.total * sizeof(float) <= 160 * 1024;
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

hipError_t fused_stage(const StageArgs &s, hipStream_t stream)
{
    return fused_dispatch<MODE_FWD>(s, stream);
}

hipError_t fused_stage_input_grad(const StageArgs &s, hipStream_t stream)
{
    return fused_dispatch<MODE_BWD_INPUT>(s, stream);
}

template <int KS, int NMB, int NB, int NW>
static hipError_t launch_batched_t(const BatchArgs &a, hipStream_t stream)
{
    FusedLds L = fused_lds(KS, NMB, NB, a.Th, a.Tw, a.Nrbf, NW, MODE_FWD);
    const size_t lds_bytes = (size_t)L.total * sizeof(float);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_batched_stage<KS, NMB, NB, NW>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipGetLastError();
        attr_set = true;
    }
    for (int t = 0; t < a.T; ++t) {
        hipLaunchKernelGGL((k_batched_stage<KS, NMB, NB, NW>), dim3(a.items_per_stage),
                           dim3(64 * NW), lds_bytes, stream, a, t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int KS, int NMB>
static hipError_t batched_nb(const BatchArgs &a, int nb, int nw, hipStream_t stream)
{
    if (nw == 4) {
        switch (nb) {
        case 2: return launch_batched_t<KS, NMB, 2, 4>(a, stream);
        case 3: return launch_batched_t<KS, NMB, 3, 4>(a, stream);
        case 4: return launch_batched_t<KS, NMB, 4, 4>(a, stream);
        }
    } else {
        switch (nb) {
        case 2: return launch_batched_t<KS, NMB, 2, 8>(a, stream);
        case 3: return launch_batched_t<KS, NMB, 3, 8>(a, stream);
        case 4: return launch_batched_t<KS, NMB, 4, 8>(a, stream);
        }
    }
    return hipErrorInvalidValue;
}

bool batched_config_ok(int ks, int nk, int nrbf, int th, int tw, int nw)
{
    const int R = ks / 2;
    const int nb = (tw + 2 * R + 15) / 16;
    if (nb < 2 || nb > 4 || th < 2 * R || tw < 2 * R) return false;  // the halo must fit in one tile
    const int nmb = (nk + 15) / 16;
    FusedLds L = fused_lds(ks, nmb <= 2 ? 2 : 3, nb, th, tw, nrbf, nw == 4 ? 4 : 8, MODE_FWD);
    return (size_t)L.total * sizeof(float) + 64 <= 160 * 1024;
}

hipError_t batched_launch(const BatchArgs &a, int ks, int nw, hipStream_t stream)
{
    const int R = ks / 2;
    const int nb = (a.Tw + 2 * R + 15) / 16;
    const int nmb = (a.Nk + 15) / 16;
    if (ks == 7) return nmb <= 2 ? batched_nb<7, 2>(a, nb, nw, stream) : batched_nb<7, 3>(a, nb, nw, stream);
    if (ks == 5) return nmb <= 2 ? batched_nb<5, 2>(a, nb, nw, stream) : batched_nb<5, 3>(a, nb, nw, stream);
    return hipErrorInvalidValue;
}

}  // namespace tnrd
