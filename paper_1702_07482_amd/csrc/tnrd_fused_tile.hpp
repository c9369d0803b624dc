// Device code of the fused stage kernel and its templated launchers; the
// translation units tnrd_fused_{fwd,mixed,bwd,batched}.hip instantiate them.
//
// Fused stage: one kernel per stage computes, for the own pixels of a tile,
//
//   z_i = K_i u        filter bank as an implicit GEMM on MFMA (v_mfma_f32_16x16x4_f32)
//   v_i = phi_i(z_i)   influence on the vector ALUs: a piecewise degree-7
//                      polynomial per unit interval of the RBF grid (of phi in the
//                      forward, of d phi / ds in the input-gradient mode) whose
//                      coefficient table is prepared once per call and copied
//                      into LDS; or, for explicit RBF windows, the windowed
//                      Gaussian sum evaluated with Horner's rule
//   Y   = K^T-GEMM     [tap slots x pixels] = [tap slots x filters] . [filters x pixels] on MFMA
//   X   = col2im(Y)    x-direction shift-add of the tap columns with DPP row shifts,
//                      y-direction sum of the tap rows through LDS
//
// without writing the Nk response maps anywhere but registers.  K^T spreads a
// tile's own pixels over the tile plus an R ring, so X is exported to the
// tile's slab (exchange form, XTiles in tnrd_fused_common.hpp); the force at
// a pixel is the sum of the slabs covering it and its border mirrors (the
// exact adjoint's fold).  The forward applies stage t's reaction,
// u_t = prox(u_{t-1} - x), in the prologue of stage t + 1 (k_react_final after
// the last stage); the input-gradient mode's g_{t-1} = e - x is formed by
// k_grad_finish.  No tile recomputes z or phi for a neighbour's pixels.
//
// Tile geometry (R = (KS-1)/2): the workgroup owns an output tile of Th x Tw
// pixels (Th, Tw >= 2R).  z on the tile needs u on the tile plus an R ring
// (the u tile staged in LDS).  Each wave takes whole tile rows; a row is cut
// into NB blocks of 16 pixels, the N dimension of every MFMA.  Pixels of a
// block that fall outside the image (or beyond Tw) carry v = 0.
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
//   Accumulator register R' = 4 mb2 + r holds tap column b = R' / HB and, in
//   lane group g, tap row a = 4 (R' % HB) + g (HB = ceil(KS / 4)): every lane
//   group of a register holds the same b for 16 consecutive pixels.
//
// col2im: Y of tap (a, b) at source pixel (e, c) belongs to padded position
// (e - a + R, c - b + R) in tile coordinates, "ring row" e - a and "ring column"
// c - b.  Shifting by b along the 16 pixels of a block is one DPP row shift per
// register (row_shl b inside the block, row_shr 16 - b for the part that lands
// in the block to the left), so the sum over b stays in registers and each row
// e leaves its tap-row partials sum_b Y_(a,b)[qx + b] in a ring of LDS rows
// indexed by the ring row they feed, P[e - a][a][qx + 2R]; every entry is
// written once, by the wave that owns row e (no atomics, deterministic).  Ring
// row o is complete once rows o .. o + 2R are done; its slab row o + 2R is
// X(o, x) = sum_a P[o][a][x + 2R] over the tap rows written by rows of the tile.
#pragma once

#include <type_traits>

#include "tnrd_device.hpp"
#include "tnrd_fused_common.hpp"
#include "tnrd_internal.hpp"

namespace tnrd {

struct FusedLds {
    int ldw;      // u tile row pitch
    int u_off, u_size;
    int e_off;    // input-gradient mode: e tile, same shape as the u tile
    int t_off, t_pitch, t_size;  // influence table (Gaussian form: weight rows of t_pitch floats;
                                 // polynomial form: [filter][2][intervals][4] coefficients)
    int ni;                      // polynomial form: intervals per filter
    int tf_pitch;                // polynomial form: floats per filter (8 ni, padded to 4 mod 16 so
                                 // that the 4 filters a wave's lane groups read start in distinct banks)
    int p_off, pw, ring, p_size; // row partials: ring of `ring` output rows x KS tap rows x pw
    int red_off;                 // 8 floats for workgroup reductions
    int dummy_off;               // 64 floats: target of the stores of masked-off lanes
    int total;
};

// Rows of a last round that join the round before it (see fused_tile).
constexpr int FUSED_MERGE = 2;
__host__ __device__ inline int fused_ring(int ks, int nw) { return 2 * nw + 2 * (ks / 2) + FUSED_MERGE; }

__host__ __device__ inline FusedLds fused_lds(int ks, int nmb, int nb, int th, int tw, int nrbf,
                                              int nw, int mode, int rbfm)
{
    const int R = ks / 2;
    FusedLds l;
    // u (and e) tile origin: R before the tile (z on the tile's own pixels)
    const int uo = R;
    (void)mode;
    const int luh = th + 2 * uo;
    l.ldw = tw + 2 * uo + 1;
    l.u_off = 0;
    l.u_size = (luh * l.ldw + 63) & ~63;  // whole 64-word chunks (the direct-to-LDS loads)
    l.e_off = l.u_off + l.u_size;
    l.t_off = l.e_off + (mode == MODE_BWD_INPUT ? l.u_size : 0);
    l.t_pitch = nrbf + 4 * RBF_WIN + 1;
    l.ni = POLY_NI;
    l.tf_pitch = POLY_TFP;
    l.t_size = rbfm == RBF_POLY || rbfm == RBF_POLY3 ? 16 * nmb * l.tf_pitch
                                                     : ((16 * nmb * l.t_pitch + 3) & ~3);
    l.p_off = l.t_off + l.t_size;
    l.pw = 16 * nb + 2 * R;
    l.ring = fused_ring(ks, nw);
    l.p_size = l.ring * ks * l.pw;
    // the prologue stages the filters in the P area (unless they come prepared)
    const int stage = 16 * nmb * ks * ks;
    if (l.p_size < stage) l.p_size = stage;
    l.red_off = l.p_off + l.p_size;
    l.dummy_off = l.red_off + 8;
    l.total = l.dummy_off + 64;
    return l;
}

// One output tile of one stage.  The pointers in `io` are those of the tile's
// image ([H][W] planes); (ty0, tx0) is the tile's origin.  The caller's
// workgroup runs it with 64 * NW threads and the dynamic LDS of fused_lds().
template <int KS, int NMB, int NB, int NW, int MODE, int PREC, int RBFM>
__device__ __forceinline__ void fused_tile(
    const FusedIO &io, int H, int W, int Th, int Tw, int ty0, int tx0,
    const float *__restrict__ filt, int Nk, const float *__restrict__ rbfw, int Nrbf,
    const FusedRbf &rb, const float *__restrict__ lam_t, float *lds)
{
    constexpr bool BWD = MODE == MODE_BWD_INPUT;
    constexpr bool POLY = RBFM == RBF_POLY || RBFM == RBF_POLY3;
    constexpr bool CUBIC = RBFM == RBF_POLY3;  // cubic half-interval table (BF16 operands)
    static_assert(!CUBIC || PREC == PREC_BF16, "the cubic half-interval form is for BF16 operands");
    // Polynomial form: the coefficient table comes ready-made from io.prep
    // (k_prep_stage); with FP32 operands the per-lane filter operands too
    constexpr bool PREP_TAB = POLY;
    constexpr bool PREP_OPS = POLY && PREC == PREC_F32;
    // the mixed kernels' BF16/FP16 filter operands come prepared as well
    constexpr bool PREP_MOPS = POLY && PREC != PREC_F32;
    const float *__restrict__ u_prev = io.u_prev;
    const float *__restrict__ f = io.f;
    using G = Geo<KS>;
    using G2 = Geo2<KS>;
    constexpr int R = G::R, KK = G::KK, KS1 = G::KS1;
    constexpr int HB = G2::HB, NREG = G2::NREG, MB2 = G2::MB2;
    constexpr int KS2 = 4 * NMB;  // GEMM2 k-steps (4 filters each)
    constexpr int THREADS = 64 * NW;
    constexpr int RING = 2 * NW + 2 * R + FUSED_MERGE;
    constexpr int PW = 16 * NB + 2 * R;  // P row pitch (fused_lds().pw)
    // Every mode computes responses on the tile's own pixels (its source region)
    // and exports the force they spread over the tile plus an R ring to its slab;
    // the u (and e) tile starts UO = R before the tile.
    constexpr int UO = R;

    const FusedLds L = fused_lds(KS, NMB, NB, Th, Tw, Nrbf, NW, MODE, RBFM);
    float *su = lds + L.u_off;
    float *se = lds + L.e_off;
    float *stab = lds + L.t_off;
    float *sp = lds + L.p_off;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;

    const int Eh = Th, Ew = Tw;  // source region
    const int luh = Th + 2 * UO, luw = Tw + 2 * UO;

    // ---- prologue: every global load of a thread is issued before the first
    // use, so the workgroup pays one memory latency, not one per element.
    // (1) the stage's filters, staged in the P area (free until the first
    // block's partials), unless the operands come prepared
    float *sf = sp;
    if (!PREP_OPS && !PREP_MOPS) {
        const int nf = Nk * KK;
        for (int base = 0; base < nf; base += 8 * THREADS) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = filt[min(base + k * THREADS + tid, nf - 1)];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (base + k * THREADS + tid < nf) sf[base + k * THREADS + tid] = v[k];
        }
    }
    // (2b) input-gradient mode: e = y * g_t over the same region, where
    // y = du_t/d(ut_t) = u_t^2 / ((1+2l) u_t^2 + 2 l f^2) is the prox derivative
    // written with the prox output (equal to the closed form of eq. derv2); for
    // the projected reaction y is the projection's derivative, 1 where u_t > c.
    float emax = 0.f;  // largest |e| of the tile (input-gradient mode)
    if (BWD) {
        const float lam0 = lam_t[0];
        const float *ucn = io.u_cur;
        const float *gcn = io.g_cur;
        const float *fcn = f;
        const int n = luh * luw;
        for (int base = 0; base < n; base += 4 * THREADS) {
            float uu[4], ff[4], gg[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int i = min(base + k * THREADS + tid, n - 1);
                int ly = i / luw, lx = i - ly * luw;
                int yy = reflect_clamp(ty0 - UO + ly, H), xx = reflect_clamp(tx0 - UO + lx, W);
                size_t q = (size_t)yy * W + xx;
                uu[k] = ucn[q];
                ff[k] = fcn[q];
                gg[k] = gcn[q];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int i = base + k * THREADS + tid;
                if (i < n) {
                    int ly = i / luw, lx = i - ly * luw;
                    const float ev = react_dut(io.react, uu[k], ff[k], lam0, io.proj_c) * gg[k];
                    se[ly * L.ldw + lx] = ev;
                    emax = fmaxf(emax, fabsf(ev));
                }
            }
        }
        // the padding word of each row (read by the mixed kernels' pad k-slots)
        for (int ly = tid; ly < luh; ly += THREADS) se[ly * L.ldw + luw] = 0.f;
    }
    // (3) Gaussian form: the RBF weights are the table itself, rows zero padded
    // by 2W on both sides
    if (!POLY) {
        float *dst = stab;
        const int pitch = L.t_pitch;
        const int pad = 2 * RBF_WIN;
        const int n = 16 * NMB * pitch;
        const int nw = Nk * Nrbf;
        for (int base = 0; base < n; base += 8 * THREADS) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                int i = base + k * THREADS + tid;
                int fi = i / pitch, jj = i - fi * pitch - pad;
                int src = min(max(fi * Nrbf + jj, 0), nw - 1);
                float w = rbfw[src];
                v[k] = (fi < Nk && jj >= 0 && jj < Nrbf) ? w : 0.f;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (base + k * THREADS + tid < n) dst[base + k * THREADS + tid] = v[k];
        }
    }
    // (2c) polynomial form: the prepared coefficient table straight into LDS in
    // 256-float chunks (lane l fills floats 4l .. 4l+3 of its wave's chunk).
    // With FP32 operands and 7x7 filters it is issued first, so that it lands
    // while the u tile is formed; the other instances issue it after the u tile
    // (measured faster for them).
    constexpr bool TAB_FIRST = PREC == PREC_F32 && KS == 7;
    auto load_table = [&]() {
        if (PREP_TAB && !io.keep_table) {
            for (int c = wave; c * 256 < L.t_size; c += NW) {
                const int k = c * 256 + 4 * lane;
                if (k < L.t_size) __builtin_amdgcn_global_load_lds(io.prep + k, stab + c * 256, 16, 0, 0);
            }
        }
    };
    if (TAB_FIRST) load_table();
    // (2) the u tile (rows ty0-UO .. ty0+Th+UO-1, reflected at the border),
    // loaded straight into LDS in 64-word chunks (lane l of a wave fills word
    // l of its chunk).  The loads stay in flight while the filter registers
    // are set up; padding words get an in-image value.
    // Forward with the previous stage's reaction pending: u_{t-1} =
    // reaction(u_{t-2}, force gathered from the slabs, f) at every position of
    // the tile (own pixels also written back to io.u_keep for later stages).
    if (MODE != MODE_FWD || !io.pend) {
        for (int c = wave; c * 64 < L.u_size; c += NW) {
            const int k = c * 64 + lane;
            const int ly = k / L.ldw, lx = k - ly * L.ldw;
            const bool in = ly < luh && lx < luw;
            const int yy = reflect_clamp(ty0 - UO + (in ? ly : 0), H);
            const int xx = reflect_clamp(tx0 - UO + (in ? lx : 0), W);
            __builtin_amdgcn_global_load_lds(u_prev + (size_t)yy * W + xx, su + c * 64, 4, 0, 0);
        }
    } else {
        // wave w takes the tile rows w, w + NW, ...; lane l the columns l + 64 c.  A
        // row's terms (reflection, covering tiles) are wave-uniform; a column's are
        // computed once per lane.
        const float lamp = io.lam_prev[0];
        const int th_own = min(Th, H - ty0), tw_own = min(Tw, W - tx0);
        constexpr int NCX = (16 * NB + 2 * R + 63) / 64;  // column chunks of the u tile
        const int wave_u = __builtin_amdgcn_readfirstlane(wave);
        int xcol[NCX];
        AxisTerms xt[NCX];
#pragma unroll
        for (int c = 0; c < NCX; ++c) {
            const int lx = min(lane + 64 * c, luw - 1);
            xcol[c] = reflect_clamp(tx0 - UO + lx, W);
            xt[c] = col_terms<R>(io.xt, xcol[c]);
        }
        // rows in flight per wave: a 32-row tile's 38 rows in one pass with FP32
        // operands, 7x7 filters and the polynomial form; the others keep the
        // registers
        constexpr int RU = PREC == PREC_F32 && KS == 7 && POLY ? 5 : 2;
        for (int ly0 = wave_u; ly0 < luh; ly0 += RU * NW) {
            float up[RU][NCX], ff[RU][NCX], xf[RU][NCX];
#pragma unroll
            for (int k = 0; k < RU; ++k) {
                const int ly = min(ly0 + k * NW, luh - 1);
                const int yy = reflect_clamp(ty0 - UO + ly, H);
                const AxisTerms yt = row_terms<R>(io.xt, yy);
                const size_t rowq = (size_t)yy * W;
#pragma unroll
                for (int c = 0; c < NCX; ++c) {
                    up[k][c] = u_prev[rowq + xcol[c]];
                    ff[k][c] = f[rowq + xcol[c]];
                    xf[k][c] = force_at(io.x_prev, yt, xt[c]);
                }
            }
#pragma unroll
            for (int k = 0; k < RU; ++k) {
                const int ly = ly0 + k * NW;
                if (ly >= luh) break;
                const int oy = ly - UO;
#pragma unroll
                for (int c = 0; c < NCX; ++c) {
                    const int lx = lane + 64 * c;
                    if (lx < luw) {
                        const float uv = reaction_step(io.react, up[k][c], xf[k][c], ff[k][c], lamp, io.proj_c);
                        su[ly * L.ldw + lx] = uv;
                        const int ox = lx - UO;
                        if (oy >= 0 && oy < th_own && ox >= 0 && ox < tw_own)
                            io.u_keep[(size_t)(ty0 + oy) * W + tx0 + ox] = uv;
                    }
                }
            }
        }
        // the padding word of each row (read by the mixed kernels' pad k-slots)
        for (int ly = tid; ly < luh; ly += THREADS) su[ly * L.ldw + luw] = 0.f;
    }
    if (!TAB_FIRST) load_table();
    if (!PREP_OPS && !PREP_MOPS) __syncthreads();  // the staged filters (and Gaussian table)

    // Mixed-precision input gradient: e, a = K e and phi' a go through BF16/FP16
    // operands.  With FP16 a power-of-two tile scale puts max|e| at 2^10 (FP16's
    // normal range starts at 2^-14 and ends below 2^16; |K e| <= 7 max|e| for
    // unit-norm 7x7 filters), undone in FP32 when g_{t-1} is formed; BF16 has
    // FP32's exponent range and needs none.
    float escale = 1.f, einv = 1.f;
    if (BWD && PREC == PREC_F16) {
        float wmax = emax;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) wmax = fmaxf(wmax, __shfl_xor(wmax, o));
        float *red = lds + L.red_off;
        if (lane == 0) red[wave] = wmax;
        __syncthreads();
        float m = 0.f;
        for (int w = 0; w < NW; ++w) m = fmaxf(m, red[w]);
        if (m > 0.f && isfinite(m)) {
            int ex = ilogbf(m);
            escale = ldexpf(1.f, 10 - ex);
            einv = ldexpf(1.f, ex - 10);
        }
    }

    // ---- filter operands in registers (from the staged copy, or the prepared
    // per-lane operands: quad k4 of lane l at floats 4 (64 k4 + l) .. +3 after
    // the table, GEMM1's a1[mb][s] first, then GEMM2's a2[mb2][s])
    float a1[NMB][KS1];
    float a2[MB2][KS2];
    if (PREP_OPS) {
        constexpr int NA1 = NMB * KS1, NOPS = NA1 + MB2 * KS2, NQ = (NOPS + 3) / 4;
        const floatx4 *opq = reinterpret_cast<const floatx4 *>(io.prep + L.t_size) + lane;
        floatx4 q[NQ];
#pragma unroll
        for (int k4 = 0; k4 < NQ; ++k4) q[k4] = opq[64 * k4];
#pragma unroll
        for (int k = 0; k < NOPS; ++k) {
            if (k < NA1) a1[k / KS1][k % KS1] = q[k >> 2][k & 3];
            else a2[(k - NA1) / KS2][(k - NA1) % KS2] = q[k >> 2][k & 3];
        }
    }
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
        for (int s = 0; s < KS1; ++s) {
            int fi = 16 * mb + j, t = 4 * s + g;
            if (!PREP_OPS && PREC == PREC_F32) a1[mb][s] = (fi < Nk && t < KK) ? sf[fi * KK + t] : 0.f;
        }
    // GEMM2 A operand: lane (g, j) supplies slot row j of block mb2, i.e.
    // register R' = 4 mb2 + (j & 3) in lane group j >> 2, and k-row g of k-step s,
    // i.e. filter 16 (s >> 2) + 4 g + (s & 3).
    int slot_a[MB2], slot_b[MB2];
#pragma unroll
    for (int mb2 = 0; mb2 < MB2; ++mb2) {
        const int Rr = 4 * mb2 + (j & 3);
        slot_b[mb2] = Rr < NREG ? Rr / HB : KS;
        slot_a[mb2] = 4 * (Rr % HB) + (j >> 2);
    }
#pragma unroll
    for (int mb2 = 0; mb2 < MB2; ++mb2)
#pragma unroll
        for (int s = 0; s < KS2; ++s) {
            int fi = 16 * (s >> 2) + 4 * g + (s & 3);
            const int ta = slot_a[mb2], tb = slot_b[mb2];
            if (!PREP_OPS && PREC == PREC_F32)
                a2[mb2][s] = (fi < Nk && ta < KS && tb < KS) ? sf[fi * KK + ta * KS + tb] : 0.f;
        }

    // mixed precision: 16-wide k-steps, operands converted once to BF16/FP16
    using MX = Mix<PREC>;
    typedef typename MX::V MV;
    constexpr bool MIXED = PREC != PREC_F32;
    constexpr int KSH = (KK + 15) / 16;  // GEMM1 k-steps of 16 taps
    MV a1m[NMB][MIXED ? KSH : 1];
    MV a2m[MB2][MIXED ? NMB : 1];
    // GEMM1 k-slots (mixed): the 7 x 7 taps in a 7 x 8 grid with a pad column in
    // front, slot 16 s + 4 g + i = tap row 2 s + (g >> 1), column 4 (g & 1) + i - 1,
    // so a lane's four taps of a k-step are adjacent in one row and its B
    // operand reads take compile-time offsets from one per-lane base.  Pad
    // slots and row 7 carry zero weight.
    static_assert(!MIXED || (KS == 7 && KSH == 4), "the mixed tap grid is laid out for 7 x 7 filters");
    if constexpr (PREP_MOPS) {
        // prepared (k_prep_stage): operand v = 2 k4 + h of lane l in quad k4, a1m first
        constexpr int NV = NMB * KSH + MB2 * NMB, NQM = (NV + 1) / 2;
        const int4v *opq = reinterpret_cast<const int4v *>(io.prep + L.t_size) + lane;
        int4v q[NQM];
#pragma unroll
        for (int k4 = 0; k4 < NQM; ++k4) q[k4] = opq[64 * k4];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const MV op = __builtin_bit_cast(MV, int2v{q[v >> 1][2 * (v & 1)], q[v >> 1][2 * (v & 1) + 1]});
            if (v < NMB * KSH) a1m[v / KSH][v % KSH] = op;
            else a2m[(v - NMB * KSH) / NMB][(v - NMB * KSH) % NMB] = op;
        }
    } else if (MIXED) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int s = 0; s < KSH; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int fi = 16 * mb + j, ta = 2 * s + (g >> 1), tb = 4 * (g & 1) + i - 1;
                    const bool ok = fi < Nk && ta < KS && tb >= 0 && tb < KS;
                    a1m[mb][s][i] = MX::cvt(ok ? sf[fi * KK + ta * KS + tb] : 0.f);
                }
#pragma unroll
        for (int mb2 = 0; mb2 < MB2; ++mb2)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int fi = 16 * mb + 4 * g + i;
                    const int ta = slot_a[mb2], tb = slot_b[mb2];
                    a2m[mb2][mb][i] =
                        MX::cvt((fi < Nk && ta < KS && tb < KS) ? sf[fi * KK + ta * KS + tb] : 0.f);
                }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the direct-to-LDS u tile and table loads have landed
    __syncthreads();  // u tile and table complete; the staged filters have been read

    // GEMM1 B-operand offsets: tap t = 4 s + g -> (a, b) = (t / KS, t % KS)
    int off1[KS1];
#pragma unroll
    for (int s = 0; s < KS1; ++s) {
        int t = 4 * s + g;
        off1[s] = t < KK ? (t / KS) * L.ldw + (t % KS) : 0;
    }
    // mixed GEMM1 B operands: lane group g's taps of k-step s sit at compile-time
    // offsets 2 s ldw + i below the per-lane base ub - gofs; in the last k-step
    // the rows past KS - 1 (zero weights) read row KS - 1 instead (gofs_last),
    // so no read leaves the tile.  Column -1 (the pad slot) is the tile row's
    // padding word past the last column, which holds a finite value.
    const int gofs = (g >> 1) * L.ldw + 4 * (g & 1) - 1;
    const int gofs_last = (min(2 * (KSH - 1) + (g >> 1), KS - 1) - 2 * (KSH - 1)) * L.ldw + 4 * (g & 1) - 1;

    const float lam = lam_t[0];
    // per-lane part of the polynomial table address: filter 16 mb + 4 g + r
    const int tab_g = 4 * g * POLY_TFP;

    // GEMM1 of block (row e, 16-pixel block cb): z = K u (and a = K e in
    // input-gradient mode).  The B operands are read first (gemm1_load), the
    // MFMAs run in k-step ranges (gemm1_steps) spread over the next block's work.
    constexpr int K1 = MIXED ? KSH : KS1;  // GEMM1 k-steps
    float bu[MIXED ? 1 : KS1], be[MIXED || !BWD ? 1 : KS1];
    MV bum[MIXED ? KSH : 1], bem[MIXED && BWD ? KSH : 1];
    auto gemm1_load = [&](int e, int cb) {
        const int c = 16 * cb + j;
        const int cc = c < Ew ? c : Ew - 1;
        const float *ub = su + (e + 2 * R) * L.ldw + cc + 2 * R;
        const float *eb = se + (e + 2 * R) * L.ldw + cc + 2 * R;
        if (MIXED) {
            const float *ubg = ub - gofs, *ubl = ub - gofs_last;
            const float *ebg = eb - gofs, *ebl = eb - gofs_last;
#pragma unroll
            for (int s = 0; s < KSH; ++s) {
                const float *up = s == KSH - 1 ? ubl : ubg;
                const float *ep = s == KSH - 1 ? ebl : ebg;
                floatx4 xu, xe;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    xu[i] = up[-(2 * s * L.ldw + i)];
                    xe[i] = BWD ? escale * ep[-(2 * s * L.ldw + i)] : 0.f;
                }
                bum[s] = MX::cvt4(xu);
                if (BWD) bem[s] = MX::cvt4(xe);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KS1; ++s) {
                bu[s] = ub[-off1[s]];
                if (BWD) be[s] = eb[-off1[s]];
            }
        }
    };
    auto gemm1_steps = [&](int s0, int s1, floatx4 *acc1, floatx4 *acca) {
#pragma unroll
        for (int s = s0; s < s1; ++s)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) {
                if (MIXED) {
                    acc1[mb] = MX::mfma(a1m[mb][s], bum[s], acc1[mb]);
                    if (BWD) acca[mb] = MX::mfma(a1m[mb][s], bem[s], acca[mb]);
                } else {
                    acc1[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[mb][s], bu[s], acc1[mb], 0, 0, 0);
                    if (BWD)
                        acca[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[mb][s], be[s], acca[mb], 0, 0, 0);
                }
            }
    };
    auto gemm1 = [&](int e, int cb, floatx4 *acc1, floatx4 *acca) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
            acc1[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
            acca[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        gemm1_load(e, cb);
        gemm1_steps(0, K1, acc1, acca);
    };

    // Polynomial form: table reads of one filter group (the four filters of an
    // accumulator register quad) into one of two buffers.  The interval index is
    // s = z / step - mu0 / step + W + 1 rounded; a lane whose pixel is masked off
    // takes scale 0 and offset POLY_OFF_MASKED instead, which selects the all-zero
    // last interval, so its influence comes out exactly 0 with no select.  The
    // cubic half-interval form indexes halves with 2 s + 1 (the caller's scale
    // and offset): half 2q + h = floor(2 s + 1) of interval q, e = the fraction
    // in [0, 1), one 4-float read.
    float dq[2][4];
    floatx4 lo[2][4], hi[2][4];
    auto fetch = [&](const floatx4 *acc1, int mb, int slot, float sscale, float soff) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float s = fmaf(acc1[mb][r], sscale, soff);
            int q;
            if (CUBIC) {
                // s = 2 (interval coordinate) + 1: half q = floor(s), e = its fraction
                const float sc = __builtin_amdgcn_fmed3f(s, 0.f, (float)(2 * POLY_NI) - 0.5f);
                q = (int)sc;
                dq[slot][r] = __builtin_amdgcn_fractf(sc);
            } else {
                const float jr = rintf(s);
                dq[slot][r] = s - jr;
                q = (int)__builtin_amdgcn_fmed3f(jr, 0.f, (float)(POLY_NI - 1));
            }
            const float *cp = stab + (16 * mb + r) * POLY_TFP + tab_g + 4 * q;
            lo[slot][r] = *reinterpret_cast<const floatx4 *>(cp);
            if (!CUBIC) hi[slot][r] = *reinterpret_cast<const floatx4 *>(cp + 4 * POLY_NI);
        }
    };
    // influence of filter group mb, in place: v = phi(z) (times phi' and a in
    // input-gradient mode), lane-local (pixel j, filters 16 mb + 4 g + r)
    auto influence = [&](floatx4 *acc1, const floatx4 *acca, int mb, bool valid) {
        if (POLY) {
            const int cur = mb & 1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float d = dq[cur][r];
                const floatx4 l = lo[cur][r];
                float p;
                if (CUBIC) {
                    p = fmaf(l[3], d, l[2]);
                } else {
                    const floatx4 h = hi[cur][r];
                    p = fmaf(h[3], d, h[2]);
                    p = fmaf(p, d, h[1]);
                    p = fmaf(p, d, h[0]);
                    p = fmaf(p, d, l[3]);
                    p = fmaf(p, d, l[2]);
                }
                p = fmaf(p, d, l[1]);
                p = fmaf(p, d, l[0]);
                // input-gradient mode: p = d phi / ds, so phi'(z) a = p a / step
                if (BWD) p *= rb.inv_step * acca[mb][r];
                acc1[mb][r] = p;  // 0 for a masked-off pixel (see fetch)
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float s = fmaf(acc1[mb][r], rb.inv_step, -rb.mu0_over_step);
                const float jr = fminf(fmaxf(rintf(s), -(float)RBF_WIN), rb.jmax);
                const float d = s - jr;
                const float *w = stab + (16 * mb + 4 * g + r) * L.t_pitch + (int)jr + RBF_WIN;
                const float q = __builtin_amdgcn_exp2f(rb.rho_log2e * d);
                const float E = __builtin_amdgcn_exp2f(-rb.rho_log2e * d * fmaf(0.5f, d, (float)RBF_WIN));
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
                    const float dphi = rb.rho_over_step * E * fmaf(q, accd, -(d + (float)RBF_WIN) * acc);
                    v = dphi * acca[mb][r];
                } else {
                    v = E * acc;
                }
                acc1[mb][r] = (valid && fabsf(d) <= 0.5f) ? v : 0.f;
            }
        }
    };
    // GEMM2 k-steps of filter group mb: Y += K^T-slots . v
    auto gemm2_group = [&](const floatx4 *acc1, int mb, floatx4 *acc2) {
        if (MIXED) {
            const MV vb = MX::cvt4(acc1[mb]);  // filters 16 mb + 4 g + i of pixel j: GEMM1's quad
#pragma unroll
            for (int mb2 = 0; mb2 < MB2; ++mb2) acc2[mb2] = MX::mfma(a2m[mb2][mb], vb, acc2[mb2]);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int mb2 = 0; mb2 < MB2; ++mb2)
                    acc2[mb2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[mb2][4 * mb + r], acc1[mb][r],
                                                                     acc2[mb2], 0, 0, 0);
        }
    };

    // Block (e, cb) from its responses c1 (and a = K e in ca), interleaved with
    // GEMM1 of the next block (en, cbn) into n1/na: influence, K^T GEMM and
    // the x-direction col2im.  xa[h] enters holding block cb-1's partial X (tap
    // rows a = 4h + g) and leaves holding block cb's; block cb-1 is complete
    // then and goes to the P ring slot of output row e - a:
    //   P[(e - a) mod RING][a][qx + 2R] = sum_b Y_(a,b)[qx + b]   (qx relative to the row)
    // The scheduling fences split the work into NMB + 1 segments; in each, the
    // table reads of the next filter group and a third of the next GEMM1 are
    // in flight while the current group's influence and GEMM2 run.  The wave's
    // last block has no next block (next_c false): its instance leaves GEMM1 out.
    auto process = [&](auto next_c, int e, int cb, floatx4 *c1, const floatx4 *ca, float *xa, int en,
                       int cbn, floatx4 *n1, floatx4 *na) {
        constexpr bool NEXT = decltype(next_c)::value;
        const int c = 16 * cb + j;
        const int xi = tx0 + c;
        const bool valid = (c < Ew) && (xi < W);
        // input-gradient mode with export: z and a of this lane's pixel (every image
        // pixel is own to exactly one tile), stored before anything else of the
        // block, when the fewest registers are live
        if (BWD && io.za && valid) {
            const size_t zi = za_index((size_t)(ty0 + e) * W + xi, Nk, 4 * g);
            if constexpr (PREC == PREC_BF16) {
                // BF16 words: the quad's four z and four a (unscaled) in one 16-byte store
                unsigned short *q = reinterpret_cast<unsigned short *>(io.za) + zi;
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
                    if (16 * mb + 4 * g < Nk) {
                        floatx4 av = ca[mb];
#pragma unroll
                        for (int i = 0; i < 4; ++i) av[i] *= einv;
                        const MV zb = MX::cvt4(c1[mb]), ab = MX::cvt4(av);
                        *reinterpret_cast<int4v *>(q + 32 * mb) =
                            int4v{__builtin_bit_cast(int2v, zb)[0], __builtin_bit_cast(int2v, zb)[1],
                                  __builtin_bit_cast(int2v, ab)[0], __builtin_bit_cast(int2v, ab)[1]};
                    }
            } else {
                float *q = io.za + zi;
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
                    if (16 * mb + 4 * g < Nk) {
                        *reinterpret_cast<floatx4 *>(q + 8 * 4 * mb) = c1[mb];
                        *reinterpret_cast<floatx4 *>(q + 8 * 4 * mb + 4) = ca[mb];
                    }
            }
        }
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
            n1[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
            na[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        floatx4 acc2[MB2];
#pragma unroll
        for (int mb2 = 0; mb2 < MB2; ++mb2) acc2[mb2] = floatx4{0.f, 0.f, 0.f, 0.f};
        // polynomial form: interval coordinate of this lane's pixel, or the
        // masked-off coordinate
        const float sscale = valid ? (CUBIC ? 2.f : 1.f) * rb.inv_step : 0.f;
        const float soff = valid ? (CUBIC ? 2.f * ((float)(RBF_WIN + 1) - rb.mu0_over_step) + 1.f
                                          : (float)(RBF_WIN + 1) - rb.mu0_over_step)
                                 : POLY_OFF_MASKED;
        if constexpr (NEXT) gemm1_load(en, cbn);
        if (POLY) fetch(c1, 0, 0, sscale, soff);
        if constexpr (NEXT) gemm1_steps(0, K1 / NMB, n1, na);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 1; m <= NMB; ++m) {
            if (POLY && m < NMB) fetch(c1, m, m & 1, sscale, soff);
            influence(c1, ca, m - 1, valid);
            gemm2_group(c1, m - 1, acc2);
            if (NEXT && m < NMB) gemm1_steps(m * K1 / NMB, (m + 1) * K1 / NMB, n1, na);
            __builtin_amdgcn_sched_barrier(0);
        }

        // x-direction col2im with row shifts: tap column b moves pixel c to
        // output column c - b, inside this block (row_shl b) or into block cb-1
        // (row_shr 16 - b).
        float xb[HB];
#pragma unroll
        for (int h = 0; h < HB; ++h) xb[h] = 0.f;
#pragma unroll
        for (int b = 0; b < KS; ++b)
#pragma unroll
            for (int h = 0; h < HB; ++h) {
                const int Rr = b * HB + h;
                const float y = acc2[Rr >> 2][Rr & 3];
                if (b == 0) {
                    xb[h] += y;
                } else {
                    xb[h] += row_shl(y, b);
                    xa[h] += row_shr(y, 16 - b);
                }
            }
        // branch-free stores: masked-off lanes write their own dummy word
        const int em = e % RING;  // wave-uniform
        const int dummy = L.dummy_off + lane;
#pragma unroll
        for (int h = 0; h < HB; ++h) {
            const int a = 4 * h + g;
            const int sl = em - a < 0 ? em - a + RING : em - a;
            const int prow = L.p_off + (sl * KS + a) * PW;
            // block cb-1: output columns 16 (cb-1) + j; block -1 only reaches j >= 16 - 2R
            const bool ok_a = a < KS && (cb > 0 || j >= 16 - 2 * R);
            lds[ok_a ? prow + 16 * (cb - 1) + j + 2 * R : dummy] = xa[h];
            if (cb == NB - 1) lds[a < KS ? prow + 16 * cb + j + 2 * R : dummy] = xb[h];
            xa[h] = xb[h];
        }
    };

    const int e_lo = 0, e_hi = min(Eh, H - ty0);  // source rows in the image
    auto slot_of = [&](int qy) {  // ring slot of output row qy (-RING < qy)
        const int m = (qy + RING) % RING;
        return sp + m * KS * PW;
    };

    // ---- export of completed ring rows to the tile's slab.  Ring row o (source
    // row e feeds ring row e - a with its tap row a) is slab row o + 2R; slab
    // column dx is P column dx.  Tap rows written by source rows outside
    // [0, e_hi) count as zero.  The input-gradient mode's slab holds the force
    // in the gradient's own scale (FP16: einv undoes the tile's e scale).
    const int sw = Tw + 2 * R;
    const int sw_own = min(Tw, W - tx0) + 2 * R;
    auto export_rows = [&](int o0, int o1) {
        float *xo = io.x_out;
        const int nx = (o1 - o0) * sw;
        for (int i = tid; i < nx; i += THREADS) {
            const int xdy = i / sw, xdx = i - xdy * sw;
            const int o = o0 + xdy, dx = xdx;
            if (dx >= sw_own) continue;
            const float *b = slot_of(o) + dx;
            float xs = 0.f;
#pragma unroll
            for (int a = 0; a < KS; ++a) {
                const int e = o + a;  // the source row that wrote tap row a
                const float v = b[a * PW];
                xs += (e >= 0 && e < e_hi) ? v : 0.f;
            }
            xo[(o + 2 * R) * sw + dx] = BWD ? xs * einv : xs;
        }
    };

    // ---- main loop: rounds of NW tile rows, one per wave.  After round k the
    // partials of every row below NW (k+1) are in the ring; the ring rows they
    // complete are exported after its barrier, before the next round's rows are
    // stored.  A last round of at most FUSED_MERGE rows follows the
    // round before it without a barrier between them, instead of running as a
    // round of its own in which most waves wait.  The ring holds
    // 2 NW + 2R + FUSED_MERGE rows, so the rows written between two barriers
    // never share a slot with the rows the previous round's outputs still read.
    // GEMM1 of the wave's next block is issued before the influence of the
    // current one.
    const int rounds = (e_hi + NW - 1) / NW;
    const bool merge = rounds >= 2 && e_hi - NW * (rounds - 1) <= FUSED_MERGE;
    bool have = false;
    floatx4 c1[NMB], ca[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
        c1[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
        ca[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    int o_done = -2 * R;  // ring rows exported so far
    for (int k = 0; k < rounds; ++k) {
        const bool sync = !(merge && k == rounds - 2);
        const int e = NW * k + wave;
        if (e >= e_lo && e < e_hi) {
            if (!have) gemm1(e, 0, c1, ca);
            float xa[HB];
#pragma unroll
            for (int h = 0; h < HB; ++h) xa[h] = 0.f;
            // the GEMM1 after the row's last block is that of the wave's next
            // row.  After the wave's last block there is none.  With FP32
            // operands the forward on two-block rows and the input-gradient
            // mode (two GEMM1s per block) on rows of up to three blocks leave it
            // out there (a second instance of the block code), which pays where
            // a wave has few blocks; elsewhere the saving does not pay for the
            // larger code, or the registers are not there, and a row of this
            // tile is repeated there and its result dropped.
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                floatx4 n1[NMB], na[NMB];
                const int en = cb + 1 < NB ? e : min(e + NW, e_hi - 1);
                const int cbn = cb + 1 < NB ? cb + 1 : 0;
                if constexpr (PREC == PREC_F32 && (MODE == MODE_FWD ? NB == 2 : NB <= 3)) {
                    if (cb + 1 < NB || e + NW < e_hi)
                        process(std::true_type{}, e, cb, c1, ca, xa, en, cbn, n1, na);
                    else
                        process(std::false_type{}, e, cb, c1, ca, xa, en, cbn, n1, na);
                } else {
                    process(std::true_type{}, e, cb, c1, ca, xa, en, cbn, n1, na);
                }
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb) {
                    c1[mb] = n1[mb];
                    ca[mb] = na[mb];
                }
            }
            have = true;
        } else {
            have = false;
        }
        if (!sync) continue;
        __syncthreads();
        // ring rows below every source row still to come are complete
        const int o_end = e_hi <= NW * (k + 1) ? e_hi : NW * (k + 1) - 2 * R;
        export_rows(o_done, o_end);
        o_done = o_end;
    }
    __syncthreads();  // LDS is free for the workgroup's next tile
}

template <int KS, int NMB, int NB, int NW, int MODE, int PREC, int RBFM>
__global__ void __launch_bounds__(64 * NW) k_fused_stage(
    FusedIO io, int H, int W, int Th, int Tw, int tiles_x, int tiles_per_img,
    const float *__restrict__ filt, int Nk, const float *__restrict__ rbfw, int Nrbf,
    FusedRbf rb, const float *__restrict__ lam_t)
{
    extern __shared__ float lds[];
    const int bid = xcd_tile_order((int)blockIdx.x, (int)gridDim.x);
    const int img = bid / tiles_per_img;
    const int trem = bid - img * tiles_per_img;
    const int ty = trem / tiles_x, tx = trem - ty * tiles_x;
    const size_t plane = (size_t)H * W;
    FusedIO ii = io;  // per-image pointers below; every other field as launched
    ii.u_prev = io.u_prev + img * plane;
    ii.f = io.f + img * plane;
    ii.out = io.out ? io.out + img * plane : nullptr;
    ii.u_cur = io.u_cur ? io.u_cur + img * plane : nullptr;
    ii.g_cur = io.g_cur ? io.g_cur + img * plane : nullptr;
    ii.za = !io.za ? nullptr
            : PREC == PREC_BF16
                ? reinterpret_cast<float *>(reinterpret_cast<unsigned short *>(io.za) + img * plane * za_stride(Nk))
                : io.za + img * plane * za_stride(Nk);
    const size_t sl = (size_t)io.xt.sl;
    ii.x_out = io.x_out + ((size_t)img * tiles_per_img + trem) * sl;
    ii.x_prev = io.x_prev ? io.x_prev + (size_t)img * tiles_per_img * sl : nullptr;
    ii.u_keep = io.u_keep ? io.u_keep + img * plane : nullptr;
    fused_tile<KS, NMB, NB, NW, MODE, PREC, RBFM>(ii, H, W, Th, Tw, ty * Th, tx * Tw, filt, Nk, rbfw,
                                                  Nrbf, rb, lam_t, lds);
}

// Final reaction of a forward in exchange form: u_T = reaction(u_{T-1}, force
// gathered from the last stage's slabs, f), one pixel per thread: workgroup
// (b, c) covers pixels 256 c .. 256 c + 255 of tile b mod tiles_per_img of
// image b / tiles_per_img.
template <int R>
__global__ void __launch_bounds__(256) k_react_final(const float *__restrict__ u_prev,
                                                     const float *__restrict__ f,
                                                     const float *__restrict__ xs, float *__restrict__ out,
                                                     XTiles xt, int tiles_per_img,
                                                     const float *__restrict__ lam, int react, float proj_c)
{
    const int img = blockIdx.x / tiles_per_img;
    const int tile = blockIdx.x - img * tiles_per_img;
    const int ty = tile / xt.nx, tx = tile - ty * xt.nx;
    const int y0 = ty * xt.Th, x0 = tx * xt.Tw;
    const int th = min(xt.Th, xt.H - y0), tw = min(xt.Tw, xt.W - x0);
    const size_t plane = (size_t)xt.H * xt.W;
    const float *up = u_prev + img * plane;
    const float *fp = f + img * plane;
    float *op = out + img * plane;
    const float *xi = xs + (size_t)img * tiles_per_img * xt.sl;
    const float l = lam[0];
    const int i = blockIdx.y * 256 + threadIdx.x;
    if (i < th * tw) {
        const int y = y0 + i / tw, x = x0 + i % tw;
        const size_t q = (size_t)y * xt.W + x;
        op[q] = reaction_step(react, up[q], pixel_force<R>(xi, xt, y, x), fp[q], l, proj_c);
    }
}

// ------------------------------------------------------------------ batched
// One launch per stage covers the tiles of every image of an uneven batch:
// workgroup b takes the b-th (image, tile) item of the stage and runs the
// fused stage on it with that image's model (chosen by its look number).
// Stages are ordered by the kernel boundaries, so no workgroup ever waits on
// another.  State planes: u_t (t >= 1) lives in u_out if T - t is even, else
// in the image's scratch plane (u_0 = f); stage t reads u_{t-1}, applies the
// pending reaction of stage t - 1 in its prologue (writing u_t), and writes its
// slabs to xs[t & 1]; k_batched_final applies the last reaction into u_out.
__device__ __forceinline__ XTiles batch_xtiles(const BatchImage &im, int Th, int Tw, int R)
{
    return make_xtiles(im.H, im.W, Th, Tw, R);
}

__device__ __forceinline__ float *batch_plane(const BatchImage &im, int T, int t)
{
    return ((T - t) & 1) == 0 ? im.u_out : im.u_tmp;
}

// Stage t (< T) of batch item k.  keep_table: the LDS already holds this
// stage's coefficient table for this item's model.
template <int KS, int NMB, int NB, int NW, int RBFM>
__device__ __forceinline__ void batched_stage_item(const BatchArgs &a, int t, int k, float *lds,
                                                   int keep_table = 0)
{
    constexpr int KK = KS * KS, R = KS / 2;
    const BatchItem it = a.items[k];
    const BatchImage im = a.imgs[it.image];
    const int ty = it.tile / im.tiles_x, tx = it.tile - ty * im.tiles_x;
    const BatchModel md = a.models[im.model];
    FusedIO io{};
    io.f = im.f;
    io.xt = batch_xtiles(im, a.Th, a.Tw, R);
    io.pend = t > 0;
    io.u_prev = t <= 1 ? im.f : batch_plane(im, a.T, t - 1);
    io.u_keep = t > 0 ? batch_plane(im, a.T, t) : nullptr;
    // (selects, not an indexed load: an indexed member array would put the
    // descriptor copy in scratch memory)
    float *const xs_even = im.xs[0], *const xs_odd = im.xs[1];
    io.x_prev = t > 0 ? ((t & 1) ? xs_even : xs_odd) : nullptr;
    io.x_out = ((t & 1) ? xs_odd : xs_even) + (size_t)it.tile * io.xt.sl;
    io.lam_prev = md.lam + (t > 0 ? t - 1 : 0);
    io.out = nullptr;
    io.u_cur = nullptr;
    io.g_cur = nullptr;
    io.za = nullptr;
    io.react = md.react;
    io.proj_c = md.proj_c;
    io.prep = md.prep + (size_t)t * a.prep_stage;
    io.keep_table = keep_table;
    fused_tile<KS, NMB, NB, NW, MODE_FWD, PREC_F32, RBFM>(
        io, im.H, im.W, a.Th, a.Tw, ty * a.Th, tx * a.Tw, md.filt + (size_t)t * a.Nk * KK, a.Nk,
        md.rbfw + (size_t)t * a.Nk * a.Nrbf, a.Nrbf, a.rb, md.lam + t, lds);
}

// The last stage's reaction at own pixel i of batch item k: u_T into u_out.
template <int R>
__device__ __forceinline__ void batched_final_pixel(const BatchArgs &a, int k, int i)
{
    const BatchItem it = a.items[k];
    const BatchImage im = a.imgs[it.image];
    const BatchModel md = a.models[im.model];
    const XTiles xt = batch_xtiles(im, a.Th, a.Tw, R);
    const int ty = it.tile / xt.nx, tx = it.tile - ty * xt.nx;
    const int y0 = ty * xt.Th, x0 = tx * xt.Tw;
    const int th = min(xt.Th, xt.H - y0), tw = min(xt.Tw, xt.W - x0);
    if (i >= th * tw) return;
    const int T = a.T;
    const float *up = T == 1 ? im.f : batch_plane(im, T, T - 1);
    const float *xs = ((T - 1) & 1) ? im.xs[1] : im.xs[0];
    const int y = y0 + i / tw, x = x0 + i % tw;
    const size_t q = (size_t)y * xt.W + x;
    im.u_out[q] = reaction_step(md.react, up[q], pixel_force<R>(xs, xt, y, x), im.f[q], md.lam[T - 1],
                                md.proj_c);
}

template <int KS, int NMB, int NB, int NW, int RBFM>
__global__ void __launch_bounds__(64 * NW) k_batched_stage(BatchArgs a, int t)
{
    extern __shared__ float lds[];
    batched_stage_item<KS, NMB, NB, NW, RBFM>(a, t, blockIdx.x, lds);
}

// The last stage's reaction of every image: u_T into u_out, one pixel per
// thread; workgroup (b, c) covers pixels 256 c .. 256 c + 255 of item b.
template <int R>
__global__ void __launch_bounds__(256) k_batched_final(BatchArgs a)
{
    batched_final_pixel<R>(a, blockIdx.x, blockIdx.y * 256 + threadIdx.x);
}

// Platform of the persistent launch's scheduling loop (tnrd_persist.hpp) on
// the GPU: workgroup barriers, device-scope atomics on the workspace's
// counter and flags, the broadcast word in the workgroup's LDS.
template <int KS, int NMB, int NB, int NW, int RBFM>
struct BatchPersist {
    const BatchArgs *a;
    float *lds;
    int *sh;
    int table_key;  // (model, stage) whose coefficient table the LDS holds, -1: none
    __device__ int tid() const { return threadIdx.x; }
    __device__ void barrier() { __syncthreads(); }
    __device__ int fetch_next(int *p)
    {
        return __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void set_shared(int v) { *sh = v; }
    __device__ int get_shared() { return *sh; }
    __device__ int poll(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
    __device__ void store_release(int *p, int v)
    {
        __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // every counter to zero: the wave's stores have been acknowledged by the L2
    __device__ void stores_done() { __builtin_amdgcn_s_waitcnt(0); }
    __device__ void pause() { __builtin_amdgcn_s_sleep(2); }
    __device__ long long now() { return (long long)wall_clock64(); }
    __device__ void neighbours(int k, int *nb)
    {
        const BatchItem it = a->items[k];
        const BatchImage im = a->imgs[it.image];
        persist_neighbours(k - it.tile, it.tile, im.tiles_x, im.tiles / im.tiles_x, nb);
    }
    __device__ void work(int t, int k)
    {
        if (t < a->T) {
            // consecutive items mostly share the stage and the model: their table
            // stays in LDS (every thread computes the same key)
            const int key = a->imgs[a->items[k].image].model * (a->T + 1) + t;
            const int keep = RBFM == RBF_POLY && key == table_key;
            table_key = key;
            batched_stage_item<KS, NMB, NB, NW, RBFM>(*a, t, k, lds, keep);
        } else {
            for (int i = threadIdx.x; i < a->Th * a->Tw; i += 64 * NW) batched_final_pixel<KS / 2>(*a, k, i);
        }
    }
};

// Every stage of every tile of the batch in one launch: workgroups take
// (stage, item) pairs in stage-major order and wait for the item's
// neighbourhood to finish the stage before (persist_loop).  The broadcast
// word sits in the LDS's reduction slot, which the forward never uses.
template <int KS, int NMB, int NB, int NW, int RBFM>
__global__ void __launch_bounds__(64 * NW) k_batched_persist(BatchArgs a)
{
    extern __shared__ float lds[];
    const FusedLds L = fused_lds(KS, NMB, NB, a.Th, a.Tw, a.Nrbf, NW, MODE_FWD, RBFM);
    BatchPersist<KS, NMB, NB, NW, RBFM> p{&a, lds, reinterpret_cast<int *>(lds + L.red_off), -1};
    persist_loop(p, a.ctl);
}

// p[0 .. n) = 0 (a kernel, not a memset: the launch sequence is recorded in graphs)
static __global__ void __launch_bounds__(256) k_clear_ints(int *__restrict__ p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <int KS, int NMB, int NB, int NW, int MODE, int PREC, int RBFM>
inline hipError_t launch_fused(const StageArgs &s, int th, int tw, hipStream_t stream)
{
    FusedLds L = fused_lds(KS, NMB, NB, th, tw, s.grid.nrbf, NW, MODE, RBFM);
    size_t lds_bytes = (size_t)L.total * sizeof(float);
    raise_lds_limit((const void *)k_fused_stage<KS, NMB, NB, NW, MODE, PREC, RBFM>);
    if (lds_bytes > 160 * 1024) return hipErrorInvalidValue;
    FusedRbf rb = make_fused_rbf(s.grid);
    FusedIO io{};
    io.u_prev = s.u_prev;
    io.f = s.f;
    io.out = s.u_next;
    io.u_cur = s.u_cur;
    io.g_cur = s.g_cur;
    io.za = MODE == MODE_BWD_INPUT && (PREC == PREC_F32 || PREC == PREC_BF16) ? s.za : nullptr;
    io.react = s.react;
    io.proj_c = s.proj_c;
    io.prep = s.prep;
    if ((RBFM == RBF_POLY || RBFM == RBF_POLY3) && !s.prep) return hipErrorInvalidValue;
    const int tiles_x = (s.W + tw - 1) / tw, tiles_y = (s.H + th - 1) / th;
    const int tiles = tiles_x * tiles_y;
    if (!s.x_out) return hipErrorInvalidValue;
    io.x_out = s.x_out;
    io.xt = make_xtiles(s.H, s.W, th, tw, KS / 2);
    io.lam_prev = s.lam;
    if (MODE == MODE_FWD && s.pend) {
        if (!s.x_prev || !s.u_keep || !s.lam_prev) return hipErrorInvalidValue;
        io.x_prev = s.x_prev;
        io.u_keep = s.u_keep;
        io.lam_prev = s.lam_prev;
        io.pend = 1;
    }
    dim3 grid(tiles * s.N);
    hipLaunchKernelGGL((k_fused_stage<KS, NMB, NB, NW, MODE, PREC, RBFM>), grid, dim3(64 * NW),
                       lds_bytes, stream, io, s.H, s.W, th, tw, tiles_x, tiles, s.filt, s.Nk, s.rbfw,
                       s.grid.nrbf, rb, s.lam);
    return hipGetLastError();
}

// Input gradient of a stage from the input-gradient kernel's slabs (tiling
// (th, tw)): g_{t-1} = e - x - r e, e = y g_t, with y the reaction's derivative
// in ut_t and r its explicit derivative in u_{t-1} (prox: 0; projected:
// psi_u(u_{t-1}); quadratic: lambda), one pixel per thread as k_react_final.
template <int R>
__global__ void __launch_bounds__(256) k_grad_finish(const float *__restrict__ u_prev,
                                                     const float *__restrict__ u_cur,
                                                     const float *__restrict__ f,
                                                     const float *__restrict__ g_cur,
                                                     const float *__restrict__ xs, float *__restrict__ out,
                                                     XTiles xt, int tiles_per_img,
                                                     const float *__restrict__ lam, int react, float proj_c)
{
    const int img = blockIdx.x / tiles_per_img;
    const int tile = blockIdx.x - img * tiles_per_img;
    const int ty = tile / xt.nx, tx = tile - ty * xt.nx;
    const int y0 = ty * xt.Th, x0 = tx * xt.Tw;
    const int th = min(xt.Th, xt.H - y0), tw = min(xt.Tw, xt.W - x0);
    const size_t plane = (size_t)xt.H * xt.W;
    const float *xi = xs + (size_t)img * tiles_per_img * xt.sl;
    const float l = lam[0];
    const int i = blockIdx.y * 256 + threadIdx.x;
    if (i < th * tw) {
        const int y = y0 + i / tw, x = x0 + i % tw;
        const size_t q = img * plane + (size_t)y * xt.W + x;
        out[q] = grad_step(react, u_prev[q], u_cur[q], f[q], g_cur[q],
                           pixel_force<R>(xi, xt, y, x), l, proj_c);
    }
}

template <int KS>
inline hipError_t launch_grad_finish(const StageArgs &s, int th, int tw, hipStream_t stream)
{
    if (!s.x_prev || !s.u_prev || !s.u_cur || !s.g_cur || !s.u_next) return hipErrorInvalidValue;
    const XTiles xt = make_xtiles(s.H, s.W, th, tw, KS / 2);
    const int tiles = xt.nx * xt.ny;
    hipLaunchKernelGGL((k_grad_finish<KS / 2>), dim3(tiles * s.N, (th * tw + 255) / 256), dim3(256), 0,
                       stream, s.u_prev, s.u_cur, s.f, s.g_cur, s.x_prev, s.u_next, xt, tiles, s.lam,
                       s.react, s.proj_c);
    return hipGetLastError();
}

// Final reaction of a forward in exchange form on the tiling (th, tw).
template <int KS>
inline hipError_t launch_react_final(const StageArgs &s, int th, int tw, hipStream_t stream)
{
    if (!s.x_prev || !s.lam_prev || !s.u_prev || !s.u_next) return hipErrorInvalidValue;
    const XTiles xt = make_xtiles(s.H, s.W, th, tw, KS / 2);
    const int tiles = xt.nx * xt.ny;
    hipLaunchKernelGGL((k_react_final<KS / 2>), dim3(tiles * s.N, (th * tw + 255) / 256), dim3(256), 0,
                       stream, s.u_prev, s.f,
                       s.x_prev, s.u_next, xt, tiles, s.lam_prev, s.react, s.proj_c);
    return hipGetLastError();
}

template <int KS, int NMB, int NW, int MODE, int PREC, int RBFM>
inline hipError_t fused_nb(const StageArgs &s, int th, int tw, int nb, hipStream_t stream)
{
    switch (nb) {
    case 2: return launch_fused<KS, NMB, 2, NW, MODE, PREC, RBFM>(s, th, tw, stream);
    case 3: return launch_fused<KS, NMB, 3, NW, MODE, PREC, RBFM>(s, th, tw, stream);
    case 4: return launch_fused<KS, NMB, 4, NW, MODE, PREC, RBFM>(s, th, tw, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int KS, int NMB, int MODE, int PREC, int RBFM>
inline hipError_t fused_nw(const StageArgs &s, int th, int tw, int nb, int nw, hipStream_t stream)
{
    if (nw == 4) return fused_nb<KS, NMB, 4, MODE, PREC, RBFM>(s, th, tw, nb, stream);
    return fused_nb<KS, NMB, 8, MODE, PREC, RBFM>(s, th, tw, nb, stream);
}

template <int KS, int NMB, int MODE, int PREC>
inline hipError_t fused_form(const StageArgs &s, int th, int tw, int nb, int nw, int rbfm,
                             hipStream_t stream)
{
    if constexpr (PREC == PREC_BF16)
        if (rbfm == RBF_POLY3) return fused_nw<KS, NMB, MODE, PREC, RBF_POLY3>(s, th, tw, nb, nw, stream);
    if (rbfm == RBF_POLY) return fused_nw<KS, NMB, MODE, PREC, RBF_POLY>(s, th, tw, nb, nw, stream);
    return fused_nw<KS, NMB, MODE, PREC, RBF_HORNER>(s, th, tw, nb, nw, stream);
}

template <int KS, int NMB, int NB, int NW, int RBFM>
inline hipError_t launch_batched_t(const BatchArgs &a, hipStream_t stream)
{
    FusedLds L = fused_lds(KS, NMB, NB, a.Th, a.Tw, a.Nrbf, NW, MODE_FWD, RBFM);
    const size_t lds_bytes = (size_t)L.total * sizeof(float);
    raise_lds_limit((const void *)k_batched_stage<KS, NMB, NB, NW, RBFM>);
    if (lds_bytes > 160 * 1024) return hipErrorInvalidValue;
    if (a.persistent) {
        // counter, abort flag and flags are contiguous: [next][abort][flags...]
        const int nctl = 2 + a.items_per_stage;
        hipLaunchKernelGGL(k_clear_ints, dim3((nctl + 255) / 256), dim3(256), 0, stream, a.ctl.next, nctl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const void *kp = (const void *)k_batched_persist<KS, NMB, NB, NW, RBFM>;
        raise_lds_limit(kp);
        int per_cu = 0, dev = 0, cus = 0, khz = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kp, 64 * NW, lds_bytes) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        // the clock wall_clock64() reads (kHz)
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz < 1)
            khz = 100000;
        (void)hipGetLastError();
        long grid = (long)per_cu * cus;
        if (grid > a.ctl.n_items) grid = a.ctl.n_items;
        BatchArgs b = a;
        b.ctl.budget = (long long)(a.budget_s * 1e3 * khz);
        hipLaunchKernelGGL((k_batched_persist<KS, NMB, NB, NW, RBFM>), dim3((int)grid), dim3(64 * NW),
                           lds_bytes, stream, b);
        return hipGetLastError();
    }
    for (int t = 0; t < a.T; ++t) {
        hipLaunchKernelGGL((k_batched_stage<KS, NMB, NB, NW, RBFM>), dim3(a.items_per_stage),
                           dim3(64 * NW), lds_bytes, stream, a, t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_batched_final<KS / 2>), dim3(a.items_per_stage, (a.Th * a.Tw + 255) / 256),
                       dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <int KS, int NMB, int RBFM>
inline hipError_t batched_nb(const BatchArgs &a, int nb, int nw, hipStream_t stream)
{
    if (nw == 4) {
        switch (nb) {
        case 2: return launch_batched_t<KS, NMB, 2, 4, RBFM>(a, stream);
        case 3: return launch_batched_t<KS, NMB, 3, 4, RBFM>(a, stream);
        case 4: return launch_batched_t<KS, NMB, 4, 4, RBFM>(a, stream);
        }
    } else {
        switch (nb) {
        case 2: return launch_batched_t<KS, NMB, 2, 8, RBFM>(a, stream);
        case 3: return launch_batched_t<KS, NMB, 3, 8, RBFM>(a, stream);
        case 4: return launch_batched_t<KS, NMB, 4, 8, RBFM>(a, stream);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace tnrd
