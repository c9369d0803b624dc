// Per-call preparation of the fused stage kernel's stage constants
// (polynomial influence form).
//
// Every workgroup of a stage launch needs the same two things, which depend
// only on the stage's parameters, not on the image:
//   - the coefficient table of the piecewise-polynomial influence function
//     (phi in the forward, d phi / ds in the input-gradient mode), built from
//     the RBF weights (the polynomial form of the fused kernel);
//   - the filter bank in the order the MFMA lanes hold it (GEMM1's A operand
//     a1[mb][s] and the K^T GEMM's a2[mb2][s] per lane).
// k_prep_stage builds both once per stage into global memory, in the exact
// layout the fused kernel copies: per stage,
//   [16 NMB filters][tf_pitch]      table (fused_lds().t_size floats)
//   [ceil(NOPS / 4)][64 lanes][4]   operands, quad k4 of lane l
// so a workgroup's prologue is a straight copy (table into LDS, FP32 operands
// into registers) instead of ~1200 VALU instructions per wave.  The BF16/FP16
// kernels copy the table and stage their own operands.
#include "tnrd_fused_tile.hpp"

namespace tnrd {

template <int KS, int NMB>
struct PrepGeo {
    using G = Geo<KS>;
    using G2 = Geo2<KS>;
    static constexpr int NA1 = NMB * G::KS1;      // GEMM1 operands per lane
    static constexpr int KS2 = 4 * NMB;           // GEMM2 k-steps
    static constexpr int NOPS = NA1 + G2::MB2 * KS2;
    static constexpr int NQ = (NOPS + 3) / 4;     // operand quads per lane
};

// Floats of one stage's prepared block (table + operands), rounded to 64.
template <int KS, int NMB>
static size_t prep_stage_floats_t(int nrbf)
{
    const FusedLds L = fused_lds(KS, NMB, 2, KS, KS, nrbf, 8, MODE_FWD, RBF_POLY);
    const size_t n = (size_t)L.t_size + (size_t)PrepGeo<KS, NMB>::NQ * 256;
    return (n + 63) & ~(size_t)63;
}

// Thread idx of stage t: table interval (fi, q) for idx < 16 NMB ni (its 8
// coefficients, plus the row's zero padding), then operand quad (k4, lane).
// form: bit 0 = d phi / ds instead of phi, bit 1 = the cubic half-interval
// form (two cubics per interval, floats 8 q .. 8 q + 7 of the row); the
// operand part holds the FP32 operands, or with PREP_MIXED_BF16/F16 the
// mixed kernels' BF16/FP16 ones.
template <int KS, int NMB>
__device__ void prep_stage_body(const float *__restrict__ filt, const float *__restrict__ rbfw, int Nk,
                                int Nrbf, const FusedRbf &rb, int form, float *__restrict__ out,
                                int idx)
{
    const int deriv = form & 1;
    const bool cubic = (form & 2) != 0;
    using G = Geo<KS>;
    using G2 = Geo2<KS>;
    using P = PrepGeo<KS, NMB>;
    constexpr int KK = G::KK, KS1 = G::KS1, HB = G2::HB, NREG = G2::NREG;
    const FusedLds L = fused_lds(KS, NMB, 2, KS, KS, Nrbf, 8, MODE_FWD, RBF_POLY);
    const int ni = L.ni, ni_used = poly_intervals(Nrbf);
    const int ntab = 16 * NMB * ni;
    if (idx < ntab) {
        // c_k = M[k][0] w_j0 + sum_{m>=1} M[k][m] (w_{j0+m} +- w_{j0-m}), j0 = q - 1 - W,
        // weights outside [0, Nrbf) taken as 0
        const int fi = idx / ni, q = idx - fi * ni;
        if (cubic) {
            // c_k of half h = sum_m P3[h][k][m + MW] w_{j0+m}, j0 = q - 1 - W
            floatx4 c[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
            if (fi < Nk && q >= 1 && q <= ni_used - 2) {
                const int j0 = q - 1 - RBF_WIN;
#pragma unroll
                for (int mi = 0; mi < POLY3_NM; ++mi) {
                    const int jj = j0 + mi - POLY_MW;
                    const float w = (jj >= 0 && jj < Nrbf) ? rbfw[fi * Nrbf + jj] : 0.f;
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int k = 0; k < POLY3_NC; ++k)
                            c[h][k] = fmaf(deriv ? rb.p3d[h][k][mi] : rb.p3[h][k][mi], w, c[h][k]);
                }
            }
            float *dst = out + fi * L.tf_pitch + 8 * q;
            *reinterpret_cast<floatx4 *>(dst) = c[0];
            *reinterpret_cast<floatx4 *>(dst + 4) = c[1];
            if (4 * q < L.tf_pitch - POLY_NC * ni)
                *reinterpret_cast<floatx4 *>(out + fi * L.tf_pitch + POLY_NC * ni + 4 * q) =
                    floatx4{0.f, 0.f, 0.f, 0.f};
            return;
        }
        const float(*pm)[POLY_MW + 1] = deriv ? rb.pmd : rb.pm;
        const int par = deriv ? 1 : 0;  // parity of k whose terms are sums
        float c[POLY_NC];
#pragma unroll
        for (int k = 0; k < POLY_NC; ++k) c[k] = 0.f;
        if (fi < Nk && q >= 1 && q <= ni_used - 2) {
            const int j0 = q - 1 - RBF_WIN;
            auto w = [&](int jj) { return (jj >= 0 && jj < Nrbf) ? rbfw[fi * Nrbf + jj] : 0.f; };
            const float w0 = w(j0);
#pragma unroll
            for (int k = 0; k < POLY_NC; ++k)
                if ((k & 1) == par) c[k] = pm[k][0] * w0;
#pragma unroll
            for (int m = 1; m <= POLY_MW; ++m) {
                const float wp = w(j0 + m), wn = w(j0 - m);
                const float sum = wp + wn, dif = wp - wn;
#pragma unroll
                for (int k = 0; k < POLY_NC; ++k) c[k] = fmaf(pm[k][m], ((k & 1) == par) ? sum : dif, c[k]);
            }
        }
        float *dst = out + fi * L.tf_pitch + 4 * q;
        *reinterpret_cast<floatx4 *>(dst) = floatx4{c[0], c[1], c[2], c[3]};
        *reinterpret_cast<floatx4 *>(dst + 4 * ni) = floatx4{c[4], c[5], c[6], c[7]};
        // zero padding at the end of the row (a multiple of 4 floats)
        if (4 * q < L.tf_pitch - POLY_NC * ni)
            *reinterpret_cast<floatx4 *>(out + fi * L.tf_pitch + POLY_NC * ni + 4 * q) =
                floatx4{0.f, 0.f, 0.f, 0.f};
        return;
    }
    idx -= ntab;
    if (idx >= P::NQ * 64) return;
    const int k4 = idx >> 6, lane = idx & 63;
    const int g = lane >> 4, j = lane & 15;
    if (form & (PREP_MIXED_BF16 | PREP_MIXED_F16)) {
        // BF16/FP16 operands of the mixed kernels, lane-ordered: operand v = 2 k4 + h
        // of lane l (four 16-bit words, element i in word i): GEMM1's a1m[mb][s]
        // first (v < NMB KSH), then the K^T GEMM's a2m[mb2][mb]
        constexpr int KSH = (KK + 15) / 16, NV = NMB * KSH + G2::MB2 * NMB;
        if (KS != 7 || 2 * k4 >= NV) return;
        unsigned wd[4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int v = 2 * k4 + h;
            float x[4] = {0.f, 0.f, 0.f, 0.f};
            if (v < NMB * KSH) {
                // the 7 x 7 taps in a 7 x 8 grid with a pad column in front: slot
                // 16 s + 4 g + i = tap row 2 s + (g >> 1), column 4 (g & 1) + i - 1
                const int mb = v / KSH, s = v - mb * KSH;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int fi = 16 * mb + j, ta = 2 * s + (g >> 1), tb = 4 * (g & 1) + i - 1;
                    if (fi < Nk && ta < KS && tb >= 0 && tb < KS) x[i] = filt[fi * KK + ta * KS + tb];
                }
            } else if (v < NV) {
                // slot row j of block mb2 (as below), k-row g of k-step mb: filter 16 mb + 4 g + i
                const int vv = v - NMB * KSH, mb2 = vv / NMB, mb = vv - mb2 * NMB;
                const int Rr = 4 * mb2 + (j & 3);
                const int tb = Rr < NREG ? Rr / HB : KS;
                const int ta = 4 * (Rr % HB) + (j >> 2);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int fi = 16 * mb + 4 * g + i;
                    if (fi < Nk && ta < KS && tb < KS) x[i] = filt[fi * KK + ta * KS + tb];
                }
            }
            unsigned short hw[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                hw[i] = (form & PREP_MIXED_BF16) ? __builtin_bit_cast(unsigned short, (__bf16)x[i])
                                                  : __builtin_bit_cast(unsigned short, (_Float16)x[i]);
            wd[2 * h] = (unsigned)hw[0] | ((unsigned)hw[1] << 16);
            wd[2 * h + 1] = (unsigned)hw[2] | ((unsigned)hw[3] << 16);
        }
        *reinterpret_cast<uint4 *>(out + L.t_size + 4 * (64 * k4 + lane)) = uint4{wd[0], wd[1], wd[2], wd[3]};
        return;
    }
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * k4 + i;
        float x = 0.f;
        if (k < P::NA1) {
            // GEMM1 A operand: lane (g, j) holds filter 16 mb + j, tap 4 s + g
            const int mb = k / KS1, s = k - mb * KS1;
            const int fi = 16 * mb + j, t = 4 * s + g;
            if (fi < Nk && t < KK) x = filt[fi * KK + t];
        } else if (k < P::NOPS) {
            // K^T GEMM A operand: slot row j of block mb2 is register R' = 4 mb2 + (j & 3)
            // in lane group j >> 2 (tap column R' / HB, tap row 4 (R' % HB) + (j >> 2));
            // k-row g of k-step s is filter 16 (s >> 2) + 4 g + (s & 3)
            const int kk = k - P::NA1;
            const int mb2 = kk / P::KS2, s = kk - mb2 * P::KS2;
            const int Rr = 4 * mb2 + (j & 3);
            const int tb = Rr < NREG ? Rr / HB : KS;
            const int ta = 4 * (Rr % HB) + (j >> 2);
            const int fi = 16 * (s >> 2) + 4 * g + (s & 3);
            if (fi < Nk && ta < KS && tb < KS) x = filt[fi * KK + ta * KS + tb];
        }
        v[i] = x;
    }
    *reinterpret_cast<floatx4 *>(out + L.t_size + 4 * (64 * k4 + lane)) = floatx4{v[0], v[1], v[2], v[3]};
}

template <int KS, int NMB>
__global__ void __launch_bounds__(256) k_prep_stage(const float *filt, const float *rbfw, int Nk,
                                                    int Nrbf, FusedRbf rb, int form, float *prep,
                                                    size_t stage_floats)
{
    const int t = blockIdx.y;
    prep_stage_body<KS, NMB>(filt + (size_t)t * Nk * KS * KS, rbfw + (size_t)t * Nk * Nrbf, Nk, Nrbf,
                             rb, form, prep + (size_t)t * stage_floats,
                             blockIdx.x * blockDim.x + threadIdx.x);
}

// Batched forward: stage t of every model of the batch (descriptors in device memory).
template <int KS, int NMB>
__global__ void __launch_bounds__(256) k_prep_batched(BatchArgs a)
{
    const int t = blockIdx.y;
    const BatchModel md = a.models[blockIdx.z];
    prep_stage_body<KS, NMB>(md.filt + (size_t)t * a.Nk * KS * KS, md.rbfw + (size_t)t * a.Nk * a.Nrbf,
                             a.Nk, a.Nrbf, a.rb, 0, md.prep + (size_t)t * a.prep_stage,
                             blockIdx.x * blockDim.x + threadIdx.x);
}

template <int KS, int NMB>
static int prep_threads(int)
{
    return 16 * NMB * POLY_NI + PrepGeo<KS, NMB>::NQ * 64;
}

static int prep_nmb(int nk) { return (nk + 15) / 16 <= 2 ? 2 : 3; }

size_t fused_prep_floats(int ks, int nk, int nrbf)
{
    const int nmb = prep_nmb(nk);
    if (ks == 7) return nmb == 2 ? prep_stage_floats_t<7, 2>(nrbf) : prep_stage_floats_t<7, 3>(nrbf);
    if (ks == 5) return nmb == 2 ? prep_stage_floats_t<5, 2>(nrbf) : prep_stage_floats_t<5, 3>(nrbf);
    return 0;
}

hipError_t fused_prep(const float *filt, const float *rbfw, int T, int ks, int nk, const RbfGrid &grid,
                      int form, float *prep, hipStream_t stream)
{
    if (T <= 0) return hipSuccess;
    const int nmb = prep_nmb(nk);
    const size_t sf = fused_prep_floats(ks, nk, grid.nrbf);
    const FusedRbf rb = make_fused_rbf(grid);
    auto go = [&](auto kern, int threads) {
        dim3 gridd((threads + 255) / 256, T);
        hipLaunchKernelGGL(kern, gridd, dim3(256), 0, stream, filt, rbfw, nk, grid.nrbf, rb, form,
                           prep, sf);
        return hipGetLastError();
    };
    if (ks == 7)
        return nmb == 2 ? go(k_prep_stage<7, 2>, prep_threads<7, 2>(grid.nrbf))
                        : go(k_prep_stage<7, 3>, prep_threads<7, 3>(grid.nrbf));
    if (ks == 5)
        return nmb == 2 ? go(k_prep_stage<5, 2>, prep_threads<5, 2>(grid.nrbf))
                        : go(k_prep_stage<5, 3>, prep_threads<5, 3>(grid.nrbf));
    return hipErrorInvalidValue;
}

hipError_t batched_prep(const BatchArgs &a, int ks, int n_models, hipStream_t stream)
{
    if (a.T <= 0 || n_models <= 0) return hipSuccess;
    const int nmb = prep_nmb(a.Nk);
    auto go = [&](auto kern, int threads) {
        dim3 gridd((threads + 255) / 256, a.T, n_models);
        hipLaunchKernelGGL(kern, gridd, dim3(256), 0, stream, a);
        return hipGetLastError();
    };
    if (ks == 7)
        return nmb == 2 ? go(k_prep_batched<7, 2>, prep_threads<7, 2>(a.Nrbf))
                        : go(k_prep_batched<7, 3>, prep_threads<7, 3>(a.Nrbf));
    if (ks == 5)
        return nmb == 2 ? go(k_prep_batched<5, 2>, prep_threads<5, 2>(a.Nrbf))
                        : go(k_prep_batched<5, 3>, prep_threads<5, 3>(a.Nrbf));
    return hipErrorInvalidValue;
}

}  // namespace tnrd
