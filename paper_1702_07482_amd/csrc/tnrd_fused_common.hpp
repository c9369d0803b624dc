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

// Operand types of the 16x16x16 MFMAs used by the mixed-precision path
// (v_mfma_f32_16x16x16_{bf16,f16}): lane l holds A[l % 16][4 (l / 16) + i]
// and B[4 (l / 16) + i][l % 16], i = 0..3; D is laid out as for 16x16x4 f32.
// Conversions round to nearest even.
enum Prec { PREC_F32 = 0, PREC_BF16 = 1, PREC_F16 = 2 };
template <int P> struct Mix;
template <> struct Mix<PREC_BF16> {
    typedef short4v V;
    static __device__ __forceinline__ short cvt(float x) { return __builtin_bit_cast(short, (__bf16)x); }
    static __device__ __forceinline__ floatx4 mfma(V a, V b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};
template <> struct Mix<PREC_F16> {
    typedef half4v V;
    static __device__ __forceinline__ _Float16 cvt(float x) { return (_Float16)x; }
    static __device__ __forceinline__ floatx4 mfma(V a, V b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mix<PREC_F32> {  // placeholder so templates instantiate; never used
    typedef short4v V;
    static __device__ __forceinline__ short cvt(float) { return 0; }
    static __device__ __forceinline__ floatx4 mfma(V, V, floatx4 c) { return c; }
};

constexpr int RBF_WIN = 5;                // Horner window half-width (11 centres)
constexpr int RBF_TERMS = 2 * RBF_WIN + 1;

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
};

// Kernel arguments of one stage (forward or input-gradient mode).
struct FusedIO {
    const float *u_prev;  // u_{t-1}
    const float *f;
    float *out;           // forward: u_t;  input gradient: g_{t-1}
    const float *u_cur;   // input gradient: u_t
    const float *g_cur;   // input gradient: g_t = dl/du_t
};

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

}  // namespace tnrd
