// Device helpers shared by the stage kernels of libtnrd (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnrd {

// Half-sample symmetric reflection into [0, n) for -n <= q < 2n:
// -1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2 (the border extension of K).
__device__ __forceinline__ int reflect(int q, int n)
{
    q = q < 0 ? -q - 1 : q;
    return q >= n ? 2 * n - 1 - q : q;
}

// Reflect, then clamp: a safe index for any q (used where the value is
// discarded anyway, e.g. responses of positions outside the image).
__device__ __forceinline__ int reflect_clamp(int q, int n)
{
    q = reflect(q, n);
    return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

// RBF grid constants, precomputed on the host for the Gaussian influence
// function phi(z) = sum_j w_j exp(-(z - mu_j)^2 / (2 sigma^2)), mu_j = mu0 + j*step.
struct RbfGrid {
    float mu0;       // first centre
    float inv_step;  // 1 / step
    float neg_half_inv_var;  // -1 / (2 sigma^2)
    float step;
    int nrbf;
    int window;      // 0: all terms; w > 0: the 2w+1 centres nearest to z
};

// Direct windowed evaluation: one exp per term.
__device__ __forceinline__ float rbf_phi_direct(float z, const float *__restrict__ w,
                                                const RbfGrid &g)
{
    int lo = 0, hi = g.nrbf - 1;
    if (g.window > 0) {
        int j0 = __float2int_rn((z - g.mu0) * g.inv_step);  // saturating; NaN -> 0
        j0 = min(max(j0, -g.window), g.nrbf - 1 + g.window);
        lo = max(lo, j0 - g.window);
        hi = min(hi, j0 + g.window);
    }
    float acc = 0.f;
    for (int j = lo; j <= hi; ++j) {
        float d = z - (g.mu0 + (float)j * g.step);
        acc = fmaf(w[j], __expf(d * d * g.neg_half_inv_var), acc);
    }
    return acc;
}

// phi and phi' together (phi'(z) = sum_j w_j * (-(z - mu_j)/sigma^2) * G_j(z)).
__device__ __forceinline__ void rbf_phi_dphi_direct(float z, const float *__restrict__ w,
                                                    const RbfGrid &g, float &phi, float &dphi)
{
    int lo = 0, hi = g.nrbf - 1;
    if (g.window > 0) {
        int j0 = __float2int_rn((z - g.mu0) * g.inv_step);  // saturating; NaN -> 0
        j0 = min(max(j0, -g.window), g.nrbf - 1 + g.window);
        lo = max(lo, j0 - g.window);
        hi = min(hi, j0 + g.window);
    }
    float a = 0.f, b = 0.f;
    for (int j = lo; j <= hi; ++j) {
        float d = z - (g.mu0 + (float)j * g.step);
        float G = w[j] * __expf(d * d * g.neg_half_inv_var);
        a += G;
        b = fmaf(G, d, b);
    }
    phi = a;
    dphi = b * (2.f * g.neg_half_inv_var);  // -(z - mu)/sigma^2 = 2 * d * (-1/(2 sigma^2))
}

// Closed-form prox of lambda <u^2 - 2 f^2 log u, 1>:
//   u = (ut + s) / (2(1+2l)),  s = sqrt(ut^2 + 8(1+2l) l f^2).
// For ut < 0 the same root is evaluated as c / ((s - ut) 2(1+2l)), c = 8(1+2l) l f^2,
// which avoids the cancellation in ut + s ((ut + s)(s - ut) = c).
// Correctly rounded square root and divisions: the states feed the lambda
// gradient, a sum over all pixels with heavy cancellation, which 1-ulp
// hardware approximations here move by several 1e-4 relative.
__device__ __forceinline__ float prox(float ut, float f, float lam)
{
    float c1 = 1.f + 2.f * lam;
    float c = 8.f * c1 * lam * f * f;
    float s = sqrtf(fmaf(ut, ut, c));
    float num = ut >= 0.f ? (ut + s) : c / (s - ut);
    return num / (2.f * c1);
}

// Reaction of the projected variant (eq. diffusion_backP), psi(u) =
// (l/u)(1 - f^2/u^2), evaluated as l (u - f)(u + f) / u^3 (no cancellation in
// 1 - f^2/u^2 when u is close to f), and its partial derivatives
// d psi/du = l (3 f^2 - u^2) / u^4, d psi/dl = (u - f)(u + f) / u^3,
// d psi/df = -2 l f / u^3.
__device__ __forceinline__ float proj_psi(float u, float f, float lam)
{
    return lam * ((u - f) * (u + f)) / (u * u * u);
}
__device__ __forceinline__ float proj_psi_du(float u, float f, float lam)
{
    const float u2 = u * u;
    return lam * fmaf(3.f * f, f, -u2) / (u2 * u2);
}
__device__ __forceinline__ float proj_psi_dlam(float u, float f)
{
    return ((u - f) * (u + f)) / (u * u * u);
}
__device__ __forceinline__ float proj_psi_df(float u, float f, float lam)
{
    return -2.f * lam * f / (u * u * u);
}

// Reaction step of a stage from u_{t-1} and the diffusion force x = sum_i K_i^T v_i:
// react 0: u_t = prox(u_{t-1} - x)                      (eq. diffusionprocessfinal)
// react 1: u_t = max(u_{t-1} - (x + psi(u_{t-1})), c)   (eq. diffusion_backP)
// react 2: u_t = u_{t-1} - (x + l (u_{t-1} - f))         (eq. diffusion, quadratic data term)
__device__ __forceinline__ float reaction_step(int react, float u_prev, float x, float f, float lam,
                                               float c)
{
    if (react == 1) return fmaxf(u_prev - (x + proj_psi(u_prev, f, lam)), c);
    if (react == 2) return u_prev - fmaf(lam, u_prev - f, x);
    return prox(u_prev - x, f, lam);
}

// Derivative of the reaction step in ut_t written with its output u_t (prox:
// y = u^2 / ((1+2l) u^2 + 2 l f^2), the closed form of eq. derv2 by the prox's
// optimality condition; projected: 1 where u_t > c, else 0; quadratic: 1).
__device__ __forceinline__ float react_dut(int react, float u_cur, float f, float lam, float c)
{
    if (react == 1) return u_cur > c ? 1.f : 0.f;
    if (react == 2) return 1.f;
    const float u2 = u_cur * u_cur;
    return u2 / fmaf(1.f + 2.f * lam, u2, 2.f * lam * f * f);
}

// dl/du_{t-1} of a stage from g = dl/du_t and the diffusion force x = sum_i K_i^T
// (phi_i'(z_i) a_i) of e = y g (transposed eq. derv1-1): g_{t-1} = e - x, and the
// projected reaction adds -(d psi/du)(u_{t-1}) e, the quadratic one -l e.
__device__ __forceinline__ float grad_step(int react, float u_prev, float u_cur, float f, float g, float x,
                                           float lam, float c)
{
    const float e = react_dut(react, u_cur, f, lam, c) * g;
    float gv = e - x;
    if (react == 1) gv -= proj_psi_du(u_prev, f, lam) * e;
    else if (react == 2) gv -= lam * e;
    return gv;
}

}  // namespace tnrd
