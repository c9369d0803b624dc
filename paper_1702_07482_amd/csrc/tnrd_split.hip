// Split (unfused) stage: two vector-ALU kernels per stage.
//
//   k_split_phi      v_i = phi_i(K_i u)  for all Nk filters -> Nk response maps in HBM
//   k_split_adj_prox u'  = prox(u - sum_i K_i^T v_i)
//
// This is the straightforward design in which every response map goes
// through HBM (4*Nk bytes written and read per pixel and stage).  It is kept
// as the comparison point for the fused kernel and as a second, independent
// GPU implementation in the tests.
#include "tnrd_device.hpp"
#include "tnrd_internal.hpp"

namespace tnrd {

constexpr int SPLIT_TILE = 16;

// grid (ceil(W/16), ceil(H/16), N); block 16x16.
template <int KS>
__global__ void __launch_bounds__(256) k_split_phi(
    const float *__restrict__ u, int H, int W,
    const float *__restrict__ filt,   // [Nk][KS*KS] of this stage
    const float *__restrict__ rbfw,   // [Nk][Nrbf] of this stage
    int Nk, RbfGrid g,
    float *__restrict__ V,            // [Nk][N][H][W]
    size_t v_filter_stride)
{
    constexpr int R = KS / 2;
    constexpr int LW = SPLIT_TILE + 2 * R;
    __shared__ float su[LW][LW + 1];

    const int n = blockIdx.z;
    const size_t img = (size_t)H * W;
    const float *un = u + n * img;
    const int ty0 = blockIdx.y * SPLIT_TILE, tx0 = blockIdx.x * SPLIT_TILE;
    const int tid = threadIdx.y * SPLIT_TILE + threadIdx.x;

    for (int i = tid; i < LW * LW; i += 256) {
        int ly = i / LW, lx = i % LW;
        int yy = reflect_clamp(ty0 - R + ly, H), xx = reflect_clamp(tx0 - R + lx, W);
        su[ly][lx] = un[(size_t)yy * W + xx];
    }
    __syncthreads();

    const int y = ty0 + threadIdx.y, x = tx0 + threadIdx.x;
    if (y >= H || x >= W) return;
    float nb[KS * KS];
#pragma unroll
    for (int a = 0; a < KS; ++a)
#pragma unroll
        for (int b = 0; b < KS; ++b)
            // ubar[p - (a-R, b-R)] sits at local (ty + R - (a-R), tx + R - (b-R))
            nb[a * KS + b] = su[threadIdx.y + 2 * R - a][threadIdx.x + 2 * R - b];

    float *vout = V + n * img + (size_t)y * W + x;
    for (int i = 0; i < Nk; ++i) {
        const float *k = filt + i * KS * KS;
        float z = 0.f;
#pragma unroll
        for (int t = 0; t < KS * KS; ++t) z = fmaf(k[t], nb[t], z);
        vout[i * v_filter_stride] = rbf_phi_direct(z, rbfw + (size_t)i * g.nrbf, g);
    }
}

// grid (ceil(W/16), ceil(H/16), N); block 16x16.
// x[p] = sum over padded q with reflect(q) = p of X[q],
// X[q] = sum_i sum_{a,b} k_i[a][b] v_i[q + (a-R, b-R)]  (v = 0 outside the image).
template <int KS>
__global__ void __launch_bounds__(256) k_split_adj_prox(
    const float *__restrict__ V, size_t v_filter_stride,
    const float *__restrict__ u, const float *__restrict__ f, int H, int W,
    const float *__restrict__ filt, int Nk, const float *__restrict__ lam_t, int react, float proj_c,
    float *__restrict__ u_next)
{
    constexpr int R = KS / 2;
    constexpr int HALO = 2 * R;                  // mirrored ring positions reach 2R out
    constexpr int LW = SPLIT_TILE + 2 * HALO;
    __shared__ float sv[LW][LW + 1];

    const int n = blockIdx.z;
    const size_t img = (size_t)H * W;
    const int ty0 = blockIdx.y * SPLIT_TILE, tx0 = blockIdx.x * SPLIT_TILE;
    const int tid = threadIdx.y * SPLIT_TILE + threadIdx.x;
    const int y = ty0 + threadIdx.y, x = tx0 + threadIdx.x;
    const bool inside = (y < H) && (x < W);

    // preimages of this pixel under the reflection, within [-R, n-1+R]
    int qy[2], qx[2], nqy = 1, nqx = 1;
    qy[0] = y;
    qx[0] = x;
    if (y < R) qy[nqy++] = -y - 1;
    else if (y >= H - R) qy[nqy++] = 2 * H - 1 - y;
    if (x < R) qx[nqx++] = -x - 1;
    else if (x >= W - R) qx[nqx++] = 2 * W - 1 - x;

    float acc = 0.f;
    for (int i = 0; i < Nk; ++i) {
        const float *vi = V + i * v_filter_stride + n * img;
        __syncthreads();
        for (int e = tid; e < LW * LW; e += 256) {
            int ly = e / LW, lx = e % LW;
            int yy = ty0 - HALO + ly, xx = tx0 - HALO + lx;
            bool ok = yy >= 0 && yy < H && xx >= 0 && xx < W;
            sv[ly][lx] = ok ? vi[(size_t)yy * W + xx] : 0.f;
        }
        __syncthreads();
        if (!inside) continue;
        const float *k = filt + i * KS * KS;
        for (int iy = 0; iy < nqy; ++iy) {
            for (int ix = 0; ix < nqx; ++ix) {
#pragma unroll
                for (int a = 0; a < KS; ++a) {
                    int ly = qy[iy] + a - R - ty0 + HALO;
                    if (ly < 0 || ly >= LW) continue;
#pragma unroll
                    for (int b = 0; b < KS; ++b) {
                        int lx = qx[ix] + b - R - tx0 + HALO;
                        if (lx < 0 || lx >= LW) continue;
                        acc = fmaf(k[a * KS + b], sv[ly][lx], acc);
                    }
                }
            }
        }
    }
    if (!inside) return;
    const size_t p = n * img + (size_t)y * W + x;
    u_next[p] = reaction_step(react, u[p], acc, f[p], lam_t[0], proj_c);
}

template <int KS>
static hipError_t split_stage_ks(const StageArgs &s, hipStream_t stream)
{
    dim3 grid((s.W + SPLIT_TILE - 1) / SPLIT_TILE, (s.H + SPLIT_TILE - 1) / SPLIT_TILE, s.N);
    dim3 block(SPLIT_TILE, SPLIT_TILE);
    size_t vstride = (size_t)s.N * s.H * s.W;
    hipLaunchKernelGGL(k_split_phi<KS>, grid, block, 0, stream, s.u_prev, s.H, s.W, s.filt,
                       s.rbfw, s.Nk, s.grid, s.scratch, vstride);
    hipLaunchKernelGGL(k_split_adj_prox<KS>, grid, block, 0, stream, s.scratch, vstride,
                       s.u_prev, s.f, s.H, s.W, s.filt, s.Nk, s.lam, s.react, s.proj_c, s.u_next);
    return hipGetLastError();
}

hipError_t split_stage(const StageArgs &s, hipStream_t stream)
{
    switch (s.ks) {
    case 3: return split_stage_ks<3>(s, stream);
    case 5: return split_stage_ks<5>(s, stream);
    case 7: return split_stage_ks<7>(s, stream);
    default: return hipErrorInvalidValue;
    }
}

size_t split_scratch_floats(int N, int H, int W, int Nk)
{
    return (size_t)Nk * N * H * W;
}

}  // namespace tnrd
