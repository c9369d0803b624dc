// Internal interfaces between the host API (tnrd_api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>

#include "tnrd_device.hpp"
#include "tnrd_fused_common.hpp"

// the scheduling loop of the persistent batched launch, plain C++ shared with
// its host model: every function in it becomes host and device
#pragma clang force_cuda_host_device begin
#include "tnrd_persist.hpp"
#pragma clang force_cuda_host_device end

namespace tnrd {

// Raises a kernel's dynamic LDS limit to the compute unit's 160 KB, once per
// (kernel, device), safely from any number of host threads, without
// allocating (a fixed table; past its capacity the attribute is simply set
// again, which is idempotent).  A failure shows up as a launch error of the
// kernel, so the status is cleared here.
inline void raise_lds_limit(const void *kernel)
{
    constexpr int CAP = 1024;
    static std::mutex mu;
    static const void *done_k[CAP];
    static int done_d[CAP];
    static int n_done = 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < n_done; ++i)
        if (done_k[i] == kernel && done_d[i] == dev) return;
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    if (n_done < CAP) {
        done_k[n_done] = kernel;
        done_d[n_done] = dev;
        ++n_done;
    }
}

// One forward stage over N equally sized images.  The forward runs in
// exchange form (see XTiles): stage t writes its diffusion force to slabs, and
// its reaction is applied by stage t + 1's prologue or by fused_finish.
struct StageArgs {
    const float *u_prev;  // [N][H][W] u_{t-1} (forward with pend: u_{t-2}, input of the
                          // pending reaction)
    const float *f;       // [N][H][W]
    float *u_next;        // [N][H][W] input-gradient mode: g_{t-1}; split forward and
                          // fused_finish: the stage output
    const float *u_cur;   // input-gradient mode: u_t
    const float *g_cur;   // input-gradient mode: g_t
    int N, H, W;
    int ks, Nk;
    const float *filt;    // [Nk][ks*ks] stage t
    const float *rbfw;    // [Nk][Nrbf] stage t
    const float *lam;     // &lambda[t]
    RbfGrid grid;
    float *scratch;       // implementation scratch (split: Nk response maps)
    int prec;             // tnrd_prec
    int tile_h, tile_w;   // 0 = automatic
    int waves;            // fused: waves per workgroup (4 or 8; 0 = automatic)
    int poly;             // fused kernel: the polynomial influence form may be used
    int react = 0;        // tnrd_reaction of the model
    float proj_c = 1.f;   // projected reaction: threshold c
    float *za = nullptr;  // input-gradient mode, FP32 or BF16 operands: if set, z = K u and
                          // a = K e at every pixel (za_index layout; BF16 words with BF16
                          // operands), the parameter-gradient kernels' input
    const float *prep = nullptr;  // polynomial form: this stage's block written by fused_prep
                                  // (phi table in the forward, d phi / ds in the input-gradient
                                  // mode; FP32 operands use its filter block too); required there
    // fused forward (exchange form)
    int pend = 0;                  // the previous stage's reaction is still to be applied
    const float *x_prev = nullptr; // pend / fused_finish: the previous stage's slabs
    float *x_out = nullptr;        // this stage's slabs
    float *u_keep = nullptr;       // pend: where u_{t-1} (own pixels) goes
    const float *lam_prev = nullptr;  // pend / fused_finish: lambda of the pending reaction
};

// Batched forward (device descriptors, filled on the host).
struct BatchImage {
    const float *f;
    float *u_out;
    float *u_tmp;
    float *xs[2];  // slabs of even and odd stages (tiles x (Th + 2R)(Tw + 2R) floats each)
    int H, W, tiles_x, tiles, model;
};

struct BatchModel {
    const float *filt;  // [T][Nk][KK]
    const float *rbfw;  // [T][Nk][Nrbf]
    const float *lam;   // [T]
    int react;          // tnrd_reaction
    float proj_c;       // projected reaction: threshold c
    float *prep;        // [T][BatchArgs::prep_stage] prepared stage blocks (polynomial form)
};

struct BatchItem {
    int image, tile;
};

struct BatchArgs {
    const BatchImage *imgs;
    const BatchModel *models;
    const BatchItem *items;  // one stage's items, image-major
    int items_per_stage, T, Th, Tw, Nk, Nrbf;
    int poly;  // the polynomial influence form may be used
    size_t prep_stage;  // floats per prepared stage block
    int n_models;
    FusedRbf rb;
    int persistent;   // one persistent launch for every stage (else one launch per stage)
    PersistCtl ctl;   // persistent: counter, flags, abort flag (in the workspace)
    double budget_s;  // persistent: ctl.budget in seconds (converted at launch)
};

// Runs the T stages of a batch: one persistent launch over every (stage, item)
// (a.persistent), or one launch per stage over all (image, tile) items and a
// last-reaction launch.
hipError_t batched_launch(const BatchArgs &a, int ks, int nw, hipStream_t stream);
bool batched_config_ok(int ks, int nk, int nrbf, int th, int tw, int nw);

// Prepared stage blocks of the fused kernel (FP32 operands, polynomial form):
// floats per stage, and the build of T stages' blocks (stage t at
// prep + t * fused_prep_floats) from [T][Nk][ks*ks] filters and [T][Nk][Nrbf]
// weights; deriv selects the d phi / ds table of the input-gradient mode.
size_t fused_prep_floats(int ks, int nk, int nrbf);
// form: bit 0 = tables of d phi / ds (input-gradient mode), bit 1 = the cubic
// half-interval form (the BF16 kernels, fused_prep_form)
hipError_t fused_prep(const float *filt, const float *rbfw, int T, int ks, int nk, const RbfGrid &grid,
                      int form, float *prep, hipStream_t stream);
// The table form bit of the kernels that read stage s's prepared blocks, and the
// operand format of the mixed kernels (their filter operands come prepared too).
inline int fused_prep_form(const StageArgs &s)
{
    return s.prec == PREC_BF16 ? 2 | PREP_MIXED_BF16 : s.prec == PREC_F16 ? PREP_MIXED_F16 : 0;
}
// The same for stage 0 .. T-1 of every model of a batch (into BatchModel::prep).
hipError_t batched_prep(const BatchArgs &a, int ks, int n_models, hipStream_t stream);
// Whether a stage with these options runs the fused kernel's prepared form.
bool fused_uses_prep(const StageArgs &s);

hipError_t split_stage(const StageArgs &s, hipStream_t stream);
size_t split_scratch_floats(int N, int H, int W, int Nk);

hipError_t fused_stage(const StageArgs &s, hipStream_t stream);
// The pending reaction of the last forward stage: u_next = reaction(u_prev,
// force from x_prev, f) with lam_prev, on the tiling fused_stage used.
hipError_t fused_finish(const StageArgs &s, hipStream_t stream);
// Floats of one set of slabs of a fused forward with these arguments (0 when
// the fused kernel cannot run them).
size_t fused_slab_floats(int ks, int nk, int nrbf, int N, int H, int W, int tile_h, int tile_w,
                         int waves, bool poly, int mode = MODE_FWD);
// The input gradient of a stage after fused_stage_input_grad wrote its slabs
// (x_prev): u_next = g_{t-1} from u_prev = u_{t-1}, u_cur = u_t, g_cur = g_t, f, lam.
hipError_t fused_grad_finish(const StageArgs &s, hipStream_t stream);
hipError_t fused_stage_input_grad(const StageArgs &s, hipStream_t stream);
bool fused_supported(int ks, int Nk, int nrbf, int window, int prec);
bool fused_config_ok(int ks, int Nk, int nrbf, int H, int W, int tile_h, int tile_w, int waves,
                     int mode);
size_t fused_scratch_floats(int N, int H, int W, int Nk, int prec);
bool poly_form_ok(const RbfGrid &grid, int automatic_window);

// Per-family launchers of the fused stage kernel (one translation unit each).
hipError_t fused_launch_fwd_f32(const StageArgs &s, int th, int tw, int nb, int nw, int rbfm,
                                hipStream_t stream);
hipError_t fused_launch_fwd_mixed(const StageArgs &s, int th, int tw, int nb, int nw, int rbfm,
                                  hipStream_t stream);
hipError_t fused_launch_bwd(const StageArgs &s, int th, int tw, int nb, int nw, int rbfm,
                            hipStream_t stream);
hipError_t fused_launch_final(const StageArgs &s, int th, int tw, hipStream_t stream);
hipError_t fused_launch_grad_finish(const StageArgs &s, int th, int tw, hipStream_t stream);
hipError_t batched_launch_impl(const BatchArgs &a, int ks, int nb, int nw, int rbfm,
                               hipStream_t stream);

}  // namespace tnrd
