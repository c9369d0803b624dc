// Host-side helpers shared by the forward, backward and batched entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "tnrd.h"
#include "tnrd_device.hpp"

namespace tnrd {

int check_model(const tnrd_model *m);
int check_image_args(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                     const float *u_out);
void resolve_opts(const tnrd_opts *o, tnrd_opts *out);
int rbf_window_for(const tnrd_model *m, int requested);
RbfGrid make_grid(const tnrd_model *m, int window);
int choose_impl(const tnrd_model *m, const tnrd_opts &o, int window);
int checkpoint_slot(int t, int T, int s);
size_t forward_ws_bytes(int N, int H, int W, const tnrd_model *m, const tnrd_opts &o, int impl);
// Largest f the FP16 operands accept (validate: TNRD_ERR_UNSUPPORTED from it on).
constexpr float FP16_FMAX = 32768.f;
// validate: TNRD_ERR_DOMAIN if some f <= 0 or is not finite, TNRD_ERR_UNSUPPORTED
// if prec is FP16 and some f >= FP16_FMAX; synchronises `stream`.
int run_domain_check(const float *f, size_t n, int *dflag, hipStream_t stream, int prec);
// Runs stages [t_begin, t_end) of m.  prep: room for the prepared blocks of
// t_end - t_begin stages (prep_region_floats), used by the fused FP32 form.
// slabs: two regions of slab_region_floats each (the fused forward's exchange buffers).
int run_stages(const float *f, int N, int H, int W, const tnrd_model *m, const tnrd_opts &o,
               int impl, int window, int t_begin, int t_end, const float *u_start,
               float *const *dst, float *scratch, float *prep, float *const *slabs,
               hipStream_t stream);
// Floats of one set of slabs of the fused forward (0 for the split path).
size_t slab_region_floats(int N, int H, int W, const tnrd_model *m, const tnrd_opts &o, int impl,
                          int window);
// Floats of the prepared blocks of `stages` stages of m (0 where the fused
// kernel builds its constants itself).
size_t prep_region_floats(const tnrd_model *m, const tnrd_opts &o, int impl, int window,
                          int stages);

// Argument checks and plan of a forward call (tnrd_forward): the stage
// implementation, the influence window and the workspace bytes it needs (0 for
// N = 0).  Returns TNRD_OK or the status tnrd_forward returns for these arguments.
struct ForwardPlan {
    int impl, window;
    size_t ws_bytes;
};
int plan_forward(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                 const float *u_out, const float *states, const tnrd_opts &oo, ForwardPlan *p);
// Runs a planned forward (N > 0) on a workspace of at least p.ws_bytes.  Allocates
// nothing, host or device.
int run_forward(const float *f, int N, int H, int W, const tnrd_model *m, float *u_out,
                float *states, const tnrd_opts &oo, const ForwardPlan &p, void *ws,
                hipStream_t stream);

size_t backward_ws_bytes(int N, int H, int W, const tnrd_model *m, const tnrd_opts &o,
                         int window);

}  // namespace tnrd
