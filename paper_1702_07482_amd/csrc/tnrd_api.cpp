// Host side of libtnrd: argument checks, workspace layout and launch sequencing
// for the C ABI declared in include/tnrd.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>


#include "tnrd.h"
#include "tnrd_api_internal.hpp"
#include "tnrd_internal.hpp"

using namespace tnrd;

namespace {

constexpr size_t WS_ALIGN = 256;

size_t align_up(size_t x) { return (x + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

// Domain check of f: flag[0] |= 1 if any f <= 0 or not finite.
// flag bit 0: some f <= 0 or not finite; bit 1: some f >= fmax
__global__ void k_check_domain(const float *__restrict__ f, size_t n, float fmax, int *flag)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += stride) {
        float v = f[i];
        bad |= (!(v > 0.f) || !isfinite(v)) ? 1 : 0;
        bad |= v >= fmax ? 2 : 0;
    }
    if (bad) atomicOr(flag, bad);
}

// flag[0] = 0 (a kernel rather than a memset node, safe where callers capture graphs)
__global__ void k_clear_flag(int *flag) { flag[0] = 0; }

}  // namespace

namespace tnrd {

int check_model(const tnrd_model *m)
{
    if (!m || !m->filters || !m->rbf_w || !m->lambda) return TNRD_ERR_ARG;
    if (m->T < 1 || m->Nk < 1 || m->ksize < 1 || (m->ksize % 2) == 0) return TNRD_ERR_ARG;
    if (m->Nrbf < 1 || m->Nrbf > 255) return TNRD_ERR_ARG;
    if (!(m->rbf_step > 0.f) || !isfinite(m->rbf_step)) return TNRD_ERR_ARG;
    if (!(m->rbf_sigma > 0.f) || !isfinite(m->rbf_sigma)) return TNRD_ERR_ARG;
    if (!isfinite(m->rbf_mu0)) return TNRD_ERR_ARG;
    if (m->L < 0) return TNRD_ERR_ARG;
    if (m->reaction != TNRD_REACT_PROX && m->reaction != TNRD_REACT_PROJECTED &&
        m->reaction != TNRD_REACT_L2)
        return TNRD_ERR_ARG;
    if (m->reaction == TNRD_REACT_PROJECTED && (!(m->proj_c > 0.f) || !isfinite(m->proj_c)))
        return TNRD_ERR_ARG;
    if (m->ksize != 3 && m->ksize != 5 && m->ksize != 7) return TNRD_ERR_UNSUPPORTED;
    return TNRD_OK;
}

int check_image_args(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                     const float *u_out)
{
    int st = check_model(m);
    if (st != TNRD_OK) return st;
    if (N < 0) return TNRD_ERR_ARG;
    if (N > 0 && (!f || !u_out || f == u_out)) return TNRD_ERR_ARG;
    if (H < m->ksize || W < m->ksize) return TNRD_ERR_ARG;
    if ((size_t)H * (size_t)W > ((size_t)1 << 31)) return TNRD_ERR_ARG;
    if (L < 1 || (m->L != 0 && m->L != L)) return TNRD_ERR_ARG;
    return TNRD_OK;
}

void resolve_opts(const tnrd_opts *o, tnrd_opts *out)
{
    if (o) {
        *out = *o;
    } else {
        tnrd_default_opts(out);
    }
}

int rbf_window_for(const tnrd_model *m, int requested)
{
    if (requested == 0) return 0;
    int w = requested;
    if (requested < 0) {
        // smallest w with exp(-rho (w + 1/2)^2 / 2) < 1e-6, rho = (step / sigma)^2:
        // every dropped centre is at least w + 1/2 spacings from z, so each
        // dropped Gaussian is below 1e-6 of its weight (w = 5 for step = sigma).
        double rho = (double)m->rbf_step / m->rbf_sigma;
        rho *= rho;
        w = (int)ceil(sqrt(2.0 * 13.82 / rho) - 0.5);
        if (w < 1) w = 1;
    }
    if (2 * w + 1 >= m->Nrbf) return 0;
    return w;
}

RbfGrid make_grid(const tnrd_model *m, int window)
{
    RbfGrid g;
    g.mu0 = m->rbf_mu0;
    g.step = m->rbf_step;
    g.inv_step = 1.0f / m->rbf_step;
    g.neg_half_inv_var = (float)(-1.0 / (2.0 * (double)m->rbf_sigma * m->rbf_sigma));
    g.nrbf = m->Nrbf;
    g.window = window;
    return g;
}

// Implementation chosen for a forward with these options (TNRD_IMPL_FUSED or
// TNRD_IMPL_SPLIT), or a negative status.
int choose_impl(const tnrd_model *m, const tnrd_opts &o, int window)
{
    bool fused_ok = fused_supported(m->ksize, m->Nk, m->Nrbf, window, o.prec);
    switch (o.impl) {
    case TNRD_IMPL_AUTO:
        if (fused_ok) return TNRD_IMPL_FUSED;
        if (o.prec == TNRD_PREC_FP32) return TNRD_IMPL_SPLIT;
        return TNRD_ERR_UNSUPPORTED;
    case TNRD_IMPL_FUSED:
        return fused_ok ? TNRD_IMPL_FUSED : TNRD_ERR_UNSUPPORTED;
    case TNRD_IMPL_SPLIT:
        return o.prec == TNRD_PREC_FP32 ? TNRD_IMPL_SPLIT : TNRD_ERR_UNSUPPORTED;
    default:
        return TNRD_ERR_ARG;
    }
}

int checkpoint_slot(int t, int T, int s)
{
    if (t == T) return tnrd_num_checkpoints(T, s) - 1;
    if (t % s == 0) return t / s;
    return -1;
}

size_t prep_region_floats(const tnrd_model *m, const tnrd_opts &o, int impl, int window,
                          int stages)
{
    if (impl != TNRD_IMPL_FUSED || o.rbf_window >= 0) return 0;
    if (!poly_form_ok(make_grid(m, window), 1)) return 0;
    return (size_t)stages * fused_prep_floats(m->ksize, m->Nk, m->Nrbf);
}

size_t slab_region_floats(int N, int H, int W, const tnrd_model *m, const tnrd_opts &o, int impl,
                          int window)
{
    if (impl != TNRD_IMPL_FUSED) return 0;
    const bool poly = o.rbf_window < 0 && poly_form_ok(make_grid(m, window), 1);
    return fused_slab_floats(m->ksize, m->Nk, m->Nrbf, N, H, W, o.tile_h, o.tile_w, o.wg_waves, poly);
}

// Forward workspace: [flags 256 B][scratch][ping A][ping B][prepared stage blocks][slabs x 2]
size_t forward_ws_bytes(int N, int H, int W, const tnrd_model *m, const tnrd_opts &o, int impl)
{
    size_t img = (size_t)N * H * W;
    size_t scratch = impl == TNRD_IMPL_SPLIT ? split_scratch_floats(N, H, W, m->Nk)
                                             : fused_scratch_floats(N, H, W, m->Nk, o.prec);
    size_t bytes = WS_ALIGN + align_up(scratch * sizeof(float));
    if (m->T > 1) bytes += 2 * align_up(img * sizeof(float));
    const int window = rbf_window_for(m, o.rbf_window);
    bytes += align_up(prep_region_floats(m, o, impl, window, m->T) * sizeof(float));
    bytes += 2 * align_up(slab_region_floats(N, H, W, m, o, impl, window) * sizeof(float));
    return bytes;
}

int run_domain_check(const float *f, size_t n, int *dflag, hipStream_t stream, int prec)
{
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, stream, dflag);
    if (hipGetLastError() != hipSuccess) return TNRD_ERR_HIP;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    // FP16 operands hold u unscaled: f below 2^15 keeps the states (which stay
    // near the data's range) well inside FP16's largest value, 65504
    const float fmax = prec == TNRD_PREC_FP16 ? FP16_FMAX : INFINITY;
    hipLaunchKernelGGL(k_check_domain, dim3(blocks), dim3(256), 0, stream, f, n, fmax, dflag);
    if (hipGetLastError() != hipSuccess) return TNRD_ERR_HIP;
    int host = 0;
    if (hipMemcpyAsync(&host, dflag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return TNRD_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return TNRD_ERR_HIP;
    return (host & 1) ? TNRD_ERR_DOMAIN : (host & 2) ? TNRD_ERR_UNSUPPORTED : TNRD_OK;
}

// Runs stages [t_begin, t_end) (0-based stage index t computes u_{t+1})
// starting from u_start = u_{t_begin}; the output of stage t goes to dst(t).
// The fused forward runs in exchange form: the launch of stage t applies
// stage t-1's reaction in its prologue (writing u_t to its destination) and
// leaves its own diffusion force in slabs[t mod 2]; a final launch applies
// the last reaction.
int run_stages(const float *f, int N, int H, int W, const tnrd_model *m, const tnrd_opts &o,
               int impl, int window, int t_begin, int t_end, const float *u_start,
               float *const *dst, float *scratch, float *prep, float *const *slabs,
               hipStream_t stream)
{
    StageArgs s;
    s.u_cur = nullptr;
    s.g_cur = nullptr;
    s.f = f;
    s.N = N;
    s.H = H;
    s.W = W;
    s.ks = m->ksize;
    s.Nk = m->Nk;
    s.grid = make_grid(m, window);
    s.scratch = scratch;
    s.prec = o.prec;
    s.tile_h = o.tile_h;
    s.tile_w = o.tile_w;
    s.waves = o.wg_waves;
    s.poly = o.rbf_window < 0;
    s.react = m->reaction;
    s.proj_c = m->proj_c;
    const float *cur = u_start;
    const size_t kk = (size_t)m->ksize * m->ksize;
    // the fused FP32 form reads its stage constants ready-made: one launch
    // prepares the blocks of all stages of this call
    const bool use_prep = impl == TNRD_IMPL_FUSED && fused_uses_prep(s) && t_end > t_begin;
    const size_t prep_sf = use_prep ? fused_prep_floats(m->ksize, m->Nk, m->Nrbf) : 0;
    if (use_prep) {
        if (!prep) return TNRD_ERR_WORKSPACE;
        if (fused_prep(m->filters + (size_t)t_begin * m->Nk * kk, m->rbf_w + (size_t)t_begin * m->Nk * m->Nrbf,
                       t_end - t_begin, m->ksize, m->Nk, s.grid, fused_prep_form(s), prep, stream) !=
            hipSuccess)
            return TNRD_ERR_HIP;
    }
    if (impl == TNRD_IMPL_SPLIT) {
        for (int t = t_begin; t < t_end; ++t) {
            s.u_prev = cur;
            s.u_next = dst[t - t_begin];
            s.filt = m->filters + (size_t)t * m->Nk * kk;
            s.rbfw = m->rbf_w + (size_t)t * m->Nk * m->Nrbf;
            s.lam = m->lambda + t;
            if (split_stage(s, stream) != hipSuccess) return TNRD_ERR_HIP;
            cur = s.u_next;
        }
        return TNRD_OK;
    }
    if (t_end <= t_begin) return TNRD_OK;
    if (!slabs || !slabs[0] || !slabs[1]) return TNRD_ERR_WORKSPACE;
    // plane holding u_{t_begin + i}
    auto state = [&](int i) -> const float * { return i == 0 ? u_start : dst[i - 1]; };
    for (int t = t_begin; t < t_end; ++t) {
        const int i = t - t_begin;
        s.pend = i > 0;
        s.u_prev = s.pend ? state(i - 1) : u_start;
        s.u_keep = s.pend ? dst[i - 1] : nullptr;
        s.x_prev = s.pend ? slabs[(i - 1) & 1] : nullptr;
        s.lam_prev = s.pend ? m->lambda + t - 1 : nullptr;
        s.x_out = slabs[i & 1];
        s.u_next = nullptr;
        s.filt = m->filters + (size_t)t * m->Nk * kk;
        s.rbfw = m->rbf_w + (size_t)t * m->Nk * m->Nrbf;
        s.lam = m->lambda + t;
        s.prep = use_prep ? prep + (size_t)i * prep_sf : nullptr;
        if (fused_stage(s, stream) != hipSuccess) return TNRD_ERR_HIP;
    }
    const int n = t_end - t_begin;
    s.pend = 1;
    s.u_prev = state(n - 1);
    s.x_prev = slabs[(n - 1) & 1];
    s.lam_prev = m->lambda + t_end - 1;
    s.u_next = dst[n - 1];
    if (fused_finish(s, stream) != hipSuccess) return TNRD_ERR_HIP;
    return TNRD_OK;
}

int plan_forward(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                 const float *u_out, const float *states, const tnrd_opts &oo, ForwardPlan *p)
{
    int st = check_image_args(f, N, H, W, L, m, u_out);
    if (st != TNRD_OK) return st;
    if (oo.prec < TNRD_PREC_FP32 || oo.prec > TNRD_PREC_FP16) return TNRD_ERR_ARG;
    if (states && (states == f || states == u_out)) return TNRD_ERR_ARG;
    p->window = rbf_window_for(m, oo.rbf_window);
    p->impl = choose_impl(m, oo, p->window);
    if (p->impl < 0) return p->impl;
    p->ws_bytes = 0;
    if (N == 0) return TNRD_OK;
    if (p->impl == TNRD_IMPL_FUSED &&
        !fused_config_ok(m->ksize, m->Nk, m->Nrbf, H, W, oo.tile_h, oo.tile_w, oo.wg_waves, 0))
        return TNRD_ERR_UNSUPPORTED;
    p->ws_bytes = forward_ws_bytes(N, H, W, m, oo, p->impl);
    return TNRD_OK;
}

int run_forward(const float *f, int N, int H, int W, const tnrd_model *m, float *u_out,
                float *states, const tnrd_opts &oo, const ForwardPlan &p, void *ws,
                hipStream_t stream)
{
    const int impl = p.impl, window = p.window;
    char *base = (char *)ws;
    int *dflag = (int *)base;
    size_t img = (size_t)N * H * W;
    size_t scratch_floats = impl == TNRD_IMPL_SPLIT ? split_scratch_floats(N, H, W, m->Nk)
                                                    : fused_scratch_floats(N, H, W, m->Nk, oo.prec);
    float *scratch = (float *)(base + WS_ALIGN);
    float *ping[2] = {nullptr, nullptr};
    char *after = base + WS_ALIGN + align_up(scratch_floats * sizeof(float));
    if (m->T > 1) {
        ping[0] = (float *)after;
        ping[1] = (float *)((char *)ping[0] + align_up(img * sizeof(float)));
        after += 2 * align_up(img * sizeof(float));
    }
    const size_t prep_floats = prep_region_floats(m, oo, impl, window, m->T);
    float *prep = prep_floats ? (float *)after : nullptr;
    after += align_up(prep_floats * sizeof(float));
    const size_t slab_floats = slab_region_floats(N, H, W, m, oo, impl, window);
    float *slabs[2] = {nullptr, nullptr};
    if (slab_floats) {
        slabs[0] = (float *)after;
        slabs[1] = (float *)(after + align_up(slab_floats * sizeof(float)));
    }

    if (oo.validate) {
        int st = run_domain_check(f, img, dflag, stream, oo.prec);
        if (st != TNRD_OK) return st;
    }

    const int T = m->T;
    const int s = oo.recompute_every < 1 ? 1 : oo.recompute_every;
    if (states) {
        if (hipMemcpyAsync(states, f, img * sizeof(float), hipMemcpyDeviceToDevice, stream) !=
            hipSuccess)
            return TNRD_ERR_HIP;
    }
    // destinations: stage t (0-based) writes u_{t+1}: u_out at the last stage, its
    // checkpoint slot if it has one, else the ping-pong plane the input is not in.
    // Stages run in chunks of a fixed number (one preparation launch per chunk),
    // so the destination list lives on the stack.
    constexpr int CHUNK = 64;
    float *dsts[CHUNK];
    const float *cur = f;
    for (int t0 = 0; t0 < T; t0 += CHUNK) {
        const int t1 = T < t0 + CHUNK ? T : t0 + CHUNK;
        const float *start = cur;
        for (int t = t0; t < t1; ++t) {
            int slot = states ? checkpoint_slot(t + 1, T, s) : -1;
            float *d;
            if (t + 1 == T) d = u_out;
            else if (slot >= 0) d = states + (size_t)slot * img;
            else d = (cur == ping[0]) ? ping[1] : ping[0];
            dsts[t - t0] = d;
            cur = d;
        }
        int st = run_stages(f, N, H, W, m, oo, impl, window, t0, t1, start, dsts, scratch, prep, slabs,
                            stream);
        if (st != TNRD_OK) return st;
    }
    if (states) {
        float *last = states + (size_t)(tnrd_num_checkpoints(T, s) - 1) * img;
        if (hipMemcpyAsync(last, u_out, img * sizeof(float), hipMemcpyDeviceToDevice, stream) !=
            hipSuccess)
            return TNRD_ERR_HIP;
    }
    return TNRD_OK;
}

}  // namespace tnrd

extern "C" {

void tnrd_default_opts(tnrd_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->prec = TNRD_PREC_FP32;
    o->impl = TNRD_IMPL_AUTO;
    o->rbf_window = -1;
    o->recompute_every = 1;
    o->validate = 0;
    o->use_graph = 1;
    o->persistent = 0;
}

int tnrd_num_checkpoints(int T, int recompute_every)
{
    if (T < 1) return 0;
    int s = recompute_every < 1 ? 1 : recompute_every;
    return (T + s - 1) / s + 1;
}

size_t tnrd_workspace_bytes(int N, int H, int W, const tnrd_model *m, const tnrd_opts *o,
                            int which)
{
    tnrd_opts oo;
    resolve_opts(o, &oo);
    if (check_model(m) != TNRD_OK || N < 0 || H < m->ksize || W < m->ksize) return 0;
    int window = rbf_window_for(m, oo.rbf_window);
    if (which == 0) {
        int impl = choose_impl(m, oo, window);
        if (impl < 0) return 0;
        return forward_ws_bytes(N, H, W, m, oo, impl);
    }
    if (which == 1) return backward_ws_bytes(N, H, W, m, oo, window);
    return 0;
}

int tnrd_forward(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                 float *u_out, float *states, const tnrd_opts *o,
                 void *ws, size_t ws_bytes, void *stream_)
{
    tnrd_opts oo;
    resolve_opts(o, &oo);
    ForwardPlan p;
    int st = plan_forward(f, N, H, W, L, m, u_out, states, oo, &p);
    if (st != TNRD_OK) return st;
    if (N == 0) return TNRD_OK;
    if (!ws || ws_bytes < p.ws_bytes) return TNRD_ERR_WORKSPACE;
    return run_forward(f, N, H, W, m, u_out, states, oo, p, ws, (hipStream_t)stream_);
}

int tnrd_selected_impl(const tnrd_model *m, const tnrd_opts *o)
{
    if (!m || m->T < 1 || m->Nk < 1 || m->Nrbf < 1 || (m->ksize != 3 && m->ksize != 5 && m->ksize != 7))
        return TNRD_ERR_ARG;
    tnrd_opts oo;
    resolve_opts(o, &oo);
    return choose_impl(m, oo, rbf_window_for(m, oo.rbf_window));
}

const char *tnrd_status_str(int status)
{
    switch (status) {
    case TNRD_OK: return "ok";
    case TNRD_ERR_ARG: return "invalid argument";
    case TNRD_ERR_DOMAIN: return "input outside the domain (f must be > 0 and finite)";
    case TNRD_ERR_WORKSPACE: return "workspace missing or too small";
    case TNRD_ERR_HIP: return "HIP runtime error";
    case TNRD_ERR_UNSUPPORTED: return "unsupported configuration";
    case TNRD_ERR_TIMEOUT: return "a persistent batched launch gave up waiting (results not valid)";
    case TNRD_ERR_CAPACITY:
        return "problem larger than the fixed scratch of tnrd_forward_noalloc (TNRD_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
    }
}

}  // extern "C"
