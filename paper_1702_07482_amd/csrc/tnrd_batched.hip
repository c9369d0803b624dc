// tnrd_forward_batched: a batch of images with different sizes and look
// numbers, one launch per stage over every (image, tile) item, with the
// per-image model chosen by L.  The descriptor upload and the T stage launches
// are recorded once per batch signature into a HIP graph and replayed on
// later calls.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "tnrd.h"
#include "tnrd_api_internal.hpp"
#include "tnrd_internal.hpp"

using namespace tnrd;

namespace {

constexpr size_t AL = 256;
size_t al(size_t x) { return (x + AL - 1) / AL * AL; }

struct BatchPlan {
    int th, tw, nw;
    int ntiles;                  // items per stage
    int n_models;
    size_t prep_stage;           // floats per prepared stage block (0: none)
    size_t off_imgs, off_models, off_items, off_tmp, off_prep, off_ctl, desc_bytes, total;
    std::vector<size_t> tmp_off; // per image, from the workspace base
    std::vector<size_t> xs_off;  // per image: its two slab regions, from the workspace base
    std::vector<size_t> xs_len;  // per image: floats of one slab region
};

int resolve_model(const tnrd_image &im, int n_models, const tnrd_model *models)
{
    int any = -1;
    for (int k = 0; k < n_models; ++k) {
        if (models[k].L == im.L) return k;
        if (models[k].L == 0 && any < 0) any = k;
    }
    return any;
}

int check_batch(int B, const tnrd_image *imgs, int n_models, const tnrd_model *models,
                const tnrd_opts &o, BatchPlan &plan, std::vector<int> &model_of)
{
    if (B < 0 || n_models < 1 || !models) return TNRD_ERR_ARG;
    if (B > 0 && !imgs) return TNRD_ERR_ARG;
    for (int k = 0; k < n_models; ++k) {
        int st = check_model(&models[k]);
        if (st != TNRD_OK) return st;
        const tnrd_model &a = models[0], &b = models[k];
        if (a.T != b.T || a.Nk != b.Nk || a.ksize != b.ksize || a.Nrbf != b.Nrbf ||
            a.rbf_mu0 != b.rbf_mu0 || a.rbf_step != b.rbf_step || a.rbf_sigma != b.rbf_sigma)
            return TNRD_ERR_ARG;
    }
    const tnrd_model &m = models[0];
    if (o.prec != TNRD_PREC_FP32) return o.prec > TNRD_PREC_FP16 || o.prec < 0 ? TNRD_ERR_ARG
                                                                                : TNRD_ERR_UNSUPPORTED;
    const int window = rbf_window_for(&m, o.rbf_window);
    if (!fused_supported(m.ksize, m.Nk, m.Nrbf, window, o.prec)) return TNRD_ERR_UNSUPPORTED;
    plan.th = o.tile_h > 0 ? o.tile_h : 32;
    plan.tw = o.tile_w > 0 ? o.tile_w : 32;
    plan.nw = o.wg_waves == 4 ? 4 : 8;
    if (!batched_config_ok(m.ksize, m.Nk, m.Nrbf, plan.th, plan.tw, plan.nw))
        return TNRD_ERR_UNSUPPORTED;
    model_of.assign(B, -1);
    plan.ntiles = 0;
    size_t tmp_total = 0;
    plan.tmp_off.assign(B, 0);
    for (int b = 0; b < B; ++b) {
        const tnrd_image &im = imgs[b];
        if (!im.f || !im.u_out || im.f == im.u_out) return TNRD_ERR_ARG;
        if (im.H < m.ksize || im.W < m.ksize || im.L < 1) return TNRD_ERR_ARG;
        if ((size_t)im.H * im.W > ((size_t)1 << 31)) return TNRD_ERR_ARG;
        model_of[b] = resolve_model(im, n_models, models);
        if (model_of[b] < 0) return TNRD_ERR_ARG;
        const int tx = (im.W + plan.tw - 1) / plan.tw, ty = (im.H + plan.th - 1) / plan.th;
        plan.ntiles += tx * ty;
    }
    size_t off = AL;  // domain-check flag
    plan.off_imgs = off;
    off += al((size_t)B * sizeof(BatchImage));
    plan.off_models = off;
    off += al((size_t)n_models * sizeof(BatchModel));
    plan.off_items = off;
    off += al((size_t)plan.ntiles * sizeof(BatchItem));
    plan.desc_bytes = off - plan.off_imgs;
    plan.off_tmp = off;
    const int R = m.ksize / 2;
    plan.xs_off.assign(B, 0);
    plan.xs_len.assign(B, 0);
    for (int b = 0; b < B; ++b) {
        plan.tmp_off[b] = off;
        off += al((size_t)imgs[b].H * imgs[b].W * sizeof(float));
        tmp_total += (size_t)imgs[b].H * imgs[b].W;
        // the image's slabs: one per tile of (Th + 2R) x (Tw + 2R) floats, two sets
        const size_t tiles = (size_t)((imgs[b].W + plan.tw - 1) / plan.tw) *
                             ((imgs[b].H + plan.th - 1) / plan.th);
        plan.xs_len[b] = tiles * (size_t)(plan.th + 2 * R) * (plan.tw + 2 * R);
        plan.xs_off[b] = off;
        off += 2 * al(plan.xs_len[b] * sizeof(float));
    }
    (void)tmp_total;
    // prepared stage blocks of the polynomial form, [model][T][prep_stage]
    plan.n_models = n_models;
    plan.prep_stage = o.rbf_window < 0 && poly_form_ok(make_grid(&m, window), 1)
                          ? fused_prep_floats(m.ksize, m.Nk, m.Nrbf)
                          : 0;
    plan.off_prep = off;
    off += al((size_t)n_models * m.T * plan.prep_stage * sizeof(float));
    // persistent launch: [item counter][abort flag][stages finished per item]
    plan.off_ctl = off;
    off += al((size_t)(2 + plan.ntiles) * sizeof(int));
    plan.total = off;
    return TNRD_OK;
}

// Host images of the device descriptors (imgs | models | items), laid out as
// in the workspace starting at off_imgs.
void build_descriptors(int B, const tnrd_image *imgs, int n_models, const tnrd_model *models,
                       const BatchPlan &plan, const std::vector<int> &model_of, char *ws,
                       unsigned char *host)
{
    memset(host, 0, plan.desc_bytes);
    BatchImage *di = (BatchImage *)(host + (plan.off_imgs - plan.off_imgs));
    BatchModel *dm = (BatchModel *)(host + (plan.off_models - plan.off_imgs));
    BatchItem *dt = (BatchItem *)(host + (plan.off_items - plan.off_imgs));
    int flag = 0;
    for (int b = 0; b < B; ++b) {
        const tnrd_image &im = imgs[b];
        const int tx = (im.W + plan.tw - 1) / plan.tw, ty = (im.H + plan.th - 1) / plan.th;
        di[b].f = im.f;
        di[b].u_out = im.u_out;
        di[b].u_tmp = (float *)(ws + plan.tmp_off[b]);
        di[b].xs[0] = (float *)(ws + plan.xs_off[b]);
        di[b].xs[1] = (float *)(ws + plan.xs_off[b] + al(plan.xs_len[b] * sizeof(float)));
        di[b].H = im.H;
        di[b].W = im.W;
        di[b].tiles_x = tx;
        di[b].tiles = tx * ty;
        di[b].model = model_of[b];
        for (int k = 0; k < tx * ty; ++k) dt[flag + k] = BatchItem{b, k};
        flag += tx * ty;
    }
    for (int k = 0; k < n_models; ++k) {
        dm[k].filt = models[k].filters;
        dm[k].rbfw = models[k].rbf_w;
        dm[k].lam = models[k].lambda;
        dm[k].react = models[k].reaction;
        dm[k].proj_c = models[k].proj_c;
        dm[k].prep = plan.prep_stage
                         ? (float *)(ws + plan.off_prep) + (size_t)k * models[k].T * plan.prep_stage
                         : nullptr;
    }
}

// Polls a persistent launch's wait makes before it gives up (about 1 s of polling)
constexpr int PERSIST_SPIN_LIMIT = 1 << 21;
// Seconds after its start at which a persistent workgroup's waits give up: 2 s,
// or 20 us per item for batches of over 10^5 items (the whole forward runs at
// well under 1 us per item)
inline double persist_budget_s(int n_items) { return n_items > 100000 ? 2e-5 * n_items : 2.0; }

BatchArgs make_args(const BatchPlan &plan, const tnrd_model &m, int window, int automatic_window,
                    int persistent, char *ws)
{
    BatchArgs a;
    a.imgs = (const BatchImage *)(ws + plan.off_imgs);
    a.models = (const BatchModel *)(ws + plan.off_models);
    a.items = (const BatchItem *)(ws + plan.off_items);
    a.items_per_stage = plan.ntiles;
    a.T = m.T;
    a.Th = plan.th;
    a.Tw = plan.tw;
    a.Nk = m.Nk;
    a.Nrbf = m.Nrbf;
    const RbfGrid grid = make_grid(&m, window);
    a.rb = make_fused_rbf(grid);
    a.poly = poly_form_ok(grid, automatic_window) && plan.prep_stage > 0;
    a.prep_stage = plan.prep_stage;
    a.n_models = plan.n_models;
    a.persistent = persistent;
    int *ctl = (int *)(ws + plan.off_ctl);
    a.ctl.next = ctl;
    a.ctl.abort_flag = ctl + 1;
    a.ctl.flags = ctl + 2;
    a.ctl.per_stage = plan.ntiles;
    a.ctl.n_items = (m.T + 1) * plan.ntiles;
    a.ctl.spin_limit = PERSIST_SPIN_LIMIT;
    a.ctl.budget = 0;  // set in ticks of the device clock at launch
    a.budget_s = persist_budget_s(a.ctl.n_items);
    return a;
}

// ---- graph cache: one recorded graph per (stream, workspace, batch signature)
struct GraphEntry {
    hipStream_t stream;
    std::vector<unsigned long long> sig;
    hipGraphExec_t exec;
    unsigned char *host_desc;  // pinned source of the recorded descriptor upload
};
std::mutex g_mu;
std::vector<GraphEntry> g_cache;
constexpr size_t G_CACHE_MAX = 8;

std::vector<unsigned long long> signature(int B, const tnrd_image *imgs, int n_models,
                                          const tnrd_model *models, const tnrd_opts &o,
                                          void *ws, size_t ws_bytes)
{
    std::vector<unsigned long long> s;
    auto P = [&](const void *p) { s.push_back((unsigned long long)(uintptr_t)p); };
    auto I = [&](long long v) { s.push_back((unsigned long long)v); };
    P(ws);
    I((long long)ws_bytes);
    I(B);
    I(n_models);
    I(o.tile_h);
    I(o.tile_w);
    I(o.wg_waves);
    I(o.rbf_window);
    I(o.persistent);
    for (int b = 0; b < B; ++b) {
        P(imgs[b].f);
        P(imgs[b].u_out);
        I(imgs[b].H);
        I(imgs[b].W);
        I(imgs[b].L);
    }
    for (int k = 0; k < n_models; ++k) {
        const tnrd_model &m = models[k];
        P(m.filters);
        P(m.rbf_w);
        P(m.lambda);
        I(m.T);
        I(m.Nk);
        I(m.ksize);
        I(m.Nrbf);
        I(m.L);
        I(m.reaction);
        // every float field by its bits (the recorded descriptor copy carries
        // reaction and proj_c, so a replay must not serve a model that differs there)
        float fl[4] = {m.rbf_mu0, m.rbf_step, m.rbf_sigma, m.proj_c};
        unsigned int u[4];
        memcpy(u, fl, sizeof(u));
        I(u[0]);
        I(u[1]);
        I(u[2]);
        I(u[3]);
    }
    return s;
}

}  // namespace

extern "C" size_t tnrd_batched_workspace_bytes(int B, const tnrd_image *imgs, int n_models,
                                               const tnrd_model *models, const tnrd_opts *o)
{
    tnrd_opts oo;
    resolve_opts(o, &oo);
    BatchPlan plan;
    std::vector<int> model_of;
    if (check_batch(B, imgs, n_models, models, oo, plan, model_of) != TNRD_OK) return 0;
    return plan.total;
}

extern "C" int tnrd_forward_batched(int B, const tnrd_image *imgs, int n_models,
                                    const tnrd_model *models, const tnrd_opts *o, void *ws,
                                    size_t ws_bytes, void *stream_)
{
    tnrd_opts oo;
    resolve_opts(o, &oo);
    BatchPlan plan;
    std::vector<int> model_of;
    int st = check_batch(B, imgs, n_models, models, oo, plan, model_of);
    if (st != TNRD_OK) return st;
    if (B == 0) return TNRD_OK;
    if (!ws || ws_bytes < plan.total) return TNRD_ERR_WORKSPACE;
    hipStream_t stream = (hipStream_t)stream_;
    const tnrd_model &m = models[0];
    const int window = rbf_window_for(&m, oo.rbf_window);
    char *wsb = (char *)ws;
    if (oo.validate) {
        for (int b = 0; b < B; ++b) {
            st = run_domain_check(imgs[b].f, (size_t)imgs[b].H * imgs[b].W, (int *)ws, stream, oo.prec);
            if (st != TNRD_OK) return st;
        }
    }
    const BatchArgs a = make_args(plan, m, window, oo.rbf_window < 0, oo.persistent != 0, wsb);
    const bool graph = oo.use_graph != 0 && stream != nullptr;
    // validate: a persistent launch whose waits gave up is reported (a direct
    // launch only; graph replays are not checked)
    auto check_abort = [&]() -> int {
        if (!oo.validate || !a.persistent) return TNRD_OK;
        int host = 0;
        if (hipMemcpyAsync(&host, a.ctl.abort_flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return TNRD_ERR_HIP;
        return host ? TNRD_ERR_TIMEOUT : TNRD_OK;
    };

    if (!graph) {
        std::vector<unsigned char> host(plan.desc_bytes);
        build_descriptors(B, imgs, n_models, models, plan, model_of, wsb, host.data());
        if (hipMemcpyAsync(wsb + plan.off_imgs, host.data(), plan.desc_bytes, hipMemcpyHostToDevice,
                           stream) != hipSuccess)
            return TNRD_ERR_HIP;
        if (batched_launch(a, m.ksize, plan.nw, stream) != hipSuccess)
            return TNRD_ERR_HIP;
        // the pageable source must outlive the copy
        if (hipStreamSynchronize(stream) != hipSuccess) return TNRD_ERR_HIP;
        st = check_abort();
        if (st != TNRD_OK) return st;
    } else {
        std::lock_guard<std::mutex> lock(g_mu);
        std::vector<unsigned long long> sig = signature(B, imgs, n_models, models, oo, ws, ws_bytes);
        GraphEntry *hit = nullptr;
        for (auto &e : g_cache)
            if (e.stream == stream && e.sig == sig) hit = &e;
        if (!hit) {
            if (g_cache.size() >= G_CACHE_MAX) {
                GraphEntry &old = g_cache.front();
                (void)hipStreamSynchronize(old.stream);
                (void)hipGraphExecDestroy(old.exec);
                (void)hipHostFree(old.host_desc);
                g_cache.erase(g_cache.begin());
            }
            GraphEntry e;
            e.stream = stream;
            e.sig = sig;
            e.exec = nullptr;
            if (hipHostMalloc((void **)&e.host_desc, plan.desc_bytes, hipHostMallocDefault) != hipSuccess)
                return TNRD_ERR_HIP;
            build_descriptors(B, imgs, n_models, models, plan, model_of, wsb, e.host_desc);
            // first launch outside the graph settles the kernels' one-time setup
            // (LDS limit), which must not happen during capture
            if (hipMemcpyAsync(wsb + plan.off_imgs, e.host_desc, plan.desc_bytes,
                               hipMemcpyHostToDevice, stream) != hipSuccess ||
                batched_launch(a, m.ksize, plan.nw, stream) != hipSuccess) {
                (void)hipHostFree(e.host_desc);
                return TNRD_ERR_HIP;
            }
            st = check_abort();
            if (st != TNRD_OK) {
                (void)hipStreamSynchronize(stream);
                (void)hipHostFree(e.host_desc);
                return st;
            }
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                (void)hipHostFree(e.host_desc);
                return TNRD_ERR_HIP;
            }
            hipError_t e1 = hipMemcpyAsync(wsb + plan.off_imgs, e.host_desc, plan.desc_bytes,
                                           hipMemcpyHostToDevice, stream);
            hipError_t e2 = e1 == hipSuccess
                                ? batched_launch(a, m.ksize, plan.nw, stream)
                                : e1;
            hipError_t e3 = hipStreamEndCapture(stream, &g);
            if (e2 != hipSuccess || e3 != hipSuccess ||
                hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0) != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                (void)hipStreamSynchronize(stream);
                (void)hipHostFree(e.host_desc);
                return TNRD_ERR_HIP;
            }
            (void)hipGraphDestroy(g);
            g_cache.push_back(e);
            // this call's result was already produced by the direct launch above
        } else {
            if (hipGraphLaunch(hit->exec, stream) != hipSuccess) return TNRD_ERR_HIP;
        }
    }
    return TNRD_OK;
}
