/*
 * tnrd.h -- C ABI of libtnrd.so, the MI355X (gfx950) implementation of the
 * trained reaction-diffusion despeckling filter of Feng & Chen, "Speckle
 * Reduction with Trained Nonlinear Diffusion Filtering" (2017).
 *
 * The filter (Sec. 3.1, eq. diffusionprocessfinal) runs T stages on an
 * observed speckled amplitude image f > 0 (Sec. 2.1, eq. mul), starting from
 * u_0 = f:
 *
 *   z_i   = k_i^t * u_{t-1}                      i = 1..Nk, true 2-D convolution
 *   v_i   = phi_i^t(z_i)                         influence function
 *   ut_t  = u_{t-1} - sum_i K_i^T v_i            diffusion step (eq. diffusion)
 *   u_t   = (ut_t + sqrt(ut_t^2 + 8(1+2l)l f^2)) / (2(1+2l)),  l = lambda^t
 *                                                prox of lambda<u^2-2f^2 log u,1>
 *                                                (eqs. subproblemGpoisson, subproblemGIdiv)
 *
 * Readings fixed by this library where the paper leaves a choice open:
 *   - influence function: phi_i(z) = sum_j w_ij exp(-(z - mu_j)^2 / (2 sigma^2)),
 *     mu_j = rbf_mu0 + j * rbf_step, j = 0..Nrbf-1 (Gaussian radial basis);
 *   - k * u is a true convolution, z[p] = sum_{a,b} k[a][b] ubar[p - (a-r, b-r)],
 *     r = (ksize-1)/2, so weights trained for correlation must be rotated by 180 degrees;
 *   - ubar is the half-sample symmetric extension (-1 -> 0, -2 -> 1, n -> n-1);
 *   - K_i^T is the exact adjoint of K_i including the folded border ring;
 *   - u_0 = f.
 *
 * Conventions for every entry point:
 *   - Image and parameter pointers are DEVICE pointers owned by the caller.
 *     Images are FP32, row-major, contiguous, [N][H][W].
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null stream)
 *     and allocate no device memory: scratch space comes from the caller's
 *     workspace `ws` of `ws_bytes` bytes (size from tnrd_workspace_bytes).
 *   - Arguments are checked on the host before anything is enqueued; on error
 *     nothing is written and a negative tnrd_status is returned.
 *   - Outputs are overwritten, never accumulated.  Outputs may not alias inputs.
 *   - Calls on distinct streams with distinct workspaces are independent.
 */
#ifndef TNRD_H
#define TNRD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tnrd_status {
    TNRD_OK = 0,
    TNRD_ERR_ARG = -1,         /* NULL pointer, bad size or parameter (see each call) */
    TNRD_ERR_DOMAIN = -2,      /* validate: f <= 0 or not finite (the prox needs f > 0) */
    TNRD_ERR_WORKSPACE = -3,   /* ws_bytes smaller than tnrd_workspace_bytes() */
    TNRD_ERR_HIP = -4,         /* a HIP runtime call or launch failed */
    TNRD_ERR_UNSUPPORTED = -5, /* valid but not built: ksize not in {3,5,7}, precision, ... */
    TNRD_ERR_TIMEOUT = -7,     /* validate: a persistent batched launch gave up waiting for a
                                  neighbour tile (its results are not valid) */
    TNRD_ERR_CAPACITY = -6     /* tnrd_forward_noalloc: the call needs more scratch than its
                                  fixed TNRD_NOALLOC_SCRATCH_BYTES */
} tnrd_status;

/* Operand precision of the two filter-bank contractions (K and K^T, forward
 * and backward).  The influence function, the prox and all accumulation stay
 * FP32 in every mode.  In tnrd_backward, BF16 also keeps z = K u and a = K e
 * of the input-gradient contraction as BF16 values for the parameter
 * gradients (fastest; dK and dW then carry z's BF16 rounding, a few percent of
 * their maximum), while FP16 recomputes z on FP32 operands for them (closer
 * to FP32). */
typedef enum tnrd_prec {
    TNRD_PREC_FP32 = 0,
    TNRD_PREC_BF16 = 1,
    TNRD_PREC_FP16 = 2
} tnrd_prec;

/* Which stage implementation runs the forward. */
typedef enum tnrd_impl {
    TNRD_IMPL_AUTO = 0,   /* the fused MFMA stage kernel where it covers the model (ksize 5 or 7,
                             Nk <= 48, the automatic or the 11-centre RBF window); otherwise, with
                             FP32 operands, the split path, about 10x slower (ksize 3, Nk > 48, an
                             explicit window such as rbf_window = 0); tnrd_selected_impl reports
                             the choice */
    TNRD_IMPL_FUSED = 1,  /* one kernel per stage: K (MFMA), phi, K^T (MFMA), prox, responses kept on chip */
    TNRD_IMPL_SPLIT = 2   /* two kernels per stage on the vector ALUs: (K, phi) -> Nk response maps in
                             the workspace, then (K^T, prox).  Reference design for comparison. */
} tnrd_impl;

/* Reaction step of a stage.
 *   TNRD_REACT_PROX       the proximal step of the paper's model (Sec. 3.1, eqs. subproblemGIdiv,
 *                         diffusionprocessfinal): u_t = prox(ut_t), ut_t = u_{t-1} - sum_i K_i^T v_i
 *   TNRD_REACT_PROJECTED  the paper's comparison model (Sec. 3.1, eq. diffusion_backP): a gradient
 *                         step on the data term followed by the projection onto u >= c,
 *                         ut_t = u_{t-1} - (sum_i K_i^T v_i + (l/u_{t-1})(1 - f^2/u_{t-1}^2)),
 *                         u_t = max(ut_t, c), c = proj_c (the paper uses c = 1).  Its backward
 *                         takes the projection's derivative as 1 where ut_t > c, else 0.
 *   TNRD_REACT_L2         the framework's Gaussian-denoising reaction (Sec. 2.2.1, eq. diffusion
 *                         with G = 0 and D = (l/2)||u - f||^2): a gradient step,
 *                         u_t = u_{t-1} - (sum_i K_i^T v_i + l (u_{t-1} - f)); f may be any sign. */
typedef enum tnrd_reaction {
    TNRD_REACT_PROX = 0,
    TNRD_REACT_PROJECTED = 1,
    TNRD_REACT_L2 = 2
} tnrd_reaction;

/* Per-stage parameters Theta^t = {lambda^t, phi_i^t, k_i^t} (Sec. 2.2.2, eq. learning). */
typedef struct tnrd_model {
    int32_t T;            /* stages, >= 1 */
    int32_t Nk;           /* filters per stage, >= 1 */
    int32_t ksize;        /* odd filter side; 3, 5 and 7 are built */
    int32_t Nrbf;         /* radial basis functions per filter, 1..255 */
    int32_t L;            /* number of looks the model was trained for; 0 = any */
    float rbf_mu0;        /* centre of the first RBF */
    float rbf_step;       /* spacing of the centres, > 0 */
    float rbf_sigma;      /* standard deviation of every RBF, > 0 */
    const float *filters; /* device [T][Nk][ksize][ksize], k_i^t (convolution kernels) */
    const float *rbf_w;   /* device [T][Nk][Nrbf], w_ij^t */
    const float *lambda;  /* device [T], lambda^t >= 0 (the backward needs lambda^t > 0) */
    int32_t reaction;     /* tnrd_reaction */
    float proj_c;         /* TNRD_REACT_PROJECTED: the projection threshold c > 0 */
} tnrd_model;

typedef struct tnrd_opts {
    int32_t prec;         /* tnrd_prec */
    int32_t impl;         /* tnrd_impl */
    int32_t rbf_window;   /* -1: automatic truncation window (every dropped Gaussian term is
                                 below 1e-6 of its weight; 5 when rbf_step == rbf_sigma),
                                 0: every RBF term, w > 0: the 2w+1 centres nearest to z */
    int32_t recompute_every; /* backward checkpointing, see tnrd_forward(states) */
    int32_t validate;     /* nonzero: check f > 0 and finite on the device first (synchronises
                             `stream`; TNRD_ERR_DOMAIN on failure); with FP16 operands also that
                             f < 2^15 (the states enter the FP16 GEMMs unscaled and stay near the
                             data's range, so this keeps them below FP16's 65504;
                             TNRD_ERR_UNSUPPORTED otherwise) */
    int32_t tile_h, tile_w; /* 0 = automatic; otherwise the fused kernel's output tile */
    int32_t wg_waves;     /* fused kernel: wavefronts per workgroup, 4 or 8; 0 = automatic */
    int32_t use_graph;    /* tnrd_forward_batched: 1 (default) records the launch sequence in a HIP
                             graph once per batch signature and replays it; 0 launches directly */
    int32_t persistent;   /* tnrd_forward_batched: 1 runs every stage of every image in one
                             persistent launch (workgroups take (stage, tile) items in stage-major
                             order and wait for the tile's neighbours to finish the stage before);
                             0 (default) launches once per stage */
} tnrd_opts;

/* Fills `o` with the defaults (FP32, AUTO, automatic window, no checkpointing,
 * no validation, automatic tiles). */
void tnrd_default_opts(tnrd_opts *o);

/* Bytes of workspace a call needs for N images of H x W (which = 0: forward,
 * 1: backward).  Returns 0 on invalid arguments.  The workspace holds the
 * ping-pong image planes, the stage constants prepared once per call for the
 * fused FP32 kernel (influence coefficient tables and lane-ordered filters,
 * about 134 KB per stage for 48 filters of 7x7), and in the backward the z/a
 * export and the per-tile gradient partials.  Its contents are scratch: no
 * call reads what an earlier call left there. */
size_t tnrd_workspace_bytes(int N, int H, int W, const tnrd_model *m, const tnrd_opts *o,
                            int which);

/* Number of checkpoint slots the forward writes into `states` and the
 * backward reads: with s = max(1, recompute_every), the states u_t for
 * t = 0, s, 2s, ... < T, followed by u_T; that is T + 1 slots when s = 1. */
int tnrd_num_checkpoints(int T, int recompute_every);

/* Forward pass (Sec. 3.1, eq. diffusionprocessfinal, Fig. feedforwardCNNspeckle; with
 * m->reaction == TNRD_REACT_PROJECTED, eq. diffusion_backP).
 *   f       [N][H][W]  observed amplitude, f > 0 (the prox is positive only then)
 *   L       number of looks of f, >= 1; must equal m->L unless m->L == 0.  L does not
 *           enter the arithmetic (the paper trains one model per L).
 *   u_out   [N][H][W]  u_T
 *   states  NULL, or [tnrd_num_checkpoints(T, recompute_every)][N][H][W]: the states
 *           the backward needs (u_0 = f first, u_T last)
 * Errors: TNRD_ERR_ARG for NULL f/u_out/m/parameter pointers, N < 0, H or W < ksize,
 * even ksize, T/Nk < 1, Nrbf outside 1..255, rbf_step or rbf_sigma <= 0 or not finite,
 * L < 1 or m->L not in {0, L}, u_out == f, a reaction outside tnrd_reaction, proj_c <= 0
 * or not finite for the projected reaction; TNRD_ERR_UNSUPPORTED for ksize not in
 * {3,5,7}, a precision the chosen implementation lacks, or a tile that does not fit
 * the fused kernel's local memory; TNRD_ERR_WORKSPACE. */
int tnrd_forward(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                 float *u_out, float *states, const tnrd_opts *o,
                 void *ws, size_t ws_bytes, void *stream);

/* Backward pass (Sec. 3.2, eqs. iterstep, derv1, derv1-1, derv2, derv4).
 * Given grad_uT = dl/du_T (e.g. u_T - u_gt for the paper's loss), the states
 * written by tnrd_forward with the same recompute_every, returns, summed over
 * the N images:
 *   grad_filters [T][Nk][ksize][ksize]  dl/dk_i^t
 *   grad_rbf_w   [T][Nk][Nrbf]          dl/dw_ij^t
 *   grad_lambda  [T]                    dl/dlambda^t  (for lambda = e^beta, eq. derv5:
 *                                       dl/dbeta^t = lambda^t * dl/dlambda^t)
 *   grad_u0      NULL or [N][H][W]      dl/du_0 through the diffusion chain, with f
 *                                       held fixed in the reaction steps
 *   grad_f       NULL or [N][H][W]      dl/df in full: grad_u0 (u_0 = f) plus, at every
 *                                       stage, dl/du_t times the reaction's explicit
 *                                       derivative in f (prox: 4 l f / s with
 *                                       s = sqrt(ut^2 + 8(1+2l) l f^2); projected:
 *                                       2 l f / u_{t-1}^3 where ut_t > c, else 0; l2: l)
 * lambda^t must be > 0.  Results are deterministic: the same inputs give the
 * same bits for every recompute_every.  N = 0 needs no workspace and writes
 * zeros to the three parameter gradients.  Errors as tnrd_forward, and
 * TNRD_ERR_ARG for NULL states/grad pointers or grad_f aliasing grad_u0. */
int tnrd_backward(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                  const float *states, const float *grad_uT,
                  float *grad_filters, float *grad_rbf_w, float *grad_lambda,
                  float *grad_u0, float *grad_f, const tnrd_opts *o,
                  void *ws, size_t ws_bytes, void *stream);

/* One image of an uneven batch. */
typedef struct tnrd_image {
    const float *f;  /* device [H][W] */
    float *u_out;    /* device [H][W] */
    int32_t H, W;
    int32_t L;       /* looks; selects the model whose L matches (or one with L == 0) */
} tnrd_image;

/* Batched forward over B images of different sizes and look numbers (per-L
 * models: the paper trains one model per noise level, Sec. 4.5).  With
 * opts->persistent every stage of every tile runs in one persistent launch:
 * workgroups take (stage, tile) items in stage-major order from an atomic
 * counter and start an item once the tile's 3 x 3 neighbourhood has finished
 * the stage before (per-tile flags, device-scope release/acquire).  A wait
 * gives up after 2^21 polls or once its workgroup has run for its clock budget
 * (2 s, more for batches of over 10^5 items) and then marks an abort flag, so
 * a launch always ends; with opts->validate such a launch returns
 * TNRD_ERR_TIMEOUT.  Otherwise (default) each stage is one launch over the
 * tiles of every image.  `imgs` and `models` are HOST
 * arrays; the models must share T, Nk, ksize, Nrbf and the RBF grid; an image
 * uses the model whose L equals its own, else one with L == 0.  Workspace from
 * tnrd_batched_workspace_bytes.  With opts->use_graph (default) and a non-null
 * stream, the descriptor upload and the launches are recorded once into a HIP
 * graph per (stream, workspace, batch signature: image pointers, sizes and
 * looks; every model field, parameter pointers, reaction and proj_c included;
 * tiles) and replayed on later calls.  Host resources of that path, the one
 * exception to "allocates nothing": the first call of a new signature records
 * the graph and allocates one pinned host buffer holding the descriptors (a
 * few bytes per tile, the source of the recorded upload); both live until the
 * entry is evicted.  The cache holds 8 entries across all callers; evicting
 * the oldest waits for the stream it was recorded on.  The cache is guarded
 * by a mutex, so concurrent calls are safe.  Tiles: opts->tile_h/tile_w
 * (default 32 x 32; both must be >= ksize - 1) and opts->wg_waves.  Errors as
 * tnrd_forward, plus TNRD_ERR_ARG for an image whose L matches no model or
 * models that disagree in shape. */
size_t tnrd_batched_workspace_bytes(int B, const tnrd_image *imgs, int n_models,
                                    const tnrd_model *models, const tnrd_opts *o);
int tnrd_forward_batched(int B, const tnrd_image *imgs, int n_models, const tnrd_model *models,
                         const tnrd_opts *o, void *ws, size_t ws_bytes, void *stream);

/* Allocation-free forward, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, checks, kernels and results (bit for bit) as
 * tnrd_forward without `ws`/`ws_bytes`: the scratch tnrd_forward takes from
 * the caller's workspace comes from one fixed device array of
 * TNRD_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, which each GPU the library runs
 * on holds until the process ends.  The call allocates nothing, host or
 * device (its first call on a device looks the array's address up once).
 * The caller still passes f, u_out and states.  A call whose tnrd_workspace_bytes
 * (which = 0) exceeds the array returns TNRD_ERR_CAPACITY before anything is
 * enqueued: with the fused FP32 kernel and 48 filters of 7x7 over 8 stages
 * that is N*H*W above about 8.2 million pixels.  All calls on one GPU share
 * its array: calls that overlap in time on one GPU (two streams, or two host
 * threads) race and must be serialised by the caller; calls on different GPUs
 * are independent.  Nothing in the array needs to start at zero (the call
 * clears its own domain flag).  Errors as tnrd_forward, plus TNRD_ERR_CAPACITY,
 * and TNRD_ERR_HIP if the array's address cannot be obtained. */
#define TNRD_NOALLOC_SCRATCH_BYTES (64u << 20)
int tnrd_forward_noalloc(const float *f, int N, int H, int W, int L, const tnrd_model *m,
                         float *u_out, float *states, const tnrd_opts *o, void *stream);

/* The implementation tnrd_forward would run for model m with options o (NULL:
 * defaults): TNRD_IMPL_FUSED or TNRD_IMPL_SPLIT, or TNRD_ERR_ARG (NULL model,
 * bad ksize or sizes) or TNRD_ERR_UNSUPPORTED (no implementation covers the
 * model at o->prec).  Host-only, no device call. */
int tnrd_selected_impl(const tnrd_model *m, const tnrd_opts *o);

/* Static description of a status code. */
const char *tnrd_status_str(int status);

/* ---- Measurement aid (not part of the filter) ----------------------------
 * Throughput probes of the units the stage kernels run on, so that their rates
 * can be read against measured rather than published peaks.  Each probe runs a
 * fixed launch on `stream` and is timed with HIP events over several launches
 * after a warm-up; the call synchronises with the stream.
 *   copy_gbs              device-to-device copy of copy_bytes (read + write bytes / s)
 *   mfma_f32_tflops       v_mfma_f32_16x16x4_f32 (the FP32 filter-bank instruction)
 *   mfma_bf16_k16_tflops  v_mfma_f32_16x16x16_bf16 (the mixed-precision instruction)
 *   mfma_bf16_k32_tflops  v_mfma_f32_16x16x32_bf16
 *   valu_f32_tflops       FP32 vector FMA, unpacked (2 flop per lane)
 *   exp_per_s             hardware exp2 (v_exp_f32) results per second
 * copy_src/copy_dst: device buffers of copy_bytes each (>= 16 MiB, a multiple
 * of 16); sink: device buffer of tnrd_peaks_sink_floats() floats (overwritten
 * with throw-away values).  Returns TNRD_ERR_ARG for a NULL pointer or a bad
 * size, TNRD_ERR_HIP if a launch or event call fails. */
typedef struct tnrd_peaks {
    double copy_gbs, mfma_f32_tflops, mfma_bf16_k16_tflops, mfma_bf16_k32_tflops;
    double valu_f32_tflops, exp_per_s;
} tnrd_peaks;
size_t tnrd_peaks_sink_floats(void);
int tnrd_measure_peaks(const void *copy_src, void *copy_dst, size_t copy_bytes, float *sink,
                       tnrd_peaks *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TNRD_H */
