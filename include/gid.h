/*
 * gid.h -- C ABI of libgid, an MI355X (gfx950) solver for the global-illumination
 * decomposition of videos of Meka et al., "Real-Time Global Illumination
 * Decomposition of Videos".
 *
 * Problem (Sec. 4, eq. imageformation): every RGB frame I is factored as
 *     I(x) = R(x) * sum_{k=0..K} b_k T_k(x),   b_0 = (1,1,1),
 * into a reflectance layer R, a direct-illumination layer T_0, one indirect layer
 * T_k per base colour b_k, and K refined base colours.  The solver minimises the
 * energy of Sec. 6 (data + reflectance priors + illumination priors, l1 terms by
 * IRLS, Sec. 6.4) with the alternating scheme of Sec. 7.1: a Gauss-Newton step on
 * the per-pixel layers whose normal equations get a fixed number of Jacobi-PCG
 * iterations, then a Gauss-Newton step on the base colours whose 3K x 3K normal
 * equations are summed over all pixels.
 *
 * Conventions shared by every call
 *  - Every call returns gid_status; nothing throws across the ABI.
 *  - Device pointers are HIP device memory of the device current at gid_create.
 *    The caller owns every buffer it passes; the library owns its workspace,
 *    allocated by gid_create from (width, height, K) and freed by gid_destroy.
 *    Solve calls allocate nothing.
 *  - Layout: planes of width*height float32 in row-major order (row pitch =
 *    width), planes back to back.  A frame is 3 planes (R, G, B; linear RGB).
 *    Layers are K+4 planes: log-reflectance is optimised internally, the output
 *    planes are R_r, R_g, R_b (linear reflectance), T_0, T_1 .. T_K.
 *    Cluster ids are width*height uint8 in [0, K): id j names base colour b_{j+1}.
 *  - Work is enqueued on the HIP stream given at gid_create, in stream order.
 *    Host outputs of a solve (base colours, statistics) are valid after
 *    gid_synchronize.
 *  - On an argument error nothing is enqueued and the context is unchanged.
 *  - One context per host thread; a context is bound to one device.
 */
#ifndef GID_H
#define GID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gid_ctx gid_ctx;

typedef enum {
    GID_OK = 0,
    GID_ERR_INVALID_ARG = 1,
    GID_ERR_OUT_OF_MEMORY = 2,
    GID_ERR_HIP = 3,
    GID_ERR_NUMERIC = 4,      /* non-finite energy or input */
    GID_ERR_STATE = 5,        /* call out of order (e.g. no frame loaded) */
    GID_ERR_UNSUPPORTED = 6
} gid_status;

/* Energy weights of Sec. 8 ("Parameters"): data 5000, clustering 200,
 * reflectance sparsity 20 with exponent p = 1, consistency 10, monochromaticity 10,
 * indirect sparsity 3, smoothness 3, non-negativity 1000, base-colour intensity
 * regulariser 10 and chromaticity regulariser 100. */
typedef struct {
    float data, cluster, r_sparsity, p, r_consistency, monochrome,
          i_sparsity, smoothness, non_neg, ir, cr;
} gid_lambdas;

enum { GID_REFINE_OFF = 0, GID_REFINE_FIRST_FRAME = 1, GID_REFINE_EVERY_STEP = 2 };
enum { GID_CR_CHROMA = 0, GID_CR_LITERAL = 1 };
enum { GID_BSTEP_PER_PIXEL = 0, GID_BSTEP_SUM = 1 };

typedef struct {
    uint32_t struct_size;      /* sizeof(gid_params), set by gid_default_params */
    int32_t K;                 /* number of base colours, 1..16 */
    gid_lambdas lambda;
    float eps_nonneg;          /* 0.002, non-negativity reweighting (Sec. 6.4.1) */
    float eps_irls;            /* 0.002, guard of the l1/l_p IRLS weights */
    float retinex_k;           /* 50, soft-Retinex weight 1 - exp(-50 dC) (Sec. 6.2) */
    double chroma_gate;        /* 0.1, temporal pair gate on |C_t(x) - C_{t-1}(y)|_2 */
    double chroma_floor;       /* 1e-6, chromaticity is white below this intensity */
    int32_t gn_iters;          /* outer iterations per frame (G) */
    int32_t pcg_iters;         /* PCG iterations per layer step (P); the paper uses 16 */
    int32_t refine_mode;       /* GID_REFINE_*; default every step */
    int32_t temporal;          /* 1: consistency prior against the previous frame */
    int32_t cr_mode;           /* GID_CR_* */
    int32_t record_energy;     /* 1: evaluate E after every half-step (extra passes) */
    int32_t use_graph;         /* 1: replay the per-frame schedule as a hipGraph */
    int32_t bstep_scale;       /* GID_BSTEP_*: data sum of the base-colour refinement energy
                                  (Sec. 6.3, eq. basecolorrefinement) divided by the pixel
                                  count (default) or the printed pixel sum */
    int32_t spatial_pairs;     /* 1: spatial pairs of the consistency prior (Sec. 6.1): every
                                  pixel tied to a seeded random half of the edges to its eight
                                  neighbours, each active when the two chromaticities are closer
                                  than chroma_gate, weight lambda.r_consistency; 0 (default) off */
    uint32_t spatial_seed;     /* seed of that sampling (SplitMix64 of (seed << 32) | (4 i + d)) */
} gid_params;

#define GID_MAX_HALF_STEPS 128
#define GID_NUM_TERMS 8        /* data, cluster, rsparsity, rconsist, mono, isparsity, smooth, nonneg */

typedef struct {
    double energy_final;                        /* E of Sec. 6 at the frame's final state, FP64 */
    double energy_terms[GID_NUM_TERMS];         /* its terms */
    double energy_half[GID_MAX_HALF_STEPS];     /* E after each half-step (record_energy) */
    double pcg_rz_last[64];                     /* <r, z> after the last PCG iteration of each GN step */
    int32_t n_half;                             /* entries of energy_half */
    int32_t gn_done;                            /* outer iterations run */
    int32_t pcg_breakdowns;                     /* PCG stopped early by a breakdown guard */
    int32_t bstep_rejected;                     /* base-colour steps rejected by a guard */
    int32_t frame_index;                        /* 0 for the first frame of the clip */
    int32_t warm_start_learned;                 /* 1 network start taken, 0 previous frame kept,
                                                   -1 not evaluated (no network, or first frame) */
    double energy_start_previous;               /* E at the previous frame's result (judge), else NaN */
    double energy_start_learned;                /* E at the network's prediction (judge), else NaN */
} gid_frame_stats;

/* Fill *out with the paper's parameters for K base colours (Sec. 8) and the
 * schedule defaults G = 3, P = 8, refinement every step, temporal prior on.
 * Errors: GID_ERR_INVALID_ARG for K outside 1..16 or out == NULL. */
gid_status gid_default_params(int32_t K, gid_params *out);

/* Create a solver context for frames of width x height (each >= 2) and K base
 * colours, enqueuing on hip_stream (a hipStream_t; NULL = the null stream).
 * Allocates the whole workspace.  Errors: GID_ERR_INVALID_ARG (bad params or
 * size), GID_ERR_OUT_OF_MEMORY, GID_ERR_HIP. */
gid_status gid_create(const gid_params *params, int32_t width, int32_t height,
                      void *hip_stream, gid_ctx **out);

/* Free the context and its workspace (waits for its stream first). NULL is a no-op. */
gid_status gid_destroy(gid_ctx *ctx);

/* Set the initial base-colour estimate b_k^init (K x 3 linear RGB, host memory,
 * FP64, every component > 0) and start a new clip: the next solve is a first frame
 * (Sec. 5.1 initialisation, no temporal prior).  Errors: GID_ERR_INVALID_ARG. */
gid_status gid_set_base_colors(gid_ctx *ctx, const double *rgb_Kx3_host);

/* Start a new clip with the current initial colours (as after gid_set_base_colors). */
gid_status gid_reset_clip(gid_ctx *ctx);

/* Decompose one frame (Sec. 7.1 schedule).
 *   frame_dev       3 planes float32 (device), read during the call's stream work
 *   cluster_ids_dev width*height uint8 (device), values in [0, K); NULL assigns every
 *                   pixel to the current base colour of nearest chromaticity (squared
 *                   L2 in FP64, ties to the lowest index), the rule of Sec. 5.1 against
 *                   the refined colours, for the frames after the clustered first one
 *   layers_dev      K+4 planes float32 (device) written: R_r, R_g, R_b, T_0..T_K; may be NULL
 *   base_colors_host K x 3 double written after gid_synchronize; may be NULL
 *   stats           filled after gid_synchronize; may be NULL
 * The first frame of a clip starts from r = ln b_id, T_0 = clip(|I|/|R|, 0, 4),
 * T_k = 0.01; later frames start from the previous frame's result and, with
 * params.temporal, add the consistency prior against it.
 * A frame is pending from this call until gid_synchronize; a second frame (or
 * gid_load_frame) before that returns GID_ERR_STATE, so every frame's status
 * reaches the caller and a rejected first frame never seeds the next one.
 * Errors: GID_ERR_INVALID_ARG (NULL frame), GID_ERR_STATE (no base
 * colours set, or a frame pending), GID_ERR_HIP. */
gid_status gid_decompose_frame(gid_ctx *ctx, const float *frame_dev, const uint8_t *cluster_ids_dev,
                               float *layers_dev, double *base_colors_host, gid_frame_stats *stats);

/* Wait for the context's stream; completes pending host outputs.  In
 * energy-target mode (gid_set_energy_target) with checks starting before the
 * last outer iteration, a pending frame's iterations after its first check and
 * its output pass are enqueued here, on the context's stream, once the device's
 * flags show the frame has not met its target; a frame that has met it goes
 * straight to its output pass.  Returns GID_ERR_NUMERIC if the last frame's
 * final energy is not finite. */
gid_status gid_synchronize(gid_ctx *ctx);

/* Energy-target continuation (used by the learned warm start's matched-energy
 * runs; not part of the paper's fixed schedule of Sec. 7.1).  With target > 0
 * every following frame runs up to max_gn (1..64) outer iterations instead of
 * params.gn_iters and evaluates E of Sec. 6 after each one; once E <= target the
 * frame's remaining iterations are skipped: those after the first check are not
 * enqueued at all (gid_synchronize decides from the device's flags), later ones
 * return on the device.  gid_frame_stats.gn_done then reports the iterations run and
 * energy_half their energies (n_half = gn_done); energy_final is the energy after
 * the last iteration run.  Call it between frames: target applies to every
 * following frame until changed; target <= 0 restores the fixed schedule.
 * Errors: GID_ERR_INVALID_ARG (NaN target, max_gn outside 1..64),
 * GID_ERR_STATE (a frame is pending). */
gid_status gid_set_energy_target(gid_ctx *ctx, double target, int32_t max_gn);

/* In energy-target mode, evaluate and check the energy only after outer
 * iterations first_gn, first_gn + 1, ... (and always after the last; default 1),
 * for callers that know no frame meets its target earlier: the frame runs at
 * least first_gn outer iterations and saves the earlier evaluations; the
 * energy_half entries of unchecked iterations are NaN.  Applies to every
 * following frame.  Errors: GID_ERR_INVALID_ARG (first_gn outside 1..64),
 * GID_ERR_STATE (a frame is pending). */
gid_status gid_set_energy_check_from(gid_ctx *ctx, int32_t first_gn);

/* ---- single-step access (each step of the schedule on the current frame) ----
 * These run one step of the hot path on the frame loaded by gid_load_frame and
 * the state set by gid_set_state, so that each step can be checked on its own. */

/* Load a frame without solving: per-frame precompute (chromaticity, soft-Retinex
 * weight Sec. 6.2, temporal pairs against the previous frame when params.temporal
 * and a previous frame exists).  Initialises the state for a first frame. */
gid_status gid_load_frame(gid_ctx *ctx, const float *frame_dev, const uint8_t *cluster_ids_dev);

/* Overwrite the unknowns: u_dev = K+4 planes (r_0, r_1, r_2 = ln R, T_0..T_K,
 * device) and b (K x 3 doubles, host, may be NULL to keep the current colours). */
gid_status gid_set_state(gid_ctx *ctx, const float *u_dev, const double *b_host);

/* Continue a clip from an external decomposition: frame_prev_dev is the
 * previous frame (3 planes, device) and r_prev_dev its final log-reflectance
 * (3 planes, device).  The next frame is solved as a continuation (temporal
 * prior against these when params.temporal), starting from the state set by
 * gid_set_state.  Errors: GID_ERR_INVALID_ARG (NULL), GID_ERR_STATE (no colours). */
gid_status gid_set_prev_frame(gid_ctx *ctx, const float *frame_prev_dev, const float *r_prev_dev);

/* Copy out the unknowns (same layout as gid_set_state); b_host may be NULL.
 * Synchronous. */
gid_status gid_get_state(gid_ctx *ctx, float *u_dev, double *b_host);

/* E of Sec. 6 and its GID_NUM_TERMS terms at the current state, FP64. Synchronous. */
gid_status gid_eval_energy(gid_ctx *ctx, double *energy_out, double *terms_out);

/* Gauss-Newton right-hand side g = -J^T F and Jacobi diagonal diag(J^T J) of the
 * IRLS surrogate linearised at the current state (K+4 planes each, device). */
gid_status gid_eval_rhs(gid_ctx *ctx, float *g_dev, float *diag_dev);

/* q = J^T J p for the surrogate linearised at the current state (device planes). */
gid_status gid_apply_normal(gid_ctx *ctx, const float *p_dev, float *q_dev);

/* One layer step: PCG on the normal equations, then u += delta.  *rz_out (host,
 * may be NULL) gets the final <r, z>.  Synchronous. */
gid_status gid_layer_step(gid_ctx *ctx, double *rz_out);

/* Base-colour step sums at the current state (Sec. 7.1): A[c][k][l] =
 * lam_d sum_x R_c^2 T_k T_l and h[c][k] = lam_d sum_x R_c T_k (I_c - R_c S_c),
 * FP64, host arrays of 3*K*K and 3*K doubles.  Synchronous. */
gid_status gid_bstep_sums(gid_ctx *ctx, double *A_host, double *h_host);

/* One base-colour step (sums + small FP64 solve + update).  *accepted (host,
 * may be NULL) is 0 when a guard rejected the step.  Synchronous. */
gid_status gid_base_step(gid_ctx *ctx, int32_t *accepted);

/* ---- kernel timing ----
 * With profiling on, the following solves launch kernels directly (no graph)
 * with a HIP event pair around every launch on the context's stream; the
 * elapsed times are accumulated per kernel kind at gid_synchronize.
 * GID_KERNEL_PCG is one Jacobi-PCG iteration (vector updates fused with the
 * J^T J product, Sec. 7.1), launched pcg_iters times per layer step. */
enum {
    GID_KERNEL_SCAN = 0, GID_KERNEL_PRECOMPUTE, GID_KERNEL_GN_BUILD, GID_KERNEL_PCG,
    GID_KERNEL_APPLY_BSUM, GID_KERNEL_BSOLVE, GID_KERNEL_ENERGY, GID_KERNEL_OUTPUT,
    GID_NUM_KERNEL_KINDS
};
/* Turn profiling on (1) or off (0); turning it on clears the accumulated times. */
gid_status gid_set_profiling(gid_ctx *ctx, int32_t enable);
/* Accumulated milliseconds and launch counts per kernel kind (arrays of
 * GID_NUM_KERNEL_KINDS entries, host). */
gid_status gid_get_kernel_times(gid_ctx *ctx, double *ms_out, int64_t *launches_out);

/* ---- batches of clips of uneven size ----
 * Independent clips solved together (each clip is its own instance of the
 * per-frame solve of Sec. 7.1, so batching changes no result).  A batch groups
 * contexts (each with its own frame size and K) that share the stream, the
 * schedule (gn_iters, pcg_iters, refine_mode) and record_energy = 0.  Each
 * workgroup of a batched launch finds its clip from a prefix table of workgroup
 * counts and runs that clip's kernel body over the clip's own launch shape;
 * reductions stay per clip, so every clip's results equal a single-clip run bit
 * for bit.  Two launch layouts:
 *   GID_BATCH_ONE_LAUNCH (default): every kernel of a step is one launch over all
 *     active clips whatever their K; the clip descriptors sit in a device table
 *     uploaded ahead of the step, and the kernel carries the bodies of every K up
 *     to the batch's largest (rounded up to 4, 8, 12 or 16), with that body's
 *     registers and LDS;
 *   GID_BATCH_PER_K: one launch per K among the active clips (per eight clips of
 *     one K), the descriptors travelling in the kernel arguments and each kernel
 *     compiled for exactly its K.
 * With use_graph the outer iterations of a step are replayed from a graph cached
 * per set of active clips, refinement, layout and set of clips with the temporal
 * prior on. */
typedef struct gid_batch gid_batch;
enum { GID_BATCH_ONE_LAUNCH = 0, GID_BATCH_PER_K = 1 };

/* Group n (1..64) distinct contexts into a batch.  Tune the contexts (gid_autotune,
 * gid_set_workgroups) before creating the batch.  Errors: GID_ERR_INVALID_ARG
 * (mismatched streams or schedules, record_energy on, duplicates). */
gid_status gid_batch_create(gid_ctx *const *ctxs, int32_t n, gid_batch **out);
gid_status gid_batch_destroy(gid_batch *b);

/* One step: decompose the next frame of every clip i with frames_dev[i] != NULL
 * (clips that have run out of frames pass NULL and are skipped).  ids_dev[i] as
 * for gid_decompose_frame; layers_dev may be NULL or hold NULL entries.  Each
 * step must be followed by gid_batch_synchronize before the next. */
gid_status gid_batch_decompose(gid_batch *b, const float *const *frames_dev,
                               const uint8_t *const *ids_dev, float *const *layers_dev);

/* Wait for the step; energies_out (n doubles, may be NULL) receives each active
 * clip's final energy (NaN for skipped clips).  GID_ERR_NUMERIC if a clip's frame
 * was rejected (its state is unchanged) or its energy is not finite. */
gid_status gid_batch_synchronize(gid_batch *b, double *energies_out);
const char *gid_batch_last_error(const gid_batch *b);

/* Choose the launch layout of later steps (GID_BATCH_ONE_LAUNCH or
 * GID_BATCH_PER_K).  Errors: GID_ERR_INVALID_ARG (unknown layout), GID_ERR_STATE
 * (a step is pending). */
gid_status gid_batch_set_launch(gid_batch *b, int32_t mode);
gid_status gid_batch_get_launch(const gid_batch *b, int32_t *mode_out);

/* Time one outer iteration of every clip without its updates (the build, the
 * pcg_iters PCG iterations and the base-colour sums, on each clip's loaded frame;
 * unknowns and colours are not changed) under both layouts, best of five, and
 * keep the one-launch layout unless the per-K one is 5% faster (the kernels left
 * out of the timing favour the one-launch layout); chosen_out (may be NULL)
 * receives the choice.  Synchronizes the stream.
 * Errors: GID_ERR_STATE (a step is pending, or a clip has no loaded frame yet:
 * run a step first). */
gid_status gid_batch_autotune(gid_batch *b, int32_t *chosen_out);

/* ---- launch-shape autotuner ----
 * Choose the number of workgroups of the per-pixel launches for this context's
 * (width, height, K) by timing the real layer-step kernels (the build and the
 * params.pcg_iters PCG iterations) on the loaded frame over the default (one
 * tile per workgroup) and every multiple of 64 from 64 to 2048 up to the tile
 * count; another shape replaces the default only when it times at least 3%
 * faster.
 * cache_path (may be NULL) is a text file of "width height K workgroups" lines:
 * a cached choice is reused, a new one appended.  Synchronous.  Needs a frame
 * loaded (gid_load_frame or a decomposed frame; GID_ERR_STATE otherwise); the
 * unknowns and colours are not changed, the PCG vectors are scratch, and the
 * frame's breakdown count and logged <r, z> are left to the next frame's reset. */
gid_status gid_autotune(gid_ctx *ctx, const char *cache_path, int32_t *workgroups_out);
/* Set / read the workgroup count directly (8..2048, rounded to a multiple of 8). */
gid_status gid_set_workgroups(gid_ctx *ctx, int32_t workgroups);
int32_t gid_get_workgroups(const gid_ctx *ctx);

/* ---- checkpoint / resume ---- */
/* Serialise the solver state (unknowns, colours, previous-frame data, frame
 * index).  With buf == NULL, *inout_bytes receives the required size. Synchronous. */
gid_status gid_save_state(gid_ctx *ctx, void *buf, size_t *inout_bytes);
gid_status gid_load_state(gid_ctx *ctx, const void *buf, size_t bytes);

/* ---- learned warm start ----
 * A network of six 3x3 convolutions (32 channels, ReLU after the first five,
 * zero padding), BF16 weights and activations with FP32 accumulation on the
 * matrix cores, predicting from the frame I_t and the previous unknowns
 * u_{t-1} (3 + K + 4 input channels) the change du (K + 4 channels,
 * u_t = u_{t-1} + du) and, through a linear head on the global average of the
 * fifth layer's features, the change of the base colours db (3K).  It is this
 * project's component, not the paper's (which names learned priors only as
 * future work, Sec. 9).  The solver keeps judging it: see gid_set_warmstart.
 *
 * Parameters are one FP32 vector, in this order: for conv layer l = 0..5 its
 * weights w[o][c][dy][dx] (c_out x c_in x 3 x 3 with c_in = K + 7 for l = 0
 * and 32 otherwise, c_out = 32 except K + 4 for l = 5), then its bias b[c_out];
 * then the head hw[3K][32] and hb[3K].  The caller provides the initial values
 * (random numbers are drawn by the caller); the library keeps FP32 master
 * weights, Adam moments and BF16 copies.  A network serves frames of exactly
 * the width, height and K it was created for. */
typedef struct gid_net gid_net;

/* Number of parameters for K base colours, or -1 for K outside 1..16. */
int64_t gid_net_num_params(int32_t K);

/* Create a network and its workspace (activations of width x height pixels),
 * enqueuing on hip_stream (NULL = null stream).  Parameters start at zero.
 * Errors: GID_ERR_INVALID_ARG, GID_ERR_UNSUPPORTED (K + 7 > 32 input channels),
 * GID_ERR_OUT_OF_MEMORY, GID_ERR_HIP. */
gid_status gid_net_create(int32_t K, int32_t width, int32_t height, void *hip_stream, gid_net **out);
gid_status gid_net_destroy(gid_net *net);

/* Copy count (== gid_net_num_params(K)) FP32 parameters from host memory and
 * reset the Adam state; get copies them back.  Synchronous. */
gid_status gid_net_set_params(gid_net *net, const float *params_host, int64_t count);
gid_status gid_net_get_params(gid_net *net, float *params_host, int64_t count);

/* Inference: u_out = u_prev + du (K + 4 planes float32, device, planar like the
 * solver's unknowns: r_0..r_2 log reflectance, T_0..T_K), db_out (3K float32,
 * host, may be NULL; synchronous when given).  frame_dev: 3 planes float32. */
gid_status gid_net_forward(gid_net *net, const float *frame_dev, const float *u_prev_dev, float *u_out_dev,
                           float *db_out_host);

/* Gradient of the loss 0.5 mean((du - du_target)^2) + 0.5 w_b mean((db - db_target)^2)
 * with respect to every parameter (FP32, host, parameter layout) and the loss
 * value; du_target: K + 4 planes (device), db_target: 3K float32 (host).
 * The parameters are not changed.  Synchronous. */
gid_status gid_net_gradients(gid_net *net, const float *frame_dev, const float *u_prev_dev,
                             const float *du_target_dev, const float *db_target_host, float w_b,
                             float *grad_host, double *loss_out);

/* One training step: the gradient as above, then Adam (beta 0.9, 0.999,
 * eps 1e-8, bias-corrected) with step size lr on the FP32 master weights.
 * loss_out (may be NULL) receives the loss before the update (then synchronous). */
gid_status gid_net_train_step(gid_net *net, const float *frame_dev, const float *u_prev_dev,
                              const float *du_target_dev, const float *db_target_host, float w_b, float lr,
                              double *loss_out);

/* Single-layer access for verification: conv layer `layer` (0..5) applied to a
 * width x height x 32 BF16 pixel-major input (device), out = conv + bias as
 * width x height x 32 float32 (device); and its weight and bias gradients
 * (host, layout of the layer's parameters) for input x and output gradient gy
 * (both width x height x 32 BF16, device).  Synchronous. */
gid_status gid_net_layer_forward(gid_net *net, int32_t layer, const void *in_dev, float *out_dev);
gid_status gid_net_layer_wgrad(gid_net *net, int32_t layer, const void *x_dev, const void *gy_dev,
                               float *gw_host, float *gb_host);

/* Launch shape of the convolutions: at most `workgroups` workgroups, each taking
 * the 4 x 64-pixel tiles i, i + workgroups, ... in turn (0, the default: two per
 * compute unit, the resident grid).  Every shape gives bit-identical results.
 * Errors: GID_ERR_INVALID_ARG for a negative count. */
gid_status gid_net_set_conv_workgroups(gid_net *net, int32_t workgroups);
const char *gid_net_last_error(const gid_net *net);

/* Attach a network as the warm start of a solver context (NULL detaches).  On
 * every frame after the first the solver evaluates the energy at the previous
 * frame's result and at the network's prediction from it, keeps the lower as
 * the start of the schedule (a prediction with a non-finite energy or a colour
 * outside (1e-4, inf) is never kept) and reports both in gid_frame_stats.  The
 * network must match the context's width, height and K and enqueue on the same
 * stream.  Errors: GID_ERR_INVALID_ARG, GID_ERR_OUT_OF_MEMORY. */
gid_status gid_set_warmstart(gid_ctx *ctx, gid_net *net);

/* ---- base-colour initialisation (Sec. 5.1, chromaticity clustering) ----
 * Cluster a clip's first frame: a histogram of its chromaticity C = I / |I|
 * (|.| the channel mean) with 10 partitions per axis over [0, 3], weighted
 * k-means on the bin mid-points (populations as weights, at most k_max
 * centres; seeded with the most populated bin, then the farthest non-empty
 * bin), centres closer than merge_dist merged (the smaller cluster joins the
 * larger; the paper uses 0.2), every pixel assigned to its nearest centre and
 * the mean RGB of each cluster's pixels returned as its initial base colour.
 *   frame_dev    3 planes width*height float32 (device)
 *   k_max        upper bound on the clusters, 1..16 (the paper uses 10)
 *   hip_stream   stream to enqueue on (NULL = null stream); the call is synchronous
 *   ids_dev      width*height uint8 (device) written: the pixel's cluster, 0..*k_out-1
 *   colors_host  k_max x 3 doubles written (rows below *k_out): mean RGB per cluster
 *   centres_host k_max x 3 doubles (may be NULL): the centres in chromaticity
 *   k_out        number of clusters found
 * The ids and colours go to gid_set_base_colors / gid_decompose_frame with K =
 * *k_out.  Allocates (and frees) a device scratch buffer of at most
 * GID_CLUSTER_SCRATCH_BYTES.  Errors: GID_ERR_INVALID_ARG, GID_ERR_NUMERIC (a
 * non-finite frame value; nothing written), GID_ERR_OUT_OF_MEMORY, GID_ERR_HIP. */
#define GID_CLUSTER_SCRATCH_BYTES 2621440u
gid_status gid_cluster_frame(const float *frame_dev, int32_t width, int32_t height, int32_t k_max,
                             double merge_dist, void *hip_stream, uint8_t *ids_dev, double *colors_host,
                             double *centres_host, int32_t *k_out);

/* ---- misclustering correction (Sec. 5.2.2) ----
 * Choose the reflectance of a region whose cluster ids are suspect: every base
 * colour j = 0..K-1 is tried as the region's colour (ids set to j inside the
 * region), each candidate frame is decomposed in full as a first frame with the
 * schedule of params (gn_iters x pcg_iters, refine_mode; the K decompositions
 * run as one batch through shared launches), and the colour whose indirect
 * layers are sparsest over the region, by the illumination sparsity term of
 * Sec. 6.2, lambda_is sum_{x in region} sum_{k>=1} |T_k(x)|, is kept (ties: the
 * lowest index).  The region itself (the paper's clicks, flood fill and
 * tracking, Sec. 5.2.1) is the caller's.
 *   params       K = the number of base colours; record_energy is ignored
 *   frame_dev    3 planes float32 (device); ids_dev width*height uint8 in [0, K)
 *   region_dev   width*height uint8 (device), nonzero inside the region
 *   colors_host  K x 3 doubles: the base colours (also the refinement's initial estimate)
 *   ids_out_dev  width*height uint8 (device) written: ids with the region set to the best colour
 *   sparsity_host K doubles written: each candidate's region sparsity
 *   best_out     the chosen colour index
 * Synchronous on hip_stream.  Allocates its workspace (K contexts, K id maps and
 * K layer sets) and frees it before returning.
 * Errors: GID_ERR_INVALID_ARG, GID_ERR_OUT_OF_MEMORY, GID_ERR_NUMERIC (a
 * candidate's frame was rejected or its energy is not finite), GID_ERR_HIP. */
gid_status gid_correct_region(const gid_params *params, int32_t width, int32_t height, const float *frame_dev,
                              const uint8_t *ids_dev, const uint8_t *region_dev, const double *colors_host,
                              void *hip_stream, uint8_t *ids_out_dev, double *sparsity_host, int32_t *best_out);

/* ---- re-synthesis for the live applications (Sec. 8.4) ----
 * Recombine layers by the image formation of Sec. 4 with edits:
 *     I'_c(x) = R_c(x) s_{id(x),c} (T_0(x) + sum_{k=1..K} g_k b'_{k,c} T_k(x)).
 * Recolouring an object (Sec. 8.4.1) passes its new colour in b_new and the
 * ratio new / old as its row of refl_scale; colour keying (Sec. 8.4.2) edits the
 * background's row of b_new; spill suppression (Sec. 8.4.3) sets its gain to 0.
 *   layers_dev      K+4 planes float32 (device): R_r, R_g, R_b (linear), T_0..T_K,
 *                   the layout gid_decompose_frame writes
 *   b_new_host      K x 3 doubles: the base colours to light with
 *   gain_host       K floats (may be NULL: all 1)
 *   ids_dev         width*height uint8 (device) with refl_scale_host (K x 3 floats), or
 *                   both NULL for no reflectance edit; ids outside [0, K) keep R
 *   out_dev         3 planes float32 (device) written
 * Asynchronous on hip_stream (NULL = null stream); FP32 arithmetic.
 * Errors: GID_ERR_INVALID_ARG (NULL layers / colours / output, size, K outside
 * 1..16, ids without scales or the reverse, non-finite colours or gains), GID_ERR_HIP. */
gid_status gid_resynthesize(const float *layers_dev, int32_t width, int32_t height, int32_t K,
                            const double *b_new_host, const float *gain_host, const uint8_t *ids_dev,
                            const float *refl_scale_host, void *hip_stream, float *out_dev);

/* gid_cluster_frame for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and results, with the scratch in a fixed device array
 * of GID_CLUSTER_SCRATCH_BYTES (2.5 MiB) that every device the library runs on
 * holds until the process ends, instead of a per-call allocation.  It calls no
 * allocating routine; the host-side k-means works in fixed-size host arrays.
 * Any frame size fits (the launches stride over the pixels with at most 512
 * workgroups).  Calls on one device share that device's array and must not
 * overlap (two concurrent calls race); each call writes every scratch value
 * it reads, so nothing carries over from the previous call.
 * Errors: as gid_cluster_frame, without GID_ERR_OUT_OF_MEMORY. */
gid_status gid_cluster_frame_noalloc(const float *frame_dev, int32_t width, int32_t height, int32_t k_max,
                                     double merge_dist, void *hip_stream, uint8_t *ids_dev, double *colors_host,
                                     double *centres_host, int32_t *k_out);

const char *gid_status_string(gid_status s);
/* Last error message of this context (valid until its next call). */
const char *gid_last_error(const gid_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GID_H */
