/*
 * dmwf.h -- C ABI of the MI355X dual messenger Wiener filter library.
 *
 * The library solves the Wiener filter equation of Kodi Ramanah, Lavaux &
 * Wandelt (2017), Section 1,
 *
 *        (S^-1 + N^-1) s_WF = N^-1 d,
 *
 * for a temperature map d on the HEALPix sphere, with a diagonal signal
 * covariance S = diag(C_l) in spherical harmonic space and a diagonal noise
 * covariance N in pixel space (N^-1 = 0 marks masked pixels).  It uses the
 * paper's dual messenger iteration (Section 2.2, Algorithm 2, hybrid form
 * with cooling of xi) where the paper's flat-sky Fourier transform is replaced
 * by the spherical harmonic transform pair on the HEALPix ring grid:
 *
 *   F^-1 = Y          synthesis, s(p) = sum_lm a_lm Y_lm(p)
 *   F    = Omega Y^H  Omega = 4 pi / Npix times the adjoint of Y
 *
 * and the harmonic step is taken in residual form (see dmwf_dm_iterate).
 * Everything is FP64 on one GPU, except the Legendre contractions of plans
 * created with a reduced precision (dmwf_precision).
 *
 * Conventions shared by every entry point
 *   Maps    [nmaps][Npix] doubles, HEALPix RING order, Npix = 12 nside^2.
 *   a_lm    [nmaps][n_alm][2] doubles (re, im), m-major: the slot of (l, m)
 *           is m (2 lmax + 1 - m) / 2 + l for 0 <= m <= l <= lmax,
 *           n_alm = (lmax+1)(lmax+2)/2.  Y_lm are orthonormal with the
 *           Condon-Shortley phase, the field is real (a_{l,-m} =
 *           (-1)^m conj(a_lm)); Im a_l0 is ignored on input and 0 on output.
 *   C_l     [nmaps][lmax+1] doubles, C_l >= 0; modes with C_l = 0 stay 0.
 *   N^-1    [nmaps][Npix] doubles, >= 0 and finite; 0 = masked.
 *   Pointers named dev_* are device pointers owned by the caller.  The plan
 *   owns only its constant tables.  The workspace is caller-allocated device
 *   memory of at least dmwf_workspace_bytes() bytes, 256-byte aligned.
 *   stream is a hipStream_t passed as void*; NULL means the null stream.
 *   All work is enqueued on that stream.  One call at a time per plan and
 *   workspace.
 *   Every function validates its host-visible arguments before enqueueing
 *   anything; on DMWF_ERR_INVALID_ARG no output is touched.  A failing HIP
 *   call returns DMWF_ERR_HIP; dmwf_last_error() then describes it.
 */
#ifndef DMWF_H
#define DMWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMWF_OK = 0,
    DMWF_ERR_INVALID_ARG = 1,   /* a size, pointer or parameter is out of range    */
    DMWF_ERR_WORKSPACE = 2,     /* workspace too small or misaligned               */
    DMWF_ERR_HIP = 3,           /* a HIP runtime call failed                       */
    DMWF_ERR_NOT_CONVERGED = 4, /* max_iter reached; outputs hold the last iterate */
    DMWF_ERR_NONFINITE = 5,     /* NaN/Inf in the inputs or in the Cauchy ratio    */
    DMWF_ERR_UNSUPPORTED = 6,   /* valid request this build does not implement     */
    DMWF_ERR_OOM = 7            /* device allocation for the plan tables failed    */
} dmwf_status;

/* Precision of the Legendre contractions (the sums over l and over rings of
 * the transform pair).  The recurrence that generates lambda_lm, its exponent
 * rescaling near the poles, the ring FFTs, the pixel and harmonic steps, the
 * Cauchy sums and the residual are FP64 in every form.
 *   DMWF_FP64         FP64 on the vector ALUs.
 *   DMWF_FP32_GEMM    lambda_lm and the coefficients rounded to FP32, products
 *                     on the matrix cores (v_mfma_f32_*_f32) with FP32
 *                     accumulation.
 *   DMWF_BF16X3_GEMM  each FP32 operand split into two BF16 parts (hi + lo),
 *                     the three products hi*hi + hi*lo + lo*hi on the matrix
 *                     cores with FP32 accumulation. */
typedef enum { DMWF_FP64 = 0, DMWF_FP32_GEMM = 1, DMWF_BF16X3_GEMM = 2 } dmwf_precision;

typedef struct dmwf_plan dmwf_plan;

typedef struct {
    int nside;     /* power of two, 1 .. 8192 (above 1024: DMWF_ERR_UNSUPPORTED) */
    int lmax;      /* 0 .. 3 nside - 1                                         */
    int nmaps;     /* 1 .. 65535; the maps of a plan are transformed and solved together */
    int precision; /* dmwf_precision                                           */
} dmwf_plan_desc;

/* Cooling schedule and stopping rule of the solve (paper Algorithm 2 and
 * Section 4).  Level k has messenger covariance xi_k: xi_0 = alpha + sigma
 * mu0 (sigma = Npix / 4 pi), xi_{k+1} = beta xi_k, and the first value
 * <= alpha is replaced by alpha, the last level.  A level repeats iterations
 * until the Cauchy ratio ||s_i - s_{i-1}|| / ||s_i|| (pixel space) falls below
 * its tolerance. */
typedef struct {
    double beta;             /* (0,1); <= 0 selects 0.75                          */
    double mu0;              /* initial mu (harmonic units); < 0 selects beta*max C_l */
    double eps_final;        /* tolerance at xi = alpha, > 0                      */
    double eps_coarse;       /* tolerance on levels with xi > alpha, > 0          */
    int max_iter;            /* cap on iterations per map, >= 1                   */
    int start_final;         /* 1: run only xi = alpha, warm start from alm_out   */
    const int* replay_iters; /* host; if non-NULL, exactly replay_iters[k]
                                iterations on level k (n_replay = level count)    */
    int n_replay;
    int want_residual;       /* 1: compute stats.wf_residual (two extra transforms) */
    int warm_start;          /* 1: start the cooling schedule (from level 0, or
                                the last level with start_final) from the a_lm
                                given in alm_out instead of a = 0; the first
                                residual is c (d - Y a) at that level's xi    */
    double eps_reduced;      /* reduced-precision plans: the last level runs the
                                matrix-core contractions until the Cauchy ratio
                                falls below this (or stops improving: 64
                                iterations without a 1% gain), then continues in
                                FP64 down to eps_final; coarse levels run reduced
                                throughout, and replayed solves never switch.
                                <= 0 selects eps_final: the reduced iterations
                                meet the final tolerance, FP64 ones confirm it */
} dmwf_schedule;

/* Per-solve statistics (host memory).  The three arrays are optional
 * (NULL) caller buffers of cap_levels entries each. */
typedef struct {
    int n_levels;          /* levels run                                       */
    int n_iter;            /* iterations run (all levels)                      */
    double alpha;          /* min N over unmasked pixels                       */
    double final_cauchy;   /* last Cauchy ratio                                */
    double wf_residual;    /* ||A x - y|| / ||y||, paper Section 4 / Appendix C, or -1 */
    int cap_levels;
    int* iters_per_level;
    double* xi_per_level;
    int* lmax_per_level;   /* l_iter: largest l with C_l > mu on that level    */
    int iters_reduced;     /* iterations whose contractions ran in reduced precision */
} dmwf_stats;

/* Create a plan: geometry, Legendre recurrence tables and the per-(m, ring)
 * starting values of the recurrence, built on the current device with
 * exponent rescaling near the poles.  *out is NULL on failure. */
dmwf_status dmwf_plan_create(const dmwf_plan_desc* desc, dmwf_plan** out);

/* Free the plan's tables.  NULL is accepted. */
void dmwf_plan_destroy(dmwf_plan* plan);

/* Workspace size in bytes needed by every call on this plan. */
dmwf_status dmwf_workspace_bytes(const dmwf_plan* plan, size_t* bytes);

/* Synthesis F^-1: map = Y alm for each of the plan's maps (one batched pass). */
dmwf_status dmwf_alm2map(dmwf_plan* plan, const double* dev_alm, double* dev_map,
                         void* dev_ws, size_t ws_bytes, void* stream);

/* Synthesis without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same result as dmwf_alm2map, bit for bit, computed
 * by the same kernels, with their scratch (the g-scaled a_lm and the ring
 * Fourier rows of every map) in a fixed 64 MiB device array of the library
 * instead of a caller's workspace.  Each GPU the library runs on holds that
 * array until the process ends; its address is looked up when a plan is
 * created on the device.  The call allocates nothing (no hipMalloc, hipFree
 * or event creation; kernel timing does not apply to it) and needs nothing
 * zeroed.  Plans whose scratch exceeds 64 MiB (16 B x nmaps x (n_alm + 64 +
 * 4 nside lp) with lp = 4 ceil((lmax+1)/4), plus alignment: one map up to
 * Nside 512 / lmax 1024) get DMWF_ERR_WORKSPACE.  All calls on one GPU share the
 * array and it keeps the last call's contents: calls that overlap on one GPU
 * (from several streams or threads) race and give wrong maps. */
dmwf_status dmwf_alm2map_static(dmwf_plan* plan, const double* dev_alm, double* dev_map,
                                void* stream);

/* Adjoint: alm_lm = sum_p map_p conj(Y_lm(p)), times Omega = 4 pi / Npix if
 * scale_by_pixel_area != 0 (then it is the method's forward transform F). */
dmwf_status dmwf_adjoint(dmwf_plan* plan, const double* dev_map, double* dev_alm,
                         int scale_by_pixel_area, void* dev_ws, size_t ws_bytes, void* stream);

/* One dual messenger iteration at messenger covariance xi (paper Algorithm 2,
 * the body of the repeat loop), single map (map 0 of the plan):
 *
 *   a <- f (a + Omega Y^H r),    f_l = S_bar_l / (S_bar_l + xi / sigma),
 *                                S_bar_l = max(C_l - mu, 0), mu = (xi - alpha) / sigma
 *   s <- Y a
 *   cauchy2 <- (sum_p (s_p - s_prev_p)^2, sum_p s_p^2)
 *   r <- c (d - s),              c = xi w / (1 + (xi - alpha) w),  w = N^-1
 *
 * r = t - s is the pixel-space messenger step with N_bar = N - alpha.  With
 * first != 0 the residual is d on unmasked pixels (t = d, s = 0) and s_prev
 * is taken as 0; otherwise r is the one left in the workspace by the previous
 * call on the same plan and workspace.  dev_alm_state [n_alm][2] and
 * dev_s_map [Npix] are read and overwritten; dev_cauchy2 receives 2 doubles.
 * Requires alpha > 0 and xi >= alpha. */
dmwf_status dmwf_dm_iterate(dmwf_plan* plan, double xi, double alpha, const double* dev_cl,
                            const double* dev_d, const double* dev_ninv, double* dev_alm_state,
                            double* dev_s_map, double* dev_cauchy2, int first,
                            void* dev_ws, size_t ws_bytes, void* stream);

/* Full solve for every map of the plan.  Outputs the Wiener filter a_lm and
 * map s_WF = Y a_WF.  Cold start from a = 0 unless sched->start_final.  The
 * level decisions (Cauchy ratio against each level's tolerance, the next xi,
 * the stop) are taken on the device after every iteration; the host enqueues
 * iterations in batches and synchronises with the stream once per batch.
 * Iterations after the first are replays of one HIP graph of the iteration
 * (launch by launch while every launch is timed; all paths give the same bits).
 * The maps of the plan iterate together, one launch per stage for all of
 * them, each with its own alpha, schedule, level and stop; a map that has
 * stopped is left untouched while the others go on.  Every map comes out
 * exactly as a one-map plan would compute it.  A schedule may have at most
 * 1024 levels (else DMWF_ERR_INVALID_ARG); with replay_iters, every map's
 * schedule must have n_replay levels.  stats may be NULL or point to nmaps
 * records, one per map.
 * Returns DMWF_ERR_NONFINITE for NaN/Inf or negative values in d, N^-1 or
 * C_l of any map (checked on the device before the first iteration) or a NaN
 * Cauchy ratio, DMWF_ERR_INVALID_ARG if every pixel of a map is masked, and
 * DMWF_ERR_NOT_CONVERGED if some map ran max_iter iterations (outputs hold
 * the last iterate); dmwf_last_error() names the map. */
dmwf_status dmwf_solve(dmwf_plan* plan, const double* dev_cl, const double* dev_d,
                       const double* dev_ninv, const dmwf_schedule* sched,
                       double* dev_alm_out, double* dev_map_out, dmwf_stats* stats,
                       void* dev_ws, size_t ws_bytes, void* stream);

/* Several plans solved together, e.g. groups of maps of different Nside
 * (Algorithm 2 for every map of every plan).  Plan i takes dev_cl[i],
 * dev_d[i], dev_ninv[i], writes dev_alm_out[i] and dev_map_out[i], fills
 * stats[i] (NULL, or its plan's nmaps records; stats itself may be NULL) and
 * uses its own workspace dev_ws[i] of ws_bytes[i] bytes.  After the first,
 * every iteration of every plan is one replay of a single HIP graph (the
 * plans' launches one after another), and every map keeps its own device-side
 * level control and stop; the host waits only once per batch of iterations.
 * Every map comes out bit for bit as dmwf_solve on its own plan computes it.
 * The schedule is shared; with replay_iters every map's schedule must have
 * n_replay levels.  Plans and workspaces must be distinct (else
 * DMWF_ERR_INVALID_ARG), 1 <= nplans <= 64; other errors as dmwf_solve. */
dmwf_status dmwf_solve_plans(int nplans, dmwf_plan* const* plans, const double* const* dev_cl,
                             const double* const* dev_d, const double* const* dev_ninv,
                             const dmwf_schedule* sched, double* const* dev_alm_out,
                             double* const* dev_map_out, dmwf_stats* const* stats,
                             void* const* dev_ws, const size_t* ws_bytes, void* stream);

/* Pick the tiles of the Legendre stages for this plan by timing each
 * candidate on the device.  Synthesis: ring pairs per lane {1, 2} x maps per
 * wave {1, 2, 4, 8}.  Analysis: ring pairs per lane {4, 8} (4 only for
 * nside <= 256) x maps per wave {1, 2}.  Maps per wave are at most nmaps; a
 * wave of several maps computes the recurrence once for all of them.  The
 * maps per wave and the synthesis ring pairs per lane change no result (each
 * map's sums run in the same order); the analysis ring pairs per lane change
 * the order in which ring pairs are summed (rounding only).  Overwrites the
 * workspace and synchronises the stream.  choice (may be NULL) receives
 * {synthesis ring pairs per lane, synthesis maps per wave, analysis ring
 * pairs per lane, analysis maps per wave}; ms_out (may be NULL) receives 12
 * per-launch times in milliseconds: synthesis at 4 (rings - 1) + log2(maps),
 * analysis at 8 + 2 (rings == 8) + (maps - 1); -1 for candidates not tried. */
dmwf_status dmwf_autotune(dmwf_plan* plan, void* dev_ws, size_t ws_bytes, void* stream,
                          int* choice, float* ms_out);

/* Set the Legendre tiles explicitly (the candidates dmwf_autotune times);
 * maps per wave above nmaps act as nmaps.  The workspace's analysis partial
 * sums and residual spectrum are invalid afterwards (the next dmwf_dm_iterate
 * call needs first != 0).  DMWF_ERR_INVALID_ARG for other values. */
dmwf_status dmwf_set_tiles(dmwf_plan* plan, int syn_k, int syn_mb, int ana_k, int ana_mb);

/* Pipelined iteration (overlap of the synthesis and the ring stage by
 * ring-pair groups): NOT BUILT.  It was removed after its first solve ended
 * the process with a host segmentation fault whose cause was not found.
 * groups 0 or 1 (no pipeline) return DMWF_OK; 2..8 return
 * DMWF_ERR_UNSUPPORTED; other values DMWF_ERR_INVALID_ARG. */
dmwf_status dmwf_set_pipeline(dmwf_plan* plan, int groups);
/* Groups in use: always 0 (no pipeline); -1 for a NULL plan. */
int dmwf_pipeline_groups(const dmwf_plan* plan);

/* ||A x - y|| / ||y|| with A = 1 + C^1/2 Y^H W Y C^1/2, x = C^-1/2 a,
 * y = C^1/2 Y^H W d over modes with C_l > 0 (paper Section 4, Appendix C),
 * norms on a_lm counting m > 0 twice, for every map of the plan: host_out
 * receives nmaps values.  Synchronises the stream. */
dmwf_status dmwf_wf_residual(dmwf_plan* plan, const double* dev_cl, const double* dev_d,
                             const double* dev_ninv, const double* dev_alm, double* host_out,
                             void* dev_ws, size_t ws_bytes, void* stream);

/* Work of one FP64 Legendre launch at band limit ell (0..lmax), counted on
 * the host from the plan's recurrence starts and its current tiles:
 * out[0] = nq (ell+1)(ell+2)/2 triples (m, l, ring pair), the full work;
 * out[1] = triples at or after each (m, ring pair)'s recurrence start (the
 * polar terms below 2^-100 skipped); out[2] / out[3] = lane-steps the
 * synthesis / analysis kernel issues (each a recurrence step and its
 * contraction for one ring pair: wave-wide starts, whole blocks, idle slots
 * skipped by the analysis).  Synchronizes the device on its first call. */
dmwf_status dmwf_legendre_work(dmwf_plan* plan, int ell, long long* out);

/* Kernel timing.  enable = 1: every launch is bracketed by HIP events on the
 * launch stream (the solve loop then launches every iteration kernel by
 * kernel).  enable = 2: only the Legendre analysis launches are (the solve
 * loop launches the analysis between its events and replays the rest of each
 * iteration from its graph).  0 switches timing off; other values are
 * DMWF_ERR_INVALID_ARG.  dmwf_profile_read returns, for each kernel class,
 * the launch count and the summed device time in milliseconds (it
 * synchronises the recorded events) and clears the record.  names[i] is a
 * static string. */
#define DMWF_NPROF 16
dmwf_status dmwf_profile_enable(dmwf_plan* plan, int enable);
dmwf_status dmwf_profile_read(dmwf_plan* plan, int* n_classes, const char** names,
                              long* counts, double* total_ms);

/* ---- Learned warm start -------------------------------------------------
 * A per-mode harmonic-space network estimates the Wiener filter a_lm of a
 * map from its masked data, as the starting point of a solve (the paper's
 * solver starts from zero, Algorithm 2's initialisation; a warm start enters
 * through dmwf_schedule.warm_start or start_final).  Architecture: F = 24
 * features of one mode (l, m) -> 128 -> 128 -> 2, ReLU after the first two
 * layers, FP32.  Features of mode (l, m), with d_lm = Omega Y^H (masked data)
 * (dmwf_adjoint with the pixel area) and the map's white-noise level N_w:
 *   0..17  d_{l+k, m} / sqrt(C_l + N_w), k = -4..4, re and im (0 outside
 *          m <= l+k <= lmax; Im 0 for m = 0)
 *   18 C_l / (C_l + N_w)   19 m / (l + 1)   20 sky fraction
 *   21 log10(N_w / C_l) / 10   22, 23 zero
 * Output: a_lm = sqrt(C_l) (y0 + i y1); modes with l < 2 or C_l = 0 get 0.
 * Parameters are one flat FP32 vector: W1 [24][128], b1 [128], W2 [128][128],
 * b2 [128], W3 [128][2], b3 [2] (row-major, y = x W + b).  Training minimises
 * the mean over a batch of |y - t|^2 (t the whitened Wiener filter a_lm) with
 * Adam (beta 0.9, 0.999, eps 1e-8).  All device pointers are caller-owned;
 * the network owns its parameters, optimizer state and activation buffers
 * for batches up to max_batch rows.  One call at a time per network. */
typedef struct dmwf_nn dmwf_nn;
int dmwf_nn_param_count(void);
/* Parameters zero until dmwf_nn_set_params. */
dmwf_status dmwf_nn_create(int max_batch, dmwf_nn** out);
void dmwf_nn_destroy(dmwf_nn* net);
/* Copy the flat parameters out / in (device FP32); set also resets Adam. */
dmwf_status dmwf_nn_get_params(dmwf_nn* net, float* dev_out, void* stream);
dmwf_status dmwf_nn_set_params(dmwf_nn* net, const float* dev_in, void* stream);
/* N_w = Omega / mean of N^-1 over unmasked pixels, and the unmasked sky
 * fraction, of one map (synchronizes the stream). */
dmwf_status dmwf_nn_noise_stats(const double* dev_ninv, long long npix, double* noise_w,
                                double* fsky, void* stream);
/* Feature rows [n][24] for the a_lm slots dev_slots[0..n-1] (NULL: slots
 * 0..n-1) of one map; with dev_target (a Wiener filter a_lm) also the
 * training targets [n][2]. */
dmwf_status dmwf_nn_features(int lmax, const double* dev_dlm, const double* dev_cl,
                             double noise_w, double fsky, const int* dev_slots, int n,
                             const double* dev_target, float* dev_x, float* dev_t, void* stream);
/* y [n][2] = network(x [n][24]), n <= max_batch. */
dmwf_status dmwf_nn_forward(dmwf_nn* net, const float* dev_x, int n, float* dev_y, void* stream);
/* Gradient of the batch loss with respect to the flat parameters into
 * dev_grad, the loss into dev_loss[0]; parameters unchanged. */
dmwf_status dmwf_nn_gradient(dmwf_nn* net, const float* dev_x, const float* dev_t, int n,
                             float* dev_grad, float* dev_loss, void* stream);
/* One Adam step on the batch (loss before the step into dev_loss[0]). */
dmwf_status dmwf_nn_train_step(dmwf_nn* net, const float* dev_x, const float* dev_t, int n,
                               float lr, float* dev_loss, void* stream);
/* The network's estimate of every a_lm of one map into dev_alm_out [n_alm][2]. */
dmwf_status dmwf_nn_warm_start(dmwf_nn* net, int lmax, const double* dev_dlm,
                               const double* dev_cl, double noise_w, double fsky,
                               double* dev_alm_out, void* stream);

/* Human-readable status and the last error message of the calling thread. */
const char* dmwf_status_string(dmwf_status status);
const char* dmwf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DMWF_H */
