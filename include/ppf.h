/*
 * ppf.h — C ABI of the MI355X (gfx950) SIR particle-filter library.
 *
 * The library runs one step of the sequential importance resampling (SIR)
 * filter of Algorithm 1 (Section 2 of "PPF – A Parallel Particle Filtering
 * Library", Demirel et al., arXiv:1310.5045) per call, entirely in HIP kernels:
 *
 *   propagate   bootstrap proposal under the near-constant-velocity model of
 *               Section 6.1, state x = (x, y, vx, vy, I0);
 *   weight      Gaussian-spot observation model of Eq. 3 evaluated on a local
 *               P x P image patch (Eq. 4, Section 5.5 "Image Patches");
 *   normalise   weight normalisation and effective sample size of Algorithm 1,
 *               done in the log domain; MMSE estimate of Section 2;
 *   resample    when ESS < threshold (Algorithm 1): either global systematic
 *               resampling, or RNA — distributed resampling with
 *               non-proportional allocation (Section 3) with one GPU workgroup
 *               standing in for each process and a ring exchange of a fixed
 *               fraction of each group's particles.
 *
 * Conventions shared by every entry point
 *   - Every function returns int: PPF_OK (0) or a negative PPF_E* code. None
 *     aborts, none lets a C++ exception escape.
 *   - "_dev" pointers are HIP device pointers on the current device; "_host"
 *     pointers are ordinary host memory. The library never frees memory it did
 *     not allocate. Nothing here allocates device memory: state lives in the
 *     caller's workspace.
 *   - A handle is used by one host thread at a time. All device work of a
 *     handle is enqueued on the hipStream_t given to ppf_create (NULL = the
 *     null stream). Functions documented as "async" return before the GPU has
 *     finished; functions documented as "syncs" wait for that stream.
 *   - Random numbers come from Philox4x32-10 (Salmon et al., SC'11), keyed by
 *     the 64-bit seed. Counter words are (particle or group index, frame k,
 *     purpose << 24 | block, track_id) with purposes INIT=1, PROPAGATE=2,
 *     RESAMPLE=3, RNA=4, so every draw of a run is a pure function of
 *     (seed, track_id, k, index): a run is reproducible and restartable.
 *     A particle's five process-noise normals come from one block (block 0):
 *     three 24-bit radius and three 18-bit angle fields, laid end to end from
 *     bit 0 of word 0, through Box-Muller.
 */
#ifndef PPF_H
#define PPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
  PPF_OK = 0,
  PPF_EINVAL = -1,    /* bad argument or parameter                          */
  PPF_ENOMEM = -2,    /* workspace / scratch smaller than required          */
  PPF_EDEVICE = -3,   /* a HIP runtime call failed                          */
  PPF_ESTATE = -4,    /* null, destroyed or otherwise unusable handle       */
  PPF_ENUMERIC = -5,  /* a step produced no finite normaliser; rolled back   */
  PPF_ENOTIMPL = -6   /* option recognised but not built                    */
};

enum { PPF_RESAMPLE_SYSTEMATIC = 0, PPF_RESAMPLE_RNA = 1, PPF_RESAMPLE_RPA = 2,
       PPF_RESAMPLE_ARNA = 3 };
/* DLB schedules of Section 4: Greedy (Alg. 2), Sorted Greedy (Alg. 3),
 * Largest Gradient (Alg. 4). */
enum { PPF_DLB_GS = 0, PPF_DLB_SGS = 1, PPF_DLB_LGS = 2 };
enum { PPF_OBS_SPOT = 0, PPF_OBS_LINEAR_GAUSSIAN = 1 };
enum { PPF_INIT_UNIFORM = 0, PPF_INIT_GAUSSIAN = 1, PPF_INIT_STRATIFIED = 2,
       PPF_INIT_UNIFORM_ZORDER = 3 };

/* Largest patch edge P the kernels are built for. */
#define PPF_MAX_PATCH 25

typedef struct ppf_ctx* ppf_handle;

/*
 * Filter parameters. Field meanings follow the paper's notation.
 *
 * state_dim     must be 5: x = (x, y, vx, vy, I0), Section 6.1.
 * obs_model     PPF_OBS_SPOT: the frame is a W x H image, Eq. 3 + Eq. 4.
 *               PPF_OBS_LINEAR_GAUSSIAN: the observation is three floats
 *               (x, y, I0) + N(0, diag(lg_r^2)); a linear-Gaussian variant of
 *               the same state-space model whose exact posterior is the Kalman
 *               filter (Eqs. 1-2), used to validate the whole recursion.
 * n_particles   N, 1 <= N <= 2^31 - 1.
 * width,height  frame size in pixels; frames are row-major fp32 Z[y][x]
 *               (spot model only; ignored for the linear-Gaussian model).
 * psf_sigma     sigma_PSF of Eq. 3 in pixels (> 0).
 * background    I_bg of Eq. 3.
 * noise_sigma   sigma_xi of Eq. 4 (> 0).
 * patch         P, the edge of the square pixel set S_x of Eq. 4, odd,
 *               1..PPF_MAX_PATCH; 0 selects 2*floor(3*psf_sigma)+1, the
 *               integer reading of the +-3 sigma_PSF box. EINVAL when
 *               (h + 1/2)^2 / (2 psf_sigma^2) > 350, h = (P - 1) / 2 (a patch
 *               so wide that its edge factors would leave the fp64 range).
 * q[5]          process-noise standard deviations of (x, y, vx, vy, I0).
 * init_kind     PPF_INIT_UNIFORM: x0[d] ~ U[init_a[d], init_b[d]) i.i.d. (the
 *               paper initialises uniformly at random, Section 6.3);
 *               PPF_INIT_GAUSSIAN: x0[d] ~ N(init_a[d], init_b[d]^2);
 *               PPF_INIT_STRATIFIED: uniform as above, but the (x, y) box is
 *               cut into 2^t cells (t = max(0, floor(log2 N) - 2), x taking
 *               ceil(t/2) bits, y floor(t/2)) visited in Z order; particle i
 *               lies uniformly inside cell floor(i 2^t / N). Consecutive
 *               indices are then neighbours in the image, which keeps the
 *               first frame's image tiles small;
 *               PPF_INIT_UNIFORM_ZORDER: the draws of PPF_INIT_UNIFORM, i.i.d.
 *               uniform, with the particles placed in the stable order of the
 *               Morton key of the top 16 bits of their x and y uniform words
 *               (x bits at the even positions; ties by draw index): the same
 *               cloud as a set, ordered so that neighbours in the index are
 *               neighbours in the image. Its initialisation sorts N keys on
 *               the device (about 17 N bytes more workspace). Single filters
 *               only.
 * lg_r[3]       observation noise sds of the linear-Gaussian model (> 0).
 * resample      PPF_RESAMPLE_SYSTEMATIC, PPF_RESAMPLE_RNA, or PPF_RESAMPLE_RPA:
 *               resampling with proportional allocation (Section 3) over
 *               groups of rna_group consecutive particles standing in for
 *               processes. Group g's offspring are its share N_g of the
 *               global systematic resampling (so the resampled multiset is
 *               that of PPF_RESAMPLE_SYSTEMATIC); it keeps its first
 *               min(N_g, n) offspring in its own slots, and the surplus of
 *               groups with N_g > n fills the free slots of groups with
 *               N_g < n following the DLB schedule `dlb` (GS or SGS, which
 *               balance exactly). Weights afterwards 1/N.
 * ess_threshold resample iff ESS < ess_threshold (Algorithm 1); +INFINITY
 *               resamples every step, 0 never.
 * rna_group     n, particles per RNA group (one workgroup each); N % n == 0,
 *               1 <= n <= 1024. For RPA the group size: N % n == 0 (any
 *               number of groups, under GS and SGS alike). Ignored for
 *               systematic resampling.
 * rna_exchange  rho in [0, 1): after local resampling the last floor(rho * n)
 *               slots of group g take the particles (and weight) of the same
 *               slots of group g-1 mod G (Section 3, ring of processes).
 *               Under ARNA: the largest exchange ratio.
 *               PPF_RESAMPLE_ARNA, adaptive RNA (Section 6.4, which names its
 *               rules without defining them; this is the library's reading):
 *               RNA's local resampling over groups of rna_group, where
 *               - group g tracks when its share W_g of the normalised weight
 *                 is at least arna_track / G, G_t groups in all;
 *               - mu = mu_min + floor((mu_max - mu_min) (G - G_t) / G) slots
 *                 move per group, mu_max = floor(rna_exchange n), mu_min =
 *                 floor(arna_min n): the more groups track, the fewer move;
 *               - the last mu slots of each group take the particles (and
 *                 weight) of the same slots of its predecessor on a ring of
 *                 the groups. The object counts as lost at a frame whose
 *                 log-likelihood increment falls more than arna_lost * P
 *                 below that of the last frame at which it was not lost;
 *                 each loss redraws the ring order (a permutation keyed by
 *                 the seed, track_id and the frame of the loss: an 8-round
 *                 Feistel network on Philox4x32-10 over the smallest even
 *                 number of bits b with 2^b >= G, restricted to the groups by
 *                 cycle walking), which is kept until the next loss; before
 *                 any loss the ring is the index order g-1 -> g of RNA.
 *               With arna_min = rna_exchange and no loss, ARNA is RNA.
 * seed          Philox key.
 * track_id      Philox counter word 3 (distinguishes independent filters).
 * dlb           PPF_DLB_GS or PPF_DLB_SGS: the schedule of RPA.
 * reserved      must be 0.
 * arna_min      ARNA: the smallest exchange ratio, 0 <= arna_min <= rna_exchange.
 * arna_track    ARNA: theta > 0 of the tracking test W_g >= theta / G.
 * arna_lost     ARNA: kappa >= 0 of the lost test (+INFINITY: never lost).
 * arna_pad      must be 0.
 * grad          1: every step also accumulates the derivatives of log p^ in
 *               theta (see ppf_grad). Needs the spot model, systematic
 *               resampling and ess_threshold = +INFINITY; the workspace then
 *               also holds 2 x 7 tangents per particle (fp32) and 9 doubles
 *               per 256-particle block. 0: none.
 */
typedef struct ppf_params {
  int32_t state_dim;
  int32_t obs_model;
  int64_t n_particles;
  int32_t width;
  int32_t height;
  float psf_sigma;
  float background;
  float noise_sigma;
  int32_t patch;
  float q[5];
  int32_t init_kind;
  float init_a[5];
  float init_b[5];
  float lg_r[3];
  int32_t resample;
  double ess_threshold;
  int32_t rna_group;
  float rna_exchange;
  uint64_t seed;
  uint32_t track_id;
  int32_t grad; /* 0, or 1: also accumulate d log p^ / d theta (ppf_grad) */
  int32_t dlb;      /* PPF_DLB_* schedule of RPA */
  int32_t reserved; /* must be 0 */
  float arna_min;   /* ARNA: smallest exchange ratio */
  float arna_track; /* ARNA: tracking share theta */
  float arna_lost;  /* ARNA: lost-test kappa */
  int32_t arna_pad; /* must be 0 */
} ppf_params;

/* Scalars of the last committed step (see ppf_stats). */
typedef struct ppf_stats_t {
  int64_t k;           /* committed steps since create/reset                  */
  int32_t resampled;   /* 1 if the last committed step resampled              */
  int32_t rolled_back; /* steps rolled back (PPF_ENUMERIC) since last report  */
  double ess;          /* 1 / sum w^2 of the last step, pre-resampling        */
  double max_logw;     /* m = max_i log w~_i (unnormalised log weight)        */
  double log_sum;      /* log sum_i exp(log w~_i - m)                         */
  double delta;        /* log p^(z_k | z_1:k-1) = m + log_sum                 */
  double cum;          /* sum over committed steps of delta                   */
  double mean[5];      /* MMSE estimate sum_i w_i x~_i (Section 2)           */
} ppf_stats_t;

/* Per-kernel timing accumulated while profiling is enabled. Entries are
 * named for the step's timed units: "k_step", "k_merge" (both merge
 * launches), "k_resample" (the systematic resampling pass: the segment
 * launch and the launch that fills queued tile chunks, under one pair of
 * events), "k_rna" (RNA and ARNA), "k_rpa", and "k_init", "k_gather",
 * "k_logw" outside the step. */
typedef struct ppf_kernel_time {
  char name[32];
  int64_t launches;
  double total_ms;
} ppf_kernel_time;

/* Library version string, static storage. */
const char* ppf_version(void);

/* sizeof(ppf_params) as compiled, so bindings can check their layout. */
size_t ppf_params_size(void);

/* Fill *p with the defaults of a single-spot 128x128 tracking problem
 * (s = 1.5, b = 10, sigma_xi = 3, N = 4096, systematic every step).
 * EINVAL if p is NULL. */
int ppf_params_default(ppf_params* p);

/* Bytes of device workspace a filter with parameters *p needs (256-byte
 * aligned start required). EINVAL for invalid parameters (see ppf_create). */
int ppf_workspace_bytes(const ppf_params* p, size_t* bytes);

/*
 * Validate *p, carve the caller's device workspace and draw x0 (Algorithm 1,
 * initialisation, k = 0: w0 = 1/N, x0 ~ pi(x0)); async on hip_stream.
 *   workspace   device pointer, 256-byte aligned, at least
 *               ppf_workspace_bytes bytes; owned by the caller and must
 *               outlive the handle.
 *   hip_stream  hipStream_t used for all device work of the handle.
 *   out         receives the handle (host memory owned by the library, freed
 *               by ppf_destroy).
 * EINVAL: state_dim != 5, N out of range, even/too large patch, a sigma <= 0,
 *   N % rna_group != 0 under RNA, rho outside [0, 1), null pointers, a patch
 *   too wide for psf_sigma (edge beyond 37 sigma), frame size <= 0.
 * ENOMEM: bytes too small. EDEVICE: a HIP call failed.
 */
int ppf_create(const ppf_params* p, void* workspace, size_t bytes, void* hip_stream,
               ppf_handle* out);

/* Re-draw x0 and zero the step counter and log-likelihood; async. */
int ppf_reset(ppf_handle h);

/*
 * One SIR step k (Algorithm 1, SIS step + normalisation + ESS + optional
 * resampling) on the observation obs_dev; async.
 *   obs_dev  spot model: device frame, H*W fp32 row-major Z[y][x];
 *            linear-Gaussian model: 3 fp32 (x, y, I0) on the device.
 *            Must stay valid until the stream has passed the step.
 * Nothing is synchronised: the resampling decision is taken on the device.
 * When the step finds no finite normaliser (e.g. NaN pixels under every
 * particle) it is rolled back on the device (state and k unchanged) and the
 * next synchronising call reports PPF_ENUMERIC.
 * ESTATE for a null handle; EDEVICE if a launch fails.
 */
int ppf_step(ppf_handle h, const float* obs_dev);

/*
 * Graph mode (1 on, 0 off; off after create). When on, the next ppf_step
 * records the step's kernel launches into a HIP graph instead of launching
 * them, and that step and every later one launch the graph (hipGraphLaunch)
 * with its frame argument pointed at the call's obs_dev; results are the
 * same as without the graph. The launch sequence of a step does not depend
 * on the filter's state (every decision is taken on the device), so one
 * recording serves all steps. Switching syncs the handle's stream and drops
 * the recorded graph. ESTATE while kernel timing (ppf_profile_enable) is on:
 * the two exclude each other.
 */
int ppf_set_graph(ppf_handle h, int enable);

/*
 * Workgroup shapes of the spot-model step kernel for patches up to 13 x 13
 * (larger patches and derivative mode have one kernel each):
 *   0  LDS image tile of up to 2048 doubles, compiled for 5 waves per SIMD
 *   1  tile of up to 1792 doubles, 6 waves per SIMD (six workgroups share a
 *      CU, fewer registers per lane)
 * Both compute the same likelihood; a workgroup whose patches span between
 * 1792 and 2048 tile pixels reads them from the frame under shape 1 instead
 * of from LDS, which sums the same terms in another order. Create selects
 * shape 0.
 */
#define PPF_NUM_SHAPES 2
/* Most tuning candidates any autotune call times (size of its ms_out). */
#define PPF_TUNE_MAX 3

/* Select the step kernel's workgroup shape (0 or 1, EINVAL otherwise);
 * syncs the stream and drops a recorded graph. Has no effect where only one
 * kernel exists (see above). */
int ppf_set_shape(ppf_handle h, int32_t shape);

/*
 * Autotuner: time every workgroup shape of the step kernel on this filter's
 * current particles and the frame obs_dev, and keep the fastest for the
 * following steps. Each candidate runs the step kernel once untimed, then
 * reps times between two HIP events on the handle's stream. The step kernel
 * alone writes only the next state buffer, weights and records, so the
 * committed step, its counter and statistics, and the next ppf_step are
 * unchanged (the timed launches are not part of any step). Candidates:
 * shapes 0 and 1 for a spot model with P <= 13 without derivatives, else
 * the single kernel (one candidate, nothing changes).
 *   reps     launches timed per candidate, 1..10000 (EINVAL otherwise)
 *   ms_out   NULL or PPF_TUNE_MAX doubles: average ms per launch, by candidate
 *   n_out    NULL or the number of candidates timed
 *   chosen   NULL or the candidate kept
 * Syncs; drops a recorded graph. EINVAL for a null frame.
 */
int ppf_autotune(ppf_handle h, const float* obs_dev, int32_t reps, double* ms_out,
                 int32_t* n_out, int32_t* chosen);

/* Wait for the handle's stream. Returns PPF_ENUMERIC if any step enqueued
 * since the last report was rolled back (and clears the report), else OK. */
int ppf_sync(ppf_handle h);

/* MMSE estimate x^ = sum_i w_i x~_i of the last committed step (weights
 * before resampling, Section 2) and its ESS; syncs. mean: 5 doubles. Either
 * pointer may be NULL. Returns PPF_ENUMERIC like ppf_sync. */
int ppf_estimate(ppf_handle h, double mean[5], double* ess);

/* cum = sum_k log p^(z_k | z_1:k-1), last = the term of the last committed
 * step: the normaliser of Eq. 1 estimated by the particles (log of the sum of
 * the normalised previous weights times the likelihood); syncs. Either
 * pointer may be NULL. Returns PPF_ENUMERIC like ppf_sync. */
int ppf_loglik(ppf_handle h, double* cum, double* last);

/*
 * Derivatives of the log-likelihood estimate (the cum of ppf_loglik) with
 * respect to
 *   theta = (psf_sigma, background, noise_sigma, q[0..4], I0),
 * I0 being a common offset of every particle's initial intensity (init_a[4]
 * and init_b[4] moved together), with the Philox noise and the resampling
 * ancestors held fixed: the state draws are reparameterised and the
 * discrete ancestor choice is not differentiated (a stop-gradient through
 * resampling). The patch size stays fixed while psf_sigma varies. With
 * resampling at every step, each step adds sum_i w_i d l_i / d theta, the
 * normalised weights times the derivative of the particle's log-likelihood
 * (Eqs. 3-4) through its parameters and its state, whose tangents in q are
 * carried along the ancestral lines. cum: 9 doubles summed over committed
 * steps since create/reset; last: the last committed step's term. Either
 * pointer may be NULL; syncs. EINVAL when the filter was created with
 * grad = 0.
 */
#define PPF_NGRAD 9
int ppf_grad(ppf_handle h, double cum[PPF_NGRAD], double last[PPF_NGRAD]);

/* ARNA state after the last committed step (PPF_RESAMPLE_ARNA only, EINVAL
 * otherwise); syncs. ring_key: the frame of the latest loss, which keys the
 * ring order (0: no loss yet, the index ring); lost: 1 if that step found the
 * object lost; tracking: G_t and moved: mu of its resampling (both 0 when it
 * did not resample). Any pointer may be NULL. */
int ppf_arna_state(ppf_handle h, int64_t* ring_key, int32_t* lost, int32_t* tracking,
                   int32_t* moved);

/* All scalars of the last committed step; syncs and clears the roll-back
 * report (returns PPF_OK even if steps were rolled back: see rolled_back). */
int ppf_stats(ppf_handle h, ppf_stats_t* out);

/*
 * Copy the particle system of the last committed step to the host; syncs.
 *   state_host  5*N fp32, SoA [x | y | vx | vy | I0], the propagated states
 *               x~_k (before resampling);
 *   logw_host   N fp64, normalised log weights log w_k (before resampling);
 *   anc_host    N int32, the ancestors s(i) drawn at step k, or the identity
 *               when step k did not resample (or no step ran yet).
 * Any pointer may be NULL.
 */
int ppf_get_particles(ppf_handle h, float* state_host, double* logw_host, int32_t* anc_host);

/*
 * Replace the particle system (checkpoint restore, test injection); syncs.
 *   state_host  5*N fp32 SoA as above; logw_host N fp64 log weights,
 *   normalised (log-sum-exp 0) for ppf_loglik to keep its meaning.
 * The next step propagates particle i from state i with log weight logw[i]
 * (no resampling in between). The step counter k is kept.
 */
int ppf_set_particles(ppf_handle h, const float* state_host, const double* logw_host);

/* Write the resampled particle states x_k^i = x~_k^{s(i)} (Algorithm 1,
 * resampling copy) as 5*N fp32 SoA to out_dev; async. Equals the state of
 * ppf_get_particles when the last step did not resample. */
int ppf_gather(ppf_handle h, float* out_dev);

/* Enable (1) / disable (0) per-kernel HIP-event timing of the handle's
 * launches; enabling clears the accumulated times. ESTATE in graph mode. */
int ppf_profile_enable(ppf_handle h, int on);

/* Read accumulated kernel times; syncs. Writes at most max_entries entries
 * and the number written to *n_entries. */
int ppf_profile_read(ppf_handle h, ppf_kernel_time* out, int max_entries, int* n_entries);

/* Release the handle (host memory only; the workspace stays the caller's).
 * Waits for the handle's outstanding work first. NULL is accepted. */
int ppf_destroy(ppf_handle h);

/* Static text for a return code. */
const char* ppf_error_string(int code);

/* Text of the last error recorded on the handle ("" if none). */
const char* ppf_last_error(ppf_handle h);

/* ------------------------------------------------ standalone primitives */

/*
 * Philox4x32-10 (Salmon et al., SC'11) over n counters: out[4i..4i+3] =
 * Philox(ctr[4i..4i+3], key = (seed & 0xffffffff, seed >> 32)); async on
 * hip_stream. ctr_dev and out_dev: 4*n uint32 on the device. EINVAL for
 * n < 0 or null pointers with n > 0.
 */
int ppf_philox4x32_10(uint64_t seed, const uint32_t* ctr_dev, uint32_t* out_dev, int64_t n,
                      void* hip_stream);

/* Device scratch bytes needed by the standalone resamplers for n weights. */
int ppf_resample_scratch_bytes(int64_t n, size_t* bytes);

/*
 * Systematic resampling of the resampling step of Algorithm 1 on arbitrary
 * log weights; async.
 *   logw_dev  n fp32 unnormalised log weights (-inf allowed, not all -inf);
 *   u         the single uniform in [0, 1); slot i uses (i + u) / n;
 *   anc_dev   n int32 out: s(i) = min{ j : (i + u)/n < C_j }, C the CDF of
 *             the normalised weights (C_{n-1} taken as 1);
 *   scratch   device scratch of ppf_resample_scratch_bytes(n), 256-aligned.
 * EINVAL / ENOMEM as usual. Non-finite normaliser: anc is left unwritten and
 * the call returns OK (no sync happens); callers validate inputs.
 */
int ppf_resample_systematic(const float* logw_dev, int64_t n, double u, int32_t* anc_dev,
                            void* scratch, size_t scratch_bytes, void* hip_stream);

/*
 * The same systematic resampling without caller scratch and without any
 * allocation, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The scratch is a device array of PPF_STATIC_SCRATCH_BYTES bytes inside the
 * library, one per device, looked up on the first call on a device and held
 * until the process ends. Arguments as ppf_resample_systematic; async.
 *   n   1 <= n <= PPF_STATIC_MAX_N (EINVAL beyond: the array's limit).
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the kernels write every scratch value they read before
 * reading it, so nothing carries over): calls that overlap on one device
 * (other streams, other threads) race on it and must not be issued.
 * EDEVICE when the array's address cannot be obtained.
 */
#define PPF_STATIC_MAX_N (1 << 22)
#define PPF_STATIC_SCRATCH_BYTES (4u << 20)
int ppf_resample_systematic_static(const float* logw_dev, int64_t n, double u, int32_t* anc_dev,
                                   void* hip_stream);

/*
 * RNA resampling (Section 3): groups g of `group` consecutive weights are
 * resampled locally and systematically with uniform u_dev[g]; group g's slot
 * weight becomes W_g / group (W_g its share of the normalised weight); then
 * the last `moved` slots of each group take the ancestors and weight of the
 * same slots of group g-1 mod G. Async.
 *   u_dev    G = n / group doubles in [0, 1) on the device;
 *   anc_dev  n int32 out (global indices);
 *   lwg_dev  G doubles out: log(W_g / group) (-inf for an empty group, which
 *            keeps the identity map).
 * EINVAL: n % group != 0, group outside 1..1024, moved outside 0..group.
 */
int ppf_resample_rna(const float* logw_dev, int64_t n, int32_t group, int32_t moved,
                     const double* u_dev, int32_t* anc_dev, double* lwg_dev, void* scratch,
                     size_t scratch_bytes, void* hip_stream);

/*
 * DLB schedule of Section 4 on the device; async. For G groups whose
 * particle counts counts_dev[g] (int32) should become n each, the senders
 * (counts > n, surplus counts - n) and receivers (counts < n, deficit
 * n - counts) are matched:
 *   PPF_DLB_GS   senders and receivers in group order; each sender in turn
 *                fills the current receiver and moves to the next one when
 *                it is full (Alg. 2, read so that a filled receiver is
 *                skipped and the loop ends: the printed loop resets j to 0
 *                and has no branch for a filled receiver);
 *   PPF_DLB_SGS  the same after sorting both lists by surplus / deficit,
 *                descending, ties by group (Alg. 3);
 *   PPF_DLB_LGS  the i-th largest sender pairs with the i-th largest
 *                receiver for min(|S|, |R|) ranks, moving the smaller of the
 *                two (Alg. 4, recording the count before zeroing it).
 * sched_dev: 3 int32 per entry (sender group, receiver group, particles),
 * at most cap entries; *n_entries_dev (int32, device) receives their number,
 * or -1 when cap is too small (then no entry is written). Any number of
 * groups: the lists are radix-sorted and the entries found in parallel (the
 * greedy walk pairs each sender with the receivers whose deficit intervals
 * overlap its surplus interval, both laid end to end in list order). The
 * call allocates its device scratch on the stream (hipMallocAsync, about
 * 80 bytes per group) and frees it there after its launches; async.
 * EINVAL: G < 1, n < 0 or an unknown kind; ENOMEM: no scratch.
 */
int ppf_dlb_schedule(int32_t kind, const int32_t* counts_dev, int32_t G, int32_t n,
                     int32_t* sched_dev, int32_t cap, int32_t* n_entries_dev, void* hip_stream);

/* ------------------------------------------ batched independent filters */

/*
 * A batch runs `count` independent SIR filters (tracks) over one shared
 * frame stream: each track is exactly the filter ppf_create would build from
 * its own ppf_params (its own N, patch, spot model, noise, resampling scheme
 * and threshold, seed and track_id), and after every step its particles,
 * weights, ancestors and statistics are bit-identical to that single filter's.
 * Tracking many spots in one movie (Section 6) this way costs one launch per
 * kernel kind per frame for the whole batch instead of one set per spot.
 * Every track must use the spot observation model (Eq. 3-4) and the same
 * frame width and height. Distinct track_ids give distinct random streams.
 */
typedef struct ppf_batch_ctx* ppf_batch;

/* Workspace bytes for a batch of `count` tracks with parameters p[0..count-1].
 * EINVAL: count < 1, a track's parameters invalid, a track not on the spot
 * model, or frame sizes that differ between tracks. */
int ppf_batch_workspace_bytes(const ppf_params* p, int32_t count, size_t* bytes);

/*
 * Create a batch in a caller-owned device workspace (256-byte aligned, at
 * least ppf_batch_workspace_bytes) and initialise every track (k = 0). The
 * batch's tables are uploaded here, so this call syncs hip_stream. Errors as
 * ppf_batch_workspace_bytes, ENOMEM for a short workspace, EDEVICE.
 */
int ppf_batch_create(const ppf_params* p, int32_t count, void* workspace, size_t bytes,
                     void* hip_stream, ppf_batch* out);

/* Re-initialise every track (k = 0) on the batch's stream; async. */
int ppf_batch_reset(ppf_batch h);

/* One step of every track on the frame obs_dev (H*W fp32, device, row-major,
 * shared by all tracks); async, as ppf_step. A track whose normaliser is not
 * finite rolls back alone and reports it in ppf_batch_stats. */
int ppf_step_batched(ppf_batch h, const float* obs_dev);

/* Graph mode of a batch, as ppf_set_graph: one HIP graph holds every launch
 * of a batched step (one step launch for all patch sizes up to 13, one per
 * wider size, then the merge and resampling launches). */
int ppf_batch_set_graph(ppf_batch h, int enable);

/*
 * Workgroup shapes of a batch's fused step launches, by candidate:
 *   0  every track with P <= 13 in one launch of shape 0
 *   1  every track with P <= 13 in one launch of shape 1
 *   2  tracks with P <= 11 in a launch of shape 1, tracks with P = 13 in a
 *      launch of shape 0
 * (tracks with P > 13 keep a launch per size). EINVAL for another value.
 * Re-orders the batch's step items on the device; syncs; drops a recorded
 * graph. Create selects candidate 0.
 */
int ppf_batch_set_shapes(ppf_batch h, int32_t candidate);

/* Autotuner of a batch, as ppf_autotune: times candidates 0 and 1 above,
 * and 2 when the batch has tracks with P = 13 and with P < 13, on the
 * batch's current particles and obs_dev (the step launches of every track,
 * once untimed, then reps times), and keeps the fastest. */
int ppf_batch_autotune(ppf_batch h, const float* obs_dev, int32_t reps, double* ms_out,
                       int32_t* n_out, int32_t* chosen);

/* Statistics of every track's last committed step (out: count entries, in
 * track order), as ppf_stats; syncs and clears the roll-back reports. */
int ppf_batch_stats(ppf_batch h, ppf_stats_t* out, int32_t count);

/* Particles of one track (0 <= track < count), as ppf_get_particles with
 * that track's N; syncs. EINVAL for a track out of range. */
int ppf_batch_get_particles(ppf_batch h, int32_t track, float* state_host, double* logw_host,
                            int32_t* anc_host);

/* Per-kernel HIP-event timing of the batch's launches, as ppf_profile_*. */
int ppf_batch_profile_enable(ppf_batch h, int on);
int ppf_batch_profile_read(ppf_batch h, ppf_kernel_time* out, int max_entries, int* n_entries);

/* Release the batch (host memory only); waits for its work. NULL accepted. */
int ppf_batch_destroy(ppf_batch h);

/* Text of the last error recorded on the batch ("" if none). */
const char* ppf_batch_last_error(ppf_batch h);

#ifdef __cplusplus
}
#endif

#endif /* PPF_H */
