/*
 * FP64 CPU oracle of the SIR filter step — TEST INFRASTRUCTURE.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * import, call, link or execute anything under oracle/. The product library
 * never links it and shares no code, header or constant table with it.
 *
 * This header is the oracle's own; it does not include or mirror the
 * library's public header.
 */
#ifndef PPF_ORACLE_H
#define PPF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Model of Sections 6.1-6.2 plus the filter options of Algorithm 1 and
 * Section 3, all in double precision. */
typedef struct orc_model {
  int64_t n;            /* N particles                                        */
  int32_t obs_model;    /* 0 = Gaussian spot on an image, 1 = linear-Gaussian */
  int32_t width;        /* W                                                  */
  int32_t height;       /* H                                                  */
  int32_t patch;        /* P, odd                                             */
  double s;             /* sigma_PSF (Eq. 3)                                  */
  double b;             /* I_bg (Eq. 3)                                       */
  double sigma;         /* sigma_xi (Eq. 4)                                   */
  double q[5];          /* process-noise sds of (x, y, vx, vy, I0)            */
  int32_t init_kind;    /* 0 uniform [a,b), 1 Gaussian N(a,b^2), 2 stratified,
                           3 uniform in Z order */
  int32_t resample;     /* 0 = systematic, 1 = RNA, 2 = ARNA                  */
  double init_a[5];
  double init_b[5];
  double lg_r[3];       /* linear-Gaussian observation sds of (x, y, I0)      */
  double ess_threshold; /* resample iff ESS < threshold                       */
  int32_t rna_group;    /* n particles per RNA group                          */
  int32_t rna_moved;    /* slots moved to the ring neighbour per group        */
  uint64_t seed;        /* Philox key                                         */
  uint32_t track;       /* Philox counter word 3                              */
  int32_t arna_mu_min;  /* ARNA: least slots exchanged per group (rna_moved the most) */
  double arna_track;    /* ARNA: a group tracks when W_g >= arna_track / G     */
  double arna_lost;     /* ARNA: kappa of the lost test (see orc_arna_lost)    */
} orc_model;

/* Host threads of the per-particle loops (propagation, Eq. 4) from now on
 * (n > 0; n <= 0 leaves it); returns the count in effect (1 without OpenMP).
 * Results do not depend on it. */
int orc_set_threads(int n);

/* Philox4x32-10 block function. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* The same over n counters (4n words each), key from a 64-bit seed. */
void orc_philox_many(uint64_t seed, int64_t n, const uint32_t* ctr, uint32_t* out);

/* Conversions of Philox words to uniforms and normals. */
double orc_u24_open_hi(uint32_t a);   /* (a >> 8) / 2^24, in [0, 1)        */
double orc_u24_open_lo(uint32_t a);   /* ((a >> 8) + 1) / 2^24, in (0, 1]  */
double orc_u53(uint32_t a, uint32_t b); /* 53-bit uniform in [0, 1)        */
/* Radius (24-bit) and angle (18-bit) fields of one block, and Box-Muller
 * from one radius field and one angle field. */
void orc_normal_fields(const uint32_t r[4], uint32_t rad[3], uint32_t ang[3]);
void orc_box_muller(uint32_t rad, uint32_t ang, double* z0, double* z1);

/* Uniform of the systematic resampling at frame k; of RNA group g at k. */
double orc_resample_uniform(const orc_model* m, int64_t k);
double orc_rna_uniform(const orc_model* m, int64_t g, int64_t k);

/* Algorithm 1 initialisation: x (5*n, SoA), lw (n) = -log N. Returns 0,
 * or -1 without memory (kind 3). */
int orc_init(const orc_model* m, double* x, double* lw);

/* Initial states of the particles index[0..m->n) of a run with n_total
 * particles (5 * m->n SoA). Returns 0, or -1 without memory (kind 3). */
int orc_init_indexed(const orc_model* m, int64_t n_total, const int64_t* index, double* x);

/* Init kind 3: the Morton key of the top 16 bits of the x and y uniform
 * words, and the draw index of the particle at each position of the
 * cloud (stable sort by key). orc_zorder_perm returns 0, or -1 without
 * memory. */
uint32_t orc_zorder_key(uint32_t wx, uint32_t wy);
int orc_zorder_perm(const orc_model* m, int64_t n, int64_t* order);

/* SIS draw of frame k under the bootstrap proposal: x_new[i] from parent
 * x_prev[parent[i]] (parent NULL: identity). SoA 5*n. */
void orc_propagate(const orc_model* m, int64_t k, const double* x_prev, const int32_t* parent,
                   double* x_new);

/* The same for the particles index[0..m->n): particle j is index[j] of the
 * run (its random numbers) and starts from parents[:, j] (5 * m->n SoA). */
void orc_propagate_indexed(const orc_model* m, int64_t k, const int64_t* index,
                           const double* parents, double* x_new);

/* log p(z | x) of Eq. 4 with its normalising constant, per particle. */
void orc_loglik_spot(const orc_model* m, const float* frame, const double* x, double* ll);
void orc_loglik_lg(const orc_model* m, const float* obs3, const double* x, double* ll);

/* Normalisation of Algorithm 1 on unnormalised log weights lwt (n):
 * w (n) normalised; stats = {m, log S, ESS, delta = m + log S}. Returns 0,
 * or -1 when no finite positive normaliser exists. */
int orc_normalize(int64_t n, const double* lwt, double* w, double stats[4]);

/* MMSE estimate sum_i w_i x_i (5 values). */
void orc_estimate(int64_t n, const double* w, const double* x, double mean[5]);

/* Systematic resampling: anc[i] = min{ j : (i + u)/n < C_j }, C_{n-1} := 1. */
void orc_resample_systematic(int64_t n, const double* w, double u, int32_t* anc);

/* RNA: local systematic resampling per group with u_g[g], slot weight W_g/n,
 * then ring exchange of the last `moved` slots from group g-1. Outputs the
 * ancestors, log(W_g/n) per group (lwg, G values) and per slot (lw_slot). */
void orc_resample_rna(int64_t n, int32_t group, int32_t moved, const double* w,
                      const double* u_g, int32_t* anc, double* lwg, double* lw_slot);

/* ARNA (adaptive RNA, Section 6.4; the reading of its rules is in the
 * design notes). Ring order of G groups under ring key `key`: order[j] is the
 * group at ring position j, group order[j] passing particles to
 * order[j + 1 mod G]. Key 0 is the index order. */
void orc_ring_order(const orc_model* m, int64_t key, int64_t G, int64_t* order);
/* The object counts as lost at a frame whose log-likelihood increment delta
 * falls more than kappa P below ref (kappa = arna_lost), ref being the
 * increment of the latest frame at which it was not lost (-inf before the
 * first frame). P is the scale of the frame-to-frame spread of a good fit:
 * the residual sum / sigma_xi^2 of Eq. 4 at the true state is chi-square with
 * P^2 degrees of freedom, standard deviation P sqrt(2), so its log-likelihood
 * varies by about P / sqrt(2). Returns 1 when lost. */
int orc_arna_lost(const orc_model* m, double delta, double ref);
/* ARNA resampling: RNA's local systematic resampling per group (uniforms
 * u_g), then G_t = #{g : W_g >= theta / G} tracking groups, the exchange
 * mu = mu_min + floor((mu_max - mu_min) (G - G_t) / G), and the last mu slots
 * of each group taken (ancestors and weight) from the same slots of its ring
 * predecessor in `order`. Outputs as orc_resample_rna, plus G_t and mu. */
void orc_resample_arna(int64_t n, int32_t group, int32_t mu_min, int32_t mu_max, double theta,
                       const double* w, const double* u_g, const int64_t* order, int32_t* anc,
                       double* lwg, double* lw_slot, int32_t* tracking, int32_t* moved);

/* A whole filter run of T frames (Algorithm 1). obs: T frames of H*W fp32
 * (spot) or T*3 fp32 (linear-Gaussian). Per-frame outputs may be NULL.
 * x_out (5n), lw_out (n: normalised log weights of the last frame before
 * resampling), anc_out (n: last ancestors or identity) may be NULL.
 * Returns 0, or -k when frame k had no finite normaliser. */
int orc_run(const orc_model* m, int32_t T, const float* obs, double* mean, double* ess,
            double* delta, int32_t* resampled, double* x_out, double* lw_out, int32_t* anc_out,
            int64_t* arna_out);
/* arna_out (ARNA only, may be NULL): per frame the ring key, the tracking
 * groups G_t and the slots exchanged (both 0 when the frame did not
 * resample), T * 3 values. */

/* Derivatives of log p^ = sum_k delta_k with respect to theta = (s, b,
 * sigma_xi, q_x, q_y, q_vx, q_vy, q_I, I0), noise and ancestors fixed. */
/* Tangents (7 * n SoA: dx/dq_x, dy/dq_y, dvx/dq_vx, dx/dq_vx, dvy/dq_vy,
 * dy/dq_vy, dI/dq_I) of frame k's states from those of the parents. */
void orc_propagate_tangent(const orc_model* m, int64_t k, const double* t_prev,
                           const int32_t* parent, double* t_new);
/* Per particle dl/d(x, y, I0, s, b, sigma) of Eq. 4 (6 * n SoA). */
void orc_loglik_spot_grad(const orc_model* m, const float* frame, const double* x,
                          double* dll);
/* sum_i w_i dl_i/dtheta (9 values). */
void orc_step_grad(int64_t n, const double* w, const double* dll, const double* tang,
                   double g[9]);
/* Whole run with derivatives; systematic resampling at every step; optional
 * ancestor replay (T * n), ancestor record (T * n), state trace (T * 5 * n). */
int orc_run_grad(const orc_model* m, int32_t T, const float* obs, const int32_t* anc_replay,
                 int32_t* anc_out, double* x_trace, double* cum, double grad[9]);

/* RPA (Section 3) with the DLB schedules of Section 4 over G = n_total /
 * group groups: offspring counts from the global systematic ancestors, the
 * schedule (kind 0 GS, 1 SGS, 2 LGS; entries (sender, receiver, particles),
 * returns their number or -1), and the balanced resampling (kind 0 or 1). */
void orc_rpa_counts(int64_t n_total, int32_t group, const int32_t* anc_sys, int32_t* counts);
int64_t orc_dlb_schedule(int kind, int64_t G, int32_t n, const int32_t* counts, int64_t cap,
                         int32_t* sched);
int orc_resample_rpa(int64_t n_total, int32_t group, int kind, const int32_t* anc_sys,
                     int32_t* anc);

#ifdef __cplusplus
}
#endif

#endif
