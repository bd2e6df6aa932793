/*
 * FP64 CPU oracle of the SIR filter step — TEST INFRASTRUCTURE.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * import, call, link or execute anything under oracle/.
 *
 * Plain, slow, sequential double-precision code that follows Algorithm 1
 * (SIR, Section 2) with the dynamics of Section 6.1 and the observation
 * model of Eqs. 3-4 (Section 6.2), and the RNA scheme of Section 3. Every
 * loop runs in index order; every sum is sequential. The random numbers come
 * from this file's own Philox4x32-10 written from its published definition
 * (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - proposal: bootstrap, pi = p(x_k | x_{k-1}), so the weight update of
 *     Algorithm 1 reduces to w_{k-1} * p(z_k | x~_k);
 *   - dynamics: unit frame interval, positions advance by the previous
 *     velocity, independent Gaussian noise per state component;
 *   - S_x: the P x P pixel block centred on the pixel nearest to (x^, y^);
 *     pixels outside the frame contribute Z - I_bg = 0;
 *   - Eq. 4 keeps its Gaussian normaliser, so the per-step normaliser of
 *     Eq. 1 (the log-likelihood increment) is an absolute quantity;
 *   - resampling scheme: systematic, s(i) = min{ j : (i+u)/N < C_j };
 *   - RNA: contiguous groups, local systematic resampling, slot weight W_g/n,
 *     the last floor(rho n) slots of group g replaced by those of g-1 mod G;
 *   - ARNA (Section 6.4 names its three rules only): a group tracks when its
 *     weight share is at least theta / G; the exchange shrinks linearly with
 *     the share of tracking groups, from floor(rho n) (none tracks) to
 *     floor(rho_min n) (all track); the ring order is redrawn as a keyed
 *     permutation at every frame whose log-likelihood increment drops well
 *     below that of the last frame that tracked (the object is lost), and
 *     kept until the next loss.
 *
 * The per-particle loops of propagation and of Eq. 4 may run on several
 * host threads (OpenMP, when built with it): each particle's value is
 * computed alone by the same arithmetic, so the results do not depend on the
 * thread count. Every reduction stays one sequential loop.
 */
#include "ppf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

enum { PURPOSE_INIT = 1, PURPOSE_PROPAGATE = 2, PURPOSE_RESAMPLE = 3, PURPOSE_RNA = 4,
       PURPOSE_RING = 5 };

/* ------------------------------------------------------------- Philox */

/* One Philox round: two 32x32->64 products, their halves xored with the
 * other counter words and the round key, then a fixed word permutation. */
static void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0;
  const uint32_t n1 = lo1;
  const uint32_t n2 = hi0 ^ c[3] ^ k1;
  const uint32_t n3 = lo0;
  c[0] = n0;
  c[1] = n1;
  c[2] = n2;
  c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { /* Weyl key schedule between rounds */
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    philox_round(c, k0, k1);
  }
  memcpy(out, c, sizeof c);
}

void orc_philox_many(uint64_t seed, int64_t n, const uint32_t* ctr, uint32_t* out) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

static void draw(const orc_model* m, uint32_t index, uint32_t k, uint32_t purpose, uint32_t block,
                 uint32_t out[4]) {
  const uint32_t ctr[4] = {index, k, (purpose << 24) | block, m->track};
  const uint32_t key[2] = {(uint32_t)m->seed, (uint32_t)(m->seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* --------------------------------------------------------- conversions */

double orc_u24_open_hi(uint32_t a) { return ldexp((double)(a >> 8), -24); }

double orc_u24_open_lo(uint32_t a) { return ldexp((double)(a >> 8) + 1.0, -24); }

double orc_u53(uint32_t a, uint32_t b) {
  return ldexp((double)a * 2097152.0 + (double)(b >> 11), -53);
}

/* The bit fields of one Philox block (words r[0..3], r[0] lowest) that the
 * five normals take: three radius fields of 24 bits and three angle fields
 * of 18 bits, laid end to end from bit 0 as radius 0, angle 0, radius 1,
 * angle 1, radius 2, angle 2 (126 bits; the top two bits are unused). */
void orc_normal_fields(const uint32_t r[4], uint32_t rad[3], uint32_t ang[3]) {
  int pos = 0;
  for (int f = 0; f < 6; ++f) {
    const int width = f % 2 == 0 ? 24 : 18;
    uint32_t v = 0;
    for (int b = 0; b < width; ++b, ++pos)
      v |= ((r[pos / 32] >> (pos % 32)) & 1u) << b;
    if (f % 2 == 0)
      rad[f / 2] = v;
    else
      ang[f / 2] = v;
  }
}

/* Box-Muller from a 24-bit radius field (uniform (rad + 1) / 2^24 in (0, 1])
 * and an 18-bit angle field (uniform ang / 2^18 in [0, 1)). */
void orc_box_muller(uint32_t rad, uint32_t ang, double* z0, double* z1) {
  const double radius = sqrt(-2.0 * log(ldexp((double)rad + 1.0, -24)));
  const double angle = 2.0 * M_PI * ldexp((double)ang, -18);
  *z0 = radius * cos(angle);
  *z1 = radius * sin(angle);
}

double orc_resample_uniform(const orc_model* m, int64_t k) {
  uint32_t r[4];
  draw(m, 0u, (uint32_t)k, PURPOSE_RESAMPLE, 0u, r);
  return orc_u53(r[0], r[1]);
}

double orc_rna_uniform(const orc_model* m, int64_t g, int64_t k) {
  uint32_t r[4];
  draw(m, (uint32_t)g, (uint32_t)k, PURPOSE_RNA, 0u, r);
  return orc_u53(r[0], r[1]);
}

/* Five standard normals for (index, k, purpose) from one Philox block: the
 * field pairs (radius 0, angle 0) and (radius 1, angle 1) give z0, z1 and
 * z2, z3; (radius 2, angle 2) gives z4 (cosine branch). */
static void five_normals(const orc_model* m, uint32_t index, uint32_t k, uint32_t purpose,
                         double z[5]) {
  uint32_t r[4], rad[3], ang[3];
  double unused;
  draw(m, index, k, purpose, 0u, r);
  orc_normal_fields(r, rad, ang);
  orc_box_muller(rad[0], ang[0], &z[0], &z[1]);
  orc_box_muller(rad[1], ang[1], &z[2], &z[3]);
  orc_box_muller(rad[2], ang[2], &z[4], &unused);
}

/* ------------------------------------------------------ initialisation */

/* Stratified uniform initialisation over the (x, y) box: 2^t cells, t =
 * max(0, floor(log2 N) - 2), x taking ceil(t/2) bits and y floor(t/2);
 * particle i lies in cell c = floor(i 2^t / N), whose bits alternate x, y
 * from the lowest (Z order), at a uniform position inside the cell. */
static int strat_bits(int64_t n) {
  int t = 0;
  while (((int64_t)1 << (t + 1)) <= n) ++t;
  t -= 2;
  return t < 0 ? 0 : t;
}

static void strat_cell(int64_t i, int64_t n, int t, uint32_t* cx, uint32_t* cy) {
  const uint64_t c = ((uint64_t)i << t) / (uint64_t)n;
  uint32_t x = 0, y = 0;
  int bx = 0, by = 0;
  for (int j = 0; j < t; ++j) {
    const uint32_t bit = (uint32_t)(c >> j) & 1u;
    if (j % 2 == 0)
      x |= bit << bx++;
    else
      y |= bit << by++;
  }
  *cx = x;
  *cy = y;
}

/* Initial state of particle i of n (stride: distance between components). */
static void init_one(const orc_model* m, int64_t i, int64_t n, double* x, int64_t stride) {
  uint32_t r0[4], r1[4];
  if (m->init_kind == 1) {
    double z[5];
    five_normals(m, (uint32_t)i, 0u, PURPOSE_INIT, z);
    for (int d = 0; d < 5; ++d) x[d * stride] = m->init_a[d] + m->init_b[d] * z[d];
    return;
  }
  draw(m, (uint32_t)i, 0u, PURPOSE_INIT, 0u, r0);
  draw(m, (uint32_t)i, 0u, PURPOSE_INIT, 1u, r1);
  double f[5] = {orc_u24_open_hi(r0[0]), orc_u24_open_hi(r0[1]), orc_u24_open_hi(r0[2]),
                 orc_u24_open_hi(r0[3]), orc_u24_open_hi(r1[0])};
  if (m->init_kind == 2) {
    const int t = strat_bits(n);
    uint32_t cx, cy;
    strat_cell(i, n, t, &cx, &cy);
    f[0] = ((double)cx + f[0]) / ldexp(1.0, (t + 1) / 2);
    f[1] = ((double)cy + f[1]) / ldexp(1.0, t / 2);
  }
  for (int d = 0; d < 5; ++d) x[d * stride] = m->init_a[d] + (m->init_b[d] - m->init_a[d]) * f[d];
}

/* Init kind 3: the uniform draws of kind 0, with the particles ordered by
 * the Z-order (Morton) key of the top 16 bits of their x and y uniforms
 * (x bits at the even positions), ties by draw index. Position is monotone
 * in those bits, so neighbours in the order are neighbours in space; the
 * cloud as a set is the uniform one. */
uint32_t orc_zorder_key(uint32_t wx, uint32_t wy) {
  uint32_t k = 0;
  for (int j = 0; j < 16; ++j) {
    k |= ((wx >> (16 + j)) & 1u) << (2 * j);
    k |= ((wy >> (16 + j)) & 1u) << (2 * j + 1);
  }
  return k;
}

static int cmp_u64(const void* a, const void* b) {
  const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* order[j] = the draw index of the particle at position j (kind 3), from
 * the composite keys (key << 32 | index), whose plain sort is the stable
 * sort by key. Returns 0, or -1 without memory. */
int orc_zorder_perm(const orc_model* m, int64_t n, int64_t* order) {
  uint64_t* kk = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  if (!kk) return -1;
  for (int64_t i = 0; i < n; ++i) {
    uint32_t r0[4];
    draw(m, (uint32_t)i, 0u, PURPOSE_INIT, 0u, r0);
    kk[i] = ((uint64_t)orc_zorder_key(r0[0], r0[1]) << 32) | (uint64_t)i;
  }
  qsort(kk, (size_t)n, sizeof(uint64_t), cmp_u64);
  for (int64_t j = 0; j < n; ++j) order[j] = (int64_t)(kk[j] & 0xffffffffu);
  free(kk);
  return 0;
}

/* Algorithm 1, k = 0: w_0 = 1/N and x_0 drawn from the initial density. */
int orc_init(const orc_model* m, double* x, double* lw) {
  const int64_t n = m->n;
  int64_t* order = NULL;
  if (m->init_kind == 3) {
    order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!order || orc_zorder_perm(m, n, order) != 0) {
      free(order);
      return -1;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    init_one(m, order ? order[i] : i, n, x + i, n);
    lw[i] = -log((double)n);
  }
  free(order);
  return 0;
}

/* The initial states at the given positions of a cloud of n_total
 * particles (kind 3 orders the whole cloud first). Returns 0, or -1
 * without memory. */
int orc_init_indexed(const orc_model* m, int64_t n_total, const int64_t* index, double* x) {
  int64_t* order = NULL;
  if (m->init_kind == 3) {
    order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_total > 0 ? n_total : 1));
    if (!order || orc_zorder_perm(m, n_total, order) != 0) {
      free(order);
      return -1;
    }
  }
  for (int64_t j = 0; j < m->n; ++j)
    init_one(m, order ? order[index[j]] : index[j], n_total, x + j, m->n);
  free(order);
  return 0;
}

/* ---------------------------------------------------------- propagate */

/* Near-constant-velocity dynamics (Section 6.1) with unit time step:
 * position += velocity, then Gaussian noise with sds q on every component. */
static void propagate_one(const orc_model* m, int64_t k, int64_t i, const double* x_prev,
                          int64_t p, double* x_new, int64_t j) {
  const int64_t n = m->n;
  double z[5];
  five_normals(m, (uint32_t)i, (uint32_t)k, PURPOSE_PROPAGATE, z);
  const double px = x_prev[0 * n + p], py = x_prev[1 * n + p];
  const double pvx = x_prev[2 * n + p], pvy = x_prev[3 * n + p];
  const double pI = x_prev[4 * n + p];
  x_new[0 * n + j] = px + pvx + m->q[0] * z[0];
  x_new[1 * n + j] = py + pvy + m->q[1] * z[1];
  x_new[2 * n + j] = pvx + m->q[2] * z[2];
  x_new[3 * n + j] = pvy + m->q[3] * z[3];
  x_new[4 * n + j] = pI + m->q[4] * z[4];
}

void orc_propagate(const orc_model* m, int64_t k, const double* x_prev, const int32_t* parent,
                   double* x_new) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m->n; ++i)
    propagate_one(m, k, i, x_prev, parent ? (int64_t)parent[i] : i, x_new, i);
}

void orc_propagate_indexed(const orc_model* m, int64_t k, const int64_t* index,
                           const double* parents, double* x_new) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m->n; ++j) propagate_one(m, k, index[j], parents, j, x_new, j);
}

/* --------------------------------------------------------- likelihood */

/* Eq. 4 on the P x P pixel block around the particle, with the spot of Eq. 3
 * evaluated per pixel (one exp per pixel, no separable shortcut). */
void orc_loglik_spot(const orc_model* m, const float* frame, const double* x, double* ll) {
  const int64_t n = m->n;
  const int h = (m->patch - 1) / 2;
  const double two_s2 = 2.0 * m->s * m->s;
  const double two_sigma2 = 2.0 * m->sigma * m->sigma;
  const double log_norm =
      (double)m->patch * (double)m->patch * log(m->sigma * sqrt(2.0 * M_PI));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double xt = x[0 * n + i], yt = x[1 * n + i], It = x[4 * n + i];
    const double cx = floor(xt + 0.5), cy = floor(yt + 0.5);
    double acc = 0.0;
    for (int dy = -h; dy <= h; ++dy) {
      for (int dx = -h; dx <= h; ++dx) {
        const double u = cx + dx, v = cy + dy;
        double D = 0.0;
        if (u >= 0.0 && u < (double)m->width && v >= 0.0 && v < (double)m->height)
          D = (double)frame[(int64_t)v * m->width + (int64_t)u] - m->b;
        const double g = exp(-((u - xt) * (u - xt) + (v - yt) * (v - yt)) / two_s2);
        const double r = D - It * g;
        acc += r * r;
      }
    }
    ll[i] = -acc / two_sigma2 - log_norm;
  }
}

/* Linear-Gaussian observation of (x, y, I0) with independent noise. */
void orc_loglik_lg(const orc_model* m, const float* obs3, const double* x, double* ll) {
  const int64_t n = m->n;
  static const int comp[3] = {0, 1, 4};
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double e = (double)obs3[d] - x[comp[d] * n + i];
      const double r = m->lg_r[d];
      acc += -e * e / (2.0 * r * r) - log(r * sqrt(2.0 * M_PI));
    }
    ll[i] = acc;
  }
}

/* ------------------------------------------------------ normalisation */

/* w_i = exp(l_i - m) / S with m = max l, S = sum exp(l - m); ESS = 1/sum w^2;
 * the normaliser log sum_i exp(l_i) = m + log S. */
int orc_normalize(int64_t n, const double* lwt, double* w, double stats[4]) {
  double mx = -INFINITY;
  for (int64_t i = 0; i < n; ++i)
    if (lwt[i] > mx) mx = lwt[i];
  double S = 0.0;
  for (int64_t i = 0; i < n; ++i) S += exp(lwt[i] - mx);
  if (!isfinite(mx) || !isfinite(S) || !(S > 0.0)) return -1;
  double sum_w2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    w[i] = exp(lwt[i] - mx) / S;
    sum_w2 += w[i] * w[i];
  }
  stats[0] = mx;
  stats[1] = log(S);
  stats[2] = 1.0 / sum_w2;
  stats[3] = mx + log(S);
  return 0;
}

void orc_estimate(int64_t n, const double* w, const double* x, double mean[5]) {
  for (int d = 0; d < 5; ++d) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += w[i] * x[d * n + i];
    mean[d] = acc;
  }
}

/* ---------------------------------------------------------- resampling */

void orc_resample_systematic(int64_t n, const double* w, double u, int32_t* anc) {
  int64_t j = 0;
  double C = w[0];
  for (int64_t i = 0; i < n; ++i) {
    const double ui = ((double)i + u) / (double)n;
    while (j < n - 1 && C <= ui) {
      ++j;
      C += w[j];
    }
    anc[i] = (int32_t)j;
  }
}

void orc_resample_rna(int64_t n, int32_t group, int32_t moved, const double* w,
                      const double* u_g, int32_t* anc, double* lwg, double* lw_slot) {
  const int64_t G = n / group;
  int32_t* local = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  for (int64_t g = 0; g < G; ++g) {
    const int64_t base = g * group;
    double W = 0.0;
    for (int32_t l = 0; l < group; ++l) W += w[base + l];
    lwg[g] = log(W / (double)group);
    if (!(W > 0.0)) {
      for (int32_t l = 0; l < group; ++l) local[base + l] = (int32_t)(base + l);
      continue;
    }
    int32_t j = 0;
    double cum = w[base];
    for (int32_t l = 0; l < group; ++l) {
      const double ul = ((double)l + u_g[g]) / (double)group;
      while (j < group - 1 && cum / W <= ul) {
        ++j;
        cum += w[base + j];
      }
      local[base + l] = (int32_t)(base + j);
    }
  }
  for (int64_t g = 0; g < G; ++g) {
    const int64_t prev = (g + G - 1) % G;
    for (int32_t l = 0; l < group; ++l) {
      const int64_t i = g * group + l;
      if (l >= group - moved) {
        anc[i] = local[prev * group + l];
        lw_slot[i] = lwg[prev];
      } else {
        anc[i] = local[i];
        lw_slot[i] = lwg[g];
      }
    }
  }
  free(local);
}

/* ------------------------------------------------------------ the filter */

/* ---------------------------------------------------------------- ARNA */

/* One pass of the ring's keyed permutation of [0, 2^(2 half)): eight Feistel
 * rounds on the halves (L, R) -> (R, L xor F_r(R)), F_r(R) the low `half`
 * bits of word 0 of the Philox block with counter (R, key, RING << 24 | r,
 * track). A Feistel network is a bijection whatever its round function;
 * eight rounds (rather than four) because the halves are tiny for small
 * rings: with four, the orders of 5 groups were measurably uneven. */
static uint32_t ring_feistel(const orc_model* m, uint32_t key, int half, uint32_t x) {
  const uint32_t mask = (1u << half) - 1u;
  uint32_t L = x >> half, R = x & mask;
  for (uint32_t r = 0; r < 8; ++r) {
    uint32_t f[4];
    draw(m, R, key, PURPOSE_RING, r, f);
    const uint32_t nl = R, nr = L ^ (f[0] & mask);
    L = nl;
    R = nr;
  }
  return (L << half) | R;
}

void orc_ring_order(const orc_model* m, int64_t key, int64_t G, int64_t* order) {
  if (key == 0 || G < 2) {
    for (int64_t j = 0; j < G; ++j) order[j] = j;
    return;
  }
  /* the smallest even width b with 2^b >= G; then the permutation of
   * [0, 2^b) restricted to [0, G) by cycle walking: apply it again until the
   * value falls below G (a bijection of [0, G), since every cycle of the
   * permutation that meets [0, G) is walked in the same direction) */
  int b = 2;
  while (((int64_t)1 << b) < G) b += 2;
  for (int64_t j = 0; j < G; ++j) {
    uint32_t x = (uint32_t)j;
    do {
      x = ring_feistel(m, (uint32_t)key, b / 2, x);
    } while ((int64_t)x >= G);
    order[j] = (int64_t)x;
  }
}

int orc_arna_lost(const orc_model* m, double delta, double ref) {
  return delta < ref - m->arna_lost * (double)m->patch;
}

void orc_resample_arna(int64_t n, int32_t group, int32_t mu_min, int32_t mu_max, double theta,
                       const double* w, const double* u_g, const int64_t* order, int32_t* anc,
                       double* lwg, double* lw_slot, int32_t* tracking, int32_t* moved) {
  const int64_t G = n / group;
  int32_t* local = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* pos = (int64_t*)malloc((size_t)G * sizeof(int64_t));
  double* W = (double*)malloc((size_t)G * sizeof(double));
  /* local systematic resampling inside each group, as RNA */
  int64_t t = 0;
  for (int64_t g = 0; g < G; ++g) {
    const int64_t base = g * group;
    double Wg = 0.0;
    for (int32_t l = 0; l < group; ++l) Wg += w[base + l];
    W[g] = Wg;
    lwg[g] = log(Wg / (double)group);
    if (Wg >= theta / (double)G) ++t;
    if (!(Wg > 0.0)) {
      for (int32_t l = 0; l < group; ++l) local[base + l] = (int32_t)(base + l);
      continue;
    }
    int32_t j = 0;
    double cum = w[base];
    for (int32_t l = 0; l < group; ++l) {
      const double ul = ((double)l + u_g[g]) / (double)group;
      while (j < group - 1 && cum / Wg <= ul) {
        ++j;
        cum += w[base + j];
      }
      local[base + l] = (int32_t)(base + j);
    }
  }
  /* the exchange shrinks as more groups track */
  const int64_t mu = mu_min + ((int64_t)(mu_max - mu_min) * (G - t)) / G;
  /* each group's ring predecessor */
  for (int64_t j = 0; j < G; ++j) pos[order[j]] = j;
  for (int64_t g = 0; g < G; ++g) {
    const int64_t pred = order[(pos[g] + G - 1) % G];
    for (int32_t l = 0; l < group; ++l) {
      const int64_t i = g * group + l;
      if (l >= group - mu) {
        anc[i] = local[pred * group + l];
        lw_slot[i] = lwg[pred];
      } else {
        anc[i] = local[i];
        lw_slot[i] = lwg[g];
      }
    }
  }
  *tracking = (int32_t)t;
  *moved = (int32_t)mu;
  free(W);
  free(pos);
  free(local);
}

int orc_run(const orc_model* m, int32_t T, const float* obs, double* mean, double* ess,
            double* delta, int32_t* resampled, double* x_out, double* lw_out, int32_t* anc_out,
            int64_t* arna_out) {
  const int64_t n = m->n;
  double* x = (double*)malloc((size_t)(5 * n) * sizeof(double));
  double* xn = (double*)malloc((size_t)(5 * n) * sizeof(double));
  double* lw = (double*)malloc((size_t)n * sizeof(double));
  double* ll = (double*)malloc((size_t)n * sizeof(double));
  double* w = (double*)malloc((size_t)n * sizeof(double));
  int32_t* parent = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  double* lwg = (double*)malloc((size_t)n * sizeof(double));
  double* ug = (double*)malloc((size_t)n * sizeof(double));
  int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t ring_key = 0;
  double delta_ref = -INFINITY;
  int have_parent = 0, status = 0;
  const int64_t frame_len = m->obs_model == 0 ? (int64_t)m->width * m->height : 3;

  if (orc_init(m, x, lw) != 0) status = -1;
  for (int32_t k = 1; k <= T && status == 0; ++k) {
    const float* z = obs + (int64_t)(k - 1) * frame_len;
    orc_propagate(m, k, x, have_parent ? parent : NULL, xn);
    if (m->obs_model == 0)
      orc_loglik_spot(m, z, xn, ll);
    else
      orc_loglik_lg(m, z, xn, ll);
    for (int64_t i = 0; i < n; ++i) ll[i] += lw[i]; /* w_{k-1} p(z|x~) in logs */
    double st[4], mu[5];
    if (orc_normalize(n, ll, w, st) != 0) {
      status = -k;
      break;
    }
    orc_estimate(n, w, xn, mu);
    if (mean) memcpy(mean + 5 * (k - 1), mu, sizeof mu);
    if (ess) ess[k - 1] = st[2];
    if (delta) delta[k - 1] = st[3];
    const int do_resample = st[2] < m->ess_threshold;
    if (resampled) resampled[k - 1] = do_resample;
    if (lw_out && k == T)
      for (int64_t i = 0; i < n; ++i) lw_out[i] = ll[i] - st[3];
    /* ARNA: a lost object draws a new ring order, kept until the next loss */
    if (m->resample == 2) {
      if (orc_arna_lost(m, st[3], delta_ref))
        ring_key = k;
      else
        delta_ref = st[3];
    }
    int32_t arna_t = 0, arna_mu = 0;
    if (do_resample) {
      if (m->resample == 0) {
        orc_resample_systematic(n, w, orc_resample_uniform(m, k), parent);
        for (int64_t i = 0; i < n; ++i) lw[i] = -log((double)n);
      } else {
        const int64_t G = n / m->rna_group;
        for (int64_t g = 0; g < G; ++g) ug[g] = orc_rna_uniform(m, g, k);
        if (m->resample == 2) {
          orc_ring_order(m, ring_key, G, order);
          orc_resample_arna(n, m->rna_group, m->arna_mu_min, m->rna_moved, m->arna_track, w, ug,
                            order, parent, lwg, lw, &arna_t, &arna_mu);
        } else {
          orc_resample_rna(n, m->rna_group, m->rna_moved, w, ug, parent, lwg, lw);
        }
      }
      have_parent = 1;
    } else {
      for (int64_t i = 0; i < n; ++i) lw[i] = ll[i] - st[3];
      have_parent = 0;
    }
    if (arna_out && m->resample == 2) {
      arna_out[3 * (k - 1)] = ring_key;
      arna_out[3 * (k - 1) + 1] = arna_t;
      arna_out[3 * (k - 1) + 2] = arna_mu;
    }
    double* t = x;
    x = xn;
    xn = t;
  }
  if (status == 0) {
    if (x_out) memcpy(x_out, x, (size_t)(5 * n) * sizeof(double));
    if (anc_out)
      for (int64_t i = 0; i < n; ++i) anc_out[i] = have_parent ? parent[i] : (int32_t)i;
  }
  free(x);
  free(xn);
  free(lw);
  free(ll);
  free(w);
  free(parent);
  free(lwg);
  free(ug);
  free(order);
  return status;
}

/* ------------------------------------------------ derivatives of log p^ */

/*
 * Derivatives of the log-likelihood estimate log p^(z_1:T) = sum_k delta_k
 * (Eq. 1 with the normaliser delta_k of Algorithm 1) with respect to
 *   theta = (s, b, sigma_xi, q_x, q_y, q_vx, q_vy, q_I, I0),
 * I0 being a common offset of every particle's initial intensity, with the
 * Philox noise and the resampling ancestors held fixed (the draws are
 * reparameterised, the discrete ancestor choice is not differentiated). The
 * patch centre c = floor(x + 1/2) is piecewise constant, so it carries no
 * derivative. Under resampling at every step the carried weights are 1/N,
 * and d delta_k / d theta = sum_i w_k^i d l_k^i / d theta with w_k the
 * normalised weights and l_k^i = log p(z_k | x~_k^i).
 */

/* Tangents of the propagated state along each particle's ancestral line
 * (fixed noise z): the near-constant-velocity update x' = x + vx + q_x z_x,
 * vx' = vx + q_vx z_vx (and y, I alike) differentiated in q:
 *   0 dx/dq_x   1 dy/dq_y   2 dvx/dq_vx   3 dx/dq_vx
 *   4 dvy/dq_vy 5 dy/dq_vy  6 dI/dq_I
 * t_prev, t_new: 7 * n SoA; parent NULL = identity. dI/dI0 = 1 throughout. */
void orc_propagate_tangent(const orc_model* m, int64_t k, const double* t_prev,
                           const int32_t* parent, double* t_new) {
  const int64_t n = m->n;
  for (int64_t i = 0; i < n; ++i) {
    double z[5];
    five_normals(m, (uint32_t)i, (uint32_t)k, PURPOSE_PROPAGATE, z);
    const int64_t p = parent ? (int64_t)parent[i] : i;
    double t[7];
    for (int d = 0; d < 7; ++d) t[d] = t_prev[d * n + p];
    t_new[0 * n + i] = t[0] + z[0];        /* x' = x + vx + q_x z_x            */
    t_new[1 * n + i] = t[1] + z[1];
    t_new[2 * n + i] = t[2] + z[2];        /* vx' = vx + q_vx z_vx             */
    t_new[3 * n + i] = t[3] + t[2];        /* x' depends on q_vx through vx    */
    t_new[4 * n + i] = t[4] + z[3];
    t_new[5 * n + i] = t[5] + t[4];
    t_new[6 * n + i] = t[6] + z[4];        /* I' = I + q_I z_I                 */
  }
}

/* Partial derivatives of l = log p(z | x) of Eq. 4 (with its normaliser) per
 * particle, by the chain rule pixel by pixel on the same P x P block as
 * orc_loglik_spot: with r = (u - x)^2 + (v - y)^2, g = exp(-r / (2 s^2)) and
 * the residual R = D - I0 g (D = Z - b inside the frame, 0 outside),
 *   dl/dx     = I0 / (sigma^2 s^2) sum R g (u - x)
 *   dl/dy     = I0 / (sigma^2 s^2) sum R g (v - y)
 *   dl/dI0    = 1 / sigma^2 sum R g
 *   dl/ds     = I0 / (sigma^2 s^3) sum R g r
 *   dl/db     = 1 / sigma^2 sum_{pixels inside the frame} R
 *   dl/dsigma = sum R^2 / sigma^3 - P^2 / sigma
 * dll: 6 * n SoA in that order. */
void orc_loglik_spot_grad(const orc_model* m, const float* frame, const double* x,
                          double* dll) {
  const int64_t n = m->n;
  const int h = (m->patch - 1) / 2;
  const double s = m->s, sg = m->sigma;
  for (int64_t i = 0; i < n; ++i) {
    const double xt = x[0 * n + i], yt = x[1 * n + i], It = x[4 * n + i];
    const double cx = floor(xt + 0.5), cy = floor(yt + 0.5);
    double ss = 0.0, a_g = 0.0, a_x = 0.0, a_y = 0.0, a_r = 0.0, a_in = 0.0;
    for (int dy = -h; dy <= h; ++dy) {
      for (int dx = -h; dx <= h; ++dx) {
        const double u = cx + dx, v = cy + dy;
        const int in = u >= 0.0 && u < (double)m->width && v >= 0.0 && v < (double)m->height;
        const double D = in ? (double)frame[(int64_t)v * m->width + (int64_t)u] - m->b : 0.0;
        const double r = (u - xt) * (u - xt) + (v - yt) * (v - yt);
        const double g = exp(-r / (2.0 * s * s));
        const double R = D - It * g;
        ss += R * R;
        a_g += R * g;
        a_x += R * g * (u - xt);
        a_y += R * g * (v - yt);
        a_r += R * g * r;
        if (in) a_in += R;
      }
    }
    dll[0 * n + i] = It * a_x / (sg * sg * s * s);
    dll[1 * n + i] = It * a_y / (sg * sg * s * s);
    dll[2 * n + i] = a_g / (sg * sg);
    dll[3 * n + i] = It * a_r / (sg * sg * s * s * s);
    dll[4 * n + i] = a_in / (sg * sg);
    dll[5 * n + i] = ss / (sg * sg * sg) - (double)m->patch * (double)m->patch / sg;
  }
}

/* One step's d delta / d theta = sum_i w_i d l_i / d theta (9 values) from
 * the normalised weights w, the partial derivatives dll and the tangents. */
void orc_step_grad(int64_t n, const double* w, const double* dll, const double* tang,
                   double g[9]) {
  for (int d = 0; d < 9; ++d) g[d] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double lx = dll[0 * n + i], ly = dll[1 * n + i], lI = dll[2 * n + i];
    const double v[9] = {dll[3 * n + i], dll[4 * n + i], dll[5 * n + i],
                         lx * tang[0 * n + i], ly * tang[1 * n + i], lx * tang[3 * n + i],
                         ly * tang[5 * n + i], lI * tang[6 * n + i], lI};
    for (int d = 0; d < 9; ++d) g[d] += w[i] * v[d];
  }
}

/* A whole run (spot model, systematic resampling at every step) with the
 * derivatives of cum = sum_k delta_k. anc_replay (T * n, may be NULL)
 * replaces the resampling's ancestors of each step (ancestor replay, so that
 * perturbed runs keep the discrete choices of a base run); anc_out (T * n,
 * may be NULL) records the ancestors used; x_trace (T * 5 * n, may be NULL)
 * the propagated states. Returns 0, -1 for an unsupported model, or -k when
 * frame k had no finite normaliser. */
int orc_run_grad(const orc_model* m, int32_t T, const float* obs, const int32_t* anc_replay,
                 int32_t* anc_out, double* x_trace, double* cum, double grad[9]) {
  if (m->obs_model != 0 || m->resample != 0 || !isinf(m->ess_threshold)) return -1;
  const int64_t n = m->n;
  double* x = (double*)malloc((size_t)(5 * n) * sizeof(double));
  double* xn = (double*)malloc((size_t)(5 * n) * sizeof(double));
  double* t = (double*)calloc((size_t)(7 * n), sizeof(double));
  double* tn = (double*)malloc((size_t)(7 * n) * sizeof(double));
  double* lw = (double*)malloc((size_t)n * sizeof(double));
  double* ll = (double*)malloc((size_t)n * sizeof(double));
  double* dll = (double*)malloc((size_t)(6 * n) * sizeof(double));
  double* w = (double*)malloc((size_t)n * sizeof(double));
  int32_t* parent = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int have_parent = 0, status = 0;
  const int64_t frame_len = (int64_t)m->width * m->height;
  *cum = 0.0;
  for (int d = 0; d < 9; ++d) grad[d] = 0.0;
  if (orc_init(m, x, lw) != 0) status = -1;
  for (int32_t k = 1; k <= T && status == 0; ++k) {
    const float* z = obs + (int64_t)(k - 1) * frame_len;
    orc_propagate(m, k, x, have_parent ? parent : NULL, xn);
    orc_propagate_tangent(m, k, t, have_parent ? parent : NULL, tn);
    if (x_trace) memcpy(x_trace + (int64_t)(k - 1) * 5 * n, xn, (size_t)(5 * n) * sizeof(double));
    orc_loglik_spot(m, z, xn, ll);
    for (int64_t i = 0; i < n; ++i) ll[i] += lw[i];
    double st[4];
    if (orc_normalize(n, ll, w, st) != 0) {
      status = -k;
      break;
    }
    *cum += st[3];
    orc_loglik_spot_grad(m, z, xn, dll);
    double g[9];
    orc_step_grad(n, w, dll, tn, g);
    for (int d = 0; d < 9; ++d) grad[d] += g[d];
    if (anc_replay)
      memcpy(parent, anc_replay + (int64_t)(k - 1) * n, (size_t)n * sizeof(int32_t));
    else
      orc_resample_systematic(n, w, orc_resample_uniform(m, k), parent);
    if (anc_out) memcpy(anc_out + (int64_t)(k - 1) * n, parent, (size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) lw[i] = -log((double)n);
    have_parent = 1;
    double* sw = x;
    x = xn;
    xn = sw;
    sw = t;
    t = tn;
    tn = sw;
  }
  free(x);
  free(xn);
  free(t);
  free(tn);
  free(lw);
  free(ll);
  free(dll);
  free(w);
  free(parent);
  return status;
}

/* ------------------------------------------- RPA and its DLB schedules */

/*
 * Resampling with proportional allocation (RPA, Section 3) over G groups of
 * n consecutive particles standing in for processes: the number of
 * offspring of group g, N_g, is its share of the global systematic
 * resampling (slots i whose (i + u)/N falls in the group's CDF range), so
 * heavy groups produce more than n offspring (senders, surplus N_g - n) and
 * light ones fewer (receivers, deficit n - N_g). The DLB schedules of
 * Section 4 route the surplus so that every group ends with n particles.
 */

/* Offspring counts N_g (G values) from the ancestors of global systematic
 * resampling. */
void orc_rpa_counts(int64_t n_total, int32_t group, const int32_t* anc_sys, int32_t* counts) {
  const int64_t G = n_total / group;
  for (int64_t g = 0; g < G; ++g) counts[g] = 0;
  for (int64_t i = 0; i < n_total; ++i) counts[anc_sys[i] / group] += 1;
}

/* Sort the entries idx[0..m) by key[idx] descending, ties by index
 * ascending (insertion sort: plain and stable). */
static void sort_desc(int32_t* idx, int64_t m, const int64_t* key) {
  for (int64_t a = 1; a < m; ++a) {
    const int32_t v = idx[a];
    int64_t b = a;
    while (b > 0 && key[idx[b - 1]] < key[v]) {
      idx[b] = idx[b - 1];
      --b;
    }
    idx[b] = v;
  }
}

/*
 * DLB schedule over the groups' counts (kind 0 = Greedy, Alg. 2; 1 = Sorted
 * Greedy, Alg. 3; 2 = Largest Gradient, Alg. 4). Senders are the groups with
 * counts[g] > n, receivers those with counts[g] < n, each listed in group
 * order (GS) or by surplus / deficit descending (SGS, LGS; ties by group).
 * Writes up to `cap` entries (sender group, receiver group, particles) to
 * sched (3 per entry) and returns their number (-1 if cap is too small or
 * the working lists cannot be allocated).
 *   GS/SGS: each sender in turn fills the current receiver; a filled
 *           receiver is skipped and the next one taken (the printed loop
 *           resets j to 0 and never ends on a filled receiver; the reading
 *           keeps j and skips, which gives the balance the text states);
 *   LGS:    the i-th sender pairs with the i-th receiver for
 *           min(|S|, |R|) ranks, moving min(surplus, deficit) particles (the
 *           printed else branch zeroes the surplus before recording it; the
 *           reading records it, then zeroes it).
 */
int64_t orc_dlb_schedule(int kind, int64_t G, int32_t n, const int32_t* counts, int64_t cap,
                         int32_t* sched) {
  if (G <= 0) return 0;
  int64_t* surplus = (int64_t*)calloc((size_t)G, sizeof(int64_t));
  int64_t* deficit = (int64_t*)calloc((size_t)G, sizeof(int64_t));
  int32_t* S = (int32_t*)malloc((size_t)G * sizeof(int32_t));
  int32_t* R = (int32_t*)malloc((size_t)G * sizeof(int32_t));
  if (!surplus || !deficit || !S || !R) {
    free(surplus);
    free(deficit);
    free(S);
    free(R);
    return -1;
  }
  int64_t ns = 0, nr = 0, m = 0;
  for (int64_t g = 0; g < G; ++g) {
    surplus[g] = counts[g] > n ? (int64_t)counts[g] - n : 0;
    deficit[g] = counts[g] < n ? (int64_t)n - counts[g] : 0;
    if (surplus[g] > 0) S[ns++] = (int32_t)g;
    if (deficit[g] > 0) R[nr++] = (int32_t)g;
  }
  if (kind != 0) {
    sort_desc(S, ns, surplus);
    sort_desc(R, nr, deficit);
  }
  if (kind == 2) {
    const int64_t c = ns < nr ? ns : nr;
    for (int64_t i = 0; i < c; ++i) {
      int64_t moved;
      if (surplus[S[i]] >= deficit[R[i]]) {
        moved = deficit[R[i]];
        surplus[S[i]] -= moved;
      } else {
        moved = surplus[S[i]];
        surplus[S[i]] = 0;
      }
      if (m >= cap) { m = -1; break; }
      sched[3 * m] = S[i];
      sched[3 * m + 1] = R[i];
      sched[3 * m + 2] = (int32_t)moved;
      ++m;
    }
  } else {
    int64_t j = 0;
    for (int64_t i = 0; i < ns && m >= 0; ++i) {
      while (surplus[S[i]] != 0) {
        while (j < nr && deficit[R[j]] == 0) ++j;  /* skip filled receivers */
        if (j >= nr) break;                         /* not reached when balanced */
        const int64_t moved = surplus[S[i]] >= deficit[R[j]] ? deficit[R[j]] : surplus[S[i]];
        if (m >= cap) { m = -1; break; }
        sched[3 * m] = S[i];
        sched[3 * m + 1] = R[j];
        sched[3 * m + 2] = (int32_t)moved;
        ++m;
        surplus[S[i]] -= moved;
        deficit[R[j]] -= moved;
      }
    }
  }
  free(surplus);
  free(deficit);
  free(S);
  free(R);
  return m;
}

/*
 * RPA resampling with a balancing schedule (kind 0 = GS, 1 = SGS): the
 * offspring of each group are its slots of the global systematic resampling
 * (anc_sys, in slot order); a group keeps its first min(N_g, n) offspring in
 * its own slots [g n, g n + min(N_g, n)); then the schedule's entries, in
 * order, move `particles` of the sender's remaining offspring (in order)
 * into the receiver's next free slots. anc: n_total ancestors out. Returns
 * 0, or -1 when a group is left unbalanced.
 */
int orc_resample_rpa(int64_t n_total, int32_t group, int kind, const int32_t* anc_sys,
                     int32_t* anc) {
  const int64_t G = n_total / group;
  int32_t* counts = (int32_t*)malloc((size_t)G * sizeof(int32_t));
  int64_t* first = (int64_t*)malloc((size_t)G * sizeof(int64_t));
  int64_t* next_out = (int64_t*)malloc((size_t)G * sizeof(int64_t)); /* sender: next offspring */
  int64_t* fill = (int64_t*)malloc((size_t)G * sizeof(int64_t));     /* receiver: slots filled */
  int32_t* sched = (int32_t*)malloc((size_t)(3 * 2 * G + 3) * sizeof(int32_t));
  int status = 0;
  orc_rpa_counts(n_total, group, anc_sys, counts);
  int64_t acc = 0;
  for (int64_t g = 0; g < G; ++g) {
    first[g] = acc; /* slots of group g's offspring in anc_sys */
    acc += counts[g];
    const int64_t keep = counts[g] < group ? counts[g] : group;
    for (int64_t p = 0; p < keep; ++p) anc[g * group + p] = anc_sys[first[g] + p];
    next_out[g] = keep;
    fill[g] = keep;
  }
  const int64_t m = orc_dlb_schedule(kind, G, group, counts, 2 * G + 1, sched);
  if (m < 0) status = -1;
  for (int64_t e = 0; e < m; ++e) {
    const int32_t s = sched[3 * e], r = sched[3 * e + 1], c = sched[3 * e + 2];
    for (int32_t q = 0; q < c; ++q)
      anc[(int64_t)r * group + fill[r]++] = anc_sys[first[s] + next_out[s]++];
  }
  for (int64_t g = 0; g < G; ++g)
    if (fill[g] != group || next_out[g] != counts[g]) status = -1;
  free(counts);
  free(first);
  free(next_out);
  free(fill);
  free(sched);
  return status;
}
