// HIP kernels of the SIR filter step for gfx950 (CDNA4, wave64).
//
// One step of Algorithm 1 (Section 2) is four launches on one stream, with
// every decision taken on the device:
//   k_step      gather parent + propagate (Section 6.1) + patch likelihood
//               (Eqs. 3-4, Section 5.5) + per-workgroup log-sum-exp record
//   k_reduce    first fixed-order merge of the records (large N only)
//   k_finalize  fixed-order fp64 merge: normaliser, ESS, MMSE estimate,
//               resampling decision and uniform; commit or roll back
//   k_scan      systematic resampling: single-pass decoupled look-back scan
//               of the normalised weights in 2^60 fixed point, and the
//               ancestor walk for each tile's output slots
//   k_heavy     load-balanced ancestor writing for tiles owning many slots
//   (or k_rna   RNA of Section 3: one workgroup per group of particles)
#include "ppf_internal.hpp"

#include <cfloat>
#include <climits>
#include <cmath>

namespace ppf {
namespace {

// ------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32-bit
// multiplications whose high halves are xored with the other counter words
// and a Weyl-sequence round key.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ uint4 draw(const Model& m, uint32_t index, uint32_t k,
                                      uint32_t purpose, uint32_t block) {
  return philox(make_uint4(index, k, (purpose << 24) | block, m.track), m.key0, m.key1);
}

// Uniforms from the top 24 bits: [0, 1) and (0, 1], exact in fp32.
__device__ __forceinline__ float u24_open_hi(uint32_t a) { return (float)(a >> 8) * 0x1p-24f; }
__device__ __forceinline__ float u24_open_lo(uint32_t a) {
  return (float)((a >> 8) + 1u) * 0x1p-24f;
}
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  return ((double)a * 2097152.0 + (double)(b >> 11)) * 0x1p-53;
}

// Box-Muller in fp32: radius from (0, 1], angle 2 pi u from [0, 1).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float rad = sqrtf(-2.0f * logf(u24_open_lo(a)));
  float s, c;
  sincospif(2.0f * u24_open_hi(b), &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

__device__ __forceinline__ void box_muller64(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double rad = sqrt(-2.0 * log((double)u24_open_lo(a)));
  double s, c;
  sincospi(2.0 * (double)u24_open_hi(b), &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

// -------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Normalisation record: (m, S, S2, sum e x_d) with e = exp(l - m).
struct Rec {
  double m, S, S2, ex[5];
};

__device__ __forceinline__ Rec rec_empty() {
  Rec r;
  r.m = -INFINITY;
  r.S = r.S2 = 0.0;
#pragma unroll
  for (int d = 0; d < 5; ++d) r.ex[d] = 0.0;
  return r;
}

__device__ __forceinline__ Rec rec_load(const double* p) {
  Rec r;
  r.m = p[0];
  r.S = p[1];
  r.S2 = p[2];
#pragma unroll
  for (int d = 0; d < 5; ++d) r.ex[d] = p[3 + d];
  return r;
}

__device__ __forceinline__ void rec_store(double* p, const Rec& r) {
  p[0] = r.m;
  p[1] = r.S;
  p[2] = r.S2;
#pragma unroll
  for (int d = 0; d < 5; ++d) p[3 + d] = r.ex[d];
}

// Merge of two records onto the larger maximum; NaN sums propagate.
__device__ __forceinline__ Rec rec_merge(const Rec& a, const Rec& b) {
  const double m = fmax(a.m, b.m);
  if (m == -INFINITY) {
    Rec r = a;
    r.S = a.S + b.S;  // both empty: keeps a NaN marker if any
    r.S2 = a.S2 + b.S2;
    return r;
  }
  const double fa = (a.m == -INFINITY) ? 0.0 : exp(a.m - m);
  const double fb = (b.m == -INFINITY) ? 0.0 : exp(b.m - m);
  Rec r;
  r.m = m;
  r.S = a.S * fa + b.S * fb;
  r.S2 = a.S2 * fa * fa + b.S2 * fb * fb;
#pragma unroll
  for (int d = 0; d < 5; ++d) r.ex[d] = a.ex[d] * fa + b.ex[d] * fb;
  return r;
}

// Fixed-order tree merge of one Rec per thread in a 256-thread workgroup.
__device__ Rec block_merge_256(Rec r, Rec* sh) {
  const int t = threadIdx.x;
  sh[t] = r;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = rec_merge(sh[t], sh[t + s]);
    __syncthreads();
  }
  Rec out = sh[0];
  __syncthreads();
  return out;
}

// ------------------------------------------------------------ k_init
// Algorithm 1 initialisation, k = 0. The state is computed in fp64 and
// rounded once to fp32.
__global__ __launch_bounds__(256) void k_init(Model m, Buffers b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    Ctrl* c = b.ctrl;
    c->k = 0;
    c->cur = 0;
    c->mode = kModeInit;
    c->resampled = 0;
    c->rolled_back = 0;
    c->do_resample = 0;
    c->heavy_count = 0;
    c->tile_counter = 0;
    c->m = c->log_sum = c->ess = c->delta = c->cum = 0.0;
    for (int d = 0; d < 5; ++d) c->mean[d] = 0.0;
    c->u = 0.0;
  }
  if (i >= m.n) return;
  const uint4 r0 = draw(m, (uint32_t)i, 0u, kInit, 0u);
  const uint4 r1 = draw(m, (uint32_t)i, 0u, kInit, 1u);
  double x[5];
  if (m.init_kind == 1) {  // Gaussian
    double z[5], unused;
    box_muller64(r0.x, r0.y, z[0], z[1]);
    box_muller64(r0.z, r0.w, z[2], z[3]);
    box_muller64(r1.x, r1.y, z[4], unused);
#pragma unroll
    for (int d = 0; d < 5; ++d) x[d] = (double)m.init_a[d] + (double)m.init_b[d] * z[d];
  } else {
    const uint32_t w[5] = {r0.x, r0.y, r0.z, r0.w, r1.x};
    double f[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) f[d] = (double)u24_open_hi(w[d]);
    if (m.init_kind == 2) {  // stratified over (x, y) in Z order
      const int t = m.strat_t;
      const uint64_t cell = ((uint64_t)i << t) / (uint64_t)m.n;
      uint32_t cx = 0, cy = 0;
      int bx = 0, by = 0;
      for (int j = 0; j < t; ++j) {
        const uint32_t bit = (uint32_t)(cell >> j) & 1u;
        if ((j & 1) == 0)
          cx |= bit << bx++;
        else
          cy |= bit << by++;
      }
      const double fx = ((double)cx + (double)u24_open_hi(r0.x)) / ldexp(1.0, (t + 1) / 2);
      const double fy = ((double)cy + (double)u24_open_hi(r0.y)) / ldexp(1.0, t / 2);
      f[0] = fx;
      f[1] = fy;
      f[2] = (double)u24_open_hi(r0.z);
      f[3] = (double)u24_open_hi(r0.w);
      f[4] = (double)u24_open_hi(r1.x);
    }
#pragma unroll
    for (int d = 0; d < 5; ++d)
      x[d] = (double)m.init_a[d] + ((double)m.init_b[d] - (double)m.init_a[d]) * f[d];
  }
#pragma unroll
  for (int d = 0; d < 5; ++d) b.X0[(int64_t)d * m.n + i] = (float)x[d];
}

// ------------------------------------------------------------ k_step
// Parent, carried log weight and propagated state of particle i.
struct Prop {
  float x, y, vx, vy, I;
  double lw;
};

__device__ __forceinline__ Prop propagate(const Model& m, const Buffers& b, const Ctrl& c,
                                          int64_t i, uint32_t k) {
  const int cur = c.cur;
  const float* Xin = cur ? b.X1 : b.X0;
  const int mode = c.mode;
  int64_t p = i;
  double lw;
  if (mode == kModeSys || mode == kModeRna) p = b.anc[i];
  if (mode == kModeNone) {
    const float* Lin = cur ? b.L1 : b.L0;
    const double* Rin = cur ? b.R1 : b.R0;
    lw = (double)Lin[i] + Rin[(i / kBlock) * kRec] - c.delta;
  } else if (mode == kModeRna) {
    const int64_t g = i / m.group;
    const int64_t l = i - g * m.group;
    const int64_t src = (l >= m.group - m.moved) ? (g + m.G - 1) % m.G : g;
    lw = b.lwg[src];
  } else if (mode == kModeSet) {
    lw = b.lw64[i];
  } else {
    lw = -m.log_n;
  }
  const int64_t n = m.n;
  const float px = Xin[p], py = Xin[n + p], pvx = Xin[2 * n + p], pvy = Xin[3 * n + p],
              pI = Xin[4 * n + p];
  const uint4 r0 = draw(m, (uint32_t)i, k, kPropagate, 0u);
  const uint4 r1 = draw(m, (uint32_t)i, k, kPropagate, 1u);
  float z0, z1, z2, z3, z4, unused;
  box_muller(r0.x, r0.y, z0, z1);
  box_muller(r0.z, r0.w, z2, z3);
  box_muller(r1.x, r1.y, z4, unused);
  Prop o;
  // near-constant velocity, unit frame interval; fp64 sum rounded once
  o.x = (float)((double)px + (double)pvx + (double)m.q[0] * (double)z0);
  o.y = (float)((double)py + (double)pvy + (double)m.q[1] * (double)z1);
  o.vx = (float)((double)pvx + (double)m.q[2] * (double)z2);
  o.vy = (float)((double)pvy + (double)m.q[3] * (double)z3);
  o.I = (float)((double)pI + (double)m.q[4] * (double)z4);
  o.lw = lw;
  return o;
}

// Block-wide reduction of the step's log weights into one record, and the
// stored value l - m_b per particle.
__device__ __forceinline__ void finish_block(const Model& m, const Buffers& b, const Ctrl& c,
                                             int64_t i, bool active, double l, const Prop& o,
                                             double* red) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double mv = wave_max(active ? l : -INFINITY);
  if (lane == 0) red[w] = mv;
  __syncthreads();
  const double mb = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  double e = 0.0;
  if (active) {
    if (isnan(l))
      e = NAN;
    else if (mb != -INFINITY)
      e = exp(l - mb);
  }
  double v[7] = {e, e * e, e * (double)o.x, e * (double)o.y, e * (double)o.vx, e * (double)o.vy,
                 e * (double)o.I};
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    v[j] = wave_sum(v[j]);
    if (lane == 0) red[8 + w * 7 + j] = v[j];
  }
  const int nxt = c.cur ^ 1;
  if (active) {
    float* Lout = nxt ? b.L1 : b.L0;
    Lout[i] = (mb == -INFINITY) ? -INFINITY : (float)(l - mb);
  }
  __syncthreads();
  if (t < 7) {
    const double s = (red[8 + t] + red[8 + 7 + t]) + (red[8 + 14 + t] + red[8 + 21 + t]);
    double* Rout = nxt ? b.R1 : b.R0;
    Rout[(int64_t)blockIdx.x * kRec + 1 + t] = s;
    if (t == 0) Rout[(int64_t)blockIdx.x * kRec] = mb;
  }
}

__device__ __forceinline__ void store_state(const Model& m, const Buffers& b, const Ctrl& c,
                                            int64_t i, const Prop& o) {
  float* Xout = c.cur ? b.X0 : b.X1;
  const int64_t n = m.n;
  Xout[i] = o.x;
  Xout[n + i] = o.y;
  Xout[2 * n + i] = o.vx;
  Xout[3 * n + i] = o.vy;
  Xout[4 * n + i] = o.I;
}

// Sum over the P x P patch of (D - I g_x g_y)^2 with D = Z - b (0 outside the
// frame). g_x, g_y are the 1-D Gaussian factors of Eq. 3 at the pixel
// offsets d - f, built by the exact recurrence
//   g(d+1) = g(d) exp(-(2d+1)/(2 s^2)) exp(f/s^2).
template <int P, bool LDS>
__device__ __forceinline__ double patch_sumsq(const float* __restrict__ src, int64_t row_stride,
                                              int64_t first, int u0, int v0, int W, int H,
                                              float bf, double b, const double (&gx)[P],
                                              double gy, double by, const double* cst,
                                              double It) {
  double acc = 0.0;
  // rows stay rolled (full P x P unrolling hoists every load and spills)
#pragma unroll 1
  for (int dy = 0; dy < P; ++dy) {
    const double my = It * gy;
    if (LDS) {
      const float* row = src + first + dy * row_stride;
#pragma unroll
      for (int dx = 0; dx < P; ++dx) {
        const double r = fma(-my, gx[dx], (double)row[dx] - b);
        acc = fma(r, r, acc);
      }
    } else {
      const int v = v0 + dy;
      const bool row_in = (unsigned)v < (unsigned)H;
      const float* row = src + (int64_t)(row_in ? v : 0) * W;
#pragma unroll
      for (int dx = 0; dx < P; ++dx) {
        const int u = u0 + dx;
        const float z = (row_in && (unsigned)u < (unsigned)W) ? row[u] : bf;
        const double r = fma(-my, gx[dx], (double)z - b);
        acc = fma(r, r, acc);
      }
    }
    if (dy + 1 < P) gy *= cst[dy] * by;
  }
  return acc;
}

template <int P>
__global__ __launch_bounds__(256) void k_step_spot(Model m, Buffers b,
                                                   const float* __restrict__ obs) {
  __shared__ float tile[kTileCap];
  __shared__ double cst[P];
  __shared__ double red[8 + 4 * 7];
  __shared__ int ired[16];
  constexpr int h = (P - 1) / 2;
  const Ctrl c = *b.ctrl;
  const uint32_t k = (uint32_t)(c.k + 1);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * kBlock + t;
  const bool active = i < m.n;
  if (t < P - 1) cst[t] = exp(-(2.0 * (double)(t - h) + 1.0) * m.inv2s2);

  Prop o{};
  double fx = 0.0, fy = 0.0;
  int cx = 0, cy = 0;
  if (active) {
    o = propagate(m, b, c, i, k);
    store_state(m, b, c, i, o);
    // patch centre: pixel nearest to (x, y); the offset f is exact in fp64
    const double rx = floor((double)o.x + 0.5), ry = floor((double)o.y + 0.5);
    fx = (double)o.x - rx;
    fy = (double)o.y - ry;
    // addresses only: far-away centres are clamped where the whole patch
    // already lies outside the frame (their pixels read as background)
    const double lox = -(double)P, hix = (double)m.W + P, loy = -(double)P, hiy = (double)m.H + P;
    cx = (rx >= lox && rx <= hix) ? (int)rx : (rx > hix ? (int)hix : (int)lox);
    cy = (ry >= loy && ry <= hiy) ? (int)ry : (ry > hiy ? (int)hiy : (int)loy);
  }
  // bounding box of the workgroup's patches
  int mnx = wave_min_i(active ? cx : INT_MAX), mxx = wave_max_i(active ? cx : INT_MIN);
  int mny = wave_min_i(active ? cy : INT_MAX), mxy = wave_max_i(active ? cy : INT_MIN);
  if (lane == 0) {
    ired[w] = mnx;
    ired[4 + w] = mxx;
    ired[8 + w] = mny;
    ired[12 + w] = mxy;
  }
  __syncthreads();
  mnx = min(min(ired[0], ired[1]), min(ired[2], ired[3]));
  mxx = max(max(ired[4], ired[5]), max(ired[6], ired[7]));
  mny = min(min(ired[8], ired[9]), min(ired[10], ired[11]));
  mxy = max(max(ired[12], ired[13]), max(ired[14], ired[15]));
  const int64_t tw = (int64_t)mxx - mnx + P, th = (int64_t)mxy - mny + P;
  const bool use_lds = tw * th <= kTileCap;  // uniform across the workgroup
  const int tx0 = mnx - h, ty0 = mny - h;
  if (use_lds) {
    const int area = (int)(tw * th);
    for (int j = t; j < area; j += kBlock) {
      const int ty = j / (int)tw;
      const int u = tx0 + (j - ty * (int)tw), v = ty0 + ty;
      tile[j] = ((unsigned)u < (unsigned)m.W && (unsigned)v < (unsigned)m.H)
                    ? obs[(int64_t)v * m.W + u]
                    : m.bf;
    }
  }
  __syncthreads();

  double l = -INFINITY;
  if (active) {
    double gx[P];
    gx[0] = exp(-((double)h + fx) * ((double)h + fx) * m.inv2s2);
    const double bx = exp(2.0 * fx * m.inv2s2);
#pragma unroll
    for (int d = 0; d + 1 < P; ++d) gx[d + 1] = gx[d] * (cst[d] * bx);
    const double gy0 = exp(-((double)h + fy) * ((double)h + fy) * m.inv2s2);
    const double by = exp(2.0 * fy * m.inv2s2);
    double acc;
    if (use_lds) {
      const int64_t first = (int64_t)(cy - h - ty0) * tw + (cx - h - tx0);
      acc = patch_sumsq<P, true>(tile, tw, first, 0, 0, 0, 0, m.bf, m.b, gx, gy0, by, cst,
                                 (double)o.I);
    } else {
      acc = patch_sumsq<P, false>(obs, 0, 0, cx - h, cy - h, m.W, m.H, m.bf, m.b, gx, gy0, by,
                                  cst, (double)o.I);
    }
    l = o.lw - acc * m.inv2sig2 - m.lognorm_obs;
  }
  finish_block(m, b, c, i, active, l, o, red);
}

// Linear-Gaussian observation of (x, y, I0): three fp32 values on the device.
__global__ __launch_bounds__(256) void k_step_lg(Model m, Buffers b,
                                                 const float* __restrict__ obs) {
  __shared__ double red[8 + 4 * 7];
  const Ctrl c = *b.ctrl;
  const uint32_t k = (uint32_t)(c.k + 1);
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < m.n;
  Prop o{};
  double l = -INFINITY;
  if (active) {
    o = propagate(m, b, c, i, k);
    store_state(m, b, c, i, o);
    const double ex = (double)obs[0] - (double)o.x, ey = (double)obs[1] - (double)o.y,
                 eI = (double)obs[2] - (double)o.I;
    l = o.lw - ex * ex * m.lg_inv2r2[0] - ey * ey * m.lg_inv2r2[1] - eI * eI * m.lg_inv2r2[2] -
        m.lg_norm;
  }
  finish_block(m, b, c, i, active, l, o, red);
}

// ------------------------------------------------------- records merging
// First merge level: workgroup j merges a contiguous chunk of level-1
// records in a fixed order.
__global__ __launch_bounds__(256) void k_reduce(Buffers b, int standalone) {
  __shared__ Rec sh[256];
  // the step wrote its records into the buffer that finalize will make current
  const double* R = (!standalone && (b.ctrl->cur ^ 1)) ? b.R1 : b.R0;
  const int64_t chunk = (b.nb + b.nr2 - 1) / b.nr2;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = min(b.nb, lo + chunk);
  Rec r = rec_empty();
  for (int64_t j = lo + threadIdx.x; j < hi; j += 256) r = rec_merge(r, rec_load(R + j * kRec));
  r = block_merge_256(r, sh);
  if (threadIdx.x == 0) rec_store(b.R2 + (int64_t)blockIdx.x * kRec, r);
}

// Final merge, statistics of Algorithm 1 and the commit of the step.
__global__ __launch_bounds__(256) void k_finalize(Model m, Buffers b, int standalone,
                                                  double u_given) {
  __shared__ Rec sh[256];
  Ctrl* c = b.ctrl;
  const int which = standalone ? 0 : (c->cur ^ 1);
  const double* R = b.nr2 ? b.R2 : (which ? b.R1 : b.R0);
  const int64_t cnt = b.nr2 ? b.nr2 : b.nb;
  Rec r = rec_empty();
  for (int64_t j = threadIdx.x; j < cnt; j += 256) r = rec_merge(r, rec_load(R + j * kRec));
  r = block_merge_256(r, sh);
  const bool ok = isfinite(r.m) && isfinite(r.S) && r.S > 0.0;
  if (threadIdx.x == 0) {
    if (standalone) {
      c->cur = 0;
      c->delta = ok ? r.m + log(r.S) : 0.0;
      c->u = u_given;
      c->do_resample = ok ? 1 : 0;
      c->k = 0;
    } else if (ok) {
      const int64_t k = c->k + 1;
      const double ess = r.S * r.S / r.S2;
      const double logS = log(r.S);
      const bool res = ess < m.thr;
      c->k = k;
      c->cur ^= 1;
      c->m = r.m;
      c->log_sum = logS;
      c->ess = ess;
      c->delta = r.m + logS;
      c->cum += r.m + logS;
      for (int d = 0; d < 5; ++d) c->mean[d] = r.ex[d] / r.S;
      c->resampled = res ? 1 : 0;
      c->do_resample = res ? 1 : 0;
      c->mode = res ? (m.group > 0 ? kModeRna : kModeSys) : kModeNone;
      const uint4 rr = draw(m, 0u, (uint32_t)k, kResample, 0u);
      c->u = u53(rr.x, rr.y);
    } else {
      c->rolled_back += 1;
      c->do_resample = 0;
    }
    c->tile_counter = 0u;
    c->heavy_count = 0;
  }
  for (int64_t j = threadIdx.x; j < b.ntiles; j += 256) b.desc[j] = 0ull;
}

// --------------------------------------------------- systematic resampling
__device__ __forceinline__ uint64_t slot_u(int64_t s, double u, double inv_n) {
  const double q = ((double)s + u) * inv_n;
  return (uint64_t)(q * 0x1p60);
}

// Number of output slots s in [0, n) with U(s) < C.
__device__ int64_t slot_count(uint64_t C, double u, double inv_n, int64_t n) {
  const double est = (double)C * 0x1p-60 * (double)n - u;
  int64_t s = est <= 0.0 ? 0 : (est >= (double)n ? n : (int64_t)ceil(est));
  while (s > 0 && slot_u(s - 1, u, inv_n) >= C) --s;
  while (s < n && slot_u(s, u, inv_n) < C) ++s;
  return s;
}

__device__ __forceinline__ void weight_src(const WeightSrc& w, const Ctrl* c, const float*& val,
                                           const double*& off) {
  const int cur = w.use_cur ? c->cur : 0;
  val = cur ? w.val1 : w.val0;
  off = cur ? w.off1 : w.off0;
}

// Fixed-point weights of one tile, local inclusive CDF into C (blocked:
// thread t owns items 8t..8t+7). Returns the tile total.
__device__ uint64_t tile_cdf(const WeightSrc& ws, const Ctrl* c, int64_t base, int64_t n,
                             double lognorm, uint64_t* C, uint64_t* wsum) {
  const float* val;
  const double* off;
  weight_src(ws, c, val, off);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int li = j * kScanThreads + t;
    const int64_t idx = base + li;
    uint64_t wf = 0;
    if (idx < n) {
      const double lw = (double)val[idx] + off[(idx / kBlock) * ws.stride] - lognorm;
      wf = __double2ull_rn(exp(lw) * 0x1p60);
    }
    C[li] = wf;
  }
  __syncthreads();
  uint64_t v[kScanItems];
  uint64_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    run += C[t * kScanItems + j];
    v[j] = run;
  }
  const uint64_t incl = wave_incl_scan_u64(run, lane);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint64_t before = 0;
  for (int j = 0; j < w; ++j) before += wsum[j];
  const uint64_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  const uint64_t texcl = before + incl - run;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) C[t * kScanItems + j] = texcl + v[j];
  __syncthreads();
  return total;
}

// Ancestors of slots [s0, s1): the two-pointer walk s(i) = min{ j : U(i) <
// C_j } over the tile's global inclusive CDF (C + excl), clamped to the last
// valid item.
__device__ __forceinline__ void walk_slots(const uint64_t* C, uint64_t excl, int nvalid,
                                           int64_t base, int64_t s0, int64_t s1, double u,
                                           double inv_n, int32_t* __restrict__ anc) {
  if (s0 >= s1) return;
  uint64_t us = slot_u(s0, u, inv_n);
  int lo = 0, hi = nvalid - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid] + excl > us)
      hi = mid;
    else
      lo = mid + 1;
  }
  int j = lo;
  for (int64_t s = s0; s < s1; ++s) {
    us = slot_u(s, u, inv_n);
    while (j < nvalid - 1 && C[j] + excl <= us) ++j;
    anc[s] = (int32_t)(base + j);
  }
}

__global__ __launch_bounds__(256) void k_scan(Model m, Buffers b, WeightSrc ws) {
  __shared__ uint64_t C[kTile];
  __shared__ uint64_t wsum[4];
  __shared__ uint64_t sh_excl;
  __shared__ uint32_t sh_tile;
  Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  if (threadIdx.x == 0) sh_tile = atomicAdd(&c->tile_counter, 1u);
  __syncthreads();
  const int64_t t = sh_tile;
  const int64_t n = m.n;
  const int64_t base = t * kTile;
  const double lognorm = c->delta;
  const double u = c->u;
  const uint64_t A = tile_cdf(ws, c, base, n, lognorm, C, wsum);

  // decoupled look-back (one wave), tile ids handed out in launch order
  const int lane = threadIdx.x & 63;
  if (t == 0) {
    if (threadIdx.x == 0) {
      __hip_atomic_store(&b.desc[0], kFlagPrefix | A, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      sh_excl = 0;
    }
  } else if (threadIdx.x < 64) {
    if (lane == 0)
      __hip_atomic_store(&b.desc[t], kFlagAggregate | A, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int64_t j = t - 1;
    while (true) {
      const int64_t idx = j - lane;
      uint64_t d = kFlagPrefix;  // before tile 0: an empty prefix
      if (idx >= 0) {
        do {
          d = __hip_atomic_load(&b.desc[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } while ((d >> 62) == 0);
      }
      const uint64_t pmask = __ballot((d >> 62) == 2);
      const int first = pmask ? (__ffsll((long long)pmask) - 1) : 64;
      excl += wave_sum_u64(lane <= first ? (d & kValueMask) : 0ull);
      if (pmask) break;
      j -= 64;
    }
    if (lane == 0) {
      __hip_atomic_store(&b.desc[t], kFlagPrefix | (excl + A), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      sh_excl = excl;
    }
  }
  __syncthreads();
  const uint64_t excl = sh_excl;
  const double inv_n = m.inv_n;
  const int64_t o_lo = slot_count(excl, u, inv_n, n);
  const int64_t o_hi = (t == b.ntiles - 1) ? n : slot_count(excl + A, u, inv_n, n);
  const int64_t M = o_hi - o_lo;
  if (M > (int64_t)kHeavyFactor * kTile) {
    if (threadIdx.x == 0) {
      const int hq = atomicAdd(&c->heavy_count, 1);
      b.heavy[2 * hq] = (uint64_t)t;
      b.heavy[2 * hq + 1] = excl;
    }
    return;
  }
  const int nvalid = (int)min((int64_t)kTile, n - base);
  const int64_t per = (M + kScanThreads - 1) / kScanThreads;
  const int64_t s0 = o_lo + (int64_t)threadIdx.x * per;
  walk_slots(C, excl, nvalid, base, s0, min(o_hi, s0 + per), u, inv_n, b.anc);
}

// Tiles with many output slots: every workgroup takes chunks of each queued
// tile round-robin, so one heavy particle's offspring are written by the
// whole GPU.
__global__ __launch_bounds__(256) void k_heavy(Model m, Buffers b, WeightSrc ws) {
  __shared__ uint64_t C[kTile];
  __shared__ uint64_t wsum[4];
  Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int nh = c->heavy_count;
  const int64_t n = m.n;
  const double lognorm = c->delta, u = c->u, inv_n = m.inv_n;
  for (int hq = 0; hq < nh; ++hq) {
    const int64_t t = (int64_t)b.heavy[2 * hq];
    const uint64_t excl = b.heavy[2 * hq + 1];
    const int64_t base = t * kTile;
    const uint64_t A = tile_cdf(ws, c, base, n, lognorm, C, wsum);
    const int64_t o_lo = slot_count(excl, u, inv_n, n);
    const int64_t o_hi = (t == b.ntiles - 1) ? n : slot_count(excl + A, u, inv_n, n);
    const int64_t nchunks = (o_hi - o_lo + kHeavyChunk - 1) / kHeavyChunk;
    const int nvalid = (int)min((int64_t)kTile, n - base);
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
      const int64_t c0 = o_lo + ch * kHeavyChunk;
      const int64_t c1 = min(o_hi, c0 + kHeavyChunk);
      constexpr int per = kHeavyChunk / kScanThreads;
      const int64_t s0 = c0 + (int64_t)threadIdx.x * per;
      walk_slots(C, excl, nvalid, base, s0, min(c1, s0 + per), u, inv_n, b.anc);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------- RNA
// One workgroup per group g (Section 3): local systematic resampling of the
// group's normalised weights, slot weight W_g / n, and the last `moved` slots
// taken from group g-1's local resampling (recomputed here, so no workgroup
// waits for another).
__global__ __launch_bounds__(256) void k_rna(Model m, Buffers b, WeightSrc ws,
                                             const double* __restrict__ u_dev) {
  __shared__ uint64_t C[2][kMaxGroup];
  __shared__ double dsum[4];
  __shared__ uint64_t wsum[4];
  Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const float* val;
  const double* off;
  weight_src(ws, c, val, off);
  const int64_t g = blockIdx.x;
  const int ng = m.group;
  const int64_t G = m.G;
  const int64_t prev = (g + G - 1) % G;
  const double lognorm = c->delta;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int ipt = (ng + kScanThreads - 1) / kScanThreads;
  double Wg[2];
  double ug[2];
  for (int side = 0; side < 2; ++side) {
    const int64_t gg = side ? prev : g;
    const int64_t base = gg * ng;
    double wl[4];
    double part = 0.0;
    for (int j = 0; j < ipt; ++j) {
      const int li = t * ipt + j;
      wl[j] = 0.0;
      if (li < ng) {
        const int64_t idx = base + li;
        wl[j] = exp((double)val[idx] + off[(idx / kBlock) * ws.stride] - lognorm);
        part += wl[j];
      }
    }
    part = wave_sum(part);
    if (lane == 0) dsum[w] = part;
    __syncthreads();
    const double W = (dsum[0] + dsum[1]) + (dsum[2] + dsum[3]);
    __syncthreads();
    uint64_t run = 0, v[4];
    for (int j = 0; j < ipt; ++j) {
      const uint64_t wf = (W > 0.0) ? __double2ull_rn(wl[j] / W * 0x1p60) : 0ull;
      run += wf;
      v[j] = run;
    }
    const uint64_t incl = wave_incl_scan_u64(run, lane);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint64_t before = 0;
    for (int j = 0; j < w; ++j) before += wsum[j];
    for (int j = 0; j < ipt; ++j) {
      const int li = t * ipt + j;
      if (li < ng) C[side][li] = before + incl - run + v[j];
    }
    __syncthreads();
    Wg[side] = W;
    if (u_dev) {
      ug[side] = u_dev[gg];
    } else {
      const uint4 rr = draw(m, (uint32_t)gg, (uint32_t)c->k, kRna, 0u);
      ug[side] = u53(rr.x, rr.y);
    }
  }
  // slots of group g: own local resampling, then the received tail
  for (int l = t; l < ng; l += kScanThreads) {
    const int side = (l >= ng - m.moved) ? 1 : 0;
    const int64_t gg = side ? prev : g;
    int j = l;
    if (Wg[side] > 0.0) {
      const uint64_t us = (uint64_t)(((double)l + ug[side]) * m.inv_group * 0x1p60);
      int lo = 0, hi = ng - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (C[side][mid] > us)
          hi = mid;
        else
          lo = mid + 1;
      }
      j = lo;
    }
    b.anc[g * ng + l] = (int32_t)(gg * ng + j);
  }
  if (t == 0) b.lwg[g] = log(Wg[0] / (double)ng);
}

// ------------------------------------------------------------- utilities
__global__ __launch_bounds__(256) void k_gather(Model m, Buffers b, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  const Ctrl* c = b.ctrl;
  const float* X = c->cur ? b.X1 : b.X0;
  const int mode = c->mode;
  const int64_t p = (mode == kModeSys || mode == kModeRna) ? b.anc[i] : i;
#pragma unroll
  for (int d = 0; d < 5; ++d) out[d * m.n + i] = X[d * m.n + p];
}

// Normalised log weights of the last committed step into lw64.
__global__ __launch_bounds__(256) void k_logw(Model m, Buffers b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  const Ctrl* c = b.ctrl;
  const int mode = c->mode;
  if (mode == kModeSet) return;
  if (mode == kModeInit) {
    b.lw64[i] = -m.log_n;
    return;
  }
  const float* L = c->cur ? b.L1 : b.L0;
  const double* R = c->cur ? b.R1 : b.R0;
  b.lw64[i] = (double)L[i] + R[(i / kBlock) * kRec] - c->delta;
}

__global__ void k_set_mode(Ctrl* c, int32_t mode) { c->mode = mode; }

// Records of caller-supplied fp32 log weights (standalone resampling).
__global__ __launch_bounds__(256) void k_records(Model m, Buffers b,
                                                 const float* __restrict__ logw) {
  __shared__ double red[8 + 4 * 7];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < m.n;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double l = active ? (double)logw[i] : -INFINITY;
  const double mv = wave_max(l);
  if (lane == 0) red[w] = mv;
  __syncthreads();
  const double mb = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  double e = 0.0;
  if (active) e = isnan(l) ? NAN : (mb == -INFINITY ? 0.0 : exp(l - mb));
  const double s1 = wave_sum(e), s2 = wave_sum(e * e);
  __syncthreads();
  if (lane == 0) {
    red[8 + w] = s1;
    red[12 + w] = s2;
  }
  __syncthreads();
  if (t == 0) {
    double* R = b.R0 + (int64_t)blockIdx.x * kRec;
    R[0] = mb;
    R[1] = (red[8] + red[9]) + (red[10] + red[11]);
    R[2] = (red[12] + red[13]) + (red[14] + red[15]);
    for (int d = 0; d < 5; ++d) R[3 + d] = 0.0;
    b.zeros[blockIdx.x] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_philox(uint32_t k0, uint32_t k1,
                                                const uint4* __restrict__ ctr,
                                                uint4* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = philox(ctr[i], k0, k1);
}

template <int P>
hipError_t launch_spot(const Model& m, const Buffers& b, const float* obs, hipStream_t s) {
  hipLaunchKernelGGL(k_step_spot<P>, dim3((unsigned)b.nb), dim3(kBlock), 0, s, m, b, obs);
  return hipGetLastError();
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_init(const Model& m, const Buffers& b, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(grid_for(m.n, 256)), dim3(256), 0, s, m, b);
  return hipGetLastError();
}

hipError_t launch_step(const Model& m, const Buffers& b, const float* obs, hipStream_t s) {
  if (m.obs == 1) {
    hipLaunchKernelGGL(k_step_lg, dim3((unsigned)b.nb), dim3(kBlock), 0, s, m, b, obs);
    return hipGetLastError();
  }
  switch (m.P) {
    case 1: return launch_spot<1>(m, b, obs, s);
    case 3: return launch_spot<3>(m, b, obs, s);
    case 5: return launch_spot<5>(m, b, obs, s);
    case 7: return launch_spot<7>(m, b, obs, s);
    case 9: return launch_spot<9>(m, b, obs, s);
    case 11: return launch_spot<11>(m, b, obs, s);
    case 13: return launch_spot<13>(m, b, obs, s);
    case 15: return launch_spot<15>(m, b, obs, s);
    case 17: return launch_spot<17>(m, b, obs, s);
    case 19: return launch_spot<19>(m, b, obs, s);
    case 21: return launch_spot<21>(m, b, obs, s);
    case 23: return launch_spot<23>(m, b, obs, s);
    case 25: return launch_spot<25>(m, b, obs, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(const Model&, const Buffers& b, int standalone, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)b.nr2), dim3(256), 0, s, b, standalone);
  return hipGetLastError();
}

hipError_t launch_finalize(const Model& m, const Buffers& b, int standalone, double u_given,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, m, b, standalone, u_given);
  return hipGetLastError();
}

hipError_t launch_scan(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3((unsigned)b.ntiles), dim3(kScanThreads), 0, s, m, b, w);
  return hipGetLastError();
}

hipError_t launch_heavy(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s) {
  hipLaunchKernelGGL(k_heavy, dim3(kHeavyBlocks), dim3(kScanThreads), 0, s, m, b, w);
  return hipGetLastError();
}

hipError_t launch_rna(const Model& m, const Buffers& b, const WeightSrc& w, const double* u_dev,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_rna, dim3((unsigned)m.G), dim3(kScanThreads), 0, s, m, b, w, u_dev);
  return hipGetLastError();
}

hipError_t launch_gather(const Model& m, const Buffers& b, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(grid_for(m.n, 256)), dim3(256), 0, s, m, b, out);
  return hipGetLastError();
}

hipError_t launch_logw(const Model& m, const Buffers& b, hipStream_t s) {
  hipLaunchKernelGGL(k_logw, dim3(grid_for(m.n, 256)), dim3(256), 0, s, m, b);
  return hipGetLastError();
}

hipError_t launch_set_mode(const Buffers& b, int32_t mode, hipStream_t s) {
  hipLaunchKernelGGL(k_set_mode, dim3(1), dim3(1), 0, s, b.ctrl, mode);
  return hipGetLastError();
}

hipError_t launch_records(const Model& m, const Buffers& b, const float* logw, hipStream_t s) {
  hipLaunchKernelGGL(k_records, dim3((unsigned)b.nb), dim3(kBlock), 0, s, m, b, logw);
  return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3(grid_for(n, 256)), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), reinterpret_cast<const uint4*>(ctr),
                     reinterpret_cast<uint4*>(out), n);
  return hipGetLastError();
}

}  // namespace ppf
