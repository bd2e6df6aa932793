// HIP kernels of the SIR filter step for gfx950 (CDNA4, wave64).
//
// One step of Algorithm 1 (Section 2) is four or five launches on one
// stream, with every decision taken on the device (so the same sequence
// serves every step, and a HIP graph of it can be replayed):
//   k_step         gather parent + propagate (Section 6.1) + patch likelihood
//                  (Eqs. 3-4, Section 5.5) + per-block normalisation record
//   k_merge        merge of the block records per chunk
//   k_merge_final  fixed-order merge of the chunks: the normaliser, ESS, MMSE
//                  estimate, resampling decision and uniform; commits or rolls
//                  back the step; the fixed-point CDF prefixes of the chunks
//   k_anc          systematic resampling: one wave per segment of 1024
//                  particles, each particle's run of output slots from the
//                  segment's CDF
//   k_fill         the slots of heavy segments queued by k_anc (concentrated
//                  weights), in chunks of tiles
//   (or k_rna_local + k_rna_exchange: RNA of Section 3, one workgroup per
//                  group of particles; k_arna_* for ARNA; k_rpa_* after k_fill
//                  for RPA)
#include "ppf_internal.hpp"

#include <array>
#include <cfloat>
#include <climits>
#include <cmath>
#include <mutex>
#include <tuple>
#include <utility>

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
    // one 32 x 32 -> 64-bit product gives both halves; each three-way xor
    // is one v_bitop3 (truth table 0x96 = a ^ b ^ c)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                   __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0);
  }
  return c;
}

__device__ __forceinline__ uint4 draw(const Model& m, uint32_t index, uint32_t k,
                                      uint32_t purpose, uint32_t block) {
  return philox(make_uint4(index, k, (purpose << 24) | block, m.track), m.key0, m.key1);
}

// Uniforms from the top 24 bits: [0, 1) and (0, 1], exact in fp32.
__device__ __forceinline__ float u24_open_hi(uint32_t a) { return (float)(a >> 8) * 0x1p-24f; }
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  return ((double)a * 2097152.0 + (double)(b >> 11)) * 0x1p-53;
}

// The five normals of a particle come from one Philox block: three radius
// fields of 24 bits and three angle fields of 18 bits, laid end to end from
// bit 0 of word x as radius 0, angle 0, radius 1, angle 1, radius 2, angle 2
// (126 of the 128 bits). A radius field r is the uniform (r + 1) / 2^24 in
// (0, 1] and an angle field a the uniform a / 2^18 in [0, 1), both exact in
// fp32.
struct NormalFields {
  uint32_t r0, a0, r1, a1, r2, a2;
};
__device__ __forceinline__ NormalFields normal_fields(uint4 w) {
  NormalFields f;
  f.r0 = w.x & 0xFFFFFFu;                                           // bits 0-23
  f.a0 = __builtin_amdgcn_alignbit(w.y, w.x, 24) & 0x3FFFFu;        // bits 24-41
  f.r1 = __builtin_amdgcn_alignbit(w.z, w.y, 10) & 0xFFFFFFu;       // bits 42-65
  f.a1 = __builtin_amdgcn_ubfe(w.z, 2, 18);                         // bits 66-83
  f.r2 = __builtin_amdgcn_alignbit(w.w, w.z, 20) & 0xFFFFFFu;       // bits 84-107
  f.a2 = __builtin_amdgcn_ubfe(w.w, 12, 18);                        // bits 108-125
  return f;
}

// Box-Muller in fp32 from a radius field r and an angle field a. The radius
// sqrt(-2 ln u), u in (0, 1], uses the hardware log2 and square root
// (measured over all 2^24 uniforms: at most 1.9 ulp for ln u, 0.9 ulp for
// the root). The angle 2 pi t, t in [0, 1), is reduced exactly: x = 4 t,
// q = rint(x), r = x - q in [-1/2, 1/2], and sin, cos(2 pi t) are
// sin, cos(pi/2 r) rotated by the quadrant q, from the Taylor series in r to
// degree 9 and 10 (truncation below 2e-9; measured at most 8.8e-8 absolute
// with fp32 rounding).
__device__ __forceinline__ float bm_radius(uint32_t r) {
  // -2 ln u = -(2 ln 2) log2 u
  return __builtin_amdgcn_sqrtf(-0x1.62e430p+0f *
                                __builtin_amdgcn_logf((float)(r + 1u) * 0x1p-24f));
}

__device__ __forceinline__ float sin_halfpi(float r, float r2) {
  float p = 0x1.507834p-13f;   //  (pi/2)^9 / 9!
  p = fmaf(p, r2, -0x1.32d2ccp-8f);  // -(pi/2)^7 / 7!
  p = fmaf(p, r2, 0x1.466bc6p-4f);   //  (pi/2)^5 / 5!
  p = fmaf(p, r2, -0x1.4abbcep-1f);  // -(pi/2)^3 / 3!
  p = fmaf(p, r2, 0x1.921fb6p+0f);   //   pi/2
  return p * r;
}

__device__ __forceinline__ float cos_halfpi(float r2) {
  float p = -0x1.a6d1f2p-16f;        // -(pi/2)^10 / 10!
  p = fmaf(p, r2, 0x1.e1f506p-11f);  //  (pi/2)^8 / 8!
  p = fmaf(p, r2, -0x1.55d3c8p-6f);  // -(pi/2)^6 / 6!
  p = fmaf(p, r2, 0x1.03c1f0p-2f);   //  (pi/2)^4 / 4!
  p = fmaf(p, r2, -0x1.3bd3ccp+0f);  // -(pi/2)^2 / 2!
  return fmaf(p, r2, 1.0f);
}

__device__ __forceinline__ void box_muller(uint32_t rf, uint32_t af, float& z0, float& z1) {
  const float rad = bm_radius(rf);
  const float x = (float)af * 0x1p-16f;  // 4 t, exact
  const float q = rintf(x);
  const float r = x - q, r2 = r * r;
  const float sn = sin_halfpi(r, r2), cs = cos_halfpi(r2);
  const int qi = (int)q & 3;
  const float ss = (qi & 1) ? cs : sn, cc = (qi & 1) ? sn : cs;
  z0 = rad * (((qi + 1) & 2) ? -cc : cc);
  z1 = rad * ((qi & 2) ? -ss : ss);
}

// The cosine branch alone.
__device__ __forceinline__ float box_muller_cos(uint32_t rf, uint32_t af) {
  const float rad = bm_radius(rf);
  const float x = (float)af * 0x1p-16f;
  const float q = rintf(x);
  const float r = x - q, r2 = r * r;
  const int qi = (int)q & 3;
  const float cc = (qi & 1) ? sin_halfpi(r, r2) : cos_halfpi(r2);
  return rad * (((qi + 1) & 2) ? -cc : cc);
}

__device__ __forceinline__ void box_muller64(uint32_t r, uint32_t a, double& z0, double& z1) {
  const double rad = sqrt(-2.0 * log(((double)r + 1.0) * 0x1p-24));
  double s, c;
  sincospi((double)a * 0x1p-17, &s, &c);  // 2 t
  z0 = rad * c;
  z1 = rad * s;
}

// e^x for finite x: Cody-Waite reduction x = k ln2 + r with ln 2 split into
// a 32-bit head (k * head exact) and a tail, |r| <= ln2 / 2, and the Taylor
// polynomial of degree 11 (truncation below 7e-15 relative); the result is
// scaled by 2^k (0 below the subnormal range, inf above the finite one).
__device__ __forceinline__ double exp_fast(double x) {
  const double k = rint(x * 0x1.71547652b82fep+0);  // x / ln 2
  double r = fma(-k, 0x1.62e42fee00000p-1, x);
  r = fma(-k, 0x1.a39ef35793c76p-33, r);
  double p = 0x1.ae64567f544e4p-26;     // 1/11!
  p = fma(p, r, 0x1.27e4fb7789f5cp-22);  // 1/10!
  p = fma(p, r, 0x1.71de3a556c734p-19);  // 1/9!
  p = fma(p, r, 0x1.a01a01a01a01ap-16);  // 1/8!
  p = fma(p, r, 0x1.a01a01a01a01ap-13);  // 1/7!
  p = fma(p, r, 0x1.6c16c16c16c17p-10);  // 1/6!
  p = fma(p, r, 0x1.1111111111111p-7);   // 1/5!
  p = fma(p, r, 0x1.5555555555555p-5);   // 1/4!
  p = fma(p, r, 0x1.5555555555555p-3);   // 1/3!
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)fmax(fmin(k, 2100.0), -2100.0));
}

// ------------------------------------------------------ wave64 primitives
// Cross-lane moves use DPP within rows of 16 lanes: row shifts (row_shr:k;
// lanes whose source falls outside the row read 0 and are masked off by the
// callers) for scans, row rotations (row_ror:k) for reductions, and either
// v_readlane for the four row results or row broadcasts that carry them into
// the last row. Every helper must be called with all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, true);
}

template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return (int)dpp32<CTRL>((uint32_t)v);
}
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return dpp32<CTRL>(v);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp(uint64_t v) {
  return (uint64_t)dpp32<CTRL>((uint32_t)v) | ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32);
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  return __longlong_as_double((long long)dpp<CTRL>((uint64_t)__double_as_longlong(v)));
}
template <int K, class T>
__device__ __forceinline__ T shr(T v) {
  return dpp<0x110 + K>(v);
}
template <int K, class T>
__device__ __forceinline__ T ror(T v) {
  return dpp<0x120 + K>(v);
}

__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
// The wave's index within its workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
}
__device__ __forceinline__ uint64_t readlane(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double readlane(double v, int l) {
  return __longlong_as_double((long long)readlane((uint64_t)__double_as_longlong(v), l));
}

struct OpAdd {
  template <class T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
  __device__ __forceinline__ double operator()(double a, double b) const { return fmax(a, b); }
  __device__ __forceinline__ uint64_t operator()(uint64_t a, uint64_t b) const {
    return a > b ? a : b;
  }
  __device__ __forceinline__ int operator()(int a, int b) const { return a > b ? a : b; }
};
struct OpMin {
  __device__ __forceinline__ int operator()(int a, int b) const { return a < b ? a : b; }
};
// Elementwise minimum of two int16 pairs packed in 32 bits (v_pk_min_i16).
struct OpMin16x2 {
  __device__ __forceinline__ uint32_t operator()(uint32_t a, uint32_t b) const {
    typedef short s2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(s2, a),
                                                                  __builtin_bit_cast(s2, b)));
  }
};

// Inclusive scan within each row of 16 lanes (r = lane & 15).
template <class T, class Op>
__device__ __forceinline__ T row_scan(T v, int r, Op op) {
  T t = shr<1>(v);
  if (r >= 1) v = op(v, t);
  t = shr<2>(v);
  if (r >= 2) v = op(v, t);
  t = shr<4>(v);
  if (r >= 4) v = op(v, t);
  t = shr<8>(v);
  if (r >= 8) v = op(v, t);
  return v;
}

// Reduction within each row of 16 lanes; every lane receives its row's
// result, combined in an order fixed for each lane.
template <class T, class Op>
__device__ __forceinline__ T row_allreduce(T v, Op op) {
  v = op(v, ror<1>(v));
  v = op(v, ror<2>(v));
  v = op(v, ror<4>(v));
  v = op(v, ror<8>(v));
  return v;
}

// Reduction over the wave, in a fixed order (result uniform).
template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, int lane, Op op) {
  (void)lane;
  v = row_allreduce(v, op);
  return op(op(readlane(v, 0), readlane(v, 16)), op(readlane(v, 32), readlane(v, 48)));
}

// Row broadcasts: CTRL 0x142 (row_bcast:15) hands lane 15 of each row to the
// whole next row, CTRL 0x143 (row_bcast:31) hands lane 31 to rows 2 and 3.
// Only the rows in the mask ROWS receive; the others read `id`.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t bcast32(uint32_t v, uint32_t id) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ int bcast(int v, int id) {
  return (int)bcast32<CTRL, ROWS>((uint32_t)v, (uint32_t)id);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t bcast(uint32_t v, uint32_t id) {
  return bcast32<CTRL, ROWS>(v, id);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double bcast(double v, double id) {
  const uint64_t x = (uint64_t)__double_as_longlong(v), z = (uint64_t)__double_as_longlong(id);
  const uint64_t r = (uint64_t)bcast32<CTRL, ROWS>((uint32_t)x, (uint32_t)z) |
                     ((uint64_t)bcast32<CTRL, ROWS>((uint32_t)(x >> 32), (uint32_t)(z >> 32))
                      << 32);
  return __longlong_as_double((long long)r);
}

// Combines each odd row's result with the even row before it: after a
// row_allreduce, rows 1 and 3 hold op(row 0, row 1) and op(row 2, row 3).
template <class T, class Op>
__device__ __forceinline__ T pair_rows(T v, Op op, T id) {
  return op(v, bcast<0x142, 0xa>(v, id));
}

// Reduction over the wave whose result is exact in lane 63 only (no
// v_readlane): rows paired by row_bcast:15, then the pairs by row_bcast:31.
// id is the identity of op.
template <class T, class Op>
__device__ __forceinline__ T wave_reduce_last(T v, Op op, T id) {
  v = pair_rows(row_allreduce(v, op), op, id);
  return op(v, bcast<0x143, 0xc>(v, id));
}

// Order-preserving integer key of a float that is not NaN: a < b exactly
// when key(a) < key(b) (-0 sorts just below +0), and key + 1 is the key of
// the next float up.
__device__ __forceinline__ int ord_key(float f) {
  const int x = __float_as_int(f);
  return x ^ ((x >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float ord_val(int k) {
  return __int_as_float(k ^ ((k >> 31) & 0x7fffffff));
}
// Key of the smallest float >= x (x not NaN).
__device__ __forceinline__ int ord_key_up(double x) {
  const float f = (float)x;
  return ord_key(f) + ((double)f < x ? 1 : 0);
}

// Inclusive scan over the wave, in a fixed order.
template <class T, class Op>
__device__ __forceinline__ T wave_scan(T v, int lane, Op op) {
  v = row_scan(v, lane & 15, op);
  const T r0 = readlane(v, 15), r1 = readlane(v, 31), r2 = readlane(v, 47);
  const int row = lane >> 4;
  if (row == 1)
    v = op(r0, v);
  else if (row == 2)
    v = op(op(r0, r1), v);
  else if (row == 3)
    v = op(op(op(r0, r1), r2), v);
  return v;
}

// Reduction over a 256-thread workgroup (sh: 4 entries of LDS scratch).
template <class T, class Op>
__device__ __forceinline__ T block_reduce(T v, T* sh, Op op) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_reduce(v, lane, op);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const T r = op(op(sh[0], sh[1]), op(sh[2], sh[3]));
  __syncthreads();
  return r;
}

// Sums of K values over a 256-thread workgroup with one LDS exchange
// (sh: 4 * K doubles), each in a fixed order.
template <int K>
__device__ __forceinline__ void block_sum_n(double (&v)[K], double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_reduce_last(v[k], OpAdd(), 0.0);
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = (sh[k] + sh[K + k]) + (sh[2 * K + k] + sh[3 * K + k]);
  __syncthreads();
}

// Exclusive prefix sum of exact unsigned integers over a 256-thread
// workgroup; *total receives the sum of all.
__device__ __forceinline__ uint64_t block_excl_sum(uint64_t v, uint64_t* sh, uint64_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t inc = wave_scan(v, lane, OpAdd());
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  uint64_t before = 0;
  for (int j = 0; j < w; ++j) before += sh[j];
  *total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return before + inc - v;
}

// ------------------------------------------------------------ k_init
// The Morton key of the top 16 bits of two words: x's bits at the even
// positions, y's at the odd ones (each spread by doubling its bit distance).
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  return (v | (v << 1)) & 0x55555555u;
}
__device__ __forceinline__ uint32_t zorder_key(uint32_t wx, uint32_t wy) {
  return spread16(wx >> 16) | (spread16(wy >> 16) << 1);
}
__device__ __forceinline__ void init_state(const Model& m, int64_t i, float* xs);
// Algorithm 1 initialisation, k = 0. The state is computed in fp64 and
// rounded once to fp32.
__device__ __forceinline__ void init_body(const Model& m, const Buffers& b, int64_t blk) {
  const int64_t i = blk * kBlock + threadIdx.x;
  if (i == 0) {
    Ctrl* c = b.ctrl;
    c->k = 0;
    c->cur = 0;
    c->mode = kModeInit;
    c->resampled = 0;
    c->rolled_back = 0;
    c->do_resample = 0;
    c->heavy_count = 0;
    c->m = c->log_sum = c->ess = c->delta = c->cum = 0.0;
    for (int d = 0; d < 5; ++d) c->mean[d] = 0.0;
    c->u = 0.0;
    c->total = 0;
    for (int d = 0; d < kNGrad; ++d) c->grad_cum[d] = c->grad_last[d] = 0.0;
    c->ring_key = 0;
    c->delta_ref = -INFINITY;
    c->lost = 0;
    c->arna_tracking = 0;
    c->arna_moved = 0;
  }
  if (i >= m.n) return;
  if (m.grad)
    for (int d = 0; d < kNTan; ++d) b.T0[(int64_t)d * m.n + i] = 0.0f;
  if (m.init_kind == 3) {
    // Z order: the sort key of draw i; k_init_place writes the states
    const uint4 r0 = draw(m, (uint32_t)i, 0u, kInit, 0u);
    b.zkey0[i] = zorder_key(r0.x, r0.y);
    b.zval0[i] = (int32_t)i;
    return;
  }
  float xs[5];
  init_state(m, i, xs);
#pragma unroll
  for (int d = 0; d < 5; ++d) b.X0[(int64_t)d * m.n + i] = xs[d];
}

// The initial state of draw i (kinds 0-2; kind 3 draws as kind 0).
__device__ __forceinline__ void init_state(const Model& m, int64_t i, float* xs) {
  const uint4 r0 = draw(m, (uint32_t)i, 0u, kInit, 0u);
  const uint4 r1 = draw(m, (uint32_t)i, 0u, kInit, 1u);
  double x[5];
  if (m.init_kind == 1) {  // Gaussian
    double z[5], unused;
    const NormalFields nf = normal_fields(r0);
    box_muller64(nf.r0, nf.a0, z[0], z[1]);
    box_muller64(nf.r1, nf.a1, z[2], z[3]);
    box_muller64(nf.r2, nf.a2, z[4], unused);
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
  for (int d = 0; d < 5; ++d) xs[d] = (float)x[d];
}

__global__ __launch_bounds__(256) void k_init(Model m, Buffers b) { init_body(m, b, blockIdx.x); }

// Z-ordered init: position p takes draw zval0[p] (the keys sorted, stably).
__global__ __launch_bounds__(256) void k_init_place(Model m, Buffers b) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= m.n) return;
  float xs[5];
  init_state(m, (int64_t)b.zval0[p], xs);
#pragma unroll
  for (int d = 0; d < 5; ++d) b.X0[(int64_t)d * m.n + p] = xs[d];
}

// ------------------------------------------------------------ k_step
// Parent, carried log weight and propagated state of particle i.
struct Prop {
  float x, y, vx, vy, I;
};

// The particle's log weight before the new observation: its stored weight
// carried over (no resampling this step), its group's weight after RNA, a
// caller-set weight, or -log N after systematic resampling. Kept out of
// propagate so that kernels compute it only where the likelihood is added,
// instead of holding it across the patch sums.
// amv: the slots exchanged by the last ARNA resampling (the control block's).
__device__ __forceinline__ double prior_lw(const Model& m, const Buffers& b, int cur, int mode,
                                           double delta, int amv, int64_t i) {
  if (mode == kModeNone) {
    const float* Ein = cur ? b.E1 : b.E0;
    const double* Rin = cur ? b.R1 : b.R0;
    return log((double)Ein[i]) + Rin[(i / kBlock) * kRec] - delta;
  }
  if (mode == kModeRna) {
    const int64_t g = i / m.group;
    const int64_t l = i - g * m.group;
    const int64_t src = (l >= m.group - m.moved) ? (g + m.G - 1) % m.G : g;
    return b.lwg[src];
  }
  if (mode == kModeArna) {
    const int64_t g = i / m.group;
    const int64_t l = i - g * m.group;
    return (l >= m.group - amv) ? b.lwt[g] : b.lwg[g];
  }
  if (mode == kModeSet) return b.lw64[i];
  return -m.log_n;
}

// zo (5 normals) and po (the parent) are optional outputs for the tangents.
__device__ __forceinline__ Prop propagate(const Model& m, const Buffers& b, int cur, int mode,
                                          int64_t i, uint32_t k, float* zo = nullptr,
                                          int64_t* po = nullptr) {
  const float* Xin = cur ? b.X1 : b.X0;
  int64_t p = i;
  if (mode == kModeSys || mode == kModeRna || mode == kModeArna) p = b.anc[i];
  const int64_t n = m.n;
  const float px = Xin[p], py = Xin[n + p], pvx = Xin[2 * n + p], pvy = Xin[3 * n + p],
              pI = Xin[4 * n + p];
  const NormalFields nf = normal_fields(draw(m, (uint32_t)i, k, kPropagate, 0u));
  float z0, z1, z2, z3;
  box_muller(nf.r0, nf.a0, z0, z1);
  box_muller(nf.r1, nf.a1, z2, z3);
  const float z4 = box_muller_cos(nf.r2, nf.a2);
  if (zo) {
    zo[0] = z0;
    zo[1] = z1;
    zo[2] = z2;
    zo[3] = z3;
    zo[4] = z4;
  }
  if (po) *po = p;
  Prop o;
  // near-constant velocity, unit frame interval; in fp32 with one fused
  // multiply-add per component, the small velocity and noise terms first,
  // so a position is within half an ulp (plus the rounding of that small
  // sum) of the exact value
  o.x = px + fmaf(m.q[0], z0, pvx);
  o.y = py + fmaf(m.q[1], z1, pvy);
  o.vx = fmaf(m.q[2], z2, pvx);
  o.vy = fmaf(m.q[3], z3, pvy);
  o.I = fmaf(m.q[4], z4, pI);
  return o;
}

// The new states stream past the caches (non-temporal stores): the next
// step gathers them through the ancestors long after, and left in the
// caches as dirty lines their write-back would compete with the weight
// stream of the resampling pass that follows.
__device__ __forceinline__ void store_state(const Model& m, const Buffers& b, int cur, int64_t i,
                                            const Prop& o) {
  float* Xout = cur ? b.X0 : b.X1;
  const int64_t n = m.n;
  __builtin_nontemporal_store(o.x, Xout + i);
  __builtin_nontemporal_store(o.y, Xout + n + i);
  __builtin_nontemporal_store(o.vx, Xout + 2 * n + i);
  __builtin_nontemporal_store(o.vy, Xout + 3 * n + i);
  __builtin_nontemporal_store(o.I, Xout + 4 * n + i);
}

// Fixed-point weight of a particle whose weight relative to its block
// maximum is e in [0, 1]: round(e 2^44), an exact integer held in a double
// (e 2^44 is an exact exponent shift below 2^52; rint rounds it once, half
// to even).
__device__ __forceinline__ double item_weight(double e) {
  static_assert(kItemScale == 0x1p44, "the scale is applied as an exponent shift");
  return rint(ldexp(e, 44));
}

// e^x for x <= 0 rounded to fp32 (0 below -104, where e^x is under half the
// least fp32 subnormal). Cody-Waite reduction x = k ln 2 + r with one fp64
// constant (|k| <= 150 keeps its error below 2^-47) and the Taylor polynomial
// of degree 9 on |r| <= ln 2 / 2 (truncation below 2^-36 relative): the fp64
// value is far closer to e^x than the fp32 rounding step.
__device__ __forceinline__ float exp_neg_f32(double x) {
  const double k = rint(x * 0x1.71547652b82fep+0);
  const double r = fma(-k, 0x1.62e42fefa39efp-1, x);
  double p = 0x1.71de3a556c734p-19;     // 1/9!
  p = fma(p, r, 0x1.a01a01a01a01ap-16);  // 1/8!
  p = fma(p, r, 0x1.a01a01a01a01ap-13);  // 1/7!
  p = fma(p, r, 0x1.6c16c16c16c17p-10);  // 1/6!
  p = fma(p, r, 0x1.1111111111111p-7);   // 1/5!
  p = fma(p, r, 0x1.5555555555555p-5);   // 1/4!
  p = fma(p, r, 0x1.5555555555555p-3);   // 1/3!
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  const float v = (float)ldexp(p, (int)k);
  return x < -104.0 ? 0.0f : v;
}

// The block's normalisation record (see kRec) and the stored weights
// E = exp(l - m_b) in fp32. red: 7 x 256 doubles of LDS that no thread reads
// once it has reached this call (it may alias the caller's image tile); dsh
// and ksh: 4 doubles and 4 ints of LDS scratch.
// Returns e = E (0 for an inactive or non-finite particle).
//
// The shift m_b is any value at or above every finite l of the block and
// close to their maximum (the record carries it, so the normalisation does
// not depend on which): the maximum of the l rounded up to fp32, taken as
// order-preserving integer keys so that each DPP step is one v_max_i32, and
// within one fp32 ulp of the largest l. Where that ulp exceeds 1/8 (block
// maxima of magnitude 2^20 and above) the exact fp64 maximum is taken instead.
__device__ __forceinline__ double finish_block(const Buffers& b, int cur, int64_t i, bool active,
                                               double l, const Prop& o, double* red,
                                               double* dsh, int* ksh) {
  // lane tests compare t with wave-uniform values, so no lane index stays live
  const int t = threadIdx.x, w = wave_index(), t0 = 64 * w;
  const bool bad = active && (isnan(l) || l == INFINITY);
  const bool ok = active && !bad;
  const int wk = wave_reduce_last(ok ? ord_key_up(l) : ord_key(-INFINITY), OpMax(), INT_MIN);
  if (t == t0 + 63) ksh[w] = wk;
  __syncthreads();
  const float mf = ord_val(max(max(ksh[0], ksh[1]), max(ksh[2], ksh[3])));
  double mb = (double)mf;
  if (mf != -INFINITY && !(fabsf(mf) < 0x1p20f)) {  // uniform across the workgroup
    const double wm = wave_reduce_last(ok ? l : -INFINITY, OpMax(), (double)-INFINITY);
    if (t == t0 + 63) dsh[w] = wm;
    __syncthreads();
    mb = fmax(fmax(dsh[0], dsh[1]), fmax(dsh[2], dsh[3]));
  }
  double e = 0.0;
  if (active) {
    float Ef = 0.0f;
    if (bad) {
      Ef = NAN;
    } else if (l != -INFINITY) {  // then m_b >= l > -inf
      Ef = exp_neg_f32(l - mb);
      e = (double)Ef;
    }
    float* Eout = cur ? b.E0 : b.E1;
    Eout[i] = Ef;
  }
  const double wi = item_weight(e);
  // after the barrier above every thread is past its reads of the LDS that
  // red may alias
  red[t] = wi;
  red[256 + t] = bad ? NAN : e * e;
  red[512 + t] = e * (double)o.x;
  red[768 + t] = e * (double)o.y;
  red[1024 + t] = e * (double)o.vx;
  red[1280 + t] = e * (double)o.vy;
  red[1536 + t] = e * (double)o.I;
  __syncthreads();
  double s = 0.0;
  if (t < 224) {  // value t >> 5, eight consecutive entries (t & 31) * 8 ...
    const double* p = red + (t >> 5) * 256 + (t & 31) * 8;
    s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
  }
  // value 2w in row 1 of wave w, value 2w + 1 in row 3
  s = pair_rows(row_allreduce(s, OpAdd()), OpAdd(), 0.0);
  double* R = (cur ? b.R0 : b.R1) + (i / kBlock) * kRec;
  if (t == t0 + 16) R[1 + 2 * w] = s;
  if (t == t0 + 48 && 2 * w + 1 < 7) R[2 + 2 * w] = s;
  if (t == 0) R[0] = mb;
  return e;
}

// LDS of one step workgroup: two copies of the tile of D = Z - b, each in
// one half of `tile` (its first 7 x 256 doubles double as the record
// exchange), the table of row sums of D^2, and the reduction scratch.
// Kernels that run several patch sizes declare it once.
template <int TILE>
struct StepLds {
  static_assert(TILE >= 7 * kBlock, "the tile doubles as the record exchange buffer");
  __align__(16) double tile[TILE];
  double sq[kSqCap];
  double dsh[4];
  int ish[16];
  int ksh[4];
};

// Patch sums of one particle over P rows of an LDS tile of D = Z - b (0
// outside the frame) with row stride tw, every row starting on 16 bytes:
//   X   += sum_dy g_y(dy) sum_dx D g_x(dx)    (Gaussian-weighted residual sum)
//   G2y += g_y^2
//   sd2 += sum D^2, from the table of row sums hrow (stride hs) when TAB,
//          else pixel by pixel.
// g_y is advanced by the exact recurrence g(d+1) = g(d) gstep(d) exp(f/s^2).
// gx[0] is 1, so each row's sum starts at its first pixel (an fma with a zero
// addend would cost an add, to turn -0 into +0; D = Z - b is never -0 here).
template <int P, bool TAB>
__device__ __forceinline__ void patch_lds(const double* __restrict__ p0, int tw,
                                          const double* __restrict__ hrow, int hs,
                                          const double (&gx)[P], double gy, double by,
                                          const double* gstep, double& X, double& G2y,
                                          double& sd2) {
#pragma unroll
  for (int dy = 0; dy < P; ++dy) {
    const double* row = static_cast<const double*>(__builtin_assume_aligned(p0 + dy * tw, 16));
    double rd = row[0];
    if (!TAB) sd2 = fma(rd, rd, sd2);
#pragma unroll
    for (int dx = 1; dx < P; ++dx) {
      const double d = row[dx];
      rd = fma(d, gx[dx], rd);
      if (!TAB) sd2 = fma(d, d, sd2);
    }
    if (TAB) sd2 += hrow[dy * hs];
    X = fma(gy, rd, X);
    G2y = fma(gy, gy, G2y);
    gy *= gstep[dy] * by;
  }
}

// The same sums read straight from the frame (workgroups whose patches do
// not fit one LDS tile); pixels outside the frame read as the background.
template <int P>
__device__ __forceinline__ void patch_global(const float* __restrict__ obs, int u0, int v0,
                                             int W, int H, double bsub, const double (&gx)[P],
                                             double gy, double by, const double* gstep,
                                             double& X, double& G2y, double& sd2) {
#pragma unroll 1
  for (int dy = 0; dy < P; ++dy) {
    const int v = v0 + dy;
    const bool row_in = (unsigned)v < (unsigned)H;
    const float* row = obs + (int64_t)(row_in ? v : 0) * W;
    double rd = 0.0;
#pragma unroll
    for (int dx = 0; dx < P; ++dx) {
      const int u = u0 + dx;
      const double d = (row_in && (unsigned)u < (unsigned)W) ? (double)row[u] - bsub : 0.0;
      rd = dx == 0 ? d : fma(d, gx[dx], rd);
      sd2 = fma(d, d, sd2);
    }
    X = fma(gy, rd, X);
    G2y = fma(gy, gy, G2y);
    gy *= gstep[dy] * by;
  }
}

// Gradient mode: moments of one particle's patch. With D = Z - b (0 outside
// the frame), the Gaussian factors g = g_x g_y and the integer offsets
// a = dx - h, c = dy - h of a pixel from the patch centre:
//   X0 = sum D g,  X1 = sum D g a,  X2 = sum D g a^2,
//   Y1 = sum D g c,  Y2 = sum D g c^2,
//   B0, B1, B2 = sum_dy g_y^2 c^{0,1,2},  SD = sum D,
//   Gin = sum of g_y over the rows inside the frame,
//   sd2 = sum D^2 (from the row-sum table when TAB).
// X0, B0 and sd2 are accumulated in the same order as patch_lds, so the log
// weights equal those of the plain step.
struct Moments {
  double X0, X1, X2, Y1, Y2, B0, B1, B2, SD, Gin, sd2;
};

template <int P>
__device__ __forceinline__ void moments_row(const double (&d)[P], const double (&gx)[P], int dy,
                                            double gy, bool row_in, bool pix_sq, bool pix_sum,
                                            Moments& mo) {
  constexpr int h = (P - 1) / 2;
  // u = D g_x along the row. s0 = sum u (the plain step's order), and the
  // running sums of running sums s1 = sum_j u_j m_j, s2 = sum_j u_j m_j
  // (m_j + 1) / 2 with m_j = P - j give the moments in a = j - h = c0 - m_j
  // (c0 = h + 1) without a product per pixel:
  //   sum u a = c0 s0 - s1,   sum u a^2 = c0^2 s0 - 2 c0 s1 + 2 s2 - s1.
  // (gx[0] = 1: the sums start at the first pixel, as in patch_lds)
  double s0 = d[0], s1 = s0, s2 = s0, sd = d[0];
  if (pix_sq) mo.sd2 = fma(d[0], d[0], mo.sd2);
#pragma unroll
  for (int dx = 1; dx < P; ++dx) {
    s0 = fma(d[dx], gx[dx], s0);
    s1 += s0;
    s2 += s1;
    if (pix_sum) sd += d[dx];
    if (pix_sq) mo.sd2 = fma(d[dx], d[dx], mo.sd2);
  }
  constexpr double c0 = (double)(h + 1);
  const double r1 = fma(c0, s0, -s1);
  const double r2 = fma(c0 * c0, s0, fma(-2.0 * c0, s1, 2.0 * s2 - s1));
  const double c = (double)(dy - h);
  mo.X0 = fma(gy, s0, mo.X0);
  mo.X1 = fma(gy, r1, mo.X1);
  mo.X2 = fma(gy, r2, mo.X2);
  const double gr = gy * s0;
  mo.Y1 = fma(gr, c, mo.Y1);
  mo.Y2 = fma(gr, c * c, mo.Y2);
  mo.B0 = fma(gy, gy, mo.B0);
  const double g2 = gy * gy;
  mo.B1 = fma(g2, c, mo.B1);
  mo.B2 = fma(g2, c * c, mo.B2);
  if (pix_sum) mo.SD += sd;
  if (row_in) mo.Gin += gy;
}

// Rows from the LDS tile (TAB: sum D^2 of each row from the row-sum table
// hrow; SUMTAB: sum D from hsum as well) or from the frame; v0 is the frame
// row of the patch's first row.
template <int P, bool TAB, bool SUMTAB, bool GLOBAL>
__device__ __forceinline__ void patch_moments(const double* __restrict__ p0, int tw,
                                              const double* __restrict__ hrow,
                                              const double* __restrict__ hsum, int hs,
                                              const float* __restrict__ obs, int u0, double bsub,
                                              int W, int H, int64_t v0,
                                              const double (&gx)[P], double gy, double by,
                                              const double* gstep, Moments& mo) {
#pragma unroll 1
  for (int dy = 0; dy < P; ++dy) {
    const int64_t v = v0 + dy;
    const bool row_in = v >= 0 && v < H;
    double d[P];
    if (GLOBAL) {
      const float* row = obs + (row_in ? v : 0) * (int64_t)W;
#pragma unroll
      for (int dx = 0; dx < P; ++dx) {
        const int u = u0 + dx;
        d[dx] = (row_in && (unsigned)u < (unsigned)W) ? (double)row[u] - bsub : 0.0;
      }
    } else {
      const double* row =
          static_cast<const double*>(__builtin_assume_aligned(p0 + dy * tw, 16));
#pragma unroll
      for (int dx = 0; dx < P; ++dx) d[dx] = row[dx];
    }
    moments_row<P>(d, gx, dy, gy, row_in, !TAB, !SUMTAB, mo);
    if (TAB) mo.sd2 += hrow[dy * hs];
    if (SUMTAB) mo.SD += hsum[dy * hs];
    gy *= gstep[dy] * by;
  }
}

// Propagation and log weight of one particle per thread (Eq. 4 with the spot
// of Eq. 3 on the P x P patch). The residual sum is expanded as
//   sum (D - I g)^2 = sum D^2 - 2 I sum D g + I^2 sum g^2,   D = Z - b,
// (D = 0 for pixels outside the frame) with sum g^2 = (sum g_x^2)(sum g_y^2);
// everything in fp64. The workgroup stages D over the bounding box of its
// patches in LDS as fp64 (the conversion is paid once per pixel, not once per
// particle and pixel) and, when small enough, a table of the P-pixel row sums
// of D^2 at every patch-centre column, so a particle adds P table entries
// instead of squaring P^2 pixels.
// Five barriers per workgroup: the box, the tile, the table, the block
// maximum, and the record exchange.
template <int P, bool GRAD = false, int TILE = kTileCap>
__device__ __forceinline__ void step_spot(const Model& m, const Buffers& b,
                                          const float* __restrict__ obs, int64_t blk,
                                          StepLds<TILE>& L) {
  constexpr int h = (P - 1) / 2;
  double* const tile = L.tile;
  double* const sq = L.sq;
  double* const dsh = L.dsh;
  int* const ish = L.ish;
  const Ctrl* cp = b.ctrl;
  const int cur = cp->cur, mode = cp->mode, amv = cp->arna_moved;
  const double cdelta = cp->delta;
  const uint32_t k = (uint32_t)(cp->k + 1);
  const int t = threadIdx.x, w = wave_index();
  const int64_t i = blk * kBlock + t;
  const bool active = i < m.n;
  // Lanes past the last particle (the tail of the last workgroup) repeat the
  // work of particle n - 1, which lies in the same workgroup, and store
  // nothing: every lane runs the same instructions on valid data.
  const int64_t ia = active ? i : m.n - 1;

  Prop o;
  float tg[kNTan];  // gradient mode: the particle's new tangents
  if constexpr (GRAD) {
    float z[5];
    int64_t p;
    o = propagate(m, b, cur, mode, ia, k, z, &p);
    // tangents along the ancestral line (see kNTan): dx'/dq_x = dx/dq_x +
    // z_x, dx'/dq_vx = dx/dq_vx + dvx/dq_vx (the parent's), and alike
    const float* Tin = cur ? b.T1 : b.T0;
    float* Tout = cur ? b.T0 : b.T1;
    float tp[kNTan];
#pragma unroll
    for (int d = 0; d < kNTan; ++d) tp[d] = Tin[(int64_t)d * m.n + p];
    tg[0] = (float)((double)tp[0] + (double)z[0]);
    tg[1] = (float)((double)tp[1] + (double)z[1]);
    tg[2] = (float)((double)tp[2] + (double)z[2]);
    tg[3] = (float)((double)tp[3] + (double)tp[2]);
    tg[4] = (float)((double)tp[4] + (double)z[3]);
    tg[5] = (float)((double)tp[5] + (double)tp[4]);
    tg[6] = (float)((double)tp[6] + (double)z[4]);
    if (active)  // streamed like the states
#pragma unroll
      for (int d = 0; d < kNTan; ++d) __builtin_nontemporal_store(tg[d], Tout + (int64_t)d * m.n + i);
  } else {
    o = propagate(m, b, cur, mode, ia, k);
  }
  if (active) store_state(m, b, cur, i, o);
  // patch centre: pixel nearest to (x, y); the offset f is exact in fp64
  const double rx = floor((double)o.x + 0.5);
  const double ry = floor((double)o.y + 0.5);
  const double fx = (double)o.x - rx;
  const double fy = (double)o.y - ry;
  // addresses only: far-away centres are clamped to [-P, W + P] x [-P, H + P],
  // where the whole patch already lies outside the frame (its pixels read as
  // background); a NaN centre goes to the low corner
  const int cx = (int)fmin(fmax(rx, m.clo[0]), m.chi[0]);
  const int cy = (int)fmin(fmax(ry, m.clo[1]), m.chi[1]);
  // The 1-D Gaussian factors of Eq. 3 at the patch's pixel offsets. Only
  // their products g_x g_y enter the likelihood, so g_x is taken relative to
  // its first value, which moves into the first g_y: three exps per particle
  // (the host keeps both first values above e^-350, so the product stays
  // normal).
  double gx[P];
  gx[0] = 1.0;
  const double bx = exp_fast(2.0 * fx * m.inv2s2);
#pragma unroll
  for (int d = 0; d + 1 < P; ++d) gx[d + 1] = gx[d] * (m.gstep[d] * bx);
  double G2x = 0.0;
#pragma unroll
  for (int d = 0; d < P; ++d) G2x = fma(gx[d], gx[d], G2x);
  const double ax = (double)h + fx, ay = (double)h + fy;
  const double gy0 = exp_fast(-(ax * ax + ay * ay) * m.inv2s2);
  const double by = exp_fast(2.0 * fy * m.inv2s2);
  // Bounding box of the workgroup's patch centres (the tail lanes repeat
  // particle n - 1, whose centre is in the box anyway). Each lane packs the
  // offsets (ox, oy) of its centre from lane 0's, saturated to +-32767, as
  // two int16 (for the minima) and their negations (for the maxima); an
  // offset at the saturation bound already makes the box wider than any
  // tile, so the saturated box still selects the global path.
  {
    const int bx0 = readlane(cx, 0), by0 = readlane(cy, 0);
    const int ox = min(max(cx - bx0, -32767), 32767), oy = min(max(cy - by0, -32767), 32767);
    const uint32_t pmin = (uint32_t)(uint16_t)ox | ((uint32_t)(uint16_t)oy << 16);
    const uint32_t pneg = (uint32_t)(uint16_t)-ox | ((uint32_t)(uint16_t)-oy << 16);
    const uint32_t rmin = wave_reduce_last(pmin, OpMin16x2(), 0x7fff7fffu);
    const uint32_t rneg = wave_reduce_last(pneg, OpMin16x2(), 0x7fff7fffu);
    if (t == 64 * w + 63) {
      ish[w] = bx0 + (int16_t)(rmin & 0xffffu);
      ish[4 + w] = bx0 - (int16_t)(rneg & 0xffffu);
      ish[8 + w] = by0 + (int16_t)(rmin >> 16);
      ish[12 + w] = by0 - (int16_t)(rneg >> 16);
    }
  }
  __syncthreads();
  const int mnx = min(min(ish[0], ish[1]), min(ish[2], ish[3]));
  const int mxx = max(max(ish[4], ish[5]), max(ish[6], ish[7]));
  const int mny = min(min(ish[8], ish[9]), min(ish[10], ish[11]));
  const int mxy = max(max(ish[12], ish[13]), max(ish[14], ish[15]));
  // The tile is staged twice, copy B shifted one column left of copy A, each
  // in half of the LDS block with an even row stride: a patch row starting
  // at an even column is read from A, one starting at an odd column from B,
  // so every row starts on 16 bytes and is read with 128-bit LDS loads.
  // 128-bit reads meet the banks in 16-byte granules, 16 granules to a bank
  // row; copy B starts 8 granules after the half, so that the patch rows of
  // two neighbouring centres (one in each copy) fall 8 granules apart.
  constexpr int kCopy = TILE / 2;  // doubles per half
  constexpr int kOffB = 16;        // copy B's start within its half, in doubles
  static_assert(kCopy % 2 == 0, "copies must keep 16-byte alignment");
  const int64_t tw64 = (int64_t)mxx - mnx + P, th64 = (int64_t)mxy - mny + P;
  const int64_t ts2min = (tw64 + 1) >> 1;  // row stride in pairs of doubles
  const bool use_lds = 2 * ts2min * th64 <= kCopy - kOffB;  // uniform across the workgroup
  const int tw = (int)tw64, th = (int)th64;
  const int tx0 = mnx - h, ty0 = mny - h;
  const int64_t acx = (int64_t)mxx - mnx + 1;
  const int64_t nH = th64 * acx;
  const bool use_tab = use_lds && nH <= kSqCap;
  // gradient mode also tables the row sums of D, in the upper half, when both
  // fit (the D^2 table is used exactly when the plain step uses it, so the log
  // weights stay the plain step's)
  constexpr int kTab = kSqCap / 2;
  const bool use_sum = GRAD && use_lds && nH <= kTab;
  // Row stride ts = 2 ts2, with ts2 padded to ceil(acx / 2) (mod 16): the
  // granule where a patch row of the centre (cx, cy) starts is then
  // (cy - mny) ceil(acx / 2) + (cx - mnx) / 2 (+ 8 in copy B) (mod 16), so
  // lanes at distinct centres of a small box meet distinct granules (this
  // layout measured a fifth of the bank-conflict cycles of 8-granule rules).
  int ts2 = (int)ts2min;
  {
    const int padh = ((int)(((acx + 1) >> 1) & 15) - (ts2 & 15)) & 15;
    if ((int64_t)2 * (ts2 + padh) * th <= kCopy - kOffB) ts2 += padh;
  }
  const int ts = 2 * ts2;
  if (use_lds) {
    // one pass over the tile's pixels (row r = e / tw from the hardware
    // reciprocal, corrected by one step: e < 2^11 and the reciprocal is
    // within 1 ulp, so the estimate is off by at most 1)
    const int nt = tw * th;
    const float rcpw = __builtin_amdgcn_rcpf((float)tw);
    for (int e = t; e < nt; e += 256) {
      int r = (int)((float)e * rcpw);
      if (r * tw > e) --r;
      else if ((r + 1) * tw <= e) ++r;
      const int c = e - r * tw, v = ty0 + r, u = tx0 + c;
      const double dv = ((unsigned)v < (unsigned)m.H && (unsigned)u < (unsigned)m.W)
                            ? (double)obs[(int64_t)v * m.W + u] - m.b
                            : 0.0;
      tile[r * ts + c] = dv;
      if (c > 0) tile[kCopy + kOffB + r * ts + c - 1] = dv;
    }
  }
  __syncthreads();
  if (use_tab) {
    // sq[r * acx + c] = sum_dx (Z[r][c + dx] - b)^2 over the tile's rows r and
    // the centres' columns c (gradient mode: sq[kTab + r * acx + c] = sum_dx
    // (Z[r][c + dx] - b), both in the per-pixel order)
    const int ax = (int)acx, nh = (int)nH;
    const float rcp = __builtin_amdgcn_rcpf((float)ax);
    for (int e = t; e < nh; e += 256) {
      int r = (int)((float)e * rcp);
      if (r * ax > e) --r;
      else if ((r + 1) * ax <= e) ++r;
      const double* src = tile + r * ts + (e - r * ax);
      double sacc = 0.0, dsum = 0.0;
#pragma unroll
      for (int dx = 0; dx < P; ++dx) {
        sacc = fma(src[dx], src[dx], sacc);
        if (GRAD) dsum += src[dx];
      }
      sq[e] = sacc;
      if (GRAD && use_sum) sq[kTab + e] = dsum;
    }
  }
  __syncthreads();

  // every lane's patch lies in the tile (the tail lanes' is particle
  // n - 1's); finish_block ignores the tail lanes' l
  double l;
  int64_t il = i;  // the particle index where the record is written
  double gth[GRAD ? kNGrad : 1] = {};
  // the particle's first patch row in copy A (even first column) or B (odd)
  const int col0 = cx - h - tx0;
  const double* p0 =
      tile + ((cy - h - ty0) * ts + (col0 & ~1) + ((col0 & 1) ? kCopy + kOffB : 0));
  if constexpr (GRAD) {
    Moments mo{};
    // frame row of the patch's first row; centres far outside are clamped,
    // as for the addresses (every row of such a patch is outside the frame)
    const int64_t v0 = (int64_t)fmin(fmax(ry, -(double)P - 1.0), (double)m.H + P + 1.0) - h;
    // table index of the centre (below nH <= kSqCap where a table is used)
    const int at = use_tab ? (cy - mny) * (int)acx + (cx - mnx) : 0;
    if (use_sum) {
      patch_moments<P, true, true, false>(p0, ts, sq + at, sq + kTab + at, (int)acx, obs, 0,
                                          m.b, m.W, m.H, v0, gx, gy0, by, m.gstep, mo);
    } else if (use_tab) {
      patch_moments<P, true, false, false>(p0, ts, sq + at, sq, (int)acx, obs, 0, m.b, m.W,
                                           m.H, v0, gx, gy0, by, m.gstep, mo);
    } else if (use_lds) {
      patch_moments<P, false, false, false>(p0, ts, sq, sq, 0, obs, 0, m.b, m.W, m.H, v0, gx,
                                            gy0, by, m.gstep, mo);
    } else {
      patch_moments<P, false, false, true>(p0, 0, sq, sq, 0, obs, cx - h, m.b, m.W, m.H, v0, gx,
                                           gy0, by, m.gstep, mo);
    }
    const double I = (double)o.I;
    const double ssq = mo.sd2 - 2.0 * I * mo.X0 + I * I * (G2x * mo.B0);
    l = prior_lw(m, b, cur, mode, cdelta, amv, ia) - ssq * m.inv2sig2 - m.lognorm_obs;
    // 1-D moments of g_x^2 and the in-frame sum of g_x (true centre rx)
    double A1 = 0.0, A2 = 0.0, Gin_x = 0.0;
#pragma unroll
    for (int dx = 0; dx < P; ++dx) {
      const double g2 = gx[dx] * gx[dx];
      A1 = fma(g2, (double)(dx - h), A1);
      A2 = fma(g2, (double)((dx - h) * (dx - h)), A2);
      const double u = rx + (double)(dx - h);
      if (u >= 0.0 && u < (double)m.W) Gin_x += gx[dx];
    }
    const double A0 = G2x, B0 = mo.B0;
    // moments in the offsets from the particle, e = a - f
    const double ex1 = mo.X1 - fx * mo.X0;
    const double ex2 = mo.X2 - 2.0 * fx * mo.X1 + fx * fx * mo.X0;
    const double ey1 = mo.Y1 - fy * mo.X0;
    const double ey2 = mo.Y2 - 2.0 * fy * mo.Y1 + fy * fy * mo.X0;
    const double gx1 = A1 - fx * A0, gx2 = A2 - 2.0 * fx * A1 + fx * fx * A0;
    const double gy1 = mo.B1 - fy * B0, gy2 = mo.B2 - 2.0 * fy * mo.B1 + fy * fy * B0;
    const double isg2 = 2.0 * m.inv2sig2, is2 = 2.0 * m.inv2s2;
    const double lI = (mo.X0 - I * A0 * B0) * isg2;
    const double lx = I * isg2 * is2 * (ex1 - I * B0 * gx1);
    const double ly = I * isg2 * is2 * (ey1 - I * A0 * gy1);
    const double ls = I * isg2 * is2 / m.s_psf * (ex2 + ey2 - I * (B0 * gx2 + A0 * gy2));
    const double lb = isg2 * (mo.SD - I * Gin_x * mo.Gin);
    const double lsig = ssq / (m.sig * m.sig * m.sig) - (double)(P * P) / m.sig;
    gth[0] = ls;
    gth[1] = lb;
    gth[2] = lsig;
    gth[3] = lx * (double)tg[0];
    gth[4] = ly * (double)tg[1];
    gth[5] = lx * (double)tg[3];
    gth[6] = ly * (double)tg[5];
    gth[7] = lI * (double)tg[6];
    gth[8] = lI;
  } else {
    double X = 0.0, G2y = 0.0, sd2 = 0.0;
    if (use_tab) {
      // the table index is below nH <= kSqCap: 32-bit arithmetic
      patch_lds<P, true>(p0, ts, sq + ((cy - mny) * (int)acx + (cx - mnx)), (int)acx, gx, gy0,
                         by, m.gstep, X, G2y, sd2);
    } else if (use_lds) {
      patch_lds<P, false>(p0, ts, sq, 0, gx, gy0, by, m.gstep, X, G2y, sd2);
    } else {
      patch_global<P>(obs, cx - h, cy - h, m.W, m.H, m.b, gx, gy0, by, m.gstep, X, G2y, sd2);
    }
    if constexpr (TILE < kTileCap) {
      // the six-wave shape: the particle index again, from a fresh copy of
      // the thread index, instead of two registers held across the patch
      // sums (they made 13 x 13 spill there)
      int tl = t;
      asm volatile("" : "+v"(tl));
      il = blk * kBlock + tl;
    }
    const int64_t ial = il < m.n ? il : m.n - 1;
    const double I = (double)o.I;
    const double ssq = sd2 - 2.0 * I * X + I * I * (G2x * G2y);
    l = prior_lw(m, b, cur, mode, cdelta, amv, ial) - ssq * m.inv2sig2 - m.lognorm_obs;
  }
  const double e = finish_block(b, cur, il, active, l, o, tile, dsh, L.ksh);
  if constexpr (GRAD) {
    // the block's sum_i E_i d l_i / d theta, weighted like the MMSE sums and
    // reduced the same way: derivatives 0-7 through the tile, 8 through the
    // table's space, eight consecutive entries per thread, then rows
    static_assert(kNGrad == 9 && TILE >= 8 * kBlock && kSqCap >= kBlock,
                  "eight derivatives fill the tile, the ninth goes to the table");
    double v[kNGrad];
#pragma unroll
    for (int d = 0; d < kNGrad; ++d) v[d] = (e > 0.0) ? e * gth[d] : 0.0;
    __syncthreads();  // every thread is past finish_block's reads of the tile
#pragma unroll
    for (int d = 0; d < 8; ++d) tile[d * kBlock + t] = v[d];
    sq[t] = v[8];
    __syncthreads();
    const double* p = tile + (t >> 5) * kBlock + (t & 31) * 8;
    double s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    s = pair_rows(row_allreduce(s, OpAdd()), OpAdd(), 0.0);
    double* RGb = b.RG + blk * kNGrad;
    // derivative 2w in row 1 of wave w, 2w + 1 in row 3
    if (t == 64 * w + 16) RGb[2 * w] = s;
    if (t == 64 * w + 48) RGb[2 * w + 1] = s;
    if (w == 0) {  // uniform: the first wave sums derivative 8
      double s8 = 0.0;
      if (t < 32) {
        const double* q = sq + t * 8;
        s8 = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
      }
      s8 = pair_rows(row_allreduce(s8, OpAdd()), OpAdd(), 0.0);
      if (t == 16) RGb[8] = s8;
    }
  }
}

// Patches up to 13 x 13 come in two workgroup shapes: five waves per SIMD, or
// six with a smaller tile (13 x 13 fits six waves' registers without spilling
// because step_spot recomputes the particle index after the patch sums);
// wider patches keep the compiler's default budget.
template <int P, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kShapeWaves[S])))
void k_step_spot(Model m, Buffers b, const float* __restrict__ obs) {
  __shared__ StepLds<kShapeTile[S]> L;
  step_spot<P, false, kShapeTile[S]>(m, b, obs, blockIdx.x, L);
}

template <int P>
__global__ __launch_bounds__(256) void k_step_spot_wide(Model m, Buffers b,
                                                        const float* __restrict__ obs) {
  __shared__ StepLds<kTileCap> L;
  step_spot<P>(m, b, obs, blockIdx.x, L);
}

// Gradient mode (derivatives of log p^ alongside the step).
template <int P>
__global__ __launch_bounds__(256) void k_step_spot_grad(Model m, Buffers b,
                                                        const float* __restrict__ obs) {
  __shared__ StepLds<kTileCap> L;
  step_spot<P, true>(m, b, obs, blockIdx.x, L);
}

// Linear-Gaussian observation of (x, y, I0): three fp32 values on the device.
__global__ __launch_bounds__(256) void k_step_lg(Model m, Buffers b,
                                                 const float* __restrict__ obs) {
  __shared__ double red[7 * 256];
  __shared__ double dsh[4];
  __shared__ int ksh[4];
  const Ctrl* cp = b.ctrl;
  const int cur = cp->cur, mode = cp->mode, amv = cp->arna_moved;
  const double cdelta = cp->delta;
  const uint32_t k = (uint32_t)(cp->k + 1);
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < m.n;
  Prop o{};
  double l = -INFINITY;
  if (active) {
    o = propagate(m, b, cur, mode, i, k);
    store_state(m, b, cur, i, o);
    const double ex = (double)obs[0] - (double)o.x, ey = (double)obs[1] - (double)o.y,
                 eI = (double)obs[2] - (double)o.I;
    l = prior_lw(m, b, cur, mode, cdelta, amv, i) - ex * ex * m.lg_inv2r2[0] - ey * ey * m.lg_inv2r2[1] - eI * eI * m.lg_inv2r2[2] -
        m.lg_norm;
  }
  finish_block(b, cur, i, active, l, o, red, dsh, ksh);
}

// Records of caller-supplied absolute fp32 log weights (standalone
// resampling): the same layout, with weights e = exp(x - m) in fp64 and zero
// state sums.
__global__ __launch_bounds__(256) void k_records(Model m, Buffers b,
                                                 const float* __restrict__ logw) {
  __shared__ double red[2 * 256];
  __shared__ double dsh[4];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kBlock + t;
  if (i == 0) {
    // the standalone scratch starts uninitialised: clear the counters and
    // flags the following kernels of this call rely on
    Ctrl* c = b.ctrl;
    c->heavy_count = 0;
    c->do_resample = 0;
    c->total = 0;
    c->cur = 0;
    c->k = 0;
  }
  const bool active = i < m.n;
  const double l = active ? (double)logw[i] : -INFINITY;
  const bool bad = active && (isnan(l) || l == INFINITY);
  const double mb = block_reduce((active && !bad) ? l : -INFINITY, dsh, OpMax());
  double e = 0.0;
  if (active && !bad && mb != -INFINITY && l != -INFINITY) e = exp(l - mb);
  red[t] = item_weight(e);
  red[256 + t] = bad ? NAN : e * e;
  __syncthreads();
  double s = 0.0;
  if (t < 64) {
    const double* p = red + (t >> 5) * 256 + (t & 31) * 8;
    s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
  }
  s = row_allreduce(s, OpAdd());
  const double h0 = readlane(s, 0) + readlane(s, 16);
  const double h1 = readlane(s, 32) + readlane(s, 48);
  if (t == 0) {
    double* R = b.R0 + (int64_t)blockIdx.x * kRec;
    R[0] = mb;
    R[1] = h0;
    R[2] = h1;
    for (int d = 0; d < 5; ++d) R[3 + d] = 0.0;
  }
}

// ------------------------------------------------------------- k_merge
// Two launches. Each workgroup of the first merges one chunk of block
// records relative to the chunk's maximum: the chunk record, and per block
// the exclusive prefix of the chunk's integer weights q_b = round(B_b
// exp(m_b - M_c)). One workgroup of the second merges the chunk records in a
// fixed order, takes the statistics of Algorithm 1 (normaliser, ESS, MMSE
// estimate), decides on resampling, commits or rolls back the step, and for
// systematic resampling writes each chunk's fixed-point CDF prefix. (The
// kernel boundary makes the chunk records visible to it: waiting for the
// last chunk inside one launch costs a device-scope release and acquire in
// every workgroup, which write back and invalidate that XCD's L2.)
__device__ __forceinline__ void merge_chunk_body(const Model& m, const Buffers& b, int standalone,
                                                 int64_t ch) {
  __shared__ double dsh[4];
  __shared__ double nsh[4 * 7];
  __shared__ double gsh[4 * kNGrad];
  __shared__ uint64_t ush[4];
  const Ctrl* c = b.ctrl;
  const int t = threadIdx.x;
  const int which = standalone ? 0 : (c->cur ^ 1);  // the records this step wrote
  const double* R = which ? b.R1 : b.R0;
  const int64_t lo = ch * b.chunk, hi = min(b.nb, lo + b.chunk);
  const int per = (int)(b.chunk / 256);
  const int64_t j0 = lo + (int64_t)t * per;

  double mx = -INFINITY;
  for (int q = 0; q < per; ++q) {
    const int64_t j = j0 + q;
    if (j < hi) mx = fmax(mx, R[j * kRec]);
  }
  const double Mc = block_reduce(mx, dsh, OpMax());
  uint64_t qs = 0;
  double s2 = 0.0, ex[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double gs[kNGrad] = {};
  for (int q = 0; q < per; ++q) {
    const int64_t j = j0 + q;
    if (j < hi) {
      const double* r = R + j * kRec;
      const double f = (r[0] == -INFINITY) ? 0.0 : exp(r[0] - Mc);
      qs += (uint64_t)rint(r[1] * f);
      s2 += r[2] * (f * f);
#pragma unroll
      for (int d = 0; d < 5; ++d) ex[d] += r[3 + d] * f;
      if (m.grad && f != 0.0)
#pragma unroll
        for (int d = 0; d < kNGrad; ++d) gs[d] += b.RG[j * kNGrad + d] * f;
    }
  }
  uint64_t qtot;
  uint64_t run = block_excl_sum(qs, ush, &qtot);
  for (int q = 0; q < per; ++q) {
    const int64_t j = j0 + q;
    if (j < hi) {
      const double* r = R + j * kRec;
      const double f = (r[0] == -INFINITY) ? 0.0 : exp(r[0] - Mc);
      b.pfx[j] = run;
      run += (uint64_t)rint(r[1] * f);
    }
  }
  double sums[6] = {s2, ex[0], ex[1], ex[2], ex[3], ex[4]};
  block_sum_n(sums, nsh);
  if (t == 0) {
    double* cr = b.CR + ch * kRec;
    cr[0] = Mc;
    cr[1] = __longlong_as_double((long long)qtot);
#pragma unroll
    for (int d = 0; d < 6; ++d) cr[2 + d] = sums[d];
  }
  if (m.grad) {
    block_sum_n<kNGrad>(gs, gsh);
    if (t == 0)
#pragma unroll
      for (int d = 0; d < kNGrad; ++d) b.CRG[ch * kNGrad + d] = gs[d];
  }
}

__device__ __forceinline__ void merge_final_body(const Model& m, const Buffers& b, int standalone,
                                                 double u_given) {
  __shared__ double dsh[4];
  __shared__ double nsh[4 * 7];
  __shared__ double gsh[4 * kNGrad];
  __shared__ uint64_t ush[4];
  __shared__ int sh_pre;
  __shared__ double sh_delta;
  Ctrl* c = b.ctrl;
  const int t = threadIdx.x;
  const int64_t nch = b.nch;
  const int per2 = (int)((nch + 255) / 256);
  const int64_t c0 = (int64_t)t * per2;
  const double* CRd = b.CR;
  auto ld = [&](int64_t idx) { return CRd[idx]; };
  double mx2 = -INFINITY;
  for (int q = 0; q < per2; ++q) {
    const int64_t cc = c0 + q;
    if (cc < nch) mx2 = fmax(mx2, ld(cc * kRec));
  }
  const double M = block_reduce(mx2, dsh, OpMax());
  double S = 0.0, S2 = 0.0, E[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int q = 0; q < per2; ++q) {
    const int64_t cc = c0 + q;
    if (cc < nch) {
      const double mc = ld(cc * kRec);
      const double f = (mc == -INFINITY) ? 0.0 : exp(mc - M);
      const uint64_t Q = (uint64_t)__double_as_longlong(ld(cc * kRec + 1));
      S += (double)Q * f;
      S2 += ld(cc * kRec + 2) * (f * f);
#pragma unroll
      for (int d = 0; d < 5; ++d) E[d] += ld(cc * kRec + 3 + d) * f;
    }
  }
  {
    double tot7[7] = {S, S2, E[0], E[1], E[2], E[3], E[4]};
    block_sum_n(tot7, nsh);
    S = tot7[0] * (1.0 / kItemScale);
    S2 = tot7[1];
#pragma unroll
    for (int d = 0; d < 5; ++d) E[d] = tot7[2 + d];
  }
  double G[kNGrad] = {};
  if (m.grad) {
    for (int q = 0; q < per2; ++q) {
      const int64_t cc = c0 + q;
      if (cc < nch) {
        const double mc = ld(cc * kRec);
        if (mc != -INFINITY) {
          const double f = exp(mc - M);
#pragma unroll
          for (int d = 0; d < kNGrad; ++d) G[d] += b.CRG[cc * kNGrad + d] * f;
        }
      }
    }
    block_sum_n<kNGrad>(G, gsh);
  }
  if (t == 0) {
    bool ok = isfinite(M) && isfinite(S) && S > 0.0 && isfinite(S2);
#pragma unroll
    for (int d = 0; d < 5; ++d) ok = ok && isfinite(E[d]);
#pragma unroll
    for (int d = 0; d < kNGrad; ++d) ok = ok && isfinite(G[d]);
    int pre = 0;
    if (standalone) {
      c->cur = 0;
      c->delta = ok ? M + log(S) : 0.0;
      c->u = u_given;
      c->do_resample = ok ? 1 : 0;
      c->k = 0;
      pre = ok ? 1 : 0;
    } else if (ok) {
      const int64_t k = c->k + 1;
      const double ess = S * S / S2;
      const double logS = log(S);
      const bool res = ess < m.thr;
      c->k = k;
      c->cur ^= 1;
      c->m = M;
      c->log_sum = logS;
      c->ess = ess;
      c->delta = M + logS;
      c->cum += M + logS;
#pragma unroll
      for (int d = 0; d < 5; ++d) c->mean[d] = E[d] / S;
      if (m.grad)
#pragma unroll
        for (int d = 0; d < kNGrad; ++d) {
          c->grad_last[d] = G[d] / S;
          c->grad_cum[d] += G[d] / S;
        }
      c->resampled = res ? 1 : 0;
      c->do_resample = res ? 1 : 0;
      c->mode = res ? (m.arna ? kModeArna : (m.group > 0 ? kModeRna : kModeSys)) : kModeNone;
      if (m.arna) {
        // the object is lost when this increment falls well below that of
        // the last frame that tracked it; each loss keys a new ring order
        const double inc = M + logS;
        const bool lost = inc < c->delta_ref - m.arna_drop;
        if (lost)
          c->ring_key = k;
        else
          c->delta_ref = inc;
        c->lost = lost ? 1 : 0;
        c->arna_tracking = 0;  // counted by k_arna_local
        c->arna_moved = 0;     // set by k_arna_exchange
      }
      const uint4 rr = draw(m, 0u, (uint32_t)k, kResample, 0u);
      c->u = u53(rr.x, rr.y);
      pre = (res && m.group == 0) ? 1 : 0;
    } else {
      c->rolled_back += 1;
      c->do_resample = 0;
    }
    sh_pre = pre;
    sh_delta = c->delta;
    c->heavy_count = 0;
  }
  __syncthreads();
  if (!sh_pre) return;
  // chunk prefixes of the fixed-point CDF (2^62 = total weight)
  const double delta = sh_delta;
  uint64_t wsum = 0;
  for (int q = 0; q < per2; ++q) {
    const int64_t cc = c0 + q;
    if (cc < nch) {
      const double mc = ld(cc * kRec);
      const double phi = (mc == -INFINITY) ? 0.0 : exp(mc - delta) * kItemToCdf;
      const uint64_t Q = (uint64_t)__double_as_longlong(ld(cc * kRec + 1));
      wsum += (uint64_t)rint((double)Q * phi);
    }
  }
  uint64_t tot;
  uint64_t pre = block_excl_sum(wsum, ush, &tot);
  for (int q = 0; q < per2; ++q) {
    const int64_t cc = c0 + q;
    if (cc < nch) {
      const double mc = ld(cc * kRec);
      const double phi = (mc == -INFINITY) ? 0.0 : exp(mc - delta) * kItemToCdf;
      const uint64_t Q = (uint64_t)__double_as_longlong(ld(cc * kRec + 1));
      b.cpre[cc].P = pre;
      b.cpre[cc].phi = phi;
      pre += (uint64_t)rint((double)Q * phi);
    }
  }
  if (t == 0) c->total = tot;
}

__global__ __launch_bounds__(256) void k_merge(Model m, Buffers b, int standalone) {
  merge_chunk_body(m, b, standalone, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_merge_final(Model m, Buffers b, int standalone,
                                                     double u_given) {
  merge_final_body(m, b, standalone, u_given);
}

// --------------------------------------------------- systematic resampling
// Slot s of N takes the particle j whose CDF interval [C_{j-1}, C_j) holds
// (s + u) / N (Algorithm 1's resampling step with one uniform u), so
// particle j owns the slots [bound(C_{j-1}), bound(C_j)) with bound(C) the
// number of slots below C. Block starts of the CDF are exact 2^62 fixed-point
// integers (so the partition of the slots over segments does not depend on
// summation order); inside a segment the CDF is a running maximum in fp64,
// so particles of zero weight own no slots, and the segment's last particle
// of positive weight takes the segment's remaining slots.

// The CDF at a block start from its block prefix and its chunk's record.
__device__ __forceinline__ double block_cdf(const ChunkPre& cp, uint64_t pfx) {
  return (double)(cp.P + (uint64_t)rint((double)pfx * cp.phi)) * (1.0 / kCdfScale);
}

// Number of slots s in [0, n) with (s + u) / n < C: ceil(C n - u), clamped.
// Monotone in C (the fma rounds once), so bounds taken at non-decreasing CDF
// values never overlap.
__device__ __forceinline__ int slot_bound(double C, double u, double nd, int n) {
  const double x = ceil(fma(C, nd, -u));
  return x <= 0.0 ? 0 : (x >= nd ? n : (int)x);
}

// Systematic resampling runs one wavefront per segment of kSegItems
// particles (kPerThread consecutive per lane, so the 256 particles of a
// block are one row of 16 lanes): every scan and maximum of the segment is
// a DPP operation within the wave and no barrier waits for other waves, so
// each wave streams its weights and ancestors at its own pace. Four blocks
// per wave spread the wave's fixed work (block records, the factor's exp,
// the scans) over 1024 particles.
constexpr int kWave = 64;
constexpr int kPerThread = kSegItems / kWave;  // particles, and slots of a tile, per lane
static_assert(kPerThread == 16 && kSlotTile == kSegItems && kSegBlocks == 4 &&
                  kBlock == 16 * kPerThread,
              "a segment is four blocks of one row each, sixteen particles and slots per lane");
// A tile's slot e lives at word slot_word(e) of the LDS tile, four spare
// words after every sixteen, so that each lane reads its slots with four
// 128-bit loads 80 bytes from its neighbour's (sixteen lanes then cover the
// 64 banks once); the lane-contiguous accesses (slots 4 lane + q of a
// block) meet at most two lanes on a bank.
constexpr int kTileWords = kSlotTile / kPerThread * (kPerThread + 4);
__device__ __forceinline__ int slot_word(int e) { return e + ((e >> 4) << 2); }

// Inclusive maximum scan over the wave of values >= 0 (each DPP step folds
// into one v_max_i32: row shifts, whose lanes outside the row read 0, then
// the row broadcasts into rows 1, 3 and into rows 2, 3). exclusive_of()
// shifts an inclusive scan one lane up (lane 0 reads 0).
__device__ __forceinline__ int wave_max_scan(int v) {
  v = max(v, (int)dpp32<0x111>((uint32_t)v));
  v = max(v, (int)dpp32<0x112>((uint32_t)v));
  v = max(v, (int)dpp32<0x114>((uint32_t)v));
  v = max(v, (int)dpp32<0x118>((uint32_t)v));
  v = max(v, bcast<0x142, 0xa>(v, 0));
  return max(v, bcast<0x143, 0xc>(v, 0));
}
__device__ __forceinline__ int exclusive_of(int inclusive) {
  return (int)dpp32<0x138>((uint32_t)inclusive);  // wave_shr:1
}

// Inclusive sum of exact integers held in doubles over the lanes of one
// block, one row of 16 lanes. Lanes whose source is outside the row read 0,
// the identity.
__device__ __forceinline__ double block_scan_add(double v) {
  v += shr<1>(v);
  v += shr<2>(v);
  v += shr<4>(v);
  v += shr<8>(v);
  return v;
}

// The resampling of one segment by one wave: the segment's slot range from
// its block starts, the particles' CDF from their fixed-point weights, every
// particle's run of slots, and the slots' particles, written tile by tile.
// Slot bounds are monotone in the CDF, so the running maximum that keeps
// runs from overlapping is taken over the integer bounds. LOG: the weights
// are caller log weights (standalone resampling), else the filter's stored
// E.
//
// k_anc runs each segment whose slots span at most kCoopTiles tiles; a
// heavier segment (concentrated weights) queues its tiles in chunks of
// kChunkTiles for k_fill, whose waves each recompute the segment's runs and
// write one chunk, so that heavy segments spread over many waves.
// queued: called by k_fill for the tiles [tile_lo, tile_hi) of the segment.
// One segment's loads, raw: its lanes' weights and its block records. Every
// lane loads (indices clamped into the arrays, values masked at use), so no
// load sits in a divergent branch that would consume it at once.
// The weights arrive lane-contiguous: x[4 h + q] is particle h kBlock +
// 4 lane + q of the segment (each load instruction reads one contiguous
// kWave x 16 bytes); anc_segment hands each lane its own kPerThread
// consecutive particles through the LDS tile.
typedef int V4i __attribute__((ext_vector_type(4)));  // for the nontemporal stores

struct SegIn {
  float x[kPerThread];
  uint64_t pfx;      // the block prefix of the lane's block b0 + lane / 16 (clamped)
  ChunkPre cp;       // its chunk's prefix and factor
  double mbt;        // its record maximum
  uint64_t pfx_end;  // the block prefix of block b0 + nbs, the first after the segment (clamped)
  ChunkPre cp_end;   // its chunk's
};

__device__ __forceinline__ SegIn load_seg(const Model& m, const Buffers& b, const float* E,
                                          const double* rec, bool log_src, int64_t seg) {
  SegIn in;
  const int lane = threadIdx.x;
  const int64_t b0 = seg * kSegBlocks;
  const int nbs = (int)min((int64_t)kSegBlocks, b.nb - b0);
  const int64_t bl = min(b0 + (lane >> 4), b.nb - 1);
  const int64_t be = min(b0 + nbs, b.nb - 1);
  // chunk = 256 per with per <= 8 and blk < 2^23: 32-bit quotients
  const uint32_t cb = (uint32_t)(b.chunk >> 8);
  in.cp = b.cpre[(uint32_t)(bl >> 8) / cb];
  in.pfx = b.pfx[bl];
  in.mbt = rec[bl * kRec];
  in.cp_end = b.cpre[(uint32_t)(be >> 8) / cb];
  in.pfx_end = b.pfx[be];
  const int64_t ib0 = b0 * kBlock;
  const int64_t ib1 = min(m.n, (b0 + nbs) * kBlock);
  if (ib1 - ib0 == kSegItems && (reinterpret_cast<uintptr_t>(E) & 15) == 0) {
    // a whole segment (uniform)
    const float4* v = reinterpret_cast<const float4*>(E + ib0);
#pragma unroll
    for (int h = 0; h < kSegBlocks; ++h) {
      const float4 f = v[h * (kBlock / 4) + lane];
      in.x[4 * h] = f.x;
      in.x[4 * h + 1] = f.y;
      in.x[4 * h + 2] = f.z;
      in.x[4 * h + 3] = f.w;
    }
  } else {
    // the ragged end: weight 0 past the last particle
#pragma unroll
    for (int h = 0; h < kSegBlocks; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = ib0 + h * kBlock + 4 * lane + q;
        const float v = E[min(j, ib1 - 1)];
        in.x[4 * h + q] = (j < ib1) ? v : (log_src ? -INFINITY : 0.0f);
      }
  }
  return in;
}

// The control block's values a resampling pass reads.
struct ResIn {
  int do_res;
  double delta, u;
};

template <bool LOG>
__device__ __forceinline__ void anc_segment(const Model& m, const Buffers& b, const ResIn& ci,
                                            int64_t seg, const SegIn& in, bool queued,
                                            int tile_lo, int tile_hi) {
  __shared__ __align__(16) int A[kTileWords];
  Ctrl* c = b.ctrl;
  const int lane = threadIdx.x;
  const int lb = lane >> 4;  // this lane's block within the segment
  const int64_t b0 = seg * kSegBlocks;
  const int nbs = (int)min((int64_t)kSegBlocks, b.nb - b0);
  const int64_t ib0 = b0 * kBlock;
  const int64_t j0 = ib0 + kPerThread * (int64_t)lane;
  const double delta = ci.delta, u = ci.u;
  // the CDF at this lane's block start and at the block after the segment
  // (blocks past the data read as its end), and the block's factor from
  // integer weights to the CDF
  const bool in_seg = lb < nbs;
  const double Pblk = in_seg ? block_cdf(in.cp, in.pfx) : 1.0;
  const double Pend = b0 + nbs < b.nb ? block_cdf(in.cp_end, in.pfx_end) : 1.0;
  const double f =
      (in_seg && in.mbt != -INFINITY) ? exp(in.mbt - delta) * (1.0 / kItemScale) : 0.0;
  const int n = (int)m.n;
  const double nd = (double)m.n;
  const int fs = seg == 0 ? 0 : slot_bound(readlane(Pblk, 0), u, nd, n);
  const int fe = seg + 1 >= b.nseg ? n : slot_bound(Pend, u, nd, n);
  if (fe <= fs) return;  // uniform: no slot falls in this segment
  const int T0 = fs & ~3;  // tiles start on 16 bytes of anc
  const int ntiles = (fe - T0 + kSlotTile - 1) / kSlotTile;
  if (!queued && ntiles > kCoopTiles) {
    // a heavy segment: its tiles go to k_fill in chunks
    const int chunks = (ntiles + kChunkTiles - 1) / kChunkTiles;
    int base = 0;
    if (lane == 0) base = atomicAdd(&c->heavy_count, chunks);
    base = readlane(base, 0);
    for (int q = lane; q < chunks; q += kWave)
      if (base >= 0 && (int64_t)base + q < b.hq_cap)  // the queue's size rules out overflow
        b.hq[base + q] = TileRun{(int32_t)seg, q * kChunkTiles,
                                 min(ntiles, (q + 1) * kChunkTiles), 0};
    return;
  }

  // each lane's kPerThread consecutive particles from the lane-contiguous
  // loads, through the tile (the tile is free: every earlier call on this
  // workgroup ended with its slots cleared and a barrier); the words a lane
  // reads stay until it clears them before the first tile
  float4* const Af = reinterpret_cast<float4*>(A);
  float4* const minef = Af + (slot_word(kPerThread * lane) >> 2);
#pragma unroll
  for (int h = 0; h < kSegBlocks; ++h)
    Af[slot_word(h * kBlock + 4 * lane) >> 2] =
        make_float4(in.x[4 * h], in.x[4 * h + 1], in.x[4 * h + 2], in.x[4 * h + 3]);
  __syncthreads();
  // a particle's fixed-point weight
  auto weight = [&](float xq) {
    if (LOG)  // particles past the data hold -inf
      return item_weight(xq == -INFINITY ? 0.0 : exp((double)xq - in.mbt));
    return item_weight((double)xq);
  };
  double kl[kPerThread];
  double tsum = 0.0;
#pragma unroll
  for (int r = 0; r < kPerThread / 4; ++r) {
    const float4 v = minef[r];
    const float xr[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      tsum += weight(xr[c4]);
      kl[4 * r + c4] = tsum;
    }
  }
  // prefix of the block's integer weights before this lane's particles
  // (exact: integers < 2^53)
  const double texcl = block_scan_add(tsum) - tsum;
  // each particle's slot bound at its CDF value C = Pblk + K f, with K the
  // block's integer weights up to and including the particle (exact):
  // ceil(C n - u) = ceil(K (n f) + (Pblk n - u)), one fma, at most fe.
  // Rounding may move a bound by one where C n - u is within a few ulps of
  // an integer; the running maximum below keeps the runs disjoint and
  // ordered regardless. Bounds are non-decreasing in K and equal K give
  // equal bounds in every lane of the block, so a particle of zero weight
  // after a positive one repeats its predecessor's bound and gets an empty
  // run. A block's leading particles of zero weight (K = 0) get 0, below
  // every bound: the previous block's CDF is computed apart and may round
  // lower than this block's start.
  const double fn = f * nd;
  const double gb = fma(Pblk, nd, -u);
  const int p0 = (int)j0;  // particle indices are below n < 2^31
  int rb[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const double K = texcl + kl[q];
    // |C n - u| stays far inside the int range (C in [0, 1], n < 2^31)
    rb[q] = K > 0.0 ? min((int)ceil(fma(K, fn, gb)), fe) : 0;
  }
  // the largest bound before the lane (bounds are non-decreasing in a lane)
  const int h0 = max(fs, exclusive_of(wave_max_scan(rb[kPerThread - 1])));
  // The segment's last particle of positive weight ends its runs at fe
  // (those after it have zero weight and empty runs), so every slot has an
  // owner whatever the rounding of the last bounds. Slots after its run's
  // end already take its mark; only if its own run came out empty (its
  // bound rounded to its predecessor's, below fe) does it need a mark, at
  // the start of its extended run: xmb / xmp, uniform, from a replay of that
  // lane's runs (rare: that lane's last bound then fell short of fe).
  int xmb = -1, xmp = 0;
  {
    const uint64_t pos_lanes = __builtin_amdgcn_ballot_w64(tsum > 0.0);
    const int L = 63 - __builtin_clzll(pos_lanes | 1ull);
    if (pos_lanes != 0 && readlane(rb[kPerThread - 1], L) < fe) {
      const double tl = readlane(texcl, L), fnl = readlane(fn, L), gbl = readlane(gb, L);
      const double mL = LOG ? readlane(in.mbt, L) : 0.0;  // lane L's block maximum
      const float* xl = reinterpret_cast<const float*>(A) + slot_word(kPerThread * L);
      int pv = readlane(h0, L), lastq = -1, pstart = 0;
      bool empty = false;
      double kk = 0.0;
#pragma nounroll
      for (int q = 0; q < kPerThread; ++q) {
        const float xq = xl[q];
        const double wq = LOG ? item_weight(xq == -INFINITY ? 0.0 : exp((double)xq - mL))
                              : item_weight((double)xq);
        kk += wq;
        const double K = tl + kk;
        const int rbq = K > 0.0 ? min((int)ceil(fma(K, fnl, gbl)), fe) : 0;
        const int e = max(pv, rbq);
        if (wq > 0.0) {
          lastq = q;
          pstart = pv;
          empty = !(e > pv);
        }
        pv = e;
      }
      if (lastq >= 0 && empty && pstart < fe) {
        const int r = pstart - T0;
        xmb = 4 * r + (r & ~15);
        xmp = p0 - kPerThread * lane + kPerThread * L + lastq;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kPerThread / 4; ++r) minef[r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // particle kPerThread lane + q owns [e_{q-1}, e_q), e_q = max(e_{q-1},
  // rb[q]), e_{-1} = h0. Each non-empty run marks its first slot with the
  // particle; a slot's particle is then the largest mark at or before it.
  // mb: the LDS byte offset of the mark in tile coordinates from T0 (tile j:
  // subtract j kTileWords 4), 4 slot_word(e) = 4 e + (e & ~15), or -1.
  int mb[kPerThread];
  int prev = h0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int e = max(prev, rb[q]);
    const int r = prev - T0;
    mb[q] = e > prev ? 4 * r + (r & ~15) : -1;
    prev = e;
  }
  static_assert(kPerThread == 16, "4 slot_word(e) = 4 e + (e & ~15) for four spare words per sixteen");
  int32_t* anc = m.rpa ? b.asys : b.anc;  // RPA routes the systematic result afterwards
  const bool vec = (reinterpret_cast<uintptr_t>(anc) & 15) == 0;
  const int jt0 = queued ? tile_lo : 0, jt1 = queued ? min(tile_hi, ntiles) : ntiles;
  // the tiles before this call's first: the largest mark among them
  int carry = 0;
  if (jt0 > 0) {
    const int lim = jt0 * kTileWords * 4;  // marks at earlier bytes precede the first tile
#pragma unroll
    for (int q = 0; q < kPerThread; ++q)
      if (mb[q] >= 0 && mb[q] < lim) carry = p0 + q;  // the largest such (mb increases with q)
    carry = readlane(wave_reduce_last(carry, OpMax(), 0), 63);
    if (xmb >= 0 && xmb < lim) carry = xmp;  // the segment's last particle of positive weight
  }
  uint4* A4 = reinterpret_cast<uint4*>(A);
  uint4* mine = A4 + (slot_word(kPerThread * lane) >> 2);
  char* const Ab = reinterpret_cast<char*>(A);
  for (int j = jt0; j < jt1; ++j) {
    const int c0 = T0 + j * kSlotTile, wbase = j * kTileWords * 4;
    __syncthreads();  // one wave: orders the LDS accesses of the lanes
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int eb = mb[q] - wbase;
      if ((unsigned)eb < (unsigned)(kTileWords * 4)) *reinterpret_cast<int*>(Ab + eb) = p0 + q;
    }
    if (lane == 0 && (unsigned)(xmb - wbase) < (unsigned)(kTileWords * 4))
      *reinterpret_cast<int*>(Ab + (xmb - wbase)) = xmp;
    __syncthreads();
    // this lane's slots, their running maximum (particles increase with
    // slots), then the maximum over the lanes before it; 0 (the cleared
    // tile, and DPP's fill) is below every mark that precedes a slot from fs
    // on.
    int v[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread / 4; ++r) {
      const uint4 a = mine[r];
      v[4 * r] = (int)a.x;
      v[4 * r + 1] = (int)a.y;
      v[4 * r + 2] = (int)a.z;
      v[4 * r + 3] = (int)a.w;
    }
#pragma unroll
    for (int q = 1; q < kPerThread; ++q) v[q] = max(v[q], v[q - 1]);
    const int winc = wave_max_scan(v[kPerThread - 1]);
    const int before = max(carry, exclusive_of(winc));
    carry = max(carry, readlane(winc, 63));
    // the slots' particles back into the tile, then out lane-contiguous
    // (slots 4 lane + q of each block-sized quarter of the tile), streamed
    // past the caches; a lane clears the words it reads for the next tile
#pragma unroll
    for (int r = 0; r < kPerThread / 4; ++r)
      mine[r] = make_uint4((uint32_t)max(before, v[4 * r]), (uint32_t)max(before, v[4 * r + 1]),
                           (uint32_t)max(before, v[4 * r + 2]), (uint32_t)max(before, v[4 * r + 3]));
    __syncthreads();
#pragma unroll
    for (int h = 0; h < kSegBlocks; ++h) {
      uint4* src = A4 + (slot_word(h * kBlock + 4 * lane) >> 2);
      const uint4 a = *src;
      *src = make_uint4(0u, 0u, 0u, 0u);
      const int s0 = c0 + h * kBlock + 4 * lane;
      int32_t* out = anc + s0;
      if (vec && s0 >= fs && s0 + 4 <= fe) {
        __builtin_nontemporal_store(V4i{(int)a.x, (int)a.y, (int)a.z, (int)a.w},
                                    reinterpret_cast<V4i*>(out));
      } else {
        const int w4[4] = {(int)a.x, (int)a.y, (int)a.z, (int)a.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (s0 + q >= fs && s0 + q < fe) out[q] = w4[q];
      }
    }
  }
}

__device__ __forceinline__ ResIn res_in(const Ctrl* c) {
  ResIn ci;
  ci.do_res = c->do_resample;
  ci.delta = c->delta;
  ci.u = c->u;
  return ci;
}

// One wave per segment.
template <bool LOG>
__device__ __forceinline__ void anc_seg(const Model& m, const Buffers& b, const WeightSrc& ws,
                                        int64_t seg) {
  const Ctrl* c = b.ctrl;
  const ResIn ci = res_in(c);
  if (!ci.do_res || seg >= b.nseg) return;
  const bool second = ws.use_cur && c->cur;
  const SegIn in = load_seg(m, b, second ? ws.E1 : ws.E0, second ? ws.rec1 : ws.rec0, LOG, seg);
  anc_segment<LOG>(m, b, ci, seg, in, false, 0, 0);
}

__global__ __launch_bounds__(kWave) void k_anc(Model m, Buffers b, WeightSrc ws) {
  anc_seg<false>(m, b, ws, blockIdx.x);
}

// The same on caller log weights (standalone resampling).
__global__ __launch_bounds__(kWave) void k_anc_log(Model m, Buffers b, WeightSrc ws) {
  anc_seg<true>(m, b, ws, blockIdx.x);
}

// The tile chunks of heavy segments queued by k_anc: each wave takes queue
// entries in turn.
// Queue entry q of one filter: its chunk of tiles, then a barrier (the next
// entry clears the tile again).
template <bool LOG>
__device__ __forceinline__ void fill_entry(const Model& m, const Buffers& b, const WeightSrc& ws,
                                           const ResIn& ci, int64_t q) {
  const TileRun r = b.hq[q];
  if (r.seg < 0 || (int64_t)r.seg >= b.nseg || r.tile_lo < 0 || r.tile_hi <= r.tile_lo)
    return;  // uniform across the wave
  const bool second = ws.use_cur && b.ctrl->cur;
  const SegIn in = load_seg(m, b, second ? ws.E1 : ws.E0, second ? ws.rec1 : ws.rec0, LOG, r.seg);
  anc_segment<LOG>(m, b, ci, r.seg, in, true, r.tile_lo, r.tile_hi);
  __syncthreads();
}

template <bool LOG>
__device__ __forceinline__ void fill_body(const Model& m, const Buffers& b, const WeightSrc& ws,
                                          int64_t q0, int64_t qstep) {
  const ResIn ci = res_in(b.ctrl);
  if (!ci.do_res) return;
  const int64_t nh = min((int64_t)b.ctrl->heavy_count, b.hq_cap);
  for (int64_t q = q0; q < nh; q += qstep) fill_entry<LOG>(m, b, ws, ci, q);
}

__global__ __launch_bounds__(kWave) void k_fill(Model m, Buffers b, WeightSrc ws) {
  fill_body<false>(m, b, ws, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kWave) void k_fill_log(Model m, Buffers b, WeightSrc ws) {
  fill_body<true>(m, b, ws, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------- RNA
__device__ __forceinline__ double wave_sum_d(double v, int lane) {
  return wave_reduce(v, lane, OpAdd());
}

// One workgroup per group g (Section 3): local systematic resampling of the
// group's normalised weights, slot weight W_g / n, and the last `moved` slots
// taken from group g-1's local resampling (recomputed here, so no workgroup
// waits for another).
// The normalised weights of group gg's ng particles (E relative to its
// block maximum, or absolute fp32 log weights), their sum W (returned) and
// their local CDF in 2^60 fixed point, C[0..ng), by one 256-thread
// workgroup; dsum and wsum are 4 entries of LDS scratch each.
__device__ __forceinline__ double group_cdf(const WeightSrc& ws, const float* E, const double* rec,
                                            double lognorm, int64_t gg, int ng, uint64_t* C,
                                            double* dsum, uint64_t* wsum) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int ipt = (ng + 255) / 256;
  const int64_t base = gg * ng;
  double wl[4];
  double part = 0.0;
  for (int j = 0; j < ipt; ++j) {
    const int li = t * ipt + j;
    wl[j] = 0.0;
    if (li < ng) {
      const int64_t idx = base + li;
      if (ws.log_src) {
        wl[j] = exp((double)E[idx] - lognorm);
      } else {
        const double mb = rec[(idx / kBlock) * kRec];
        wl[j] = mb == -INFINITY ? 0.0 : (double)E[idx] * exp(mb - lognorm);
      }
      part += wl[j];
    }
  }
  part = wave_sum_d(part, lane);
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
  const uint64_t incl = wave_scan(run, lane, OpAdd());
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint64_t before = 0;
  for (int j = 0; j < w; ++j) before += wsum[j];
  for (int j = 0; j < ipt; ++j) {
    const int li = t * ipt + j;
    if (li < ng) C[li] = before + incl - run + v[j];
  }
  __syncthreads();
  return W;
}

// Local systematic resampling of slot l of a group with CDF C (ng entries)
// and uniform u: the first j with C_j > (l + u) / ng in 2^60 fixed point (the
// identity when the group has no weight).
__device__ __forceinline__ int local_slot(const uint64_t* C, int ng, double inv_ng, double W,
                                          double u, int l) {
  if (!(W > 0.0)) return l;
  const uint64_t us = (uint64_t)(((double)l + u) * inv_ng * 0x1p60);
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid] > us)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// One workgroup per group g (Section 3): local systematic resampling of the
// group's normalised weights, slot weight W_g / n, and the last `moved` slots
// taken from group g-1's local resampling (recomputed here, so no workgroup
// waits for another).
__device__ __forceinline__ void rna_body(const Model& m, const Buffers& b, const WeightSrc& ws,
                                         const double* __restrict__ u_dev, int64_t g) {
  __shared__ uint64_t C[2][kMaxGroup];
  __shared__ double dsum[4];
  __shared__ uint64_t wsum[4];
  Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const bool second = ws.use_cur && c->cur;
  const float* E = second ? ws.E1 : ws.E0;
  const double* rec = second ? ws.rec1 : ws.rec0;
  const int ng = m.group;
  const int64_t G = m.G;
  const int64_t prev = (g + G - 1) % G;
  const double lognorm = c->delta;
  const int t = threadIdx.x;
  double Wg[2];
  double ug[2];
  for (int side = 0; side < 2; ++side) {
    const int64_t gg = side ? prev : g;
    Wg[side] = group_cdf(ws, E, rec, lognorm, gg, ng, C[side], dsum, wsum);
    if (u_dev) {
      ug[side] = u_dev[gg];
    } else {
      const uint4 rr = draw(m, (uint32_t)gg, (uint32_t)c->k, kRna, 0u);
      ug[side] = u53(rr.x, rr.y);
    }
  }
  // slots of group g: own local resampling, then the received tail
  for (int l = t; l < ng; l += 256) {
    const int side = (l >= ng - m.moved) ? 1 : 0;
    const int64_t gg = side ? prev : g;
    const int j = local_slot(C[side], ng, m.inv_group, Wg[side], ug[side], l);
    b.anc[g * ng + l] = (int32_t)(gg * ng + j);
  }
  if (t == 0) b.lwg[g] = log(Wg[0] / (double)ng);
}

__global__ __launch_bounds__(256) void k_rna(Model m, Buffers b, WeightSrc ws,
                                             const double* __restrict__ u_dev) {
  rna_body(m, b, ws, u_dev, blockIdx.x);
}

// ------------------------------------------------------------------ ARNA
// Adaptive RNA (Section 6.4 names its rules; the reading): RNA's local
// resampling per group; G_t groups track (share W_g >= theta / G); mu =
// mu_min + floor((mu_max - mu_min) (G - G_t) / G) slots move per group, from
// its predecessor on a ring of the groups whose order is redrawn whenever the
// object is lost (k_merge_final keys it by the frame of the loss).

// One round value of the ring's Feistel network: the low `half` bits of word
// 0 of the Philox block with counter (R, key, RING << 24 | r, track).
__device__ __forceinline__ uint32_t ring_f(const Model& m, uint32_t key, uint32_t r, uint32_t R,
                                           uint32_t mask) {
  return draw(m, R, key, kRing, r).x & mask;
}

// Eight Feistel rounds (L, R) -> (R, L xor F_r(R)) on the two halves of x,
// and their inverse: a keyed permutation of [0, 2^(2 half)).
__device__ __forceinline__ uint32_t ring_fwd(const Model& m, uint32_t key, int half, uint32_t x) {
  const uint32_t mask = (1u << half) - 1u;
  uint32_t L = x >> half, R = x & mask;
  for (uint32_t r = 0; r < 8; ++r) {
    const uint32_t nl = R;
    R = L ^ ring_f(m, key, r, R, mask);
    L = nl;
  }
  return (L << half) | R;
}
__device__ __forceinline__ uint32_t ring_back(const Model& m, uint32_t key, int half, uint32_t x) {
  const uint32_t mask = (1u << half) - 1u;
  uint32_t L = x >> half, R = x & mask;
  for (int r = 7; r >= 0; --r) {
    const uint32_t pl = R ^ ring_f(m, key, (uint32_t)r, L, mask);
    R = L;
    L = pl;
  }
  return (L << half) | R;
}

// The ring predecessor of group g among G groups under ring key `key`: the
// ring order is the permutation of [0, 2^b) (b the smallest even width with
// 2^b >= G) restricted to [0, G) by cycle walking; g's ring position comes
// from walking the inverse, its predecessor's group from walking forward.
// Key 0: the index ring (g - 1 mod G).
__device__ int64_t ring_pred(const Model& m, uint32_t key, int64_t G, int64_t g) {
  if (key == 0 || G < 2) return (g + G - 1) % G;
  int b = 2;
  while (((int64_t)1 << b) < G) b += 2;
  const int half = b / 2;
  uint32_t x = (uint32_t)g;
  do {
    x = ring_back(m, key, half, x);
  } while ((int64_t)x >= G);
  uint32_t y = (uint32_t)(((int64_t)x + G - 1) % G);
  do {
    y = ring_fwd(m, key, half, y);
  } while ((int64_t)y >= G);
  return (int64_t)y;
}

// One workgroup per group: W_g, the local systematic resampling (global
// indices into aloc), and the tracking count.
// The local resampling of group g into aloc and its share W_g (RNA and
// ARNA; ARNA also counts the tracking groups).
template <bool ARNA>
__device__ __forceinline__ void group_local_body(const Model& m, const Buffers& b, int64_t g) {
  __shared__ uint64_t C[kMaxGroup];
  __shared__ double dsum[4];
  __shared__ uint64_t wsum[4];
  Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int cur = c->cur;
  const WeightSrc ws{b.E0, b.E1, b.R0, b.R1, 1, 0};
  const float* E = cur ? b.E1 : b.E0;
  const double* rec = cur ? b.R1 : b.R0;
  const int ng = m.group;
  const double W = group_cdf(ws, E, rec, c->delta, g, ng, C, dsum, wsum);
  const uint4 rr = draw(m, (uint32_t)g, (uint32_t)c->k, kRna, 0u);
  const double u = u53(rr.x, rr.y);
  for (int l = threadIdx.x; l < ng; l += 256)
    b.aloc[g * ng + l] = (int32_t)(g * ng + local_slot(C, ng, m.inv_group, W, u, l));
  if (threadIdx.x == 0) {
    b.Wg[g] = W;
    if (ARNA && W >= m.arna_share) atomicAdd(&c->arna_tracking, 1);
  }
}

// One workgroup per group: the exchange along the ring and the slot weights.
__device__ __forceinline__ void arna_exchange_body(const Model& m, const Buffers& b, int64_t g) {
  __shared__ int64_t sh_pred;
  Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int64_t G = m.G;
  const int ng = m.group;
  const int64_t mu =
      m.arna_mu_min + ((int64_t)(m.moved - m.arna_mu_min) * (G - c->arna_tracking)) / G;
  if (threadIdx.x == 0) sh_pred = ring_pred(m, (uint32_t)c->ring_key, G, g);
  __syncthreads();
  const int64_t pred = sh_pred;
  for (int l = threadIdx.x; l < ng; l += 256) {
    const int64_t src = (l >= ng - mu) ? pred : g;
    b.anc[g * ng + l] = b.aloc[src * ng + l];
  }
  if (threadIdx.x == 0) {
    b.lwg[g] = log(b.Wg[g] / (double)ng);
    b.lwt[g] = log(b.Wg[pred] / (double)ng);
    if (g == 0) c->arna_moved = (int32_t)mu;
  }
}

__global__ __launch_bounds__(256) void k_arna_local(Model m, Buffers b) {
  group_local_body<true>(m, b, blockIdx.x);
}

// RNA (Section 3) in two launches: the groups' local resampling
// (k_rna_local), then each group's last `moved` slots from group g-1's
// (k_rna_exchange); the same ancestors and weights as rna_body, which
// recomputes group g-1's local resampling in every workgroup instead.
__global__ __launch_bounds__(256) void k_rna_local(Model m, Buffers b) {
  group_local_body<false>(m, b, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_rna_exchange(Model m, Buffers b) {
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int64_t g = blockIdx.x, G = m.G;
  const int ng = m.group;
  const int64_t prev = (g + G - 1) % G;
  for (int l = threadIdx.x; l < ng; l += 256) {
    const int64_t src = (l >= ng - m.moved) ? prev : g;
    b.anc[g * ng + l] = b.aloc[src * ng + l];
  }
  if (threadIdx.x == 0) b.lwg[g] = log(b.Wg[g] / (double)ng);
}

__global__ __launch_bounds__(256) void k_arna_exchange(Model m, Buffers b) {
  arna_exchange_body(m, b, blockIdx.x);
}

// ------------------------------------------------------------------- RPA
// Resampling with proportional allocation (Section 3) over groups of n
// particles: group g's offspring are its share of the global systematic
// resampling (the slots whose ancestor lies in the group; the systematic
// ancestors are non-decreasing, so they form one range, found by binary
// search); a group keeps its first min(N_g, n) offspring, and the DLB
// schedule of Section 4 routes the surplus of the senders (N_g > n) into the
// free slots of the receivers (N_g < n). Greedy matching is the overlap of
// the senders' surplus intervals and the receivers' deficit intervals laid
// end to end in schedule order (group order for GS, by size descending for
// SGS), so each routed slot finds its sender by binary search.

// First index of the non-decreasing a[0..n) with a[i] >= v.
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* a, int64_t n, int64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t rpa_count(const Buffers& b, int64_t g) {
  return b.rfirst[g + 1] - b.rfirst[g];
}

// The groups' offspring ranges: one binary search per group boundary.
__global__ __launch_bounds__(256) void k_rpa_first(Model m, Buffers b) {
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t N = m.n, G = m.rpa_G;
  if (g <= G) b.rfirst[g] = g == G ? N : lower_bound_i32(b.asys, N, g * (int64_t)m.rpa_group);
}

// Surplus (side 0) or deficit (side 1) of group g; 0 when it is not a
// sender (receiver).
__device__ __forceinline__ uint64_t rpa_value(const Buffers& b, int64_t n, int64_t g, int side) {
  const int64_t cg = rpa_count(b, g);
  const int64_t v = side == 0 ? cg - n : n - cg;
  return v > 0 ? (uint64_t)v : 0;
}

// ------------------------------------------------------------ radix sort
// Stable least-significant-digit sort of (uint32 key, int32 value) pairs,
// eight bits per pass, in tiles of kSortTile pairs (256 threads x 4 rounds).
// A pass: the digit's count per tile (k_radix_hist), each digit's row of
// tile counts turned into exclusive prefixes (k_radix_rowscan, one workgroup
// per digit), then every pair written to digit start + tile prefix + its
// rank among the tile's pairs of the same digit in input order
// (k_radix_scatter). `gate`, when given, skips the pass on steps that do not
// resample.
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ key,
                                                    int64_t count, int shift,
                                                    uint32_t* __restrict__ hist, int32_t ntiles,
                                                    const Ctrl* gate) {
  if (gate && !gate->do_resample) return;
  __shared__ uint32_t h[256];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortTile / 256; ++r) {
    const int64_t j = base + r * 256 + t;
    if (j < count) atomicAdd(&h[(key[j] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)t * ntiles + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(256) void k_radix_rowscan(uint32_t* __restrict__ hist, int32_t ntiles,
                                                       uint32_t* __restrict__ rowtot,
                                                       const Ctrl* gate) {
  if (gate && !gate->do_resample) return;
  __shared__ uint64_t sh[4];
  uint32_t* row = hist + (int64_t)blockIdx.x * ntiles;
  uint64_t carry = 0;
  for (int32_t i0 = 0; i0 < ntiles; i0 += 256) {
    const int32_t i = i0 + (int32_t)threadIdx.x;
    const uint64_t v = i < ntiles ? row[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_sum(v, sh, &tot);
    if (i < ntiles) row[i] = (uint32_t)(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = (uint32_t)carry;
}

__global__ __launch_bounds__(256) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    int32_t* __restrict__ vout, int64_t count, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ rowtot, int32_t ntiles, const Ctrl* gate) {
  if (gate && !gate->do_resample) return;
  __shared__ uint32_t run[256];      // the tile's pairs of each digit in earlier rounds
  __shared__ uint32_t wcnt[4][256];  // this round's pairs per wave and digit
  __shared__ uint32_t start[256];    // each digit's first position for this tile
  __shared__ uint64_t sh[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint64_t total;
  const uint64_t dstart = block_excl_sum((uint64_t)rowtot[t], sh, &total);
  start[t] = (uint32_t)dstart + hist[(int64_t)t * ntiles + blockIdx.x];
  run[t] = 0;
  const int64_t tb = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortTile / 256; ++r) {
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) wcnt[ww][t] = 0;
    __syncthreads();
    const int64_t j = tb + r * 256 + t;
    const bool in = j < count;
    const uint32_t key = in ? kin[j] : 0u;
    const int32_t val = in ? vin[j] : 0;
    const uint32_t d = (key >> shift) & 255u;
    // the lanes of this wave holding the same digit
    uint64_t peers = __ballot(in);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t bb = __ballot(set);
      peers &= set ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    if (in && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (in) {
      uint32_t off = start[d] + run[d] + rank;
      for (int ww = 0; ww < w; ++ww) off += wcnt[ww][d];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    run[t] += (wcnt[0][t] + wcnt[1][t]) + (wcnt[2][t] + wcnt[3][t]);
  }
}

// SGS: the sort keys of the 2G list entries, senders (side 0) then
// receivers (side 1), each side by value descending; absent entries (value
// 0) sort last in their side, ties (stable) by group.
__global__ __launch_bounds__(256) void k_rpa_keys(Model m, Buffers b) {
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int64_t G = m.rpa_G;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= 2 * G) return;
  const int side = j >= G ? 1 : 0;
  const int64_t g = j - side * G;
  // values are below N < 2^31
  const uint64_t v = rpa_value(b, m.rpa_group, g, side);
  b.rkey0[j] = ((uint32_t)side << 31) | (v > 0 ? (uint32_t)(0x7fffffffu - (uint32_t)v) : 0x7fffffffu);
  b.rval0[j] = (int32_t)g;
}

// Group at position k of one side's list: group order (GS) or the sorted
// order (SGS: the sort's result is back in the ping buffers).
__device__ __forceinline__ int64_t rpa_at(const Model& m, const Buffers& b, int side, int64_t k) {
  return m.dlb == 1 ? (int64_t)b.rval0[side * (int64_t)m.rpa_G + k] : k;
}

// The plan: over each side's list in schedule order, the exclusive prefix of
// the values (and, for the senders, of their count), in three launches:
// per tile of kSortTile positions the sum and the count present
// (k_rpa_plan_tiles), their exclusive prefixes over the tiles
// (k_rpa_plan_scan, one workgroup per side), then each position's prefixes
// (k_rpa_plan_apply): each sender's position in the sender order and the
// prefix of the surplus before it, each receiver's first surplus particle.
__global__ __launch_bounds__(256) void k_rpa_plan_tiles(Model m, Buffers b) {
  __shared__ uint64_t sh[4];
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int side = blockIdx.y;
  const int64_t G = m.rpa_G, n = m.rpa_group;
  const int64_t nt2 = (G + kSortTile - 1) / kSortTile;
  const int64_t k0 = (int64_t)blockIdx.x * kSortTile + 4 * threadIdx.x;
  uint64_t sv = 0, sp = 0;
  for (int i = 0; i < 4; ++i) {
    const int64_t k = k0 + i;
    if (k < G) {
      const uint64_t v = rpa_value(b, n, rpa_at(m, b, side, k), side);
      sv += v;
      sp += v > 0 ? 1 : 0;
    }
  }
  uint64_t tv, tp;
  block_excl_sum(sv, sh, &tv);
  block_excl_sum(sp, sh, &tp);
  if (threadIdx.x == 0) {
    b.rtsum[2 * (side * nt2 + blockIdx.x)] = tv;
    b.rtsum[2 * (side * nt2 + blockIdx.x) + 1] = tp;
  }
}

__global__ __launch_bounds__(256) void k_rpa_plan_scan(Model m, Buffers b) {
  __shared__ uint64_t sh[4];
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int side = blockIdx.x;
  const int64_t G = m.rpa_G;
  const int64_t nt2 = (G + kSortTile - 1) / kSortTile;
  uint64_t* ts = b.rtsum + 2 * side * nt2;
  uint64_t cv = 0, cp = 0;
  for (int64_t i0 = 0; i0 < nt2; i0 += 256) {
    const int64_t i = i0 + threadIdx.x;
    const uint64_t v = i < nt2 ? ts[2 * i] : 0, p = i < nt2 ? ts[2 * i + 1] : 0;
    uint64_t tv, tp;
    const uint64_t ev = block_excl_sum(v, sh, &tv);
    const uint64_t ep = block_excl_sum(p, sh, &tp);
    if (i < nt2) {
      ts[2 * i] = cv + ev;
      ts[2 * i + 1] = cp + ep;
    }
    cv += tv;
    cp += tp;
  }
  if (side == 0 && threadIdx.x == 0) {
    b.rns[0] = (int32_t)cp;
    b.rscum[cp] = (int64_t)cv;
  }
}

__global__ __launch_bounds__(256) void k_rpa_plan_apply(Model m, Buffers b) {
  __shared__ uint64_t sh[4];
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int side = blockIdx.y;
  const int64_t G = m.rpa_G, n = m.rpa_group;
  const int64_t nt2 = (G + kSortTile - 1) / kSortTile;
  const int64_t k0 = (int64_t)blockIdx.x * kSortTile + 4 * threadIdx.x;
  int64_t g[4];
  uint64_t v[4];
  uint64_t sv = 0, sp = 0;
  for (int i = 0; i < 4; ++i) {
    const int64_t k = k0 + i;
    g[i] = k < G ? rpa_at(m, b, side, k) : 0;
    v[i] = k < G ? rpa_value(b, n, g[i], side) : 0;
    sv += v[i];
    sp += v[i] > 0 ? 1 : 0;
  }
  uint64_t tv, tp;
  uint64_t pv = block_excl_sum(sv, sh, &tv) + b.rtsum[2 * (side * nt2 + blockIdx.x)];
  uint64_t pp = block_excl_sum(sp, sh, &tp) + b.rtsum[2 * (side * nt2 + blockIdx.x) + 1];
  for (int i = 0; i < 4; ++i) {
    if (v[i] > 0) {
      if (side == 0) {
        b.rscum[pp] = (int64_t)pv;
        b.rsidx[g[i]] = (int32_t)pp;
      } else {
        b.rdbase[g[i]] = (int64_t)pv;
      }
      pv += v[i];
      pp += 1;
    }
  }
}

// The surplus stream: the q-th surplus offspring in schedule order is
// offspring n + j of the sender at position i of the sender order, where q =
// (surplus of the senders before i) + j. Each thread takes four consecutive
// systematic slots t: slot t is offspring t - first(g) of the group g that
// holds its ancestor (every load is issued before any store).
__global__ __launch_bounds__(256) void k_rpa_stream(Model m, Buffers b) {
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int64_t t0 = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  const int64_t N = m.n;
  if (t0 >= N) return;
  const int64_t n = m.rpa_group;
  const int32_t* __restrict__ asys = b.asys;
  int32_t a[4];
  if (t0 + 4 <= N && (reinterpret_cast<uintptr_t>(asys + t0) & 15) == 0) {
    const int4 v = *reinterpret_cast<const int4*>(asys + t0);
    a[0] = v.x;
    a[1] = v.y;
    a[2] = v.z;
    a[3] = v.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = asys[min(t0 + i, N - 1)];
  }
  int64_t q[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // ancestors are below N < 2^31: a 32-bit quotient
    const int64_t g = (int64_t)((uint32_t)a[i] / (uint32_t)n);
    const int64_t j = t0 + i - b.rfirst[g] - n;
    q[i] = (t0 + i < N && j >= 0) ? b.rscum[b.rsidx[g]] + j : -1;  // -1: kept by its group
  }
  int32_t* __restrict__ out = b.rstream;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (q[i] >= 0 && q[i] < N) out[q[i]] = a[i];  // a balanced plan has q < N
}

// Four consecutive output slots per thread: each takes its group's own
// offspring first, then the surplus stream from the receiver's first
// surplus particle (every load is issued before any store).
__global__ __launch_bounds__(256) void k_rpa_route(Model m, Buffers b) {
  const Ctrl* c = b.ctrl;
  if (!c->do_resample) return;
  const int64_t s0 = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  const int64_t N = m.n;
  if (s0 >= N) return;
  const int64_t n = m.rpa_group;
  const int32_t* __restrict__ asys = b.asys;
  const int32_t* __restrict__ stream = b.rstream;
  int32_t v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t s = min(s0 + i, N - 1);
    const int64_t g = (int64_t)((uint32_t)s / (uint32_t)n);
    const int64_t p = s - g * n;
    const int64_t f0 = b.rfirst[g];
    const int64_t keep = min(b.rfirst[g + 1] - f0, n);
    const int64_t q = min(max(b.rdbase[g] + (p - keep), (int64_t)0), N - 1);
    // (both indices stay in [0, N) whichever way the choice goes; a balanced
    // plan never clamps q)
    v[i] = p < keep ? asys[min(f0 + p, N - 1)] : stream[q];
  }
  int32_t* __restrict__ out = b.anc;
  if (s0 + 4 <= N && (reinterpret_cast<uintptr_t>(out + s0) & 15) == 0) {
    *reinterpret_cast<int4*>(out + s0) = make_int4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (s0 + i < N) out[s0 + i] = v[i];
  }
}

// ------------------------------------------------ standalone DLB schedules
// The DLB schedules of Section 4 for any number of groups. The lists: the
// 2G entries (senders, then receivers) radix-sorted by key, where GS keys a
// present entry by its group and SGS / LGS by the complement of its value
// (descending, ties in group order); absent entries sort last in their side.
__global__ __launch_bounds__(256) void k_dlb_keys(int32_t kind, const int32_t* __restrict__ counts,
                                                  int32_t G, int32_t n, uint32_t* __restrict__ key,
                                                  int32_t* __restrict__ val) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= 2 * (int64_t)G) return;
  const int side = j >= G ? 1 : 0;
  const int64_t g = j - side * (int64_t)G;
  const int64_t v = side == 0 ? (int64_t)counts[g] - n : (int64_t)n - counts[g];
  // values and groups are below 2^31
  const uint32_t low = v <= 0 ? 0x7fffffffu
                              : (kind == 0 ? (uint32_t)g : 0x7fffffffu - (uint32_t)min(v, (int64_t)0x7ffffffe));
  key[j] = ((uint32_t)side << 31) | low;
  val[j] = (int32_t)g;
}

__global__ __launch_bounds__(64) void k_zero_i32(int32_t* __restrict__ p, int32_t count) {
  if ((int32_t)threadIdx.x < count) p[threadIdx.x] = 0;
}

// The surplus (side 0) or deficit (side 1) at each list position, 0 past
// the present entries.
__global__ __launch_bounds__(256) void k_dlb_values(const int32_t* __restrict__ counts, int32_t G,
                                                    int32_t n, const int32_t* __restrict__ val,
                                                    uint64_t* __restrict__ vals) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= 2 * (int64_t)G) return;
  const int side = j >= G ? 1 : 0;
  const int64_t c = counts[val[j]];
  const int64_t v = side == 0 ? c - n : n - c;
  vals[j] = v > 0 ? (uint64_t)v : 0;
}

// Exclusive prefix sums over `len` uint64 values (tiles of kSortTile: the
// tiles' sums, their prefixes in one workgroup, then each value's prefix);
// out[len] receives the total.
__global__ __launch_bounds__(256) void k_scan_tiles(const uint64_t* __restrict__ in, int64_t len,
                                                    uint64_t* __restrict__ tsum) {
  __shared__ uint64_t sh[4];
  const int64_t k0 = (int64_t)blockIdx.x * kSortTile + 4 * threadIdx.x;
  uint64_t s = 0;
  for (int i = 0; i < 4; ++i)
    if (k0 + i < len) s += in[k0 + i];
  uint64_t tot;
  block_excl_sum(s, sh, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_top(uint64_t* __restrict__ tsum, int64_t ntiles,
                                                  uint64_t* __restrict__ total) {
  __shared__ uint64_t sh[4];
  uint64_t carry = 0;
  for (int64_t i0 = 0; i0 < ntiles; i0 += 256) {
    const int64_t i = i0 + threadIdx.x;
    const uint64_t v = i < ntiles ? tsum[i] : 0;
    uint64_t t;
    const uint64_t ex = block_excl_sum(v, sh, &t);
    if (i < ntiles) tsum[i] = carry + ex;
    carry += t;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint64_t* __restrict__ in, int64_t len,
                                                    const uint64_t* __restrict__ tsum,
                                                    uint64_t* __restrict__ out) {
  __shared__ uint64_t sh[4];
  const int64_t k0 = (int64_t)blockIdx.x * kSortTile + 4 * threadIdx.x;
  uint64_t v[4], s = 0;
  for (int i = 0; i < 4; ++i) {
    v[i] = k0 + i < len ? in[k0 + i] : 0;
    s += v[i];
  }
  uint64_t tot;
  uint64_t p = block_excl_sum(s, sh, &tot) + tsum[blockIdx.x];
  for (int i = 0; i < 4; ++i) {
    if (k0 + i < len) out[k0 + i] = p;
    p += v[i];
  }
}

// Number of the leading positive values of one side (its present entries).
__global__ __launch_bounds__(256) void k_dlb_present(const uint64_t* __restrict__ vals, int32_t G,
                                                     int32_t* __restrict__ nsr) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= 2 * (int64_t)G) return;
  const int side = j >= G ? 1 : 0;
  const int64_t k = j - side * (int64_t)G;
  // present entries come first: the last one marks the count
  if (vals[j] > 0 && (k + 1 == G || vals[j + 1] == 0)) nsr[side] = (int32_t)(k + 1);
}

// GS / SGS: the greedy walk of the two lists (Alg. 2, with filled receivers
// skipped) pairs sender i with every receiver whose deficit interval
// [cd_j, cd_j + de_j) overlaps its surplus interval [cs_i, cs_i + su_i),
// both laid end to end in list order and cut at T = min(total surplus,
// total deficit). Per sender: its first receiver and its number of entries.
__global__ __launch_bounds__(256) void k_dlb_count(const uint64_t* __restrict__ cs,
                                                   const uint64_t* __restrict__ cd,
                                                   const int32_t* __restrict__ nsr, int32_t G,
                                                   int32_t* __restrict__ jlo,
                                                   uint64_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= G) return;
  const int64_t ns = nsr[0], nr = nsr[1];
  const uint64_t T = min(cs[ns], cd[nr]);
  cnt[i] = 0;
  if (i >= ns || cs[i] >= T) return;
  const uint64_t* d = cd;
  // last j with d[j] <= cs[i], then last j with d[j] < min(cs[i + 1], T)
  int64_t lo = 0, hi = nr - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (d[mid] <= cs[i]) lo = mid;
    else hi = mid - 1;
  }
  const uint64_t end = min(cs[i + 1], T);
  int64_t lo2 = lo, hi2 = nr - 1;
  while (lo2 < hi2) {
    const int64_t mid = (lo2 + hi2 + 1) >> 1;
    if (d[mid] < end) lo2 = mid;
    else hi2 = mid - 1;
  }
  jlo[i] = (int32_t)lo;
  cnt[i] = (uint64_t)(lo2 - lo + 1);
}

// Entry e: GS / SGS its sender (the last with entry prefix <= e) and
// receiver, the overlap of their intervals; LGS the e-th sender with the e-th
// receiver and the smaller of their values (Alg. 4, the count recorded before
// it is zeroed). Thread 0 writes the number of entries, or -1 past cap.
__global__ __launch_bounds__(256) void k_dlb_entries(int32_t kind, const int32_t* __restrict__ val,
                                                     const uint64_t* __restrict__ vals,
                                                     const uint64_t* __restrict__ cs,
                                                     const uint64_t* __restrict__ cd,
                                                     const int32_t* __restrict__ nsr, int32_t G,
                                                     const int32_t* __restrict__ jlo,
                                                     const uint64_t* __restrict__ E,
                                                     int32_t* __restrict__ sched, int32_t cap,
                                                     int32_t* __restrict__ n_entries) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t ns = nsr[0], nr = nsr[1];
  const int64_t M = kind == 2 ? min(ns, nr) : (int64_t)E[G];
  if (e == 0) *n_entries = M <= cap ? (int32_t)M : -1;
  if (e >= M || M > cap) return;  // nothing is written past the capacity
  int64_t i, j;
  uint64_t amount;
  if (kind == 2) {
    i = e;
    j = e;
    amount = min(vals[i], vals[G + j]);
  } else {
    int64_t lo = 0, hi = ns - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (E[mid] <= (uint64_t)e) lo = mid;
      else hi = mid - 1;
    }
    i = lo;
    j = jlo[i] + (e - (int64_t)E[i]);
    const uint64_t* d = cd;
    const uint64_t T = min(cs[ns], d[nr]);
    amount = min(min(cs[i + 1], d[j + 1]), T) - max(cs[i], d[j]);
  }
  sched[3 * e] = val[i];
  sched[3 * e + 1] = val[G + j];
  sched[3 * e + 2] = (int32_t)amount;
}

// --------------------------------------------------------------- batches
// Independent filters (tracks) advance together: each launch covers every
// track, one workgroup per work item (track, index of the track's block,
// chunk, segment or group) from a list built on the host, with the track's
// model and buffers read from device arrays.
__device__ __forceinline__ WeightSrc own_weights(const Buffers& b) {
  WeightSrc w{};
  w.E0 = b.E0;
  w.E1 = b.E1;
  w.rec0 = b.R0;
  w.rec1 = b.R1;
  w.use_cur = 1;
  w.log_src = 0;
  return w;
}

__global__ __launch_bounds__(256) void k_init_batch(const Model* __restrict__ ms,
                                                    const Buffers* __restrict__ bs,
                                                    const BatchItem* __restrict__ items) {
  const BatchItem it = items[blockIdx.x];
  init_body(ms[it.track], bs[it.track], it.idx);
}

template <int P>
__global__ __launch_bounds__(256) void k_step_batch_wide(const Model* __restrict__ ms,
                                                         const Buffers* __restrict__ bs,
                                                         const BatchItem* __restrict__ items,
                                                         const float* __restrict__ obs) {
  __shared__ StepLds<kTileCap> L;
  const BatchItem it = items[blockIdx.x];
  step_spot<P>(ms[it.track], bs[it.track], obs, it.idx, L);
}

// Every patch size up to kFusedMaxP in one launch of workgroup shape S: each
// workgroup takes its item's patch size (uniform across the workgroup) and
// shares one LDS block.
template <int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kShapeWaves[S])))
void k_step_batch_fused(const Model* __restrict__ ms, const Buffers* __restrict__ bs,
                        const BatchItem* __restrict__ items, const float* __restrict__ obs) {
  constexpr int T = kShapeTile[S];
  __shared__ StepLds<T> L;
  const BatchItem it = items[blockIdx.x];
  const Model& m = ms[it.track];
  const Buffers& b = bs[it.track];
  switch (m.P) {
    case 1: step_spot<1, false, T>(m, b, obs, it.idx, L); break;
    case 3: step_spot<3, false, T>(m, b, obs, it.idx, L); break;
    case 5: step_spot<5, false, T>(m, b, obs, it.idx, L); break;
    case 7: step_spot<7, false, T>(m, b, obs, it.idx, L); break;
    case 9: step_spot<9, false, T>(m, b, obs, it.idx, L); break;
    case 11: step_spot<11, false, T>(m, b, obs, it.idx, L); break;
    case 13: step_spot<13, false, T>(m, b, obs, it.idx, L); break;
    default: break;  // the host puts only these sizes in a fused launch
  }
}
static_assert(kFusedMaxP == 13, "k_step_batch_fused handles the odd patch sizes up to 13");

__global__ __launch_bounds__(256) void k_merge_batch(const Model* __restrict__ ms,
                                                     const Buffers* __restrict__ bs,
                                                     const BatchItem* __restrict__ items) {
  const BatchItem it = items[blockIdx.x];
  merge_chunk_body(ms[it.track], bs[it.track], 0, it.idx);
}

// One workgroup per track.
__global__ __launch_bounds__(256) void k_merge_final_batch(const Model* __restrict__ ms,
                                                           const Buffers* __restrict__ bs) {
  merge_final_body(ms[blockIdx.x], bs[blockIdx.x], 0, 0.0);
}

__global__ __launch_bounds__(kWave) void k_anc_batch(const Model* __restrict__ ms,
                                                   const Buffers* __restrict__ bs,
                                                   const BatchItem* __restrict__ items) {
  const BatchItem it = items[blockIdx.x];
  const Buffers& b = bs[it.track];
  anc_seg<false>(ms[it.track], b, own_weights(b), it.idx);
}

// The queued chunks of all the tracks in `tracks` as one list, track after
// track (a track that did not resample this step has none). Wave w takes the
// list entries w, w + gridDim.x, ..., so a track whose weights collapsed gets
// as many waves as its chunks need. The tracks are counted kFillTracks at a
// time, their loads issued together.
constexpr int kFillTracks = 4 * kWave;
__global__ __launch_bounds__(kWave) void k_fill_batch(const Model* __restrict__ ms,
                                                    const Buffers* __restrict__ bs,
                                                    const int32_t* __restrict__ tracks,
                                                    int32_t n_tracks) {
  const int lane = threadIdx.x;
  const int64_t G = gridDim.x;
  int64_t base = 0;  // list entries of the tracks before this pass's
  for (int32_t j0 = 0; j0 < n_tracks; j0 += kFillTracks) {
    int32_t tr[4];
    int cnt[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t j = j0 + u * kWave + lane;
      tr[u] = j < n_tracks ? tracks[j] : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cnt[u] = 0;
      if (tr[u] >= 0) {
        const Buffers& b = bs[tr[u]];
        const Ctrl* c = b.ctrl;
        if (c->do_resample) cnt[u] = (int)max((int64_t)0, min((int64_t)c->heavy_count, b.hq_cap));
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int incl = wave_scan(cnt[u], lane, OpAdd());
      const int tot = readlane(incl, 63);
      // the first list entry at or after base that is this wave's
      int64_t off = ((int64_t)blockIdx.x - base % G) % G;
      if (off < 0) off += G;
      for (int64_t q = base + off; q < base + tot; q += G) {
        const int r = (int)(q - base);
        // the lane whose entries [incl - cnt, incl) hold r: the lanes below
        // it are those whose entries end at or before r
        const int owner = __popcll(__ballot(incl <= r));
        const int32_t t_own = readlane(tr[u], owner);
        const int first = readlane(incl - cnt[u], owner);
        const Buffers& b = bs[t_own];
        fill_entry<false>(ms[t_own], b, own_weights(b), res_in(b.ctrl), r - first);
      }
      base += tot;
    }
  }
}

__global__ __launch_bounds__(256) void k_rna_batch(const Model* __restrict__ ms,
                                                   const Buffers* __restrict__ bs,
                                                   const BatchItem* __restrict__ items) {
  const BatchItem it = items[blockIdx.x];
  const Buffers& b = bs[it.track];
  rna_body(ms[it.track], b, own_weights(b), nullptr, it.idx);
}

// ------------------------------------------------------------- utilities
__global__ __launch_bounds__(256) void k_gather(Model m, Buffers b, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  const Ctrl* c = b.ctrl;
  const float* X = c->cur ? b.X1 : b.X0;
  const int mode = c->mode;
  const int64_t p = (mode == kModeSys || mode == kModeRna || mode == kModeArna) ? b.anc[i] : i;
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
  const float* E = c->cur ? b.E1 : b.E0;
  const double* R = c->cur ? b.R1 : b.R0;
  b.lw64[i] = log((double)E[i]) + R[(i / kBlock) * kRec] - c->delta;
}

__global__ void k_set_mode(Ctrl* c, int32_t mode) { c->mode = mode; }

__global__ __launch_bounds__(256) void k_philox(uint32_t k0, uint32_t k1,
                                                const uint4* __restrict__ ctr,
                                                uint4* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = philox(ctr[i], k0, k1);
}

// ---------------------------------------------------------------- launches
// Every kernel goes out through launch_k: onto the stream, or, while a
// StepGraph records on the calling thread, into its graph.
thread_local StepGraph* t_rec = nullptr;

template <class... T>
struct ArgTuple final : StepGraph::Args {
  std::tuple<T...> v;
  template <class... A>
  explicit ArgTuple(A&&... a) : v(std::forward<A>(a)...) {}
};

template <class Tup, size_t... I>
std::array<void*, sizeof...(I)> arg_ptrs(Tup& t, std::index_sequence<I...>) {
  return {{static_cast<void*>(&std::get<I>(t))...}};
}

template <class T>
void note_frame(T&, const float*, std::vector<const float**>*) {}
void note_frame(const float*& p, const float* frame, std::vector<const float**>* out) {
  if (p == frame) out->push_back(&p);
}

template <class... P, class... A>
hipError_t launch_k(void (*k)(P...), dim3 grid, dim3 block, hipStream_t s, A&&... a) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  constexpr auto idx = std::index_sequence_for<P...>{};
  if (!t_rec) {
    std::tuple<P...> v(std::forward<A>(a)...);
    std::array<void*, sizeof...(P)> argv = arg_ptrs(v, idx);
    return hipLaunchKernel(reinterpret_cast<const void*>(k), grid, block, argv.data(), 0, s);
  }
  auto pack = std::make_unique<ArgTuple<P...>>(std::forward<A>(a)...);
  const std::array<void*, sizeof...(P)> argv = arg_ptrs(pack->v, idx);
  std::vector<const float**> slots;
  std::apply([&](auto&... x) { (note_frame(x, t_rec->frame(), &slots), ...); }, pack->v);
  return t_rec->add(reinterpret_cast<const void*>(k), grid, block, std::move(pack),
                    std::vector<void*>(argv.begin(), argv.end()), std::move(slots));
}

template <int P>
hipError_t launch_spot(const Model& m, const Buffers& b, const float* obs, hipStream_t s) {
  const dim3 grid((unsigned)b.nb), block(kBlock);
  if (m.grad) return launch_k(k_step_spot_grad<P>, grid, block, s, m, b, obs);
  if constexpr (P <= kFusedMaxP) {
    if (m.shape == 1) return launch_k(k_step_spot<P, 1>, grid, block, s, m, b, obs);
    return launch_k(k_step_spot<P, 0>, grid, block, s, m, b, obs);
  }
  return launch_k(k_step_spot_wide<P>, grid, block, s, m, b, obs);
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

template <int P>
hipError_t launch_spot_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                             int64_t n_items, const float* obs, hipStream_t s) {
  return launch_k(k_step_batch_wide<P>, dim3((unsigned)n_items), dim3(kBlock), s, ms, bs, items,
                  obs);
}

}  // namespace

StepGraph::~StepGraph() {
  if (t_rec == this) t_rec = nullptr;
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (graph_) (void)hipGraphDestroy(graph_);
}

hipError_t StepGraph::begin(const float* frame) {
  if (t_rec || graph_) return hipErrorInvalidValue;  // one recording per graph and thread
  const hipError_t e = hipGraphCreate(&graph_, 0);
  if (e != hipSuccess) return e;
  frame_ = frame;
  t_rec = this;
  return hipSuccess;
}

hipError_t StepGraph::end() {
  if (t_rec != this) return hipErrorInvalidValue;
  t_rec = nullptr;
  if (nodes_.empty()) return hipErrorInvalidValue;
  return hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0);
}

hipError_t StepGraph::add(const void* fn, dim3 grid, dim3 block, std::unique_ptr<Args> args,
                          std::vector<void*> argv, std::vector<const float**> frame_slots) {
  Node n;
  n.args = std::move(args);
  n.argv = std::move(argv);
  n.frame_slots = std::move(frame_slots);
  n.params.func = const_cast<void*>(fn);
  n.params.gridDim = grid;
  n.params.blockDim = block;
  n.params.sharedMemBytes = 0;
  n.params.kernelParams = n.argv.data();  // moving the vector keeps its storage
  n.params.extra = nullptr;
  const hipGraphNode_t* deps = deps_.empty() ? nullptr : deps_.data();
  const hipError_t e = hipGraphAddKernelNode(&n.node, graph_, deps, deps_.size(), &n.params);
  if (e != hipSuccess) return e;
  if (in_group_)
    group_.push_back(n.node);
  else
    deps_.assign(1, n.node);
  nodes_.push_back(std::move(n));
  return hipSuccess;
}

void StepGraph::group_begin() {
  in_group_ = true;
  group_.clear();
}

void StepGraph::group_end() {
  in_group_ = false;
  if (!group_.empty()) deps_ = group_;
  group_.clear();
}

void launch_group_begin() {
  if (t_rec) t_rec->group_begin();
}

void launch_group_end() {
  if (t_rec) t_rec->group_end();
}

hipError_t StepGraph::set_frame(const float* frame) {
  if (!exec_) return hipErrorInvalidValue;
  if (frame == frame_) return hipSuccess;
  for (Node& n : nodes_) {
    if (n.frame_slots.empty()) continue;
    for (const float** slot : n.frame_slots) *slot = frame;
    const hipError_t e = hipGraphExecKernelNodeSetParams(exec_, n.node, &n.params);
    if (e != hipSuccess) return e;
  }
  frame_ = frame;
  return hipSuccess;
}

// Scratch of the allocation-free standalone resampler: every device that
// runs it holds one copy until the process ends. Host code must not use the
// array's name as a device address (on the host it names a stand-in): the
// device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr, size_t* bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // with this device current: its own copy of the array
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

hipError_t launch_init(const Model& m, const Buffers& b, hipStream_t s) {
  hipError_t e = launch_k(k_init, dim3(grid_for(m.n, 256)), dim3(256), s, m, b);
  if (e != hipSuccess || m.init_kind != 3) return e;
  // Z order: sort the keys with their draw indices (stable), then place
  const int32_t nt = (int32_t)((m.n + kSortTile - 1) / kSortTile);
  const Ctrl* nogate = nullptr;
  for (int pass = 0; pass < 4 && e == hipSuccess; ++pass) {
    const uint32_t* kin = pass & 1 ? b.zkey1 : b.zkey0;
    const int32_t* vin = pass & 1 ? b.zval1 : b.zval0;
    uint32_t* kout = pass & 1 ? b.zkey0 : b.zkey1;
    int32_t* vout = pass & 1 ? b.zval0 : b.zval1;
    e = launch_k(k_radix_hist, dim3((unsigned)nt), dim3(256), s, kin, m.n, 8 * pass, b.zhist, nt,
                 nogate);
    if (e == hipSuccess)
      e = launch_k(k_radix_rowscan, dim3(256), dim3(256), s, b.zhist, nt, b.zrow, nogate);
    if (e == hipSuccess)
      e = launch_k(k_radix_scatter, dim3((unsigned)nt), dim3(256), s, kin, vin, kout, vout, m.n,
                   8 * pass, (const uint32_t*)b.zhist, (const uint32_t*)b.zrow, nt, nogate);
  }
  if (e == hipSuccess) e = launch_k(k_init_place, dim3(grid_for(m.n, 256)), dim3(256), s, m, b);
  return e;
}

hipError_t launch_step(const Model& m, const Buffers& b, const float* obs, hipStream_t s) {
  if (m.obs == 1) {
    return launch_k(k_step_lg, dim3((unsigned)b.nb), dim3(kBlock), s, m, b, obs);
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

hipError_t launch_init_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                             int64_t n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  return launch_k(k_init_batch, dim3((unsigned)n_items), dim3(kBlock), s, ms, bs, items);
}

hipError_t launch_step_batch_fused(int shape, const Model* ms, const Buffers* bs,
                                   const BatchItem* items, int64_t n_items, const float* obs,
                                   hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const dim3 grid((unsigned)n_items), block(kBlock);
  if (shape == 1) return launch_k(k_step_batch_fused<1>, grid, block, s, ms, bs, items, obs);
  return launch_k(k_step_batch_fused<0>, grid, block, s, ms, bs, items, obs);
}

hipError_t launch_step_batch(int P, const Model* ms, const Buffers* bs, const BatchItem* items,
                             int64_t n_items, const float* obs, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (P) {
    case 15: return launch_spot_batch<15>(ms, bs, items, n_items, obs, s);
    case 17: return launch_spot_batch<17>(ms, bs, items, n_items, obs, s);
    case 19: return launch_spot_batch<19>(ms, bs, items, n_items, obs, s);
    case 21: return launch_spot_batch<21>(ms, bs, items, n_items, obs, s);
    case 23: return launch_spot_batch<23>(ms, bs, items, n_items, obs, s);
    case 25: return launch_spot_batch<25>(ms, bs, items, n_items, obs, s);
    default: return hipErrorInvalidValue;  // sizes up to kFusedMaxP go to the fused launch
  }
}

hipError_t launch_merge_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                              int64_t n_items, int32_t n_tracks, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const hipError_t e = launch_k(k_merge_batch, dim3((unsigned)n_items), dim3(256), s, ms, bs,
                                items);
  if (e != hipSuccess) return e;
  return launch_k(k_merge_final_batch, dim3((unsigned)n_tracks), dim3(256), s, ms, bs);
}

hipError_t launch_anc_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                            int64_t n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  return launch_k(k_anc_batch, dim3((unsigned)n_items), dim3(kWave), s, ms, bs, items);
}

hipError_t launch_fill_batch(const Model* ms, const Buffers* bs, const int32_t* tracks,
                             int32_t n_tracks, hipStream_t s) {
  if (n_tracks <= 0) return hipSuccess;
  return launch_k(k_fill_batch, dim3(kFillGridBatch), dim3(kWave), s, ms, bs, tracks, n_tracks);
}

hipError_t launch_rna_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                            int64_t n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  return launch_k(k_rna_batch, dim3((unsigned)n_items), dim3(256), s, ms, bs, items);
}

hipError_t launch_rna_groups(const Model& m, const Buffers& b, hipStream_t s) {
  const hipError_t e = launch_k(k_rna_local, dim3((unsigned)m.G), dim3(256), s, m, b);
  if (e != hipSuccess) return e;
  return launch_k(k_rna_exchange, dim3((unsigned)m.G), dim3(256), s, m, b);
}

hipError_t launch_arna(const Model& m, const Buffers& b, hipStream_t s) {
  const hipError_t e = launch_k(k_arna_local, dim3((unsigned)m.G), dim3(256), s, m, b);
  if (e != hipSuccess) return e;
  return launch_k(k_arna_exchange, dim3((unsigned)m.G), dim3(256), s, m, b);
}

hipError_t launch_rpa(const Model& m, const Buffers& b, hipStream_t s) {
  const int64_t G = m.rpa_G;
  hipError_t e = launch_k(k_rpa_first, dim3(grid_for(G + 1, 256)), dim3(256), s, m, b);
  if (e == hipSuccess && m.dlb == 1) {
    const int64_t cnt = 2 * G;
    const int32_t nt = (int32_t)((cnt + kSortTile - 1) / kSortTile);
    e = launch_k(k_rpa_keys, dim3(grid_for(cnt, 256)), dim3(256), s, m, b);
    for (int pass = 0; pass < 4 && e == hipSuccess; ++pass) {
      // ping -> pong on even passes, back on odd ones: the result lands in ping
      const uint32_t* kin = pass & 1 ? b.rkey1 : b.rkey0;
      const int32_t* vin = pass & 1 ? b.rval1 : b.rval0;
      uint32_t* kout = pass & 1 ? b.rkey0 : b.rkey1;
      int32_t* vout = pass & 1 ? b.rval0 : b.rval1;
      const Ctrl* gate = b.ctrl;
      e = launch_k(k_radix_hist, dim3((unsigned)nt), dim3(256), s, kin, cnt, 8 * pass, b.rhist,
                   nt, gate);
      if (e == hipSuccess)
        e = launch_k(k_radix_rowscan, dim3(256), dim3(256), s, b.rhist, nt, b.rrow, gate);
      if (e == hipSuccess)
        e = launch_k(k_radix_scatter, dim3((unsigned)nt), dim3(256), s, kin, vin, kout, vout, cnt,
                     8 * pass, (const uint32_t*)b.rhist, (const uint32_t*)b.rrow, nt, gate);
    }
  }
  const unsigned nt2 = (unsigned)((G + kSortTile - 1) / kSortTile);
  if (e == hipSuccess) e = launch_k(k_rpa_plan_tiles, dim3(nt2, 2), dim3(256), s, m, b);
  if (e == hipSuccess) e = launch_k(k_rpa_plan_scan, dim3(2), dim3(256), s, m, b);
  if (e == hipSuccess) e = launch_k(k_rpa_plan_apply, dim3(nt2, 2), dim3(256), s, m, b);
  const int64_t quads = (m.n + 3) / 4;
  if (e == hipSuccess) e = launch_k(k_rpa_stream, dim3(grid_for(quads, 256)), dim3(256), s, m, b);
  if (e == hipSuccess) e = launch_k(k_rpa_route, dim3(grid_for(quads, 256)), dim3(256), s, m, b);
  return e;
}

namespace {
// Scratch of a standalone DLB schedule of G groups, carved from `base` (the
// pointers stay null when it is null); returns its size in bytes.
struct DlbScratch {
  uint32_t* key0;
  uint32_t* key1;
  int32_t* val0;
  int32_t* val1;
  uint32_t* hist;
  uint32_t* row;
  uint64_t* vals;  // list values, 2G
  uint64_t* cs;    // senders' prefixes, G + 1
  uint64_t* cd;    // receivers' prefixes, G + 1
  uint64_t* cnt;   // entries per sender, G
  uint64_t* E;     // their prefixes, G + 1
  int32_t* jlo;    // each sender's first receiver, G
  uint64_t* tsum;  // scan tiles
  int32_t* nsr;    // present entries per side, 2
};

size_t dlb_carve(int32_t G, char* base, DlbScratch* d) {
  const size_t L = 2 * (size_t)G, nt = (L + kSortTile - 1) / kSortTile;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  d->key0 = reinterpret_cast<uint32_t*>(take(L * 4));
  d->key1 = reinterpret_cast<uint32_t*>(take(L * 4));
  d->val0 = reinterpret_cast<int32_t*>(take(L * 4));
  d->val1 = reinterpret_cast<int32_t*>(take(L * 4));
  d->hist = reinterpret_cast<uint32_t*>(take(256 * nt * 4));
  d->row = reinterpret_cast<uint32_t*>(take(256 * 4));
  d->vals = reinterpret_cast<uint64_t*>(take(L * 8));
  d->cs = reinterpret_cast<uint64_t*>(take(((size_t)G + 1) * 8));
  d->cd = reinterpret_cast<uint64_t*>(take(((size_t)G + 1) * 8));
  d->cnt = reinterpret_cast<uint64_t*>(take((size_t)G * 8));
  d->E = reinterpret_cast<uint64_t*>(take(((size_t)G + 1) * 8));
  d->jlo = reinterpret_cast<int32_t*>(take((size_t)G * 4));
  d->tsum = reinterpret_cast<uint64_t*>(take((nt + 1) * 8));
  d->nsr = reinterpret_cast<int32_t*>(take(2 * 4));
  return off;
}

// Exclusive prefix sums of len values into out[0..len), the total into
// out[len] (tsum: scan tiles).
hipError_t scan_u64(const uint64_t* in, int64_t len, uint64_t* out, uint64_t* tsum, hipStream_t s) {
  const unsigned nt = (unsigned)((len + kSortTile - 1) / kSortTile);
  hipError_t e = launch_k(k_scan_tiles, dim3(nt), dim3(256), s, in, len, tsum);
  if (e == hipSuccess) e = launch_k(k_scan_top, dim3(1), dim3(256), s, tsum, (int64_t)nt, out + len);
  if (e == hipSuccess)
    e = launch_k(k_scan_apply, dim3(nt), dim3(256), s, in, len, (const uint64_t*)tsum, out);
  return e;
}
}  // namespace

size_t dlb_scratch_bytes(int32_t G) {
  DlbScratch d;
  return dlb_carve(G, nullptr, &d);
}

hipError_t launch_dlb_schedule(int32_t kind, const int32_t* counts, int32_t G, int32_t n,
                               int32_t* sched, int32_t cap, int32_t* n_entries, void* scratch,
                               hipStream_t s) {
  const int64_t L = 2 * (int64_t)G;
  const int32_t nt = (int32_t)((L + kSortTile - 1) / kSortTile);
  DlbScratch d;
  dlb_carve(G, static_cast<char*>(scratch), &d);
  const Ctrl* nogate = nullptr;
  hipError_t e = launch_k(k_dlb_keys, dim3(grid_for(L, 256)), dim3(256), s, kind, counts, G, n,
                          d.key0, d.val0);
  for (int pass = 0; pass < 4 && e == hipSuccess; ++pass) {
    // ping -> pong on even passes, back on odd ones: the lists land in ping
    const uint32_t* kin = pass & 1 ? d.key1 : d.key0;
    const int32_t* vin = pass & 1 ? d.val1 : d.val0;
    uint32_t* kout = pass & 1 ? d.key0 : d.key1;
    int32_t* vout = pass & 1 ? d.val0 : d.val1;
    e = launch_k(k_radix_hist, dim3((unsigned)nt), dim3(256), s, kin, L, 8 * pass, d.hist, nt,
                 nogate);
    if (e == hipSuccess)
      e = launch_k(k_radix_rowscan, dim3(256), dim3(256), s, d.hist, nt, d.row, nogate);
    if (e == hipSuccess)
      e = launch_k(k_radix_scatter, dim3((unsigned)nt), dim3(256), s, kin, vin, kout, vout, L,
                   8 * pass, (const uint32_t*)d.hist, (const uint32_t*)d.row, nt, nogate);
  }
  if (e == hipSuccess)
    e = launch_k(k_dlb_values, dim3(grid_for(L, 256)), dim3(256), s, counts, G, n,
                 (const int32_t*)d.val0, d.vals);
  if (e == hipSuccess) e = launch_k(k_zero_i32, dim3(1), dim3(64), s, d.nsr, 2);
  if (e == hipSuccess)
    e = launch_k(k_dlb_present, dim3(grid_for(L, 256)), dim3(256), s, (const uint64_t*)d.vals, G,
                 d.nsr);
  if (e == hipSuccess) e = scan_u64(d.vals, G, d.cs, d.tsum, s);
  if (e == hipSuccess) e = scan_u64(d.vals + G, G, d.cd, d.tsum, s);
  if (kind != 2) {
    if (e == hipSuccess)
      e = launch_k(k_dlb_count, dim3(grid_for(G, 256)), dim3(256), s, (const uint64_t*)d.cs,
                   (const uint64_t*)d.cd, (const int32_t*)d.nsr, G, d.jlo, d.cnt);
    if (e == hipSuccess) e = scan_u64(d.cnt, G, d.E, d.tsum, s);
  }
  if (e == hipSuccess)
    e = launch_k(k_dlb_entries, dim3(grid_for(L, 256)), dim3(256), s, kind,
                 (const int32_t*)d.val0, (const uint64_t*)d.vals, (const uint64_t*)d.cs,
                 (const uint64_t*)d.cd, (const int32_t*)d.nsr, G, (const int32_t*)d.jlo,
                 (const uint64_t*)d.E, sched, cap, n_entries);
  return e;
}

hipError_t launch_merge(const Model& m, const Buffers& b, int standalone, double u_given,
                        hipStream_t s) {
  const hipError_t e = launch_k(k_merge, dim3((unsigned)b.nch), dim3(256), s, m, b, standalone);
  if (e != hipSuccess) return e;
  return launch_k(k_merge_final, dim3(1), dim3(256), s, m, b, standalone, u_given);
}

hipError_t launch_anc(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s) {
  if (w.log_src) return launch_k(k_anc_log, dim3((unsigned)b.nseg), dim3(kWave), s, m, b, w);
  return launch_k(k_anc, dim3((unsigned)b.nseg), dim3(kWave), s, m, b, w);
}

hipError_t launch_fill(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s) {
  const unsigned grid = (unsigned)(b.hq_cap < kFillGrid ? b.hq_cap : kFillGrid);
  if (w.log_src) return launch_k(k_fill_log, dim3(grid), dim3(kWave), s, m, b, w);
  return launch_k(k_fill, dim3(grid), dim3(kWave), s, m, b, w);
}

hipError_t launch_rna(const Model& m, const Buffers& b, const WeightSrc& w, const double* u_dev,
                      hipStream_t s) {
  return launch_k(k_rna, dim3((unsigned)m.G), dim3(256), s, m, b, w, u_dev);
}

hipError_t launch_gather(const Model& m, const Buffers& b, float* out, hipStream_t s) {
  return launch_k(k_gather, dim3(grid_for(m.n, 256)), dim3(256), s, m, b, out);
}

hipError_t launch_logw(const Model& m, const Buffers& b, hipStream_t s) {
  return launch_k(k_logw, dim3(grid_for(m.n, 256)), dim3(256), s, m, b);
}

hipError_t launch_set_mode(const Buffers& b, int32_t mode, hipStream_t s) {
  return launch_k(k_set_mode, dim3(1), dim3(1), s, b.ctrl, mode);
}

hipError_t launch_records(const Model& m, const Buffers& b, const float* logw, hipStream_t s) {
  return launch_k(k_records, dim3((unsigned)b.nb), dim3(kBlock), s, m, b, logw);
}

hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  return launch_k(k_philox, dim3(grid_for(n, 256)), dim3(256), s, (uint32_t)seed,
                  (uint32_t)(seed >> 32), reinterpret_cast<const uint4*>(ctr),
                  reinterpret_cast<uint4*>(out), n);
}

}  // namespace ppf
