// Host runtime of the C ABI declared in include/ppf.h: parameter validation,
// workspace carving, the per-step launch sequence on the caller's stream,
// synchronising queries, and per-kernel event timing.
#include "ppf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "ppf_internal.hpp"

using ppf::Buffers;
using ppf::Ctrl;
using ppf::Model;

namespace {

// Timed units of a step. k_resample is the systematic resampling pass, its
// two launches (segments, then queued tile chunks) under one pair of events.
enum KernelId {
  kKStep, kKMerge, kKResample, kKRna, kKInit, kKGather, kKLogw, kKRpa, kNumKernels
};
const char* const kKernelNames[kNumKernels] = {"k_step",   "k_merge",  "k_resample", "k_rna",
                                               "k_init",   "k_gather", "k_logw",     "k_rpa"};

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int derived_patch(const ppf_params* p) {
  return p->patch ? p->patch : 2 * (int)std::floor(3.0 * (double)p->psf_sigma) + 1;
}

// Returns an empty string when *p is acceptable.
std::string validate(const ppf_params* p) {
  if (!p) return "null parameters";
  if (p->state_dim != 5) return "state_dim must be 5";
  if (p->grad != 0 && p->grad != 1) return "grad must be 0 or 1";
  if (p->grad) {
    if (p->obs_model != PPF_OBS_SPOT) return "grad needs the spot model";
    if (p->resample != PPF_RESAMPLE_SYSTEMATIC) return "grad needs systematic resampling";
    if (!(std::isinf(p->ess_threshold) && p->ess_threshold > 0))
      return "grad needs resampling at every step (ess_threshold = +inf)";
  }
  if (p->n_particles < 1 || p->n_particles > 2147483647LL) return "n_particles out of range";
  if (p->obs_model != PPF_OBS_SPOT && p->obs_model != PPF_OBS_LINEAR_GAUSSIAN)
    return "unknown obs_model";
  if (p->init_kind < PPF_INIT_UNIFORM || p->init_kind > PPF_INIT_UNIFORM_ZORDER)
    return "unknown init_kind";
  if (p->resample != PPF_RESAMPLE_SYSTEMATIC && p->resample != PPF_RESAMPLE_RNA &&
      p->resample != PPF_RESAMPLE_RPA && p->resample != PPF_RESAMPLE_ARNA)
    return "unknown resample scheme";
  if (p->reserved != 0 || p->arna_pad != 0) return "reserved must be 0";
  if (p->resample == PPF_RESAMPLE_ARNA) {
    if (p->obs_model != PPF_OBS_SPOT) return "ARNA needs the spot model";
    if (!(p->arna_min >= 0.0f && p->arna_min <= p->rna_exchange))
      return "ARNA: arna_min must be in [0, rna_exchange]";
    if (!(p->arna_track > 0.0f) || !std::isfinite(p->arna_track))
      return "ARNA: arna_track must be > 0";
    if (!(p->arna_lost >= 0.0f)) return "ARNA: arna_lost must be >= 0";
  }
  if (p->resample == PPF_RESAMPLE_RPA) {
    if (p->rna_group < 1 || p->n_particles % p->rna_group != 0)
      return "RPA: n_particles must be a multiple of rna_group";
    if (p->dlb != PPF_DLB_GS && p->dlb != PPF_DLB_SGS) return "RPA: dlb must be GS or SGS";
  }
  for (int d = 0; d < 5; ++d) {
    if (!std::isfinite(p->q[d]) || p->q[d] < 0.0f) return "q must be finite and >= 0";
    if (!std::isfinite(p->init_a[d]) || !std::isfinite(p->init_b[d]))
      return "init box must be finite";
  }
  if (std::isnan(p->ess_threshold)) return "ess_threshold is NaN";
  if (p->obs_model == PPF_OBS_SPOT) {
    if (p->width < 1 || p->height < 1) return "frame size must be positive";
    if ((int64_t)p->width * p->height > (int64_t)1 << 31) return "frame too large";
    if (!(p->psf_sigma > 0.0f) || !std::isfinite(p->psf_sigma)) return "psf_sigma must be > 0";
    if (!(p->noise_sigma > 0.0f) || !std::isfinite(p->noise_sigma))
      return "noise_sigma must be > 0";
    if (!std::isfinite(p->background)) return "background must be finite";
    const int P = derived_patch(p);
    if (P < 1 || P > PPF_MAX_PATCH || P % 2 == 0) return "patch must be odd and <= 25";
    const double s = p->psf_sigma, h = (P - 1) / 2;
    // the Gaussian factors start at the patch corner, the product of the two
    // axes' edge values: keep it normal (e^-700 > 2^-1022)
    if ((h + 0.5) * (h + 0.5) / (2.0 * s * s) > 350.0) return "patch too wide for psf_sigma";
  } else {
    for (int d = 0; d < 3; ++d)
      if (!(p->lg_r[d] > 0.0f) || !std::isfinite(p->lg_r[d])) return "lg_r must be > 0";
  }
  if (p->resample == PPF_RESAMPLE_RNA || p->resample == PPF_RESAMPLE_ARNA) {
    if (p->rna_group < 1 || p->rna_group > ppf::kMaxGroup) return "rna_group out of range";
    if (p->n_particles % p->rna_group != 0) return "n_particles must be a multiple of rna_group";
    if (!(p->rna_exchange >= 0.0f && p->rna_exchange < 1.0f)) return "rna_exchange not in [0,1)";
  }
  return "";
}

int strat_bits(int64_t n) {
  int t = 0;
  while (((int64_t)1 << (t + 1)) <= n) ++t;
  t -= 2;
  return t < 0 ? 0 : t;
}

Model make_model(const ppf_params* p) {
  Model m{};
  m.n = p->n_particles;
  m.inv_n = 1.0 / (double)m.n;
  m.log_n = std::log((double)m.n);
  m.W = p->width;
  m.H = p->height;
  m.P = p->obs_model == PPF_OBS_SPOT ? derived_patch(p) : 1;
  m.obs = p->obs_model;
  m.init_kind = p->init_kind;
  for (int d = 0; d < 5; ++d) {
    m.q[d] = p->q[d];
    m.init_a[d] = p->init_a[d];
    m.init_b[d] = p->init_b[d];
  }
  m.b = (double)p->background;
  const double s = p->psf_sigma, sg = p->noise_sigma;
  m.inv2s2 = 1.0 / (2.0 * s * s);
  m.inv2sig2 = 1.0 / (2.0 * sg * sg);
  m.lognorm_obs = (double)m.P * (double)m.P * std::log(sg * std::sqrt(2.0 * M_PI));
  m.clo[0] = m.clo[1] = -(double)m.P;
  m.chi[0] = (double)m.W + m.P;
  m.chi[1] = (double)m.H + m.P;
  // ratio of consecutive 1-D Gaussian factors at unit pixel steps from -h
  const int h = (m.P - 1) / 2;
  for (int d = 0; d < ppf::kMaxPatch; ++d)
    m.gstep[d] = d + 1 < m.P ? std::exp(-(2.0 * (double)(d - h) + 1.0) * m.inv2s2) : 0.0;
  m.lg_norm = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double r = p->lg_r[d];
    m.lg_inv2r2[d] = r > 0.0 ? 1.0 / (2.0 * r * r) : 0.0;
    m.lg_norm += r > 0.0 ? std::log(r * std::sqrt(2.0 * M_PI)) : 0.0;
  }
  m.thr = p->ess_threshold;
  if (p->resample == PPF_RESAMPLE_RNA || p->resample == PPF_RESAMPLE_ARNA) {
    m.group = p->rna_group;
    m.moved = (int32_t)std::floor((double)p->rna_exchange * (double)p->rna_group);
    m.G = (int32_t)(m.n / m.group);
    m.inv_group = 1.0 / (double)m.group;
  }
  if (p->resample == PPF_RESAMPLE_ARNA) {
    m.arna = 1;
    m.arna_mu_min = (int32_t)std::floor((double)p->arna_min * (double)p->rna_group);
    m.arna_share = (double)p->arna_track / (double)m.G;
    m.arna_drop = (double)p->arna_lost * (double)m.P;
  }
  m.key0 = (uint32_t)p->seed;
  m.key1 = (uint32_t)(p->seed >> 32);
  m.track = p->track_id;
  m.strat_t = strat_bits(m.n);
  m.grad = p->grad;
  if (p->resample == PPF_RESAMPLE_RPA) {
    m.rpa = 1;
    m.dlb = p->dlb;
    m.rpa_group = p->rna_group;
    m.rpa_G = (int32_t)(m.n / p->rna_group);
  }
  m.s_psf = s;
  m.sig = sg;
  return m;
}

int64_t record_blocks(int64_t n) { return (n + ppf::kBlock - 1) / ppf::kBlock; }
// Records per merge chunk: a multiple of 256, at most 2048 (so a chunk's sum
// of 2^52-bounded integer weights stays below 2^63), aiming at <= 256 chunks
// so that the final merge is one pass of one workgroup.
int64_t merge_chunk(int64_t nb) {
  int64_t per = (nb + 256 * 256 - 1) / (256 * 256);
  if (per < 1) per = 1;
  if (per > 8) per = 8;
  return 256 * per;
}
int64_t seg_count(int64_t n) { return (n + ppf::kSegItems - 1) / ppf::kSegItems; }
// Tile chunks queued by heavy segments (more than kCoopTiles tiles each).
// With S = kSlotTile and C = kChunkTiles: a segment with M slots spans
// ntiles <= (M + 3) / S + 1 tiles (its first tile starts up to 3 slots
// early) and queues ceil(ntiles / C) <= (M + 3) / (C S) + 1 <= M / (C S) + 2
// chunks; a heavy one has ntiles >= kCoopTiles + 1, so M >= kCoopTiles S - 2,
// and there are at most H = n / (kCoopTiles S - 2) of them. The queue holds
// at most n / (C S) + 2 H entries; the capacity adds a margin.
int64_t queue_cap(int64_t n) {
  const int64_t heavy = n / ((int64_t)ppf::kCoopTiles * ppf::kSlotTile - 2) + 1;
  return n / ((int64_t)ppf::kChunkTiles * ppf::kSlotTile) + 3 * heavy + 16;
}

void shape(int64_t n, Buffers* bb) {
  bb->nb = record_blocks(n);
  bb->chunk = merge_chunk(bb->nb);
  bb->nch = (bb->nb + bb->chunk - 1) / bb->chunk;
  bb->nseg = seg_count(n);
}

// Carve the filter workspace; base may be null to only compute the size.
// With own_ctrl false the control block is not carved (a batch keeps the
// control blocks of its tracks together) and b->ctrl is left null.
size_t carve(const ppf_params* p, char* base, Buffers* b, bool own_ctrl = true) {
  const int64_t n = p->n_particles;
  Buffers bb{};
  shape(n, &bb);
  const bool groups = p->resample == PPF_RESAMPLE_RNA || p->resample == PPF_RESAMPLE_ARNA;
  const int64_t G = groups ? n / p->rna_group : 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* ptr = base ? base + off : nullptr;
    off += align_up(bytes);
    return ptr;
  };
  if (own_ctrl) bb.ctrl = reinterpret_cast<Ctrl*>(take(sizeof(Ctrl)));
  bb.X0 = reinterpret_cast<float*>(take(sizeof(float) * 5 * n));
  bb.X1 = reinterpret_cast<float*>(take(sizeof(float) * 5 * n));
  bb.E0 = reinterpret_cast<float*>(take(sizeof(float) * n));
  bb.E1 = reinterpret_cast<float*>(take(sizeof(float) * n));
  bb.R0 = reinterpret_cast<double*>(take(sizeof(double) * ppf::kRec * bb.nb));
  bb.R1 = reinterpret_cast<double*>(take(sizeof(double) * ppf::kRec * bb.nb));
  bb.pfx = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * bb.nb));
  bb.CR = reinterpret_cast<double*>(take(sizeof(double) * ppf::kRec * bb.nch));
  bb.cpre = reinterpret_cast<ppf::ChunkPre*>(take(sizeof(ppf::ChunkPre) * bb.nch));
  bb.anc = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * n));
  bb.lw64 = reinterpret_cast<double*>(take(sizeof(double) * n));
  bb.lwg = reinterpret_cast<double*>(take(sizeof(double) * G));
  bb.hq = reinterpret_cast<ppf::TileRun*>(take(sizeof(ppf::TileRun) * queue_cap(n)));
  bb.hq_cap = queue_cap(n);
  if (p->resample == PPF_RESAMPLE_RPA) {
    const int64_t Gr = n / p->rna_group;
    bb.asys = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * n));
    bb.rfirst = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (Gr + 1)));
    bb.rdbase = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * Gr));
    bb.rscum = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (Gr + 1)));
    bb.rns = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 2));
    const int64_t nt = (2 * Gr + ppf::kSortTile - 1) / ppf::kSortTile;
    const int64_t nt2 = (Gr + ppf::kSortTile - 1) / ppf::kSortTile;
    if (p->dlb == PPF_DLB_SGS) {
      bb.rkey0 = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 2 * Gr));
      bb.rkey1 = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 2 * Gr));
      bb.rval0 = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 2 * Gr));
      bb.rval1 = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 2 * Gr));
      bb.rhist = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 256 * nt));
      bb.rrow = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 256));
    }
    bb.rtsum = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * 4 * nt2));
    bb.rsidx = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * Gr));
    bb.rstream = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * n));
  }
  if (p->init_kind == PPF_INIT_UNIFORM_ZORDER) {
    // the initialisation's sort of the particles' keys
    const int64_t nt = (n + ppf::kSortTile - 1) / ppf::kSortTile;
    bb.zkey0 = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * n));
    bb.zkey1 = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * n));
    bb.zval0 = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * n));
    bb.zval1 = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * n));
    bb.zhist = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 256 * nt));
    bb.zrow = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 256));
  }
  if (p->resample == PPF_RESAMPLE_RNA || p->resample == PPF_RESAMPLE_ARNA) {
    // the local resampling of every group and its share W_g, read by the
    // exchange launch
    bb.aloc = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * n));
    bb.Wg = reinterpret_cast<double*>(take(sizeof(double) * G));
  }
  if (p->resample == PPF_RESAMPLE_ARNA)
    bb.lwt = reinterpret_cast<double*>(take(sizeof(double) * G));
  if (p->grad) {
    bb.T0 = reinterpret_cast<float*>(take(sizeof(float) * ppf::kNTan * n));
    bb.T1 = reinterpret_cast<float*>(take(sizeof(float) * ppf::kNTan * n));
    bb.RG = reinterpret_cast<double*>(take(sizeof(double) * ppf::kNGrad * bb.nb));
    bb.CRG = reinterpret_cast<double*>(take(sizeof(double) * ppf::kNGrad * bb.nch));
  }
  if (b) *b = bb;
  return off;
}

// Scratch of the standalone resamplers.
size_t carve_scratch(int64_t n, char* base, Buffers* b) {
  Buffers bb{};
  shape(n, &bb);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* ptr = base ? base + off : nullptr;
    off += align_up(bytes);
    return ptr;
  };
  bb.ctrl = reinterpret_cast<Ctrl*>(take(sizeof(Ctrl)));
  bb.R0 = reinterpret_cast<double*>(take(sizeof(double) * ppf::kRec * bb.nb));
  bb.pfx = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * bb.nb));
  bb.CR = reinterpret_cast<double*>(take(sizeof(double) * ppf::kRec * bb.nch));
  bb.cpre = reinterpret_cast<ppf::ChunkPre*>(take(sizeof(ppf::ChunkPre) * bb.nch));
  bb.hq = reinterpret_cast<ppf::TileRun*>(take(sizeof(ppf::TileRun) * queue_cap(n)));
  bb.hq_cap = queue_cap(n);
  if (b) *b = bb;
  return off;
}

// Launch bookkeeping shared by filters and batches: the stream, the last
// error text, and optional per-kernel HIP-event timing.
struct Runner {
  hipStream_t stream = nullptr;
  std::string err;
  bool prof = false;
  struct Ev {
    int kernel;
    hipEvent_t start, stop;
  };
  std::vector<Ev> events;
  double total_ms[kNumKernels] = {};
  int64_t launches[kNumKernels] = {};

  int fail(int code, const std::string& what) {
    err = what;
    return code;
  }
  int hip_fail(hipError_t e, const char* where) {
    err = std::string(where) + ": " + hipGetErrorString(e);
    return PPF_EDEVICE;
  }
  // Launch with optional event timing around it.
  template <class F>
  int run(int kernel, F&& launch) {
    hipEvent_t a = nullptr, z = nullptr;
    if (prof) {
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&z) != hipSuccess)
        return fail(PPF_EDEVICE, "hipEventCreate failed");
      if (hipEventRecord(a, stream) != hipSuccess) return fail(PPF_EDEVICE, "hipEventRecord");
    }
    const hipError_t e = launch();
    if (prof) {
      const hipError_t ez = hipEventRecord(z, stream);
      events.push_back({kernel, a, z});
      if (ez != hipSuccess) return hip_fail(ez, "hipEventRecord");
    }
    if (e != hipSuccess) return hip_fail(e, kKernelNames[kernel]);
    return PPF_OK;
  }
  int collect() {
    for (auto& ev : events) {
      if (hipEventSynchronize(ev.stop) != hipSuccess) return fail(PPF_EDEVICE, "event sync");
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev.start, ev.stop) == hipSuccess) {
        total_ms[ev.kernel] += ms;
        launches[ev.kernel] += 1;
      }
      (void)hipEventDestroy(ev.start);
      (void)hipEventDestroy(ev.stop);
    }
    events.clear();
    return PPF_OK;
  }
  // Graph mode: a step is recorded once into a HIP graph (the first step
  // after enabling) and replayed, pointed at each call's frame.
  bool graph_on = false;
  std::unique_ptr<ppf::StepGraph> graph;
  int graph_enable(int on) {
    if (on && prof) return fail(PPF_ESTATE, "graph mode and kernel timing exclude each other");
    if (hipStreamSynchronize(stream) != hipSuccess) return fail(PPF_EDEVICE, "sync");
    graph_on = on != 0;
    graph.reset();
    return PPF_OK;
  }
  // Enqueues one step: enqueue() itself, or the graph of its launches.
  template <class F>
  int step(const float* frame, F&& enqueue) {
    if (!graph_on) return enqueue();
    if (!graph) {
      auto g = std::make_unique<ppf::StepGraph>();
      hipError_t e = g->begin(frame);
      if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
      const int rc = enqueue();
      e = g->end();
      if (rc) return rc;
      if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
      graph = std::move(g);
    }
    hipError_t e = graph->set_frame(frame);
    if (e != hipSuccess) return hip_fail(e, "hipGraphExecKernelNodeSetParams");
    e = graph->launch(stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return PPF_OK;
  }
  // Average ms of one call of launch() over reps calls, after one untimed
  // call; syncs.
  template <class F>
  int time_launches(int reps, F&& launch, double* ms) {
    hipEvent_t a = nullptr, z = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&z);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(a, stream);
    for (int r = 0; e == hipSuccess && r < reps; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(z, stream);
    if (e == hipSuccess) e = hipEventSynchronize(z);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, z);
    if (a) (void)hipEventDestroy(a);
    if (z) (void)hipEventDestroy(z);
    if (e != hipSuccess) return hip_fail(e, "timing a tuning candidate");
    *ms = (double)t / reps;
    return PPF_OK;
  }
  int profile_enable(int on) {
    if (on && graph_on) return fail(PPF_ESTATE, "graph mode and kernel timing exclude each other");
    if (hipStreamSynchronize(stream) != hipSuccess) return fail(PPF_EDEVICE, "sync");
    collect();
    prof = on != 0;
    if (prof)
      for (int k = 0; k < kNumKernels; ++k) {
        total_ms[k] = 0.0;
        launches[k] = 0;
      }
    return PPF_OK;
  }
  int profile_read(ppf_kernel_time* out, int max_entries, int* n_entries) {
    if (!n_entries || (max_entries > 0 && !out)) return PPF_EINVAL;
    const int rc = collect();
    if (rc) return rc;
    int cnt = 0;
    for (int k = 0; k < kNumKernels && cnt < max_entries; ++k) {
      if (!launches[k]) continue;
      std::snprintf(out[cnt].name, sizeof out[cnt].name, "%s", kKernelNames[k]);
      out[cnt].launches = launches[k];
      out[cnt].total_ms = total_ms[k];
      ++cnt;
    }
    *n_entries = cnt;
    return PPF_OK;
  }
  // Copy one filter's particles to the host (state, normalised fp64 log
  // weights, ancestors); syncs.
  int particles(const Model& m, const Buffers& b, float* state_host, double* logw_host,
                int32_t* anc_host) {
    Ctrl c;
    hipError_t e = hipMemcpyAsync(&c, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "reading control block");
    const int64_t n = m.n;
    if (state_host)
      e = hipMemcpyAsync(state_host, c.cur ? b.X1 : b.X0, sizeof(float) * 5 * n,
                         hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && logw_host) {
      const int rc = run(kKLogw, [&] { return ppf::launch_logw(m, b, stream); });
      if (rc) return rc;
      e = hipMemcpyAsync(logw_host, b.lw64, sizeof(double) * n, hipMemcpyDeviceToHost, stream);
    }
    const bool resampled =
        c.mode == ppf::kModeSys || c.mode == ppf::kModeRna || c.mode == ppf::kModeArna;
    if (e == hipSuccess && anc_host && resampled)
      e = hipMemcpyAsync(anc_host, b.anc, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "copying particles");
    if (anc_host && !resampled)
      for (int64_t i = 0; i < n; ++i) anc_host[i] = (int32_t)i;
    return PPF_OK;
  }
};

void fill_stats(const Ctrl& c, ppf_stats_t* out) {
  out->k = c.k;
  out->resampled = c.resampled;
  out->rolled_back = c.rolled_back;
  out->ess = c.ess;
  out->max_logw = c.m;
  out->log_sum = c.log_sum;
  out->delta = c.delta;
  out->cum = c.cum;
  for (int d = 0; d < 5; ++d) out->mean[d] = c.mean[d];
}

}  // namespace

struct ppf_ctx : Runner {
  ppf_params p{};
  Model m{};
  Buffers b{};
  int read_ctrl(Ctrl* c) {
    hipError_t e = hipMemcpyAsync(c, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "reading control block");
    return PPF_OK;
  }
  ppf::WeightSrc filter_weights() const {
    ppf::WeightSrc w{};
    w.E0 = b.E0;
    w.E1 = b.E1;
    w.rec0 = b.R0;
    w.rec1 = b.R1;
    w.use_cur = 1;
    return w;
  }
};

extern "C" {

const char* ppf_version(void) { return "ppf-mi355x 0.1 (gfx950)"; }

size_t ppf_params_size(void) { return sizeof(ppf_params); }

int ppf_params_default(ppf_params* p) {
  if (!p) return PPF_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->state_dim = 5;
  p->obs_model = PPF_OBS_SPOT;
  p->n_particles = 4096;
  p->width = p->height = 128;
  p->psf_sigma = 1.5f;
  p->background = 10.0f;
  p->noise_sigma = 3.0f;
  p->patch = 0;
  const float q[5] = {0.5f, 0.5f, 0.1f, 0.1f, 1.0f};
  const float a[5] = {0.0f, 0.0f, -1.0f, -1.0f, 15.0f};
  const float bnd[5] = {128.0f, 128.0f, 1.0f, 1.0f, 45.0f};
  for (int d = 0; d < 5; ++d) {
    p->q[d] = q[d];
    p->init_a[d] = a[d];
    p->init_b[d] = bnd[d];
  }
  p->init_kind = PPF_INIT_UNIFORM;
  p->lg_r[0] = p->lg_r[1] = p->lg_r[2] = 1.0f;
  p->resample = PPF_RESAMPLE_SYSTEMATIC;
  p->ess_threshold = INFINITY;
  p->rna_group = 256;
  p->rna_exchange = 0.1f;
  p->seed = 1;
  p->track_id = 0;
  p->arna_min = 0.0f;
  p->arna_track = 0.5f;
  p->arna_lost = 3.0f;
  return PPF_OK;
}

int ppf_workspace_bytes(const ppf_params* p, size_t* bytes) {
  if (!bytes || !validate(p).empty()) return PPF_EINVAL;
  *bytes = carve(p, nullptr, nullptr);
  return PPF_OK;
}

int ppf_create(const ppf_params* p, void* workspace, size_t bytes, void* hip_stream,
               ppf_handle* out) {
  if (!out) return PPF_EINVAL;
  *out = nullptr;
  if (!validate(p).empty() || !workspace) return PPF_EINVAL;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return PPF_EINVAL;
  const size_t need = carve(p, nullptr, nullptr);
  if (bytes < need) return PPF_ENOMEM;
  ppf_ctx* h = new (std::nothrow) ppf_ctx();
  if (!h) return PPF_ENOMEM;
  h->p = *p;
  h->m = make_model(p);
  carve(p, static_cast<char*>(workspace), &h->b);
  h->stream = static_cast<hipStream_t>(hip_stream);
  const int rc = h->run(kKInit, [&] { return ppf::launch_init(h->m, h->b, h->stream); });
  if (rc != PPF_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return PPF_OK;
}

int ppf_reset(ppf_handle h) {
  if (!h) return PPF_ESTATE;
  return h->run(kKInit, [&] { return ppf::launch_init(h->m, h->b, h->stream); });
}

namespace {
// The launches of one step; every decision between them is taken on the
// device, so the same sequence serves every step (and a graph of it).
int enqueue_step(ppf_handle h, const float* obs_dev) {
  int rc = h->run(kKStep, [&] { return ppf::launch_step(h->m, h->b, obs_dev, h->stream); });
  if (rc) return rc;
  rc = h->run(kKMerge, [&] { return ppf::launch_merge(h->m, h->b, 0, 0.0, h->stream); });
  if (rc) return rc;
  const ppf::WeightSrc w = h->filter_weights();
  if (h->p.resample == PPF_RESAMPLE_RNA)
    return h->run(kKRna, [&] { return ppf::launch_rna_groups(h->m, h->b, h->stream); });
  if (h->p.resample == PPF_RESAMPLE_ARNA)
    return h->run(kKRna, [&] { return ppf::launch_arna(h->m, h->b, h->stream); });
  rc = h->run(kKResample, [&] {
    const hipError_t e = ppf::launch_anc(h->m, h->b, w, h->stream);
    return e != hipSuccess ? e : ppf::launch_fill(h->m, h->b, w, h->stream);
  });
  if (rc || !h->m.rpa) return rc;
  return h->run(kKRpa, [&] { return ppf::launch_rpa(h->m, h->b, h->stream); });
}
}  // namespace

int ppf_step(ppf_handle h, const float* obs_dev) {
  if (!h) return PPF_ESTATE;
  if (!obs_dev) return h->fail(PPF_EINVAL, "null observation");
  return h->step(obs_dev, [&] { return enqueue_step(h, obs_dev); });
}

int ppf_set_graph(ppf_handle h, int enable) {
  if (!h) return PPF_ESTATE;
  return h->graph_enable(enable);
}

int ppf_set_shape(ppf_handle h, int32_t shape) {
  if (!h) return PPF_ESTATE;
  if (shape < 0 || shape >= ppf::kNumShapes) return h->fail(PPF_EINVAL, "shape must be 0 or 1");
  const hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "sync");
  h->m.shape = shape;
  h->graph.reset();
  return PPF_OK;
}

namespace {
void tune_report(const double* ms, int n, int best, double* ms_out, int32_t* n_out,
                 int32_t* chosen) {
  if (ms_out)
    for (int c = 0; c < n; ++c) ms_out[c] = ms[c];
  if (n_out) *n_out = n;
  if (chosen) *chosen = best;
}
}  // namespace

int ppf_autotune(ppf_handle h, const float* obs_dev, int32_t reps, double* ms_out,
                 int32_t* n_out, int32_t* chosen) {
  if (!h) return PPF_ESTATE;
  if (!obs_dev) return h->fail(PPF_EINVAL, "null observation");
  if (reps < 1 || reps > 10000) return h->fail(PPF_EINVAL, "reps must be in [1, 10000]");
  // the step kernel alone writes only the next state, weights and records:
  // the committed step, counter and statistics stay as they are
  const bool shapes = h->m.obs == 0 && !h->m.grad && h->m.P <= ppf::kFusedMaxP;
  const int n = shapes ? ppf::kNumShapes : 1;
  const int keep = h->m.shape;
  double ms[ppf::kNumShapes] = {};
  for (int c = 0; c < n; ++c) {
    if (shapes) h->m.shape = c;
    const int rc = h->time_launches(
        reps, [&] { return ppf::launch_step(h->m, h->b, obs_dev, h->stream); }, &ms[c]);
    if (rc) {
      h->m.shape = keep;
      return rc;
    }
  }
  int best = 0;
  for (int c = 1; c < n; ++c)
    if (ms[c] < ms[best]) best = c;
  h->m.shape = shapes ? best : keep;
  h->graph.reset();
  tune_report(ms, n, best, ms_out, n_out, chosen);
  return PPF_OK;
}

int ppf_sync(ppf_handle h) {
  if (!h) return PPF_ESTATE;
  Ctrl c;
  int rc = h->read_ctrl(&c);
  if (rc) return rc;
  if (c.rolled_back) {
    const int32_t zero = 0;
    hipError_t e = hipMemcpyAsync(&h->b.ctrl->rolled_back, &zero, sizeof zero,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "clearing roll-back report");
    return h->fail(PPF_ENUMERIC, "a step had no finite normaliser and was rolled back");
  }
  return PPF_OK;
}

int ppf_estimate(ppf_handle h, double mean[5], double* ess) {
  if (!h) return PPF_ESTATE;
  const int rc = ppf_sync(h);
  if (rc != PPF_OK && rc != PPF_ENUMERIC) return rc;
  Ctrl c;
  const int rc2 = h->read_ctrl(&c);
  if (rc2) return rc2;
  if (mean)
    for (int d = 0; d < 5; ++d) mean[d] = c.mean[d];
  if (ess) *ess = c.ess;
  return rc;
}

int ppf_loglik(ppf_handle h, double* cum, double* last) {
  if (!h) return PPF_ESTATE;
  const int rc = ppf_sync(h);
  if (rc != PPF_OK && rc != PPF_ENUMERIC) return rc;
  Ctrl c;
  const int rc2 = h->read_ctrl(&c);
  if (rc2) return rc2;
  if (cum) *cum = c.cum;
  if (last) *last = c.delta;
  return rc;
}

int ppf_grad(ppf_handle h, double cum[PPF_NGRAD], double last[PPF_NGRAD]) {
  if (!h) return PPF_ESTATE;
  if (!h->m.grad) return h->fail(PPF_EINVAL, "the filter was created with grad = 0");
  const int rc = ppf_sync(h);
  if (rc != PPF_OK && rc != PPF_ENUMERIC) return rc;
  Ctrl c;
  const int rc2 = h->read_ctrl(&c);
  if (rc2) return rc2;
  for (int d = 0; d < PPF_NGRAD; ++d) {
    if (cum) cum[d] = c.grad_cum[d];
    if (last) last[d] = c.grad_last[d];
  }
  return rc;
}

int ppf_arna_state(ppf_handle h, int64_t* ring_key, int32_t* lost, int32_t* tracking,
                   int32_t* moved) {
  if (!h) return PPF_ESTATE;
  if (!h->m.arna) return h->fail(PPF_EINVAL, "the filter does not use ARNA");
  Ctrl c;
  const int rc = h->read_ctrl(&c);
  if (rc) return rc;
  if (ring_key) *ring_key = c.ring_key;
  if (lost) *lost = c.lost;
  if (tracking) *tracking = c.resampled ? c.arna_tracking : 0;
  if (moved) *moved = c.resampled ? c.arna_moved : 0;
  return PPF_OK;
}

int ppf_stats(ppf_handle h, ppf_stats_t* out) {
  if (!h) return PPF_ESTATE;
  if (!out) return PPF_EINVAL;
  Ctrl c;
  int rc = h->read_ctrl(&c);
  if (rc) return rc;
  fill_stats(c, out);
  if (c.rolled_back) {
    const int32_t zero = 0;
    hipError_t e = hipMemcpyAsync(&h->b.ctrl->rolled_back, &zero, sizeof zero,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "clearing roll-back report");
  }
  return PPF_OK;
}

int ppf_get_particles(ppf_handle h, float* state_host, double* logw_host, int32_t* anc_host) {
  if (!h) return PPF_ESTATE;
  return h->particles(h->m, h->b, state_host, logw_host, anc_host);
}

int ppf_set_particles(ppf_handle h, const float* state_host, const double* logw_host) {
  if (!h) return PPF_ESTATE;
  if (!state_host || !logw_host) return h->fail(PPF_EINVAL, "null particles");
  Ctrl c;
  int rc = h->read_ctrl(&c);
  if (rc) return rc;
  const int64_t n = h->m.n;
  hipError_t e = hipMemcpyAsync(c.cur ? h->b.X1 : h->b.X0, state_host, sizeof(float) * 5 * n,
                                hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->b.lw64, logw_host, sizeof(double) * n, hipMemcpyHostToDevice,
                       h->stream);
  // gradient mode: the new states are constants (zero tangents)
  if (e == hipSuccess && h->m.grad)
    e = hipMemsetAsync(c.cur ? h->b.T1 : h->b.T0, 0, sizeof(float) * ppf::kNTan * n, h->stream);
  if (e == hipSuccess) e = ppf::launch_set_mode(h->b, ppf::kModeSet, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "setting particles");
  return PPF_OK;
}

int ppf_gather(ppf_handle h, float* out_dev) {
  if (!h) return PPF_ESTATE;
  if (!out_dev) return h->fail(PPF_EINVAL, "null output");
  return h->run(kKGather, [&] { return ppf::launch_gather(h->m, h->b, out_dev, h->stream); });
}

int ppf_profile_enable(ppf_handle h, int on) {
  if (!h) return PPF_ESTATE;
  return h->profile_enable(on);
}

int ppf_profile_read(ppf_handle h, ppf_kernel_time* out, int max_entries, int* n_entries) {
  if (!h) return PPF_ESTATE;
  return h->profile_read(out, max_entries, n_entries);
}

int ppf_destroy(ppf_handle h) {
  if (!h) return PPF_OK;
  (void)hipStreamSynchronize(h->stream);
  h->collect();
  delete h;
  return PPF_OK;
}

const char* ppf_error_string(int code) {
  switch (code) {
    case PPF_OK: return "ok";
    case PPF_EINVAL: return "invalid argument";
    case PPF_ENOMEM: return "workspace too small";
    case PPF_EDEVICE: return "HIP device error";
    case PPF_ESTATE: return "invalid handle state";
    case PPF_ENUMERIC: return "non-finite normaliser: step rolled back";
    case PPF_ENOTIMPL: return "not implemented";
    default: return "unknown error";
  }
}

const char* ppf_last_error(ppf_handle h) { return h ? h->err.c_str() : "null handle"; }

int ppf_philox4x32_10(uint64_t seed, const uint32_t* ctr_dev, uint32_t* out_dev, int64_t n,
                      void* hip_stream) {
  if (n < 0 || (n > 0 && (!ctr_dev || !out_dev))) return PPF_EINVAL;
  const hipError_t e =
      ppf::launch_philox(seed, ctr_dev, out_dev, n, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? PPF_OK : PPF_EDEVICE;
}

int ppf_dlb_schedule(int32_t kind, const int32_t* counts_dev, int32_t G, int32_t n,
                     int32_t* sched_dev, int32_t cap, int32_t* n_entries_dev, void* hip_stream) {
  if (kind < PPF_DLB_GS || kind > PPF_DLB_LGS || G < 1 || n < 0) return PPF_EINVAL;
  if (!counts_dev || !n_entries_dev || cap < 0 || (cap > 0 && !sched_dev)) return PPF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // stream-ordered scratch: freed on the stream after the schedule's launches
  void* scratch = nullptr;
  if (hipMallocAsync(&scratch, ppf::dlb_scratch_bytes(G), s) != hipSuccess) return PPF_ENOMEM;
  const hipError_t e = ppf::launch_dlb_schedule(kind, counts_dev, G, n, sched_dev, cap,
                                                n_entries_dev, scratch, s);
  const hipError_t ef = hipFreeAsync(scratch, s);
  return e == hipSuccess && ef == hipSuccess ? PPF_OK : PPF_EDEVICE;
}

int ppf_resample_scratch_bytes(int64_t n, size_t* bytes) {
  if (!bytes || n < 1 || n > 2147483647LL) return PPF_EINVAL;
  *bytes = carve_scratch(n, nullptr, nullptr);
  return PPF_OK;
}

namespace {

int standalone_prepare(const float* logw_dev, int64_t n, void* scratch, size_t scratch_bytes,
                       Model* m, Buffers* b) {
  if (!logw_dev || !scratch || n < 1 || n > 2147483647LL) return PPF_EINVAL;
  if (reinterpret_cast<uintptr_t>(scratch) % kAlign != 0) return PPF_EINVAL;
  if (scratch_bytes < carve_scratch(n, nullptr, nullptr)) return PPF_ENOMEM;
  *m = Model{};
  m->n = n;
  m->inv_n = 1.0 / (double)n;
  m->log_n = std::log((double)n);
  carve_scratch(n, static_cast<char*>(scratch), b);
  return PPF_OK;
}

}  // namespace

int ppf_resample_systematic(const float* logw_dev, int64_t n, double u, int32_t* anc_dev,
                            void* scratch, size_t scratch_bytes, void* hip_stream) {
  if (!anc_dev || !(u >= 0.0 && u < 1.0)) return PPF_EINVAL;
  Model m;
  Buffers b;
  const int rc = standalone_prepare(logw_dev, n, scratch, scratch_bytes, &m, &b);
  if (rc) return rc;
  b.anc = anc_dev;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // every scratch field the kernels read is written earlier in the same call
  // (the records by k_records, which also clears the counters of the
  // control block; the prefixes by the merge), so nothing is cleared first
  const ppf::WeightSrc w{logw_dev, logw_dev, b.R0, b.R0, 0, 1};
  hipError_t e = ppf::launch_records(m, b, logw_dev, s);
  if (e == hipSuccess) e = ppf::launch_merge(m, b, 1, u, s);
  if (e == hipSuccess) e = ppf::launch_anc(m, b, w, s);
  if (e == hipSuccess) e = ppf::launch_fill(m, b, w, s);
  return e == hipSuccess ? PPF_OK : PPF_EDEVICE;
}

int ppf_resample_systematic_static(const float* logw_dev, int64_t n, double u, int32_t* anc_dev,
                                   void* hip_stream) {
  if (!logw_dev || !anc_dev || !(u >= 0.0 && u < 1.0)) return PPF_EINVAL;
  if (n < 1 || n > PPF_STATIC_MAX_N) return PPF_EINVAL;
  void* base = nullptr;
  size_t cap = 0;
  if (ppf::static_scratch(&base, &cap) != hipSuccess) return PPF_EDEVICE;
  if (carve_scratch(n, nullptr, nullptr) > cap) return PPF_ENOMEM;  // ruled out by the limit
  return ppf_resample_systematic(logw_dev, n, u, anc_dev, base, cap, hip_stream);
}

int ppf_resample_rna(const float* logw_dev, int64_t n, int32_t group, int32_t moved,
                     const double* u_dev, int32_t* anc_dev, double* lwg_dev, void* scratch,
                     size_t scratch_bytes, void* hip_stream) {
  if (!anc_dev || !lwg_dev || !u_dev) return PPF_EINVAL;
  if (group < 1 || group > ppf::kMaxGroup || n % group != 0) return PPF_EINVAL;
  if (moved < 0 || moved > group) return PPF_EINVAL;
  Model m;
  Buffers b;
  const int rc = standalone_prepare(logw_dev, n, scratch, scratch_bytes, &m, &b);
  if (rc) return rc;
  m.group = group;
  m.moved = moved;
  m.G = (int32_t)(n / group);
  m.inv_group = 1.0 / (double)group;
  b.anc = anc_dev;
  b.lwg = lwg_dev;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const ppf::WeightSrc w{logw_dev, logw_dev, b.R0, b.R0, 0, 1};
  hipError_t e = ppf::launch_records(m, b, logw_dev, s);
  if (e == hipSuccess) e = ppf::launch_merge(m, b, 1, 0.0, s);
  if (e == hipSuccess) e = ppf::launch_rna(m, b, w, u_dev, s);
  return e == hipSuccess ? PPF_OK : PPF_EDEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
// A batch keeps its tables at the start of its workspace, then every track's
// filter workspace (carved as for a single filter, minus the control block):
//   Ctrl[count] | Model[count] | Buffers[count] | block items (grouped by
//   patch size) | merge-chunk items | segment items | RNA-group items |
//   systematic track list | track workspaces.
namespace {

struct BatchPlan {
  std::vector<Model> models;
  std::vector<Buffers> bufs;
  std::vector<ppf::BatchItem> blocks, chunks, segs, groups;
  std::vector<int32_t> sys_tracks;
  struct StepRange {
    int P;      // patch size; 0: sizes up to kFusedMaxP in one fused launch
    int shape;  // workgroup shape of a fused launch
    int64_t first, count;  // of blocks
  };
  std::vector<StepRange> step_ranges;
  std::array<int, ppf::kFusedMaxP + 1> shape_of{};  // fused sizes' shapes
  size_t off_models = 0, off_bufs = 0, off_blocks = 0, off_chunks = 0, off_segs = 0,
         off_groups = 0, off_sys = 0, off_tracks = 0, total = 0;
  std::vector<size_t> track_off;
};

std::string validate_batch(const ppf_params* p, int32_t count) {
  if (!p) return "null parameters";
  if (count < 1) return "count must be >= 1";
  for (int32_t t = 0; t < count; ++t) {
    const std::string e = validate(&p[t]);
    if (!e.empty()) return "track " + std::to_string(t) + ": " + e;
    if (p[t].obs_model != PPF_OBS_SPOT)
      return "track " + std::to_string(t) + ": batches take the spot model only";
    if (p[t].grad) return "track " + std::to_string(t) + ": batches do not take grad = 1";
    if (p[t].resample == PPF_RESAMPLE_RPA || p[t].resample == PPF_RESAMPLE_ARNA)
      return "track " + std::to_string(t) + ": batches do not take RPA or ARNA";
    if (p[t].init_kind == PPF_INIT_UNIFORM_ZORDER)
      return "track " + std::to_string(t) + ": batches do not take the Z-ordered init";
    if (p[t].width != p[0].width || p[t].height != p[0].height)
      return "track " + std::to_string(t) + ": frame size differs from track 0";
  }
  return "";
}

// Sizes, offsets and work lists of a batch (p already validated).
// Step items: the sizes up to kFusedMaxP in one fused launch per workgroup
// shape (shape_of[P]), then each wider size in a launch of its own; the
// items of one size in track order.
void order_steps(BatchPlan* bp, const std::array<int, ppf::kFusedMaxP + 1>& shape_of) {
  const int32_t count = (int32_t)bp->models.size();
  std::vector<int> sizes;
  for (int32_t t = 0; t < count; ++t) sizes.push_back(bp->models[t].P);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  bp->blocks.clear();
  bp->step_ranges.clear();
  bp->shape_of = shape_of;
  auto add_size = [&](int P) {
    for (int32_t t = 0; t < count; ++t)
      if (bp->models[t].P == P)
        for (int64_t j = 0; j < bp->bufs[t].nb; ++j) bp->blocks.push_back({t, (int32_t)j});
  };
  for (int sh = 0; sh < ppf::kNumShapes; ++sh) {
    const int64_t first = (int64_t)bp->blocks.size();
    for (int P : sizes)
      if (P <= ppf::kFusedMaxP && shape_of[P] == sh) add_size(P);
    const int64_t cnt = (int64_t)bp->blocks.size() - first;
    if (cnt) bp->step_ranges.push_back({0, sh, first, cnt});
  }
  for (int P : sizes) {
    if (P <= ppf::kFusedMaxP) continue;
    const int64_t first = (int64_t)bp->blocks.size();
    add_size(P);
    bp->step_ranges.push_back({P, 0, first, (int64_t)bp->blocks.size() - first});
  }
}

void plan_batch(const ppf_params* p, int32_t count, BatchPlan* bp) {
  bp->models.resize(count);
  bp->bufs.resize(count);
  bp->track_off.resize(count);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  take(sizeof(Ctrl) * count);
  bp->off_models = take(sizeof(Model) * count);
  bp->off_bufs = take(sizeof(Buffers) * count);
  for (int32_t t = 0; t < count; ++t) {
    bp->models[t] = make_model(&p[t]);
    carve(&p[t], nullptr, &bp->bufs[t], false);
  }
  order_steps(bp, bp->shape_of);
  for (int32_t t = 0; t < count; ++t) {
    for (int64_t j = 0; j < bp->bufs[t].nch; ++j) bp->chunks.push_back({t, (int32_t)j});
    if (p[t].resample == PPF_RESAMPLE_RNA) {
      for (int64_t g = 0; g < bp->models[t].G; ++g) bp->groups.push_back({t, (int32_t)g});
    } else {
      for (int64_t j = 0; j < bp->bufs[t].nseg; ++j) bp->segs.push_back({t, (int32_t)j});
      bp->sys_tracks.push_back(t);
    }
  }
  bp->off_blocks = take(sizeof(ppf::BatchItem) * bp->blocks.size());
  bp->off_chunks = take(sizeof(ppf::BatchItem) * bp->chunks.size());
  bp->off_segs = take(sizeof(ppf::BatchItem) * bp->segs.size());
  bp->off_groups = take(sizeof(ppf::BatchItem) * bp->groups.size());
  bp->off_sys = take(sizeof(int32_t) * bp->sys_tracks.size());
  for (int32_t t = 0; t < count; ++t) bp->track_off[t] = take(carve(&p[t], nullptr, nullptr, false));
  bp->total = off;
}

}  // namespace

struct ppf_batch_ctx : Runner {
  int32_t count = 0;
  BatchPlan plan;
  char* base = nullptr;
  Ctrl* ctrl = nullptr;
  const Model* d_models = nullptr;
  const Buffers* d_bufs = nullptr;
  const ppf::BatchItem *d_blocks = nullptr, *d_chunks = nullptr, *d_segs = nullptr,
                       *d_groups = nullptr;
  const int32_t* d_sys = nullptr;

  int init() {
    return run(kKInit, [&] {
      return ppf::launch_init_batch(d_models, d_bufs, d_blocks, (int64_t)plan.blocks.size(),
                                    stream);
    });
  }
  // The step launches of every track (one range after another).
  hipError_t launch_steps(const float* obs) {
    hipError_t e = hipSuccess;
    // each range steps its own tracks: in a graph the launches may overlap
    ppf::launch_group_begin();
    for (const auto& r : plan.step_ranges) {
      const ppf::BatchItem* it = d_blocks + r.first;
      e = r.P == 0 ? ppf::launch_step_batch_fused(r.shape, d_models, d_bufs, it, r.count, obs,
                                                  stream)
                   : ppf::launch_step_batch(r.P, d_models, d_bufs, it, r.count, obs, stream);
      if (e != hipSuccess) break;
    }
    ppf::launch_group_end();
    return e;
  }
  // Fused step launches per tuning candidate: 0 every fused size in shape 0,
  // 1 all in shape 1, 2 sizes below kFusedMaxP in shape 1 and kFusedMaxP
  // itself in shape 0. Re-orders the step items on the device; syncs. The
  // host plan changes only once the new order is on the device.
  int candidate = 0;
  int set_shapes(int cand) {
    if (cand < 0 || cand > 2) return fail(PPF_EINVAL, "shape candidate must be 0, 1 or 2");
    std::array<int, ppf::kFusedMaxP + 1> sh{};
    for (int P = 0; P <= ppf::kFusedMaxP; ++P)
      sh[P] = cand == 0 ? 0 : (cand == 1 ? 1 : (P < ppf::kFusedMaxP ? 1 : 0));
    BatchPlan next = plan;
    order_steps(&next, sh);
    hipError_t e = hipMemcpyAsync(base + plan.off_blocks, next.blocks.data(),
                                  sizeof(ppf::BatchItem) * next.blocks.size(),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      // the device items may be partly rewritten: put the current order back
      (void)hipMemcpyAsync(base + plan.off_blocks, plan.blocks.data(),
                           sizeof(ppf::BatchItem) * plan.blocks.size(), hipMemcpyHostToDevice,
                           stream);
      (void)hipStreamSynchronize(stream);
      return hip_fail(e, "uploading the step items");
    }
    plan.blocks = std::move(next.blocks);
    plan.step_ranges = std::move(next.step_ranges);
    plan.shape_of = next.shape_of;
    candidate = cand;
    graph.reset();
    return PPF_OK;
  }
};

extern "C" {

int ppf_batch_workspace_bytes(const ppf_params* p, int32_t count, size_t* bytes) {
  if (!bytes || !validate_batch(p, count).empty()) return PPF_EINVAL;
  BatchPlan bp;
  plan_batch(p, count, &bp);
  *bytes = bp.total;
  return PPF_OK;
}

int ppf_batch_create(const ppf_params* p, int32_t count, void* workspace, size_t bytes,
                     void* hip_stream, ppf_batch* out) {
  if (!out) return PPF_EINVAL;
  *out = nullptr;
  if (!validate_batch(p, count).empty() || !workspace) return PPF_EINVAL;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return PPF_EINVAL;
  ppf_batch_ctx* h = new (std::nothrow) ppf_batch_ctx();
  if (!h) return PPF_ENOMEM;
  plan_batch(p, count, &h->plan);
  if (bytes < h->plan.total) {
    delete h;
    return PPF_ENOMEM;
  }
  BatchPlan& bp = h->plan;
  h->count = count;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->base = static_cast<char*>(workspace);
  h->ctrl = reinterpret_cast<Ctrl*>(h->base);
  for (int32_t t = 0; t < count; ++t) {
    carve(&p[t], h->base + bp.track_off[t], &bp.bufs[t], false);
    bp.bufs[t].ctrl = h->ctrl + t;
  }
  h->d_models = reinterpret_cast<const Model*>(h->base + bp.off_models);
  h->d_bufs = reinterpret_cast<const Buffers*>(h->base + bp.off_bufs);
  h->d_blocks = reinterpret_cast<const ppf::BatchItem*>(h->base + bp.off_blocks);
  h->d_chunks = reinterpret_cast<const ppf::BatchItem*>(h->base + bp.off_chunks);
  h->d_segs = reinterpret_cast<const ppf::BatchItem*>(h->base + bp.off_segs);
  h->d_groups = reinterpret_cast<const ppf::BatchItem*>(h->base + bp.off_groups);
  h->d_sys = reinterpret_cast<const int32_t*>(h->base + bp.off_sys);
  struct Up {
    size_t off;
    const void* src;
    size_t n;
  };
  const Up ups[] = {
      {bp.off_models, bp.models.data(), sizeof(Model) * bp.models.size()},
      {bp.off_bufs, bp.bufs.data(), sizeof(Buffers) * bp.bufs.size()},
      {bp.off_blocks, bp.blocks.data(), sizeof(ppf::BatchItem) * bp.blocks.size()},
      {bp.off_chunks, bp.chunks.data(), sizeof(ppf::BatchItem) * bp.chunks.size()},
      {bp.off_segs, bp.segs.data(), sizeof(ppf::BatchItem) * bp.segs.size()},
      {bp.off_groups, bp.groups.data(), sizeof(ppf::BatchItem) * bp.groups.size()},
      {bp.off_sys, bp.sys_tracks.data(), sizeof(int32_t) * bp.sys_tracks.size()},
  };
  hipError_t e = hipSuccess;
  for (const Up& u : ups)
    if (e == hipSuccess && u.n)
      e = hipMemcpyAsync(h->base + u.off, u.src, u.n, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return PPF_EDEVICE;
  }
  const int rc = h->init();
  if (rc != PPF_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return PPF_OK;
}

int ppf_batch_reset(ppf_batch h) {
  if (!h) return PPF_ESTATE;
  return h->init();
}

namespace {
int enqueue_batch_step(ppf_batch h, const float* obs_dev) {
  const BatchPlan& bp = h->plan;
  const int rc0 = h->run(kKStep, [&] { return h->launch_steps(obs_dev); });
  if (rc0) return rc0;
  int rc = h->run(kKMerge, [&] {
    return ppf::launch_merge_batch(h->d_models, h->d_bufs, h->d_chunks,
                                   (int64_t)bp.chunks.size(), h->count, h->stream);
  });
  if (rc) return rc;
  if (!bp.segs.empty()) {
    rc = h->run(kKResample, [&] {
      const hipError_t e = ppf::launch_anc_batch(h->d_models, h->d_bufs, h->d_segs,
                                                 (int64_t)bp.segs.size(), h->stream);
      return e != hipSuccess ? e
                             : ppf::launch_fill_batch(h->d_models, h->d_bufs, h->d_sys,
                                                      (int32_t)bp.sys_tracks.size(), h->stream);
    });
    if (rc) return rc;
  }
  if (!bp.groups.empty())
    return h->run(kKRna, [&] {
      return ppf::launch_rna_batch(h->d_models, h->d_bufs, h->d_groups,
                                   (int64_t)bp.groups.size(), h->stream);
    });
  return PPF_OK;
}
}  // namespace

int ppf_step_batched(ppf_batch h, const float* obs_dev) {
  if (!h) return PPF_ESTATE;
  if (!obs_dev) return h->fail(PPF_EINVAL, "null observation");
  return h->step(obs_dev, [&] { return enqueue_batch_step(h, obs_dev); });
}

int ppf_batch_set_graph(ppf_batch h, int enable) {
  if (!h) return PPF_ESTATE;
  return h->graph_enable(enable);
}

int ppf_batch_set_shapes(ppf_batch h, int32_t candidate) {
  if (!h) return PPF_ESTATE;
  return h->set_shapes(candidate);
}

int ppf_batch_autotune(ppf_batch h, const float* obs_dev, int32_t reps, double* ms_out,
                       int32_t* n_out, int32_t* chosen) {
  if (!h) return PPF_ESTATE;
  if (!obs_dev) return h->fail(PPF_EINVAL, "null observation");
  if (reps < 1 || reps > 10000) return h->fail(PPF_EINVAL, "reps must be in [1, 10000]");
  bool top = false, below = false;
  for (const Model& m : h->plan.models) {
    top = top || m.P == ppf::kFusedMaxP;
    below = below || m.P < ppf::kFusedMaxP;
  }
  const int n = (top && below) ? 3 : 2;
  const int keep = h->candidate;
  double ms[3] = {};
  for (int c = 0; c < n; ++c) {
    int rc = h->set_shapes(c);
    if (!rc) rc = h->time_launches(reps, [&] { return h->launch_steps(obs_dev); }, &ms[c]);
    if (rc) {
      const std::string why = h->err;
      (void)h->set_shapes(keep);  // leave the batch in the shapes it had
      h->err = why;
      return rc;
    }
  }
  int best = 0;
  for (int c = 1; c < n; ++c)
    if (ms[c] < ms[best]) best = c;
  const int rc = h->set_shapes(best);
  if (rc) return rc;
  tune_report(ms, n, best, ms_out, n_out, chosen);
  return PPF_OK;
}

int ppf_batch_stats(ppf_batch h, ppf_stats_t* out, int32_t count) {
  if (!h) return PPF_ESTATE;
  if (!out || count != h->count) return h->fail(PPF_EINVAL, "stats buffer must hold count entries");
  std::vector<Ctrl> c(h->count);
  hipError_t e = hipMemcpyAsync(c.data(), h->ctrl, sizeof(Ctrl) * h->count, hipMemcpyDeviceToHost,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "reading control blocks");
  const int32_t zero = 0;
  for (int32_t t = 0; t < h->count; ++t) {
    fill_stats(c[t], &out[t]);
    if (c[t].rolled_back && e == hipSuccess)
      e = hipMemcpyAsync(&h->ctrl[t].rolled_back, &zero, sizeof zero, hipMemcpyHostToDevice,
                         h->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "clearing roll-back reports");
  return PPF_OK;
}

int ppf_batch_get_particles(ppf_batch h, int32_t track, float* state_host, double* logw_host,
                            int32_t* anc_host) {
  if (!h) return PPF_ESTATE;
  if (track < 0 || track >= h->count) return h->fail(PPF_EINVAL, "track out of range");
  return h->particles(h->plan.models[track], h->plan.bufs[track], state_host, logw_host, anc_host);
}

int ppf_batch_profile_enable(ppf_batch h, int on) {
  if (!h) return PPF_ESTATE;
  return h->profile_enable(on);
}

int ppf_batch_profile_read(ppf_batch h, ppf_kernel_time* out, int max_entries, int* n_entries) {
  if (!h) return PPF_ESTATE;
  return h->profile_read(out, max_entries, n_entries);
}

int ppf_batch_destroy(ppf_batch h) {
  if (!h) return PPF_OK;
  (void)hipStreamSynchronize(h->stream);
  h->collect();
  delete h;
  return PPF_OK;
}

const char* ppf_batch_last_error(ppf_batch h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
