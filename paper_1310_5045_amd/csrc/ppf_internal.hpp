// Internal declarations shared by the HIP kernels (ppf_kernels.hip) and the
// host runtime behind the C ABI (ppf_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ppf {

// Particles per k_step workgroup; also the granularity of the per-block
// normalisation records and of the stored log-weight offsets.
constexpr int kBlock = 256;
// Systematic-resampling scan tiles: 256 threads x 8 particles.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kTile = kScanThreads * kScanItems;
// A tile whose particles own more than kHeavyFactor * kTile output slots is
// handed to the load-balanced heavy pass instead of writing them itself.
constexpr int kHeavyFactor = 4;
constexpr int kHeavyBlocks = 1024;
constexpr int kHeavyChunk = 8192;  // slots per workgroup iteration (32 per thread)
// Normalisation record: m, S, S2, sum e*x[5] (doubles).
constexpr int kRec = 8;
// Up to this many level-1 records the finalize kernel merges them itself;
// beyond, a grid-wide first merge produces at most kReduceBlocks records.
constexpr int64_t kDirectRecords = 4096;
constexpr int kReduceBlocks = 1024;
// LDS image tile of one k_step workgroup, in floats.
constexpr int kTileCap = 4096;
constexpr int kMaxPatch = 25;
constexpr int kMaxGroup = 1024;

// Fixed-point CDF: weights scaled by 2^60; descriptor words carry a 2-bit
// status in bits 62-63 and the value in bits 0-61.
constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;

enum Purpose : uint32_t { kInit = 1, kPropagate = 2, kResample = 3, kRna = 4 };

// What the next k_step reads for the parent and the carried log weight.
enum Mode : int32_t {
  kModeInit = 0,  // parents identity, log w = -log N (after init)
  kModeNone = 1,  // parents identity, log w = stored normalised log weight
  kModeSys = 2,   // parents = ancestors, log w = -log N
  kModeRna = 3,   // parents = ancestors, log w = log(W_g / n) of the slot's group
  kModeSet = 4    // parents identity, log w = caller-supplied fp64 values
};

// Device-resident control block (256 bytes). Kernels read and update it, so a
// step needs no host synchronisation.
struct Ctrl {
  int64_t k;            // committed steps
  int32_t cur;          // which of the double buffers holds the current state
  int32_t mode;         // Mode for the next step
  int32_t resampled;    // last committed step resampled
  int32_t rolled_back;  // steps rolled back since the host last read this
  int32_t do_resample;  // set by finalize for the resampling kernels
  int32_t heavy_count;  // heavy tiles queued by the scan
  uint32_t tile_counter;
  uint32_t pad0;
  double m, log_sum, ess, delta, cum;
  double mean[5];
  double u;             // uniform of the systematic resampling
  double pad1[16];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl must stay 256 bytes");

// Model constants derived on the host from ppf_params (all fp32 parameters
// widened exactly).
struct Model {
  int64_t n;
  double inv_n;
  double log_n;
  int32_t W, H, P, obs;
  int32_t init_kind, group, moved, G;
  float q[5];
  float init_a[5];
  float init_b[5];
  float bf;              // background as the fp32 value used for tile padding
  double b;              // background
  double inv2s2;         // 1 / (2 s^2)
  double inv2sig2;       // 1 / (2 sigma_xi^2)
  double lognorm_obs;    // P^2 log(sigma_xi sqrt(2 pi))
  double lg_inv2r2[3];
  double lg_norm;        // sum_d log(r_d sqrt(2 pi))
  double thr;            // ESS threshold
  double inv_group;
  uint32_t key0, key1, track;
  int32_t strat_t;       // stratified init: total cell bits
};

// Device buffers carved from the caller's workspace (or a scratch area).
struct Buffers {
  Ctrl* ctrl;
  float* X0;     // states, 5*n SoA, double-buffered
  float* X1;
  float* L0;     // stored log weights minus the block maximum, double-buffered
  float* L1;
  double* R0;    // per-block records, double-buffered
  double* R1;
  double* R2;    // second-level records
  int32_t* anc;  // ancestors of the last resampling
  double* lw64;  // fp64 per-particle log weights (caller-set, or output staging)
  double* lwg;   // RNA per-group log(W_g / n)
  uint64_t* desc;   // scan tile descriptors
  uint64_t* heavy;  // heavy-tile queue: (tile, exclusive prefix) pairs
  double* zeros;    // standalone resampling: zero offsets
  int64_t nb;       // level-1 records = ceil(n / kBlock)
  int64_t nr2;      // level-2 records (0: merge level 1 directly)
  int64_t ntiles;   // scan tiles = ceil(n / kTile)
};

// Where the resampling kernels read log weights: value[i] + off[i / kBlock *
// stride] - ctrl->delta. Filter: the stored (L, R) pair selected by ctrl->cur;
// standalone: caller's fp32 log weights with zero offsets.
struct WeightSrc {
  const float* val0;
  const float* val1;
  const double* off0;
  const double* off1;
  int32_t stride;
  int32_t use_cur;
};

// Kernel launchers (ppf_kernels.hip). Each returns the launch status.
hipError_t launch_init(const Model& m, const Buffers& b, hipStream_t s);
hipError_t launch_step(const Model& m, const Buffers& b, const float* obs, hipStream_t s);
hipError_t launch_reduce(const Model& m, const Buffers& b, int standalone, hipStream_t s);
hipError_t launch_finalize(const Model& m, const Buffers& b, int standalone, double u_given,
                           hipStream_t s);
hipError_t launch_scan(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s);
hipError_t launch_heavy(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s);
hipError_t launch_rna(const Model& m, const Buffers& b, const WeightSrc& w, const double* u_dev,
                      hipStream_t s);
hipError_t launch_gather(const Model& m, const Buffers& b, float* out, hipStream_t s);
hipError_t launch_logw(const Model& m, const Buffers& b, hipStream_t s);
hipError_t launch_set_mode(const Buffers& b, int32_t mode, hipStream_t s);
hipError_t launch_records(const Model& m, const Buffers& b, const float* logw, hipStream_t s);
hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                         hipStream_t s);

}  // namespace ppf
