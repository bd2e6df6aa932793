// Internal declarations shared by the HIP kernels (ppf_kernels.hip) and the
// host runtime behind the C ABI (ppf_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <vector>

namespace ppf {

// Particles per k_step workgroup; also the granularity of the per-block
// normalisation records and of the stored log-weight offsets.
constexpr int kBlock = 256;
// LDS image tile of one k_step workgroup (D = Z - b as doubles; this is the
// widest) and its table of P-pixel row sums of D^2 at the patch-centre
// columns (doubles).
constexpr int kTileCap = 2048;
constexpr int kSqCap = 1536;
// Workgroup shapes of the step kernel for patches up to kFusedMaxP: shape s
// stages a tile of up to kShapeTile[s] doubles and is compiled for
// kShapeWaves[s] waves per SIMD, which its LDS lets as many workgroups share
// a CU with. Which is faster depends on the patch size (register demand
// grows with it); the autotuner measures them on the live workload.
constexpr int kNumShapes = 2;
constexpr int kShapeTile[kNumShapes] = {2048, 1792};
constexpr int kShapeWaves[kNumShapes] = {5, 6};
constexpr int kMaxPatch = 25;
constexpr int kMaxGroup = 1024;

// Normalisation record of one block of kBlock particles (doubles), with
// E = exp(l - m) rounded to fp32 the stored weight of a particle:
//   [0] m   maximum log weight of the block
//   [1] B   sum of the fixed-point weights round(E 2^44) (an exact integer
//           below 2^52, held in a double)
//   [2] S2  sum E^2; NaN marks a non-finite log weight
//   [3..7]  sum E x_d for the five state components
constexpr int kRec = 8;
constexpr double kItemScale = 0x1p44;   // fixed-point weight of one particle
constexpr double kCdfScale = 0x1p62;    // fixed-point scale of the global CDF
// Chunk prefixes map 2^44-scaled weights to the 2^62-scaled CDF.
constexpr double kItemToCdf = 0x1p18;

// Systematic resampling: one wave per segment of kSegBlocks blocks writes the
// segment's output slots itself when they span at most kCoopTiles tiles of
// kSlotTile slots; a heavier segment queues its tiles in chunks of
// kChunkTiles for k_fill (kFillGrid one-wave workgroups, each taking chunks
// in turn).
constexpr int kSegBlocks = 4;
constexpr int kSegItems = kSegBlocks * kBlock;
constexpr int kSlotTile = kSegItems;  // slots per LDS tile of the segment's writes
constexpr int kCoopTiles = 4;
constexpr int kChunkTiles = 2;
constexpr int kFillGrid = 4096;
constexpr int kFillGridBatch = 2048;  // waves of a batched fill, over all tracks' queues
// Batched steps run every patch size up to this one in a single launch (the
// sizes that fit five waves per SIMD); wider patches launch per size.
constexpr int kFusedMaxP = 13;
constexpr int kSortTile = 1024;      // pairs per tile of the radix sort and list scans
// The allocation-free standalone resampler keeps its scratch in a device
// array of this many bytes, one per device for the life of the process.
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;

// One work item of a batched launch: the track, and the index of the track's
// block, merge chunk, resampling segment or RNA group.
struct BatchItem {
  int32_t track;
  int32_t idx;
};

// One entry of the fill queue: the tiles [tile_lo, tile_hi) of a heavy
// resampling segment.
struct TileRun {
  int32_t seg;
  int32_t tile_lo;
  int32_t tile_hi;
  int32_t pad;
};

enum Purpose : uint32_t { kInit = 1, kPropagate = 2, kResample = 3, kRna = 4, kRing = 5 };

// What the next k_step reads for the parent and the carried log weight.
enum Mode : int32_t {
  kModeInit = 0,  // parents identity, log w = -log N (after init)
  kModeNone = 1,  // parents identity, log w = stored normalised log weight
  kModeSys = 2,   // parents = ancestors, log w = -log N
  kModeRna = 3,   // parents = ancestors, log w = log(W_g / n) of the slot's group
  kModeSet = 4,   // parents identity, log w = caller-supplied fp64 values
  kModeArna = 5   // parents = ancestors, log w = log(W_g / n) of the slot's group, or
                  // of its ring predecessor for the last arna_moved slots
};

// Derivatives of log p^ kept in gradient mode, theta = (s, b, sigma_xi,
// q_x, q_y, q_vx, q_vy, q_I, I0), and the per-particle tangents of the state
// in q (dx/dq_x, dy/dq_y, dvx/dq_vx, dx/dq_vx, dvy/dq_vy, dy/dq_vy, dI/dq_I).
constexpr int kNGrad = 9;
constexpr int kNTan = 7;

// Device-resident control block (384 bytes). Kernels read and update it, so a
// step needs no host synchronisation.
struct Ctrl {
  int64_t k;            // committed steps
  int32_t cur;          // which of the double buffers holds the current state
  int32_t mode;         // Mode for the next step
  int32_t resampled;    // last committed step resampled
  int32_t rolled_back;  // steps rolled back since the host last read this
  int32_t do_resample;  // set by the merge for the resampling kernels
  int32_t heavy_count;  // tile chunks queued for k_fill
  uint64_t pad0;
  double m, log_sum, ess, delta, cum;
  double mean[5];
  double u;             // uniform of the systematic resampling
  uint64_t total;       // fixed-point total weight (2^62 scale) of the CDF
  double grad_cum[kNGrad];   // d cum / d theta over committed steps
  double grad_last[kNGrad];  // the last committed step's term
  // ARNA: the frame of the latest loss (keys the ring order; 0: index ring),
  // the log-likelihood increment of the last frame that was not lost, whether
  // the last step lost the object, and its resampling's tracking groups
  // (counted by k_arna_local) and slots exchanged
  int64_t ring_key;
  double delta_ref;
  int32_t lost;
  int32_t arna_tracking;
  int32_t arna_moved;
  int32_t pad2;
  double pad1[9];
};
static_assert(sizeof(Ctrl) == 384, "Ctrl must stay 384 bytes");

// Prefix of one chunk of block records: P = fixed-point CDF before the chunk,
// phi = factor from the chunk's relative integer weights to the CDF scale.
struct ChunkPre {
  uint64_t P;
  double phi;
};

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
  double b;              // background
  double inv2s2;         // 1 / (2 s^2)
  double inv2sig2;       // 1 / (2 sigma_xi^2)
  double lognorm_obs;    // P^2 log(sigma_xi sqrt(2 pi))
  double gstep[kMaxPatch];  // exp(-(2 (d - h) + 1) / (2 s^2)), h = (P - 1) / 2
  double lg_inv2r2[3];
  double lg_norm;        // sum_d log(r_d sqrt(2 pi))
  double thr;            // ESS threshold
  double inv_group;
  uint32_t key0, key1, track;
  int32_t strat_t;       // stratified init: total cell bits
  int32_t grad;          // accumulate d log p^ / d theta
  int32_t rpa;           // resampling with proportional allocation
  int32_t dlb;           // its schedule (0 greedy, 1 sorted greedy)
  int32_t rpa_group;     // particles per RPA group
  int32_t rpa_G;         // RPA groups
  int32_t shape;         // step workgroup shape (patches up to kFusedMaxP)
  double s_psf;          // s
  double sig;            // sigma_xi
  double clo[2], chi[2]; // patch-centre clamp (x, y): -P and W + P, H + P
  // ARNA (group, G and moved = the largest exchange as for RNA)
  int32_t arna;          // adaptive RNA
  int32_t arna_mu_min;   // the smallest exchange, floor(arna_min n)
  double arna_share;     // a group tracks when W_g >= arna_share (= theta / G)
  double arna_drop;      // lost when delta < delta_ref - arna_drop (= kappa P)
};

// Device buffers carved from the caller's workspace (or a scratch area).
struct Buffers {
  Ctrl* ctrl;
  float* X0;     // states, 5*n SoA, double-buffered
  float* X1;
  float* E0;     // stored weights exp(l - m_block) in fp32, double-buffered
  float* E1;
  double* R0;    // per-block records, double-buffered
  double* R1;
  uint64_t* pfx;    // per block: exclusive prefix of its chunk's relative weights
  double* CR;       // per chunk: merged record (m, Q bits, S2, sum e x[5])
  ChunkPre* cpre;   // per chunk: CDF prefix
  int32_t* anc;  // ancestors of the last resampling
  double* lw64;  // fp64 per-particle log weights (caller-set, or output staging)
  double* lwg;   // RNA per-group log(W_g / n)
  TileRun* hq;   // queued tile chunks of heavy resampling segments
  float* T0;     // gradient mode: tangents, kNTan*n SoA, double-buffered with X
  float* T1;
  double* RG;    // gradient mode: per block sum E d l / d theta (kNGrad doubles)
  double* CRG;   // gradient mode: per chunk, the same merged (kNGrad doubles)
  int32_t* asys;     // RPA: ancestors of the global systematic resampling
  int64_t* rfirst;   // RPA: first systematic slot of each group's offspring (G + 1)
  int64_t* rdbase;   // RPA: per receiver group, its first surplus particle
  int64_t* rscum;    // RPA: exclusive prefix of the senders' surplus (ns + 1)
  int32_t* rns;      // RPA: number of senders
  uint32_t* rkey0;   // RPA with SGS: radix-sort keys of the 2G list entries, ping
  uint32_t* rkey1;   //   and pong
  int32_t* rval0;    // RPA with SGS: their groups (after the sort: senders in order,
  int32_t* rval1;    //   then receivers in order), ping and pong
  uint32_t* rhist;   // RPA with SGS: digit counts per sort tile (256 x tiles)
  uint32_t* rrow;    // RPA with SGS: digit totals (256)
  uint64_t* rtsum;   // RPA: per list tile, the sum of the values and the count present
  uint32_t* zkey0;   // Z-ordered init: the particles' sort keys, ping
  uint32_t* zkey1;   //   and pong
  int32_t* zval0;    // Z-ordered init: their draw indices, ping (after the sort: the
  int32_t* zval1;    //   draw index at each position) and pong
  uint32_t* zhist;   // Z-ordered init: digit counts per sort tile
  uint32_t* zrow;    // Z-ordered init: digit totals
  int32_t* rsidx;    // RPA: each sender group's position in the sender order (G)
  int32_t* rstream;  // RPA: the senders' surplus offspring in schedule order (N)
  int32_t* aloc;     // ARNA: each group's local resampling (n global indices)
  double* Wg;        // ARNA: each group's share of the normalised weight
  double* lwt;       // ARNA: per group, the weight log(W_pred / n) of its exchanged slots
  int64_t hq_cap;   // entries of hq
  int64_t nb;       // block records = ceil(n / kBlock)
  int64_t chunk;    // records per merge chunk (multiple of 256, at most 2048)
  int64_t nch;      // merge chunks = ceil(nb / chunk)
  int64_t nseg;     // resampling segments = ceil(n / kSegItems)
};

// Where the resampling kernels read weights, with the block records: the
// filter's stored E (the pair selected by ctrl->cur), or a caller's absolute
// fp32 log weights (log_src = 1, standalone resampling). A particle's weight
// relative to its block maximum is e = E, or exp(x - m_block) in fp64 for
// log weights; its fixed-point weight inside its block is round(e 2^44).
struct WeightSrc {
  const float* E0;
  const float* E1;
  const double* rec0;
  const double* rec1;
  int32_t use_cur;
  int32_t log_src;
};

// Kernel launchers (ppf_kernels.hip). Each returns the launch status.
hipError_t launch_init(const Model& m, const Buffers& b, hipStream_t s);
hipError_t launch_step(const Model& m, const Buffers& b, const float* obs, hipStream_t s);
hipError_t launch_merge(const Model& m, const Buffers& b, int standalone, double u_given,
                        hipStream_t s);
hipError_t launch_anc(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s);
hipError_t launch_fill(const Model& m, const Buffers& b, const WeightSrc& w, hipStream_t s);
hipError_t launch_rna(const Model& m, const Buffers& b, const WeightSrc& w, const double* u_dev,
                      hipStream_t s);
hipError_t launch_gather(const Model& m, const Buffers& b, float* out, hipStream_t s);
hipError_t launch_logw(const Model& m, const Buffers& b, hipStream_t s);
hipError_t launch_set_mode(const Buffers& b, int32_t mode, hipStream_t s);
hipError_t launch_records(const Model& m, const Buffers& b, const float* logw, hipStream_t s);
hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                         hipStream_t s);

// Device address and size of the current device's static scratch array
// (kStaticScratchBytes, 256-byte aligned), looked up once per device.
hipError_t static_scratch(void** ptr, size_t* bytes);

// ARNA: local resampling per group, then the exchange along the ring.
// RNA of the filter's own weights in two launches: every group's local
// resampling, then the exchange with group g-1.
hipError_t launch_rna_groups(const Model& m, const Buffers& b, hipStream_t s);
hipError_t launch_arna(const Model& m, const Buffers& b, hipStream_t s);

// RPA: the balancing plan and the routed ancestors of one filter.
hipError_t launch_rpa(const Model& m, const Buffers& b, hipStream_t s);
// DLB schedule of G groups' counts (kind 0 GS, 1 SGS, 2 LGS) with
// dlb_scratch_bytes(G) bytes of device scratch (256-byte aligned).
size_t dlb_scratch_bytes(int32_t G);
hipError_t launch_dlb_schedule(int32_t kind, const int32_t* counts, int32_t G, int32_t n,
                               int32_t* sched, int32_t cap, int32_t* n_entries, void* scratch,
                               hipStream_t s);

// Batched launches over independent filters: ms and bs are device arrays of
// the tracks' models and buffers, items the device list of work items.
hipError_t launch_init_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                             int64_t n_items, hipStream_t s);
// Items of one patch size above kFusedMaxP.
hipError_t launch_step_batch(int P, const Model* ms, const Buffers* bs, const BatchItem* items,
                             int64_t n_items, const float* obs, hipStream_t s);
// Items with patch sizes up to kFusedMaxP, whatever their size, in one
// launch of the given workgroup shape.
hipError_t launch_step_batch_fused(int shape, const Model* ms, const Buffers* bs,
                                   const BatchItem* items, int64_t n_items, const float* obs,
                                   hipStream_t s);
// The chunk merges (items), then one final merge per track.
hipError_t launch_merge_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                              int64_t n_items, int32_t n_tracks, hipStream_t s);
hipError_t launch_anc_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                            int64_t n_items, hipStream_t s);
hipError_t launch_fill_batch(const Model* ms, const Buffers* bs, const int32_t* tracks,
                             int32_t n_tracks, hipStream_t s);
hipError_t launch_rna_batch(const Model* ms, const Buffers* bs, const BatchItem* items,
                            int64_t n_items, hipStream_t s);

// A HIP graph of one step's launches, replayed with another frame. While a
// StepGraph records (begin() to end(), on the calling thread), the launch_*
// functions above add kernel nodes to it, each depending on the one before,
// instead of launching; the graph keeps every node's argument values, and
// notes the arguments equal to the frame pointer given to begin() so that
// set_frame() can point them at another frame before a replay.
class StepGraph {
 public:
  StepGraph() = default;
  StepGraph(const StepGraph&) = delete;
  StepGraph& operator=(const StepGraph&) = delete;
  ~StepGraph();
  hipError_t begin(const float* frame);
  hipError_t end();  // stops recording and instantiates the graph
  bool ready() const { return exec_ != nullptr; }
  hipError_t set_frame(const float* frame);
  hipError_t launch(hipStream_t s) const { return hipGraphLaunch(exec_, s); }

  // used by the launch functions while recording
  struct Args {
    virtual ~Args() = default;
  };
  hipError_t add(const void* fn, dim3 grid, dim3 block, std::unique_ptr<Args> args,
                 std::vector<void*> argv, std::vector<const float**> frame_slots);
  const float* frame() const { return frame_; }
  // Nodes added between group_begin and group_end depend only on what came
  // before the group, and the first node after it on all of them.
  void group_begin();
  void group_end();

 private:
  struct Node {
    hipGraphNode_t node = nullptr;
    hipKernelNodeParams params{};
    std::unique_ptr<Args> args;
    std::vector<void*> argv;
    std::vector<const float**> frame_slots;
  };
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  std::vector<Node> nodes_;
  const float* frame_ = nullptr;
  std::vector<hipGraphNode_t> deps_;   // what the next node depends on
  bool in_group_ = false;
  std::vector<hipGraphNode_t> group_;  // the nodes of the open group
};

// Launches between these two calls may run concurrently when a graph records
// them (they must touch disjoint data); on a stream they run in order.
void launch_group_begin();
void launch_group_end();

}  // namespace ppf
