// Internal structures of the index and the launch wrappers of its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "gt.h"

namespace gt {

constexpr int kWalkThreads = 512;     // threads per workgroup of the walk kernels
constexpr int kQueriesPerTile16 = 64; // queries per tile for 16/8-bit pools
constexpr int kQueriesPerTileF32 = 32;
constexpr int kMaxTiles = 1024;       // tiles per call (64K queries)
constexpr int kGroupEntries = 16;     // frontier entries per wave step (32 child rows)
constexpr int kHitStage = 192;        // per-wave LDS staging of candidate hits

// Frontier buckets.  A sparse frontier entry (pool p of level l, mask) lives
// in bucket p >> (l - nb): the subtree of node p's ancestor at level nb, so a
// child stays in its parent's bucket.  Bucket b of tile t is the slot
// b * nt + t; its entries are stored at slot * (fr_cap >> nb).  Buckets are
// dealt to the chip's 8 XCDs in contiguous ranges, so each subtree's pool
// rows are only read through one XCD's L2, where the copies needed by the
// different query tiles meet.
constexpr int kXcds = 8;
constexpr int kMaxBucketBits = 7;
constexpr int kMaxSlots = 8192;       // nt << nb
constexpr int kMaxSlotsPerXcd = kMaxSlots / kXcds;
constexpr int kMaxBucketsPerXcd = (1 << kMaxBucketBits) / kXcds;

// Largest row length (padded columns) whose whole query tile each walk
// format keeps in LDS; wider rows (up to kMaxWalkWidth: d <= 4096, or the
// 2 d_pad rows of a signed index) pass the tile through LDS in windows.
constexpr int kMaxDpBf16 = 1152, kMaxDpFp8 = 2304, kMaxDpF32 = 1152;
constexpr int kMaxWalkWidth = 8192;
__host__ __device__ constexpr int maxdp_walk(int fmt) {
  return fmt == GT_POOL_F32 ? kMaxDpF32 : fmt == GT_POOL_BF16 ? kMaxDpBf16 : kMaxDpFp8;
}

// Device scratch of the allocation-free query entry point (one array per
// device, in gt_noalloc.hip).
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

enum : uint32_t { HIT_ACCEPT = 1u, HIT_BAND = 2u, HIT_REJECT = 3u };

// One candidate (query, vector) pair.  flag: kind in bits 0-1 (HIT_*); an
// accepted pair carries in bits 2-31 its slot among its query's results, the
// value of the query's result counter when it was accepted.
struct Hit {
  uint32_t q, id;
  float sim;
  uint32_t flag;
};
__host__ __device__ inline uint32_t hit_kind(uint32_t flag) { return flag & 3u; }
__host__ __device__ inline uint32_t hit_slot(uint32_t flag) { return flag >> 2; }
constexpr uint32_t kMaxResultsPerQuery = 1u << 30;

// Counters written by the device during a query call.  Zeroed at call start.
struct DevCounters {
  unsigned long long nhits;         // candidates produced (may exceed capacity)
  unsigned long long ncand;         // exhaustive-GEMM candidate pairs
  unsigned long long total;         // results after the recheck
  unsigned long long leaf_pairs;
  unsigned long long rechecked;
  unsigned long long nband;         // candidates within the recheck band
  unsigned int err;                 // invalid query input seen
  unsigned int slot_over;           // a query reached kMaxResultsPerQuery results
  unsigned int fr_over;             // a frontier slot outgrew its capacity (entries dropped)
  unsigned int pad_;
  unsigned long long pairs[GT_MAX_LEVELS];
  unsigned long long entries[GT_MAX_LEVELS];  // frontier (pool, tile) entries per level
};

// Arguments of one level step of the frontier walk (parents at `level`,
// children at `level + 1`).
struct WalkLevelArgs {
  int level, dense, nt, dp;
  int nb;                   // bucket bits
  int64_t bcap;             // entries per bucket slot
  const void* child_rows;   // first row of level+1 in the pool format
  const uint32_t* in_node;
  const uint64_t* in_mask;
  const uint32_t* in_count;  // [slots]
  uint32_t* out_node;
  uint64_t* out_mask;
  uint32_t* out_count;      // [slots]
  const uint64_t* tile_mask;
  const void* qtile;        // [nt * TQ * dp] queries in the pool format
  const float* thr;         // [nt * TQ] lowered thresholds tau'
  const int* qexp;          // [nt * TQ] float8 query scale exponents
  int lexp;                 // float8 scale exponent of level+1
  unsigned long long* stat_pairs;
  uint32_t* bitmap;         // optional: one bit per tree row read
  int64_t bit_base;         // tree row of node 0 of level+1
  // subtraction step (bfloat16 pools): per entry, 64 bfloat16 upper bounds of
  // the pool's score for the tile's queries (entries' live queries only)
  const uint16_t* in_rec;   // [slots * bcap * 64], parallel to in_node
  uint16_t* out_rec;        // [slots * bcap * 64], parallel to out_node
  const float* sabs;        // [nt * TQ] absolute term of the lower bound
  int64_t n_epoch;          // rows visible to the call
  int depth;                // leaves are at this level
  unsigned int* over;       // set when an output slot is full (its entry is dropped)
};

// Arguments of a dense level step (children at `level`, all 2^level pools).
struct DenseLevelArgs {
  int level, nt, dp;
  int64_t rows;             // pools tested: those holding a row below the epoch
  int nb;                   // bucket bits of the sparse output
  int64_t bcap;
  const void* child_rows;   // first row of `level` in the pool format
  const void* qtile;        // [nt * 64 * dp] queries in the pool format
  const float* thr;
  const int* qexp;
  int lexp;                 // float8 scale exponent of `level`
  const uint64_t* parent;   // [2^(level-1) x nt] survival masks, or NULL: tile masks
  const uint64_t* tile_mask;
  uint64_t* out_dense;      // [2^level x nt], or NULL: sparse output below
  uint32_t* out_node;
  uint64_t* out_mask;
  uint32_t* out_count;      // [slots] entries (sparse), or [nt] non-empty masks (dense)
  unsigned long long* stat_pairs;
  uint32_t* bitmap;
  int64_t bit_base;
  uint16_t* out_rec;        // score records of the sparse output, or NULL
  unsigned int* over;       // set when an output slot is full (its entry is dropped)
};

struct LeafArgs {
  int level, dense, nt, dp, tq;
  int nb;
  int64_t bcap;
  const uint32_t* in_node;
  const uint64_t* in_mask;
  const uint32_t* in_count;
  const uint64_t* tile_mask;
  const float* leaves;      // [capacity x dp] float32
  const float* invn_f;      // [capacity]
  const float* qf;          // [nt * tq x dp] float32 queries
  const float* invn_q;      // [nt * tq]
  const double* rho;        // [nt * tq]
  int64_t n_epoch;
  Hit* hits;
  unsigned long long hit_cap;
  uint32_t* band_idx;       // [hit_cap] indices of band candidates in hits
  unsigned int* qcount;     // [nt * tq] accepted results per query
  DevCounters* ctr;
  uint32_t* bitmap;         // optional: one bit per tree row read
  int64_t bit_base;         // tree row of leaf 0
};

struct Index;

// Device workspace of one query call (query copies, frontiers, counters,
// candidate and result staging).  The index owns one for the synchronous
// entry points; gt_batch_create makes more so that calls can be in flight on
// several streams at once.
struct Batch {
  Index* ix = nullptr;
  int max_queries = 0;       // 0: grows on demand (the index's own workspace)
  // Carved out of a caller's fixed device buffer (the scratch of the
  // allocation-free entry point): nothing is ever allocated or freed; a call
  // that would need more than the carve holds fails with GT_ERR_CAPACITY.
  // No events (the host waits on the stream) and no pinned staging.
  bool fixed = false;
  unsigned char* arena = nullptr;  // the fixed buffer and how much of it is used
  size_t arena_size = 0, arena_used = 0;
  // External workspace (gt_batch_create_external): the caller hands each call
  // its device memory.  The frontier gets what the memory leaves after the
  // other buffers (a budget, not the worst case); when a level outgrows it,
  // or the candidates outgrow theirs, finish runs the call again one query
  // tile at a time, each tile with the whole memory.  The call's inputs are
  // kept for that.
  bool external = false;
  bool cont = false;                 // a continuation tile is running
  const float* q_in = nullptr;       // the call's queries (borrowed until finish)
  std::vector<double> rho_in;        // the call's thresholds
  int user_fmt = 0;
  unsigned char* ext_mem = nullptr;
  size_t ext_bytes = 0;
  int64_t ext_pairs = 0;
  int ext_max_queries = 0;           // the external workspace's call limit
  int64_t ext_epoch = 0;             // rows the call sees (kept by its continuation)
  bool hits_overflowed = false;      // the last fixed call's candidates outgrew their room
  int continued_tiles = 0;           // tiles the last call ran one by one
  bool cont_again = false;           // a continued call ended in a result overflow
  int64_t last_max_entries = 0;      // largest frontier level of the last call
  int64_t last_results = 0;
  int nt_alloc = 0;
  int nq_alloc = 0;
  uint32_t* fr_node[2] = {nullptr, nullptr};
  uint64_t* fr_mask[2] = {nullptr, nullptr};
  uint16_t* fr_rec[2] = {nullptr, nullptr};  // score records (64 per entry)
  bool maxpool = false;      // the call walks the max-pool tree
  // the last finished walk of this workspace (automatic dense level)
  bool have_last = false, last_maxpool = false;
  int last_dl = -1, last_walk_fmt = 0, last_walk_nt = 0;
  int64_t last_n_epoch = 0;
  unsigned long long last_entries[GT_MAX_LEVELS] = {};
  float* sabs = nullptr;                     // [nq_pad] lower-bound absolute terms
  int64_t fr_cap = 0;        // entries per tile per buffer
  int64_t rec_len = 0;       // entries of each fr_rec buffer
  uint32_t* lvl_count = nullptr;    // [GT_MAX_LEVELS x kMaxSlots]
  uint64_t* tile_mask = nullptr;    // [kMaxTiles]
  float* qf = nullptr;       // [nq_pad x dp]
  float* qw = nullptr;       // [nq_pad x pw] walk queries [max(q,0) | max(-q,0)] (signed)
  uint16_t* qbf = nullptr;   // [nq_pad x pw]
  uint8_t* q8 = nullptr;
  int* qexp = nullptr;
  float* invn_q = nullptr;
  double* qq = nullptr;
  double* rho = nullptr;
  float* thr = nullptr;
  float* thr_gemm = nullptr;
  unsigned int* qcount = nullptr;
  int64_t* offs = nullptr;   // [nq + 1]
  Hit* hits = nullptr;
  uint32_t* band_idx = nullptr;
  int64_t hit_cap = 0;
  uint2* cand = nullptr;     // exhaustive candidates
  int64_t cand_cap = 0;
  uint32_t* out_id = nullptr;    // results placed by query, unsorted
  float* out_sim = nullptr;
  uint32_t* tmp_id = nullptr;    // radix sort scratch
  float* tmp_sim = nullptr;
  int64_t* fin_id = nullptr;     // sorted results when the caller's buffers are not known yet
  float* fin_sim = nullptr;
  int64_t out_cap = 0;
  // Placement and sort are enqueued with the call, before the host has seen
  // the result count: into the caller's buffers (tgt_*) when the call passed
  // them, else into fin_*.  They do nothing unless the count fits spec_lim.
  int64_t* tgt_ids = nullptr;
  float* tgt_sims = nullptr;
  int64_t tgt_max = 0;
  int64_t spec_lim = -1;
  bool spec_direct = false;
  uint64_t* dmask[2] = {nullptr, nullptr};  // dense survival masks, ping-pong
  int64_t dmask_len = 0;
  uint32_t* bitmap = nullptr;
  int64_t bitmap_words = 0;
  bool counted = false;
  DevCounters* ctr = nullptr;
  DevCounters* h_ctr = nullptr;  // pinned
  double* h_rho = nullptr;       // pinned staging for thresholds
  hipEvent_t done = nullptr;     // counters copied to h_ctr
  hipEvent_t ev[8] = {};
  hipEvent_t evw[2 * GT_MAX_LEVELS] = {};
  bool evw_dense[GT_MAX_LEVELS] = {};
  int nw = 0;
  bool events = false;

  // the call in flight (between submit and finish)
  bool pending = false;
  int kind = 0;              // 1: walk, 2: exhaustive
  hipStream_t stream = nullptr;
  int fmt = 0, nq = 0, nq_pad = 0, nt = 0, tq = 0, head = 0, dense_last = -1, nb = 0;
  int64_t n_epoch = 0;       // vectors visible to the call (ids below this)
  bool profile = false;

  // counters of the last finished call
  int last_nq = 0, last_nt = 0, last_fmt = 0, last_head = -1;
  double ms[8] = {0};
  int frontier_launches = 0, dense_launches = 0;
};

struct Index {
  int device = 0;
  int n_cu = 256;
  int64_t n = 0, cap = 0;
  int d = 0, dp = 0, depth = 0;
  gt_dtype dtype = GT_F32;
  uint32_t formats = 0;
  uint64_t epoch = 0;
  int head_level = -1;       // -1: automatic
  int grid = 0;              // 0: one workgroup per CU
  int dense_last = -2;       // last level walked densely (-2: automatic, -1: none)
  int dense_start = -1;      // automatic: the first call's level (-1: the fixed rule)
  int walk_subtract = -1;    // subtraction step (bfloat16 after a dense step): 0 off,
                             // 1 every sparse level, 2 all but the last, -1 automatic
  bool profile = false;
  bool count_unique = false;
  double m_min = 0.0;        // host copy
  int64_t bytes = 0;

  // device memory of the tree
  float* leaves = nullptr;   // [cap x dp]
  float* invn = nullptr;     // [cap]
  double* ff = nullptr;      // [cap] canonical squared norms
  float* nf = nullptr;       // [cap] float32 norms rounded down (GEMM epilogue)
  double* d_mmin = nullptr;  // device copy of m_min, and a scratch slot
  float* master = nullptr;   // levels 0..depth-1, level l at row (2^l - 1)
  uint16_t* pbf16 = nullptr;
  uint8_t* pfp8 = nullptr;
  float* mmax = nullptr;     // element-wise max pools (Our-Max), same layout as master
                             // with rows of pw values
  uint16_t* pmax16 = nullptr;  // their bfloat16 copy, rounded up
  // Vectors of any sign (GT_POOL_SIGNED): mmax rows are [max + B | B - min]
  // over the members, pw = 2 dp; no sum trees.
  bool signed_mode = false;
  int pw = 0;                // row length of mmax / pmax16 (dp, or 2 dp when signed)
  float sbound = 0.0f;       // B (power of two >= every |value|), signed only
  unsigned int* d_absmax = nullptr;  // float bits of the largest |value| of an ingest
  int* d_lexp = nullptr;     // float8 scale exponents per level
  int lexp[GT_MAX_LEVELS] = {0};
  float* d_levelmax = nullptr;
  unsigned int* d_flags = nullptr;  // float8 overflow flags per level; last: input error

  Batch* def = nullptr;      // workspace of gt_query_batch / gt_exhaustive
  hipError_t scratch_err = hipSuccess;  // set-up of the device scratch at build
};

// ---- launch wrappers (kernels in k_build.hip, k_walk.hip, k_exhaustive.hip) ----
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_ingest(const void* src, int dtype, int64_t rows, int d, int dp, float* leaves,
                         double* ff, float* invn, float* nf, double* mmin, unsigned int* err,
                         bool allow_negative, unsigned int* absmax, hipStream_t s);
hipError_t launch_signed_bottom(const float* leaves, float* parent, int64_t first, int64_t nodes,
                                int dp, int d, int64_t n, float bound, hipStream_t s);
hipError_t launch_build_level(const float* child, float* parent, int64_t nodes, int dp,
                              int64_t first, hipStream_t s, bool max_pool);
hipError_t launch_level_entries(const uint32_t* lvl_count, int first, int levels,
                                DevCounters* ctr, hipStream_t s);
hipError_t launch_level_max(const float* rows, int64_t nrows, int dp, float* out_max, hipStream_t s);
hipError_t launch_quant_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t s);
hipError_t launch_quant_fp8(const float* src, uint8_t* dst, int64_t count, int lexp,
                            unsigned int* overflow, hipStream_t s);
hipError_t launch_query_prep(const float* q, int nq, int d, int dp, int tq, const double* rho,
                             const double* mmin, float* qf, uint16_t* qbf, uint8_t* q8, int* qexp,
                             float* invn_q, double* qq, float* thr, float* thr_gemm,
                             uint64_t* tile_mask, const float* root, float* sabs,
                             float* qw, int pw, float sbound,
                             unsigned int* err, int nq_pad, hipStream_t s);
hipError_t launch_walk_level(int fmt, const WalkLevelArgs& a, int grid, hipStream_t s);
hipError_t launch_walk_sub(const WalkLevelArgs& a, int grid, hipStream_t s);
hipError_t launch_leaf(const LeafArgs& a, int grid, hipStream_t s);
hipError_t launch_dense_level(int fmt, const DenseLevelArgs& a, hipStream_t s);
hipError_t launch_recheck(Hit* hits, const uint32_t* band_idx, const unsigned long long* nband,
                          unsigned long long cap, const float* qf, const float* leaves, int d,
                          int dp, const double* ff, const double* rho,
                          unsigned int* qcount, DevCounters* ctr, hipStream_t s);
hipError_t launch_scan_offsets(const unsigned int* qcount, int nq, int64_t* offs_internal,
                               int64_t* offs_out, DevCounters* ctr, hipStream_t s);
hipError_t launch_scatter(const Hit* hits, const DevCounters* ctr, unsigned long long hit_cap,
                          unsigned long long lim, const int64_t* offs, uint32_t* out_id,
                          float* out_sim, hipStream_t s);
hipError_t launch_sort_segments(const int64_t* offs, int nq, uint32_t* id, float* sim,
                                uint32_t* tmp_id, float* tmp_sim, int64_t* ids_out,
                                float* sims_out, const DevCounters* ctr,
                                unsigned long long hit_cap, unsigned long long lim,
                                int64_t id_bound, hipStream_t s);
hipError_t launch_exhaustive_gemm(const float* qf, int nq_pad, const float* leaves, int64_t n,
                                  int dp, const float* thr_gemm, const float* nf, uint2* cand,
                                  unsigned long long cand_cap, DevCounters* ctr, int nq,
                                  hipStream_t s);
hipError_t launch_pair_check(const uint2* cand, const unsigned long long* ncand,
                             unsigned long long cap, const float* qf, const float* leaves,
                             const float* invn_q, const float* invn_f, const double* rho, int dp,
                             Hit* hits, unsigned long long hit_cap, uint32_t* band_idx,
                             unsigned int* qcount, DevCounters* ctr, int grid, hipStream_t s);
// Scratch of the allocation-free entry point (gt_noalloc.hip): taken once per
// device at set-up (index build), with that device current.
hipError_t scratch_setup(int device);
void* scratch_of(int device);  // NULL until scratch_setup succeeded on the device

hipError_t launch_insert_paths(float* master, const float* leaves, int depth, int dp, int64_t lo,
                               int64_t hi, uint16_t* pbf16, uint8_t* pfp8, const int* lexp,
                               unsigned int* flags, hipStream_t s);

}  // namespace gt
