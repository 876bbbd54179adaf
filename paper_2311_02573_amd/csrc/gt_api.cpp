// Host runtime behind the C interface of gt.h: the index object, device buffer
// management and the launch sequence of each call.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gt.h"
#include "gt_internal.h"

using gt::Index;

struct gt_index : Index {};

namespace {

thread_local std::string g_err;

gt_status fail(gt_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? GT_ERR_OUT_OF_MEMORY : GT_ERR_DEVICE,    \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

template <class T>
gt_status dalloc(Index* ix, T** p, size_t count) {
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(GT_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                          " bytes failed: " + hipGetErrorString(e));
  }
  *p = static_cast<T*>(q);
  ix->bytes += (int64_t)(count * sizeof(T));
  return GT_OK;
}

template <class T>
void dfree(Index* ix, T** p, size_t count) {
  if (*p) {
    (void)hipFree(*p);
    ix->bytes -= (int64_t)(std::max<size_t>(count, 1) * sizeof(T));
  }
  *p = nullptr;
}

#define TRY(expr)                  \
  do {                             \
    gt_status s_ = (expr);         \
    if (s_ != GT_OK) return s_;    \
  } while (0)

inline int64_t level_row(int level) { return (int64_t(1) << level) - 1; }

inline size_t bitmap_words(const Index* ix) { return (size_t)((int64_t(2) << ix->depth) / 32 + 1); }

int default_head(int depth) {
  // Pools near the root hold thousands of vectors and essentially never fall
  // below the threshold; starting the walk a few levels down only skips tests
  // that cannot prune.
  int h = std::min(10, depth - 10);
  return std::max(0, std::min(h, depth - 1));
}

int head_of(const Index* ix) {
  if (ix->head_level >= 0) return std::min(ix->head_level, ix->depth - 1);
  return default_head(ix->depth);
}

int tq_of(int fmt) { return fmt == GT_POOL_F32 ? gt::kQueriesPerTileF32 : gt::kQueriesPerTile16; }

int maxdp_of(int fmt) {
  return fmt == GT_POOL_F32 ? gt::kMaxDpF32 : fmt == GT_POOL_BF16 ? gt::kMaxDpBf16 : gt::kMaxDpFp8;
}

void free_all(Index* ix) {
  const size_t cap = (size_t)ix->cap, dp = (size_t)ix->dp, tree = (cap - 1) * dp;
  dfree(ix, &ix->leaves, cap * dp);
  dfree(ix, &ix->invn, cap);
  dfree(ix, &ix->ff, cap);
  dfree(ix, &ix->nf, cap);
  dfree(ix, &ix->d_mmin, 2);
  dfree(ix, &ix->master, tree);
  dfree(ix, &ix->pbf16, tree);
  dfree(ix, &ix->pfp8, tree);
  dfree(ix, &ix->d_lexp, GT_MAX_LEVELS);
  dfree(ix, &ix->d_levelmax, GT_MAX_LEVELS);
  dfree(ix, &ix->d_flags, GT_MAX_LEVELS);
  for (int b = 0; b < 2; ++b) {
    dfree(ix, &ix->fr_node[b], (size_t)ix->nt_alloc * ix->fr_cap);
    dfree(ix, &ix->fr_mask[b], (size_t)ix->nt_alloc * ix->fr_cap);
  }
  const size_t nqa = (size_t)ix->nq_alloc;
  dfree(ix, &ix->lvl_count, (size_t)GT_MAX_LEVELS * gt::kMaxTiles);
  dfree(ix, &ix->tile_mask, gt::kMaxTiles);
  dfree(ix, &ix->qf, nqa * dp);
  dfree(ix, &ix->qbf, nqa * dp);
  dfree(ix, &ix->q8, nqa * dp);
  dfree(ix, &ix->qexp, nqa);
  dfree(ix, &ix->invn_q, nqa);
  dfree(ix, &ix->qq, nqa);
  dfree(ix, &ix->rho, nqa);
  dfree(ix, &ix->thr, nqa);
  dfree(ix, &ix->thr_gemm, nqa);
  dfree(ix, &ix->qcount, nqa);
  dfree(ix, &ix->qcursor, nqa);
  dfree(ix, &ix->offs, nqa + 1);
  dfree(ix, &ix->hits, (size_t)ix->hit_cap);
  dfree(ix, &ix->band_idx, (size_t)ix->hit_cap);
  dfree(ix, &ix->cand, (size_t)ix->cand_cap);
  dfree(ix, &ix->out_id, (size_t)ix->out_cap);
  dfree(ix, &ix->out_sim, (size_t)ix->out_cap);
  dfree(ix, &ix->tmp_id, (size_t)ix->out_cap);
  dfree(ix, &ix->tmp_sim, (size_t)ix->out_cap);
  dfree(ix, &ix->ctr, 1);
  dfree(ix, &ix->bitmap, bitmap_words(ix));
  if (ix->h_ctr) (void)hipHostFree(ix->h_ctr);
  if (ix->h_rho) (void)hipHostFree(ix->h_rho);
  ix->h_ctr = nullptr;
  ix->h_rho = nullptr;
}

gt_status zero_dev(void* p, size_t bytes, hipStream_t s) {
  HIPCHK(gt::launch_zero_u32(static_cast<uint32_t*>(p), (int64_t)(bytes / 4), s));
  return GT_OK;
}

// float8 scale exponent of a level: 2^e with (level max * 2) / 2^e <= 448, so
// a pool can grow to twice its build-time maximum through inserts before the
// level has to be rescaled.
int fp8_exp_for(float mx) {
  if (!(mx > 0.0f)) return 0;
  int ex;
  const double m = frexp((double)mx * 2.0 / 448.0, &ex);
  return m == 0.5 ? ex - 1 : ex;
}

gt_status quantize_fp8_level(Index* ix, int level, hipStream_t s, bool recompute_scale) {
  const int64_t nodes = int64_t(1) << level;
  float* rows = ix->master + level_row(level) * ix->dp;
  if (recompute_scale) {
    TRY(zero_dev(ix->d_levelmax + level, 4, s));
    HIPCHK(gt::launch_level_max(rows, nodes, ix->dp, ix->d_levelmax + level, s));
    float mx = 0.0f;
    HIPCHK(hipMemcpyAsync(&mx, ix->d_levelmax + level, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ix->lexp[level] = fp8_exp_for(mx);
    HIPCHK(hipMemcpyAsync(ix->d_lexp + level, &ix->lexp[level], 4, hipMemcpyHostToDevice, s));
  }
  HIPCHK(gt::launch_quant_fp8(rows, ix->pfp8 + level_row(level) * ix->dp, nodes * ix->dp,
                              ix->lexp[level], ix->d_flags + level, s));
  return GT_OK;
}

gt_status ensure_query_buffers(Index* ix, int nq_pad, int nt) {
  const size_t dp = (size_t)ix->dp;
  if (!ix->ctr) {
    TRY(dalloc(ix, &ix->ctr, 1));
    HIPCHK(hipHostMalloc((void**)&ix->h_ctr, sizeof(gt::DevCounters), hipHostMallocDefault));
    TRY(dalloc(ix, &ix->lvl_count, (size_t)GT_MAX_LEVELS * gt::kMaxTiles));
    TRY(dalloc(ix, &ix->tile_mask, gt::kMaxTiles));
  }
  if (nq_pad > ix->nq_alloc) {
    const size_t o = (size_t)ix->nq_alloc, nqa = (size_t)nq_pad;
    dfree(ix, &ix->qf, o * dp);
    dfree(ix, &ix->qbf, o * dp);
    dfree(ix, &ix->q8, o * dp);
    dfree(ix, &ix->qexp, o);
    dfree(ix, &ix->invn_q, o);
    dfree(ix, &ix->qq, o);
    dfree(ix, &ix->rho, o);
    dfree(ix, &ix->thr, o);
    dfree(ix, &ix->thr_gemm, o);
    dfree(ix, &ix->qcount, o);
    dfree(ix, &ix->qcursor, o);
    dfree(ix, &ix->offs, o + 1);
    if (ix->h_rho) (void)hipHostFree(ix->h_rho);
    ix->h_rho = nullptr;
    ix->nq_alloc = 0;
    TRY(dalloc(ix, &ix->qf, nqa * dp));
    TRY(dalloc(ix, &ix->qbf, nqa * dp));
    TRY(dalloc(ix, &ix->q8, nqa * dp));
    TRY(dalloc(ix, &ix->qexp, nqa));
    TRY(dalloc(ix, &ix->invn_q, nqa));
    TRY(dalloc(ix, &ix->qq, nqa));
    TRY(dalloc(ix, &ix->rho, nqa));
    TRY(dalloc(ix, &ix->thr, nqa));
    TRY(dalloc(ix, &ix->thr_gemm, nqa));
    TRY(dalloc(ix, &ix->qcount, nqa));
    TRY(dalloc(ix, &ix->qcursor, nqa));
    TRY(dalloc(ix, &ix->offs, nqa + 1));
    HIPCHK(hipHostMalloc((void**)&ix->h_rho, nqa * sizeof(double), hipHostMallocDefault));
    ix->nq_alloc = nq_pad;
  }
  const int64_t fr_cap = int64_t(1) << std::max(0, ix->depth - 1);
  if (nt > ix->nt_alloc || fr_cap != ix->fr_cap) {
    for (int b = 0; b < 2; ++b) {
      dfree(ix, &ix->fr_node[b], (size_t)ix->nt_alloc * ix->fr_cap);
      dfree(ix, &ix->fr_mask[b], (size_t)ix->nt_alloc * ix->fr_cap);
    }
    ix->nt_alloc = 0;
    for (int b = 0; b < 2; ++b) {
      TRY(dalloc(ix, &ix->fr_node[b], (size_t)nt * fr_cap));
      TRY(dalloc(ix, &ix->fr_mask[b], (size_t)nt * fr_cap));
    }
    ix->nt_alloc = nt;
    ix->fr_cap = fr_cap;
  }
  if (!ix->hits) {
    ix->hit_cap = int64_t(1) << 20;
    TRY(dalloc(ix, &ix->hits, (size_t)ix->hit_cap));
    TRY(dalloc(ix, &ix->band_idx, (size_t)ix->hit_cap));
  }
  return GT_OK;
}

gt_status grow_hits(Index* ix, int64_t need) {
  dfree(ix, &ix->hits, (size_t)ix->hit_cap);
  dfree(ix, &ix->band_idx, (size_t)ix->hit_cap);
  ix->hit_cap = 0;
  const int64_t cap = need + need / 4 + 1024;
  if (cap >= (int64_t(1) << 32)) return fail(GT_ERR_OUT_OF_MEMORY, "more than 2^32 candidates");
  TRY(dalloc(ix, &ix->hits, (size_t)cap));
  TRY(dalloc(ix, &ix->band_idx, (size_t)cap));
  ix->hit_cap = cap;
  return GT_OK;
}

gt_status ensure_out(Index* ix, int64_t need) {
  if (need <= ix->out_cap && ix->out_id) return GT_OK;
  const size_t o = (size_t)ix->out_cap;
  dfree(ix, &ix->out_id, o);
  dfree(ix, &ix->out_sim, o);
  dfree(ix, &ix->tmp_id, o);
  dfree(ix, &ix->tmp_sim, o);
  ix->out_cap = 0;
  const int64_t cap = std::max<int64_t>(need + need / 4, int64_t(1) << 16);
  TRY(dalloc(ix, &ix->out_id, (size_t)cap));
  TRY(dalloc(ix, &ix->out_sim, (size_t)cap));
  TRY(dalloc(ix, &ix->tmp_id, (size_t)cap));
  TRY(dalloc(ix, &ix->tmp_sim, (size_t)cap));
  ix->out_cap = cap;
  return GT_OK;
}

struct Timer {
  Index* ix;
  hipStream_t s;
  hipEvent_t ev[8] = {};
  hipEvent_t evw[2 * GT_MAX_LEVELS] = {};
  int nw = 0;
  bool on;
  Timer(Index* i, hipStream_t st) : ix(i), s(st), on(i->profile) {
    if (on) {
      for (auto& e : ev) (void)hipEventCreate(&e);
      for (auto& e : evw) (void)hipEventCreate(&e);
    }
  }
  ~Timer() {
    if (on) {
      for (auto& e : ev) (void)hipEventDestroy(e);
      for (auto& e : evw) (void)hipEventDestroy(e);
    }
  }
  void mark(int k) {
    if (on) (void)hipEventRecord(ev[k], s);
  }
  // events bracketing each walk-level launch
  void launch_begin() {
    if (on && nw < GT_MAX_LEVELS) (void)hipEventRecord(evw[2 * nw], s);
  }
  void launch_end() {
    if (on && nw < GT_MAX_LEVELS) (void)hipEventRecord(evw[2 * nw + 1], s), ++nw;
  }
  float walk_ms() {
    float t = 0.0f;
    for (int i = 0; on && i < nw; ++i) {
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, evw[2 * i], evw[2 * i + 1]);
      t += ms;
    }
    return t;
  }
  float between(int a, int b) {
    float ms = 0.0f;
    if (on) (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return ms;
  }
};

// Validation shared by the two query entry points.
gt_status check_query_args(const Index* ix, const float* q, int nq, const double* rho,
                           int64_t max_results, int64_t* offsets, int64_t* ids, float* sims,
                           int64_t* total_out, int tq) {
  if (!ix) return fail(GT_ERR_INVALID_ARG, "index is NULL");
  if (!total_out) return fail(GT_ERR_INVALID_ARG, "total_out is NULL");
  if (nq < 0) return fail(GT_ERR_INVALID_ARG, "nq < 0");
  if ((int64_t)nq > (int64_t)gt::kMaxTiles * tq)
    return fail(GT_ERR_INVALID_ARG, "nq exceeds " + std::to_string(gt::kMaxTiles * tq) +
                                        " queries per call for this format");
  if (max_results < 0) return fail(GT_ERR_INVALID_ARG, "max_results < 0");
  if (nq > 0 && (!q || !rho || !offsets)) return fail(GT_ERR_INVALID_ARG, "NULL query argument");
  if (max_results > 0 && (!ids || !sims)) return fail(GT_ERR_INVALID_ARG, "NULL output buffer");
  for (int i = 0; i < nq; ++i)
    if (isnan(rho[i])) return fail(GT_ERR_INVALID_ARG, "rho is NaN");
  return GT_OK;
}

// Shared tail: recheck, offsets, one host synchronisation, overflow handling,
// scatter and sort.  `rerun` relaunches the candidate-producing stage after
// the hit buffer has grown.
template <class Rerun>
gt_status finish_query(Index* ix, int nq, int nq_pad, int64_t max_results, int64_t* offsets,
                       int64_t* ids, float* sims, int64_t* total_out, hipStream_t s, Timer& tm,
                       Rerun rerun, bool* cand_overflow = nullptr) {
  for (int attempt = 0;; ++attempt) {
    HIPCHK(gt::launch_recheck(ix->hits, ix->band_idx, &ix->ctr->nband,
                              (unsigned long long)ix->hit_cap, ix->qf, ix->leaves, ix->d, ix->dp,
                              ix->qq, ix->ff, ix->rho, ix->qcount, ix->ctr, s));
    tm.mark(4);
    HIPCHK(gt::launch_scan_offsets(ix->qcount, nq, ix->offs, offsets, ix->ctr, s));
    HIPCHK(hipMemcpyAsync(ix->h_ctr, ix->ctr, sizeof(gt::DevCounters), hipMemcpyDeviceToHost, s));
    tm.mark(5);
    HIPCHK(hipStreamSynchronize(s));
    const gt::DevCounters& c = *ix->h_ctr;
    if (c.err) return fail(GT_ERR_INVALID_INPUT, "query contains a NaN, infinite or negative value");
    if (cand_overflow && (int64_t)c.ncand > ix->cand_cap) {
      *cand_overflow = true;  // the caller regrows the candidate list and starts over
      return GT_OK;
    }
    if ((int64_t)c.nhits <= ix->hit_cap) break;
    if (attempt > 2) return fail(GT_ERR_DEVICE, "candidate buffer did not converge");
    TRY(grow_hits(ix, (int64_t)c.nhits));
    TRY(zero_dev(ix->qcount, (size_t)nq_pad * 4, s));
    TRY(zero_dev(&ix->ctr->nhits, 8, s));
    TRY(zero_dev(&ix->ctr->leaf_pairs, 8, s));
    TRY(zero_dev(&ix->ctr->rechecked, 8, s));
    TRY(zero_dev(&ix->ctr->nband, 8, s));
    TRY(rerun());
  }
  const int64_t total = (int64_t)ix->h_ctr->total;
  *total_out = total;
  if (total > max_results)
    return fail(GT_ERR_RESULT_OVERFLOW, "need max_results >= " + std::to_string(total));
  if (total > 0) {
    TRY(ensure_out(ix, total));
    TRY(zero_dev(ix->qcursor, (size_t)nq_pad * 4, s));
    HIPCHK(gt::launch_scatter(ix->hits, &ix->ctr->nhits, (unsigned long long)ix->hit_cap, ix->offs,
                              ix->qcursor, ix->out_id, ix->out_sim, s));
    HIPCHK(gt::launch_sort_segments(ix->offs, nq, ix->out_id, ix->out_sim, ix->tmp_id,
                                    ix->tmp_sim, ids, sims, s));
  }
  tm.mark(6);
  if (tm.on) {
    HIPCHK(hipStreamSynchronize(s));
    ix->ms[3] = tm.between(3, 4);
    ix->ms[4] = tm.between(4, 5) + tm.between(5, 6);
    ix->ms[6] = tm.between(0, 6);
  }
  return GT_OK;
}

}  // namespace

extern "C" {

const char* gt_last_error(void) { return g_err.c_str(); }

gt_status gt_build_tree(const void* feats_dev, int64_t n, int32_t d, gt_dtype dtype,
                        int64_t capacity, uint32_t pool_formats, void* stream, gt_index** out) {
  g_err.clear();
  if (!out) return fail(GT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > 4096) return fail(GT_ERR_INVALID_ARG, "d must be in [1, 4096]");
  if (n < 0) return fail(GT_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && !feats_dev) return fail(GT_ERR_INVALID_ARG, "feats_dev is NULL");
  if (dtype != GT_F32 && dtype != GT_F16 && dtype != GT_BF16)
    return fail(GT_ERR_INVALID_ARG, "unknown dtype");
  if (pool_formats & ~(uint32_t)(GT_POOL_F32 | GT_POOL_BF16 | GT_POOL_FP8E4M3))
    return fail(GT_ERR_INVALID_ARG, "unknown pool format bits");
  if (capacity == 0) {
    capacity = 2;
    while (capacity < n) capacity <<= 1;
  }
  if (capacity < 2 || (capacity & (capacity - 1)) || capacity < n)
    return fail(GT_ERR_INVALID_ARG, "capacity must be a power of two >= max(n, 2)");
  if (capacity > (int64_t(1) << 31)) return fail(GT_ERR_INVALID_ARG, "capacity above 2^31");

  hipStream_t s = (hipStream_t)stream;
  gt_index* ix = new gt_index();
  HIPCHK(hipGetDevice(&ix->device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, ix->device));
  ix->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  ix->d = d;
  ix->dp = (d + 127) / 128 * 128;
  ix->cap = capacity;
  ix->depth = 0;
  while ((int64_t(1) << ix->depth) < capacity) ++ix->depth;
  ix->dtype = dtype;
  ix->formats = pool_formats | GT_POOL_F32;

  auto bail = [&](gt_status st) {
    std::string keep = g_err;
    free_all(ix);
    delete ix;
    g_err = keep;
    return st;
  };
#define BTRY(expr)                 \
  do {                             \
    gt_status s_ = (expr);         \
    if (s_ != GT_OK) return bail(s_); \
  } while (0)
#define BHIP(expr)                                                                    \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return bail(fail(GT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)

  const size_t cap = (size_t)capacity, dp = (size_t)ix->dp, tree = (cap - 1) * dp;
  BTRY(dalloc(ix, &ix->leaves, cap * dp));
  BTRY(dalloc(ix, &ix->invn, cap));
  BTRY(dalloc(ix, &ix->ff, cap));
  BTRY(dalloc(ix, &ix->nf, cap));
  BTRY(dalloc(ix, &ix->d_mmin, 2));
  BTRY(dalloc(ix, &ix->master, tree));
  if (ix->formats & GT_POOL_BF16) BTRY(dalloc(ix, &ix->pbf16, tree));
  if (ix->formats & GT_POOL_FP8E4M3) BTRY(dalloc(ix, &ix->pfp8, tree));
  BTRY(dalloc(ix, &ix->d_lexp, GT_MAX_LEVELS));
  BTRY(dalloc(ix, &ix->d_levelmax, GT_MAX_LEVELS));
  BTRY(dalloc(ix, &ix->d_flags, GT_MAX_LEVELS));
  BHIP(hipMemsetAsync(ix->leaves, 0, cap * dp * 4, s));
  BHIP(hipMemsetAsync(ix->invn, 0, cap * 4, s));
  BHIP(hipMemsetAsync(ix->ff, 0, cap * 8, s));
  BHIP(hipMemsetAsync(ix->nf, 0, cap * 4, s));
  BHIP(hipMemsetAsync(ix->master, 0, tree * 4, s));
  BHIP(hipMemsetAsync(ix->d_flags, 0, GT_MAX_LEVELS * 4, s));
  BHIP(hipMemsetAsync(ix->d_lexp, 0, GT_MAX_LEVELS * 4, s));
  const double inf = INFINITY;
  BHIP(hipMemcpyAsync(ix->d_mmin, &inf, 8, hipMemcpyHostToDevice, s));
  unsigned int* derr = ix->d_flags + (GT_MAX_LEVELS - 1);
  BHIP(gt::launch_ingest(feats_dev, dtype, n, d, ix->dp, ix->leaves, ix->ff, ix->invn, ix->nf,
                         ix->d_mmin, derr, s));
  unsigned int herr = 0;
  BHIP(hipMemcpyAsync(&herr, derr, 4, hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  if (herr) return bail(fail(GT_ERR_INVALID_INPUT, "features contain a NaN, infinite or negative value"));
  ix->n = n;

  // pools, bottom-up; only pools covering some of the first n leaves are non-zero
  for (int l = ix->depth - 1; l >= 0; --l) {
    const float* child = (l == ix->depth - 1) ? ix->leaves : ix->master + level_row(l + 1) * dp;
    const int64_t span = int64_t(1) << (ix->depth - l);
    const int64_t nodes = (n + span - 1) / span;
    BHIP(gt::launch_build_level(child, ix->master + level_row(l) * dp, nodes, ix->dp, 0, s));
  }
  if (ix->pbf16) BHIP(gt::launch_quant_bf16(ix->master, ix->pbf16, (int64_t)tree, s));
  if (ix->pfp8) {
    BHIP(hipMemsetAsync(ix->d_levelmax, 0, GT_MAX_LEVELS * 4, s));
    for (int l = 0; l < ix->depth; ++l)
      BHIP(gt::launch_level_max(ix->master + level_row(l) * dp, int64_t(1) << l, ix->dp,
                                ix->d_levelmax + l, s));
    float mx[GT_MAX_LEVELS] = {0};
    BHIP(hipMemcpyAsync(mx, ix->d_levelmax, GT_MAX_LEVELS * 4, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    for (int l = 0; l < ix->depth; ++l) ix->lexp[l] = fp8_exp_for(mx[l]);
    BHIP(hipMemcpyAsync(ix->d_lexp, ix->lexp, GT_MAX_LEVELS * 4, hipMemcpyHostToDevice, s));
    for (int l = 0; l < ix->depth; ++l) BTRY(quantize_fp8_level(ix, l, s, false));
  }
  BHIP(hipMemcpyAsync(&ix->m_min, ix->d_mmin, 8, hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
#undef BTRY
#undef BHIP
  *out = ix;
  return GT_OK;
}

gt_status gt_insert(gt_index* ix, const void* feats_dev, int64_t n_new, void* stream,
                    int64_t* first_id_out) {
  g_err.clear();
  if (!ix) return fail(GT_ERR_INVALID_ARG, "index is NULL");
  if (n_new < 0) return fail(GT_ERR_INVALID_ARG, "n_new < 0");
  if (first_id_out) *first_id_out = ix->n;
  if (n_new == 0) return GT_OK;
  if (!feats_dev) return fail(GT_ERR_INVALID_ARG, "feats_dev is NULL");
  if (ix->n + n_new > ix->cap)
    return fail(GT_ERR_CAPACITY, "insert of " + std::to_string(n_new) + " rows exceeds capacity " +
                                     std::to_string(ix->cap));
  hipStream_t s = (hipStream_t)stream;
  const size_t dp = (size_t)ix->dp;
  const int64_t lo = ix->n, hi = ix->n + n_new;
  unsigned int* derr = ix->d_flags + (GT_MAX_LEVELS - 1);
  double* tmp_mmin = ix->d_mmin + 1;
  const double inf = INFINITY;
  HIPCHK(hipMemsetAsync(derr, 0, 4, s));
  HIPCHK(hipMemcpyAsync(tmp_mmin, &inf, 8, hipMemcpyHostToDevice, s));
  HIPCHK(gt::launch_ingest(feats_dev, ix->dtype, n_new, ix->d, ix->dp, ix->leaves + lo * dp,
                           ix->ff + lo, ix->invn + lo, ix->nf + lo, tmp_mmin, derr, s));
  unsigned int herr = 0;
  double mnew = inf;
  HIPCHK(hipMemcpyAsync(&herr, derr, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&mnew, tmp_mmin, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (herr) {
    // leave the unused leaf slots zero, as they were
    HIPCHK(hipMemsetAsync(ix->leaves + lo * dp, 0, (size_t)n_new * dp * 4, s));
    HIPCHK(hipMemsetAsync(ix->ff + lo, 0, (size_t)n_new * 8, s));
    HIPCHK(hipMemsetAsync(ix->invn + lo, 0, (size_t)n_new * 4, s));
    HIPCHK(hipMemsetAsync(ix->nf + lo, 0, (size_t)n_new * 4, s));
    HIPCHK(hipStreamSynchronize(s));
    return fail(GT_ERR_INVALID_INPUT, "inserted rows contain a NaN, infinite or negative value");
  }
  // pools on the root-to-leaf paths of the new rows, re-derived bottom-up
  for (int l = ix->depth - 1; l >= 0; --l) {
    const int sh = ix->depth - l;
    const int64_t a = lo >> sh, b = (hi - 1) >> sh;
    const float* child = (l == ix->depth - 1) ? ix->leaves : ix->master + level_row(l + 1) * dp;
    float* par = ix->master + level_row(l) * dp;
    HIPCHK(gt::launch_build_level(child, par, b - a + 1, ix->dp, a, s));
    if (ix->pbf16)
      HIPCHK(gt::launch_quant_bf16(par + a * dp, ix->pbf16 + (level_row(l) + a) * dp,
                                   (b - a + 1) * ix->dp, s));
    if (ix->pfp8)
      HIPCHK(gt::launch_quant_fp8(par + a * dp, ix->pfp8 + (level_row(l) + a) * dp,
                                  (b - a + 1) * ix->dp, ix->lexp[l], ix->d_flags + l, s));
  }
  if (ix->pfp8) {
    unsigned int fl[GT_MAX_LEVELS] = {0};
    HIPCHK(hipMemcpyAsync(fl, ix->d_flags, GT_MAX_LEVELS * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int l = 0; l < ix->depth; ++l)
      if (fl[l]) {  // a pool outgrew the level's float8 range: new scale for the level
        HIPCHK(hipMemsetAsync(ix->d_flags + l, 0, 4, s));
        TRY(quantize_fp8_level(ix, l, s, true));
      }
  }
  if (mnew < ix->m_min) {
    ix->m_min = mnew;
    HIPCHK(hipMemcpyAsync(ix->d_mmin, &ix->m_min, 8, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  ix->n = hi;
  ix->epoch++;
  return GT_OK;
}

gt_status gt_query_batch(gt_index* ix, const float* q_dev, int32_t nq, const double* rho_host,
                         gt_pool fmt, int64_t max_results, int64_t* offsets_dev, int64_t* ids_dev,
                         float* sims_dev, int64_t* total_out, void* stream) {
  g_err.clear();
  const int f = (int)fmt;
  if (f != GT_POOL_F32 && f != GT_POOL_BF16 && f != GT_POOL_FP8E4M3)
    return fail(GT_ERR_INVALID_ARG, "unknown pool format");
  const int tq = tq_of(f);
  TRY(check_query_args(ix, q_dev, nq, rho_host, max_results, offsets_dev, ids_dev, sims_dev,
                       total_out, tq));
  if (!(ix->formats & (uint32_t)f)) return fail(GT_ERR_INVALID_ARG, "pool format was not built");
  if (ix->dp > maxdp_of(f))
    return fail(GT_ERR_INVALID_ARG, "d too large for this pool format (padded d <= " +
                                        std::to_string(maxdp_of(f)) + ")");
  hipStream_t s = (hipStream_t)stream;
  *total_out = 0;
  const int nt = (nq + tq - 1) / tq;
  const int nq_pad = std::max(128, (nq + 127) / 128 * 128);
  TRY(ensure_query_buffers(ix, nq_pad, std::max(nt, 1)));
  if (nq == 0) {
    if (offsets_dev) TRY(zero_dev(offsets_dev, 8, s));
    return GT_OK;
  }
  Timer tm(ix, s);
  tm.mark(0);
  TRY(zero_dev(ix->ctr, sizeof(gt::DevCounters), s));
  TRY(zero_dev(ix->qcount, (size_t)nq_pad * 4, s));
  TRY(zero_dev(ix->tile_mask, (size_t)gt::kMaxTiles * 8, s));
  TRY(zero_dev(ix->lvl_count, (size_t)GT_MAX_LEVELS * gt::kMaxTiles * 4, s));
  if (ix->count_unique) {
    if (!ix->bitmap) TRY(dalloc(ix, &ix->bitmap, bitmap_words(ix)));
    TRY(zero_dev(ix->bitmap, bitmap_words(ix) * 4, s));
  }
  ix->counted = ix->count_unique;
  memcpy(ix->h_rho, rho_host, (size_t)nq * 8);
  HIPCHK(hipMemcpyAsync(ix->rho, ix->h_rho, (size_t)nq * 8, hipMemcpyHostToDevice, s));
  HIPCHK(gt::launch_query_prep(q_dev, nq, ix->d, ix->dp, tq, ix->rho, ix->d_mmin, ix->qf, ix->qbf,
                               ix->q8, ix->qexp, ix->invn_q, ix->qq, ix->thr, ix->thr_gemm,
                               ix->tile_mask, &ix->ctr->err, nq_pad, s));
  tm.mark(1);

  const int D = ix->depth, h = head_of(ix);
  const int grid = ix->grid > 0 ? ix->grid : ix->n_cu;
  const size_t dp = (size_t)ix->dp;
  const void* qtile = f == GT_POOL_F32 ? (const void*)ix->qf
                      : f == GT_POOL_BF16 ? (const void*)ix->qbf : (const void*)ix->q8;
  const size_t esz = f == GT_POOL_F32 ? 4 : f == GT_POOL_BF16 ? 2 : 1;
  const unsigned char* pool_base = f == GT_POOL_F32 ? (const unsigned char*)ix->master
                                   : f == GT_POOL_BF16 ? (const unsigned char*)ix->pbf16
                                                       : (const unsigned char*)ix->pfp8;
  ix->frontier_launches = 0;
  if (ix->n > 0) {
    for (int l = h; l <= D - 2; ++l) {
      gt::WalkLevelArgs a{};
      a.level = l;
      a.dense = (l == h);
      a.nt = nt;
      a.dp = ix->dp;
      a.cap = (int)ix->fr_cap;
      a.child_rows = pool_base + (size_t)level_row(l + 1) * dp * esz;
      a.in_node = ix->fr_node[l & 1];
      a.in_mask = ix->fr_mask[l & 1];
      a.in_count = ix->lvl_count + (size_t)l * gt::kMaxTiles;
      a.out_node = ix->fr_node[(l + 1) & 1];
      a.out_mask = ix->fr_mask[(l + 1) & 1];
      a.out_count = ix->lvl_count + (size_t)(l + 1) * gt::kMaxTiles;
      a.tile_mask = ix->tile_mask;
      a.qtile = qtile;
      a.thr = ix->thr;
      a.qexp = ix->qexp;
      a.lexp = ix->lexp[l + 1];
      a.stat_pairs = &ix->ctr->pairs[l + 1];
      a.bitmap = ix->count_unique ? ix->bitmap : nullptr;
      a.bit_base = level_row(l + 1);
      tm.launch_begin();
      HIPCHK(gt::launch_walk_level(f, a, grid, s));
      tm.launch_end();
      ix->frontier_launches++;
    }
  }
  tm.mark(2);
  gt::LeafArgs la{};
  la.level = D - 1;
  la.dense = (h == D - 1);
  la.nt = nt;
  la.dp = ix->dp;
  la.cap = (int)ix->fr_cap;
  la.tq = tq;
  la.in_node = ix->fr_node[(D - 1) & 1];
  la.in_mask = ix->fr_mask[(D - 1) & 1];
  la.in_count = ix->lvl_count + (size_t)(D - 1) * gt::kMaxTiles;
  la.tile_mask = ix->tile_mask;
  la.leaves = ix->leaves;
  la.invn_f = ix->invn;
  la.qf = ix->qf;
  la.invn_q = ix->invn_q;
  la.rho = ix->rho;
  la.n_epoch = ix->n;
  la.qcount = ix->qcount;
  la.ctr = ix->ctr;
  la.bitmap = ix->count_unique ? ix->bitmap : nullptr;
  la.bit_base = level_row(D);
  auto run_leaf = [&]() -> gt_status {
    la.hits = ix->hits;
    la.band_idx = ix->band_idx;
    la.hit_cap = (unsigned long long)ix->hit_cap;
    if (ix->n > 0) HIPCHK(gt::launch_leaf(la, ix->n_cu * 4, s));
    return GT_OK;
  };
  TRY(run_leaf());
  tm.mark(3);
  ix->last_nq = nq;
  ix->last_nt = nt;
  ix->last_fmt = f;
  ix->last_head = h;
  gt_status st = finish_query(ix, nq, nq_pad, max_results, offsets_dev, ids_dev, sims_dev,
                              total_out, s, tm, run_leaf);
  if (tm.on) {
    ix->ms[0] = tm.between(0, 1);
    ix->ms[1] = tm.walk_ms();
    ix->ms[2] = tm.between(2, 3);
    ix->ms[5] = 0.0;
  }
  return st;
}

gt_status gt_exhaustive(gt_index* ix, const float* q_dev, int32_t nq, const double* rho_host,
                        int64_t max_results, int64_t* offsets_dev, int64_t* ids_dev,
                        float* sims_dev, int64_t* total_out, void* stream) {
  g_err.clear();
  TRY(check_query_args(ix, q_dev, nq, rho_host, max_results, offsets_dev, ids_dev, sims_dev,
                       total_out, gt::kQueriesPerTile16));
  hipStream_t s = (hipStream_t)stream;
  *total_out = 0;
  const int tq = gt::kQueriesPerTile16;
  const int nt = (nq + tq - 1) / tq;
  const int nq_pad = std::max(128, (nq + 127) / 128 * 128);
  TRY(ensure_query_buffers(ix, nq_pad, std::max(nt, 1)));
  if (!ix->cand) {
    ix->cand_cap = int64_t(1) << 20;
    TRY(dalloc(ix, &ix->cand, (size_t)ix->cand_cap));
  }
  if (nq == 0) {
    if (offsets_dev) TRY(zero_dev(offsets_dev, 8, s));
    return GT_OK;
  }
  Timer tm(ix, s);
  tm.mark(0);
  TRY(zero_dev(ix->ctr, sizeof(gt::DevCounters), s));
  TRY(zero_dev(ix->qcount, (size_t)nq_pad * 4, s));
  TRY(zero_dev(ix->tile_mask, (size_t)gt::kMaxTiles * 8, s));
  memcpy(ix->h_rho, rho_host, (size_t)nq * 8);
  HIPCHK(hipMemcpyAsync(ix->rho, ix->h_rho, (size_t)nq * 8, hipMemcpyHostToDevice, s));
  HIPCHK(gt::launch_query_prep(q_dev, nq, ix->d, ix->dp, tq, ix->rho, ix->d_mmin, ix->qf, ix->qbf,
                               ix->q8, ix->qexp, ix->invn_q, ix->qq, ix->thr, ix->thr_gemm,
                               ix->tile_mask, &ix->ctr->err, nq_pad, s));
  tm.mark(1);
  auto run_gemm_and_check = [&]() -> gt_status {
    HIPCHK(gt::launch_exhaustive_gemm(ix->qf, nq_pad, ix->leaves, ix->n, ix->dp, ix->thr_gemm,
                                      ix->nf, ix->cand, (unsigned long long)ix->cand_cap, ix->ctr,
                                      nq, s));
    tm.mark(2);
    HIPCHK(gt::launch_pair_check(ix->cand, &ix->ctr->ncand, (unsigned long long)ix->cand_cap,
                                 ix->qf, ix->leaves, ix->invn_q, ix->invn, ix->rho, ix->dp,
                                 ix->hits, (unsigned long long)ix->hit_cap, ix->band_idx,
                                 ix->qcount, ix->ctr, ix->n_cu * 4, s));
    tm.mark(3);
    return GT_OK;
  };
  TRY(run_gemm_and_check());
  ix->last_nq = nq;
  ix->last_nt = nt;
  ix->last_fmt = 0;
  ix->frontier_launches = 0;
  for (int attempt = 0;; ++attempt) {
    bool cand_over = false;
    gt_status st = finish_query(ix, nq, nq_pad, max_results, offsets_dev, ids_dev, sims_dev,
                                total_out, s, tm, [&]() -> gt_status {
                                  TRY(zero_dev(&ix->ctr->ncand, 8, s));
                                  return run_gemm_and_check();
                                }, &cand_over);
    if (st != GT_OK) return st;
    if (!cand_over) break;
    // the candidate list overflowed: grow it and redo the whole pass
    if (attempt > 2) return fail(GT_ERR_DEVICE, "candidate list did not converge");
    const int64_t need = (int64_t)ix->h_ctr->ncand;
    dfree(ix, &ix->cand, (size_t)ix->cand_cap);
    ix->cand_cap = 0;
    TRY(dalloc(ix, &ix->cand, (size_t)(need + need / 4 + 1024)));
    ix->cand_cap = need + need / 4 + 1024;
    TRY(zero_dev(ix->ctr, sizeof(gt::DevCounters), s));
    TRY(zero_dev(ix->qcount, (size_t)nq_pad * 4, s));
    HIPCHK(gt::launch_query_prep(q_dev, nq, ix->d, ix->dp, tq, ix->rho, ix->d_mmin, ix->qf, ix->qbf,
                                 ix->q8, ix->qexp, ix->invn_q, ix->qq, ix->thr, ix->thr_gemm,
                                 ix->tile_mask, &ix->ctr->err, nq_pad, s));
    TRY(run_gemm_and_check());
  }
  if (tm.on) {
    ix->ms[0] = tm.between(0, 1);
    ix->ms[5] = tm.between(1, 2);
    ix->ms[2] = tm.between(2, 3);
    ix->ms[1] = 0.0;
  }
  return GT_OK;
}

gt_status gt_get_stats(const gt_index* ix, gt_stats* out) {
  g_err.clear();
  if (!ix || !out) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  memset(out, 0, sizeof(*out));
  out->n = ix->n;
  out->capacity = ix->cap;
  out->d = ix->d;
  out->d_pad = ix->dp;
  out->depth = ix->depth;
  out->head_level = head_of(ix);
  out->pool_formats = ix->formats;
  out->m_min = ix->m_min;
  out->epoch = ix->epoch;
  out->bytes_device = ix->bytes;
  out->last_nq = ix->last_nq;
  out->last_tiles = ix->last_nt;
  out->last_format = ix->last_fmt;
  if (ix->ctr && ix->last_nt > 0) {
    HIPCHK(hipDeviceSynchronize());
    std::vector<uint32_t> cnt((size_t)GT_MAX_LEVELS * gt::kMaxTiles);
    HIPCHK(hipMemcpy(cnt.data(), ix->lvl_count, cnt.size() * 4, hipMemcpyDeviceToHost));
    gt::DevCounters c;
    HIPCHK(hipMemcpy(&c, ix->ctr, sizeof(c), hipMemcpyDeviceToHost));
    for (int l = 0; l < ix->depth && l < GT_MAX_LEVELS; ++l) {
      int64_t e = 0;
      for (int t = 0; t < ix->last_nt; ++t) e += cnt[(size_t)l * gt::kMaxTiles + t];
      out->entries[l] = e;
      out->pairs[l] = (int64_t)c.pairs[l];
    }
    out->leaf_pairs = (int64_t)c.leaf_pairs;
    out->candidates = (int64_t)c.nhits;
    out->rechecked = (int64_t)c.rechecked;
    out->results = (int64_t)c.total;
  }
  out->ms_prep = ix->ms[0];
  out->ms_frontier = ix->ms[1];
  out->ms_leaf = ix->ms[2];
  out->ms_recheck = ix->ms[3];
  out->ms_compact = ix->ms[4];
  out->ms_gemm = ix->ms[5];
  out->ms_total = ix->ms[6];
  out->frontier_launches = ix->frontier_launches;
  for (int l = 0; l < GT_MAX_LEVELS; ++l) out->fp8_exp[l] = ix->lexp[l];
  if (ix->counted && ix->bitmap) {
    std::vector<uint32_t> bm(bitmap_words(ix));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(bm.data(), ix->bitmap, bm.size() * 4, hipMemcpyDeviceToHost));
    for (int l = 0; l <= ix->depth && l < GT_MAX_LEVELS; ++l) {
      int64_t c = 0;
      for (int64_t r = level_row(l); r < level_row(l + 1); ++r) c += (bm[r >> 5] >> (r & 31)) & 1u;
      out->unique_rows[l] = c;
    }
  }
  return GT_OK;
}

gt_status gt_read_pools(const gt_index* ix, int32_t level, int64_t first, int64_t count,
                        gt_pool fmt, void* host_out) {
  g_err.clear();
  if (!ix || !host_out) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  if (level < 0 || level > ix->depth) return fail(GT_ERR_INVALID_ARG, "level out of range");
  const int64_t rows = int64_t(1) << level;
  if (first < 0 || count < 0 || first + count > rows)
    return fail(GT_ERR_INVALID_ARG, "row range out of the level");
  const int f = (int)fmt;
  if (!(ix->formats & (uint32_t)f) || (level == ix->depth && f != GT_POOL_F32))
    return fail(GT_ERR_INVALID_ARG, "format not available for this level");
  const size_t esz = f == GT_POOL_F32 ? 4 : f == GT_POOL_BF16 ? 2 : 1;
  const unsigned char* base =
      level == ix->depth ? (const unsigned char*)ix->leaves
      : f == GT_POOL_F32 ? (const unsigned char*)(ix->master + level_row(level) * ix->dp)
      : f == GT_POOL_BF16 ? (const unsigned char*)(ix->pbf16 + level_row(level) * ix->dp)
                          : (const unsigned char*)(ix->pfp8 + level_row(level) * ix->dp);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(host_out, base + (size_t)first * ix->dp * esz, (size_t)count * ix->dp * esz,
                   hipMemcpyDeviceToHost));
  return GT_OK;
}

gt_status gt_set_option(gt_index* ix, const char* key, int64_t value) {
  g_err.clear();
  if (!ix || !key) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  if (!strcmp(key, "profile")) {
    ix->profile = value != 0;
  } else if (!strcmp(key, "head_level")) {
    if (value < -1 || value > ix->depth - 1) return fail(GT_ERR_INVALID_ARG, "head_level out of range");
    ix->head_level = (int)value;
  } else if (!strcmp(key, "count_unique")) {
    ix->count_unique = value != 0;
  } else if (!strcmp(key, "grid")) {
    if (value < 0 || value > 65536) return fail(GT_ERR_INVALID_ARG, "grid out of range");
    ix->grid = (int)value;
  } else {
    return fail(GT_ERR_INVALID_ARG, std::string("unknown option ") + key);
  }
  return GT_OK;
}

void gt_destroy(gt_index* ix) {
  if (!ix) return;
  (void)hipDeviceSynchronize();
  free_all(ix);
  delete ix;
}

}  // extern "C"
