// Host runtime behind the C interface of gt.h: the index object, per-call
// device workspaces, and the launch sequence of each call.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "gt.h"
#include "gt_internal.h"

using gt::Batch;
using gt::Index;

struct gt_index : Index {};
struct gt_batch : Batch {};

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

#define TRY(expr)                  \
  do {                             \
    gt_status s_ = (expr);         \
    if (s_ != GT_OK) return s_;    \
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

inline int64_t level_row(int level) { return (int64_t(1) << level) - 1; }

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

// Last level walked with dense steps (every pool against every query).  Near
// the root nearly every pool is live for every query tile, so a dense matrix
// product reads each pool row once per workgroup column instead of once per
// tile; a few levels above the leaves the frontier is sparse enough that the
// per-tile walk reads less.  Float32 pools stay on the sparse walk (float32
// matrix cores are 16x slower than bfloat16 ones).
int dense_last_of(const Index* ix, int fmt, int h) {
  if (fmt == GT_POOL_F32 || ix->dense_last == -1) return -1;
  // automatic: a level given by the caller (a cost model's choice), else
  // the level whose pools hold about 16 of the populated rows
  int lg = 0;
  while ((int64_t(1) << lg) < ix->n) ++lg;
  int dl = ix->dense_last >= 0 ? ix->dense_last : ix->dense_start >= 0 ? ix->dense_start : lg - 4;
  dl = std::min(dl, ix->depth - 1);
  return dl > h ? dl : -1;
}

// Automatic dense level, per workspace, from its last walk (same format): a
// dense step at level L + 1 costs in proportion to its pools x tiles x d_pad,
// a sparse step in proportion to the entries of level L.  Measured on this
// chip (d_pad 512 and 1024), the dense step is the cheaper one while the
// entries of level L fill more than 4.6e-4 d_pad of level L's populated
// (pool, tile) pairs.  The last call counted the entries of every level from
// its own dense level down, so the level moves down while that holds; it
// moves up one level when the density at the last dense level is below half
// the threshold (the level above has about twice the density: its pools are
// half as many and the entries about as many).  Only for rows of 512
// columns or more, where the costs were measured.  Results never depend on it.
int adapt_dense_last(const Index* ix, const Batch* b, int fmt, bool maxp, int dl, int h) {
  const int width = maxp ? ix->pw : ix->dp;
  if (ix->dense_last != -2 || dl < 0 || width < 512 || !b->have_last || b->last_dl < 0 ||
      b->last_walk_fmt != fmt || b->last_maxpool != maxp || b->last_walk_nt <= 0)
    return dl;
  const int D = ix->depth;
  const double thr = 4.6e-4 * width;
  auto density = [&](int L) {
    const int64_t span = int64_t(1) << (D - L);
    const int64_t pop =
        std::min<int64_t>(int64_t(1) << L, (b->last_n_epoch + span - 1) / span);
    return pop > 0 ? (double)b->last_entries[L] / ((double)pop * b->last_walk_nt) : 0.0;
  };
  int L = std::min(b->last_dl, D - 1);
  while (L + 1 <= D - 1 && density(L) > thr) ++L;
  if (L == b->last_dl && L - 1 > h && density(L) < 0.5 * thr) --L;
  return L > h ? L : dl;
}

// Bucket bits of a call's sparse frontier: subtrees of level nb, at most
// 2^7 of them and at most kMaxSlots (bucket, tile) slots, never deeper than
// the level where the sparse frontier starts.
int bucket_bits_of(int sparse_from, int nt) {
  int nb = std::min(gt::kMaxBucketBits, std::max(0, sparse_from));
  while (nb > 0 && ((int64_t)nt << nb) > gt::kMaxSlots) --nb;
  return nb;
}

int tq_of(int fmt) { return fmt == GT_POOL_F32 ? gt::kQueriesPerTileF32 : gt::kQueriesPerTile16; }

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

// ------------------------------------------------------------------ workspaces
void free_query_arrays(Batch* b) {
  Index* ix = b->ix;
  const size_t o = (size_t)b->nq_alloc, dp = (size_t)ix->dp, pw = (size_t)ix->pw;
  dfree(ix, &b->qf, o * dp);
  dfree(ix, &b->qw, o * pw);
  dfree(ix, &b->qbf, o * pw);
  dfree(ix, &b->q8, o * dp);
  dfree(ix, &b->qexp, o);
  dfree(ix, &b->invn_q, o);
  dfree(ix, &b->qq, o);
  dfree(ix, &b->rho, o);
  dfree(ix, &b->thr, o);
  dfree(ix, &b->thr_gemm, o);
  dfree(ix, &b->sabs, o);
  dfree(ix, &b->qcount, o);
  dfree(ix, &b->offs, o + 1);
  if (b->h_rho) (void)hipHostFree(b->h_rho);
  b->h_rho = nullptr;
  b->nq_alloc = 0;
}

void free_frontier(Batch* b) {
  for (int k = 0; k < 2; ++k) {
    dfree(b->ix, &b->fr_node[k], (size_t)b->nt_alloc * b->fr_cap);
    dfree(b->ix, &b->fr_mask[k], (size_t)b->nt_alloc * b->fr_cap);
    dfree(b->ix, &b->fr_rec[k], (size_t)b->rec_len * 64);
  }
  b->nt_alloc = 0;
  b->rec_len = 0;
}

void free_batch(Batch* b) {
  if (!b) return;
  Index* ix = b->ix;
  if (b->external) {
    // device buffers were the caller's: only the host-side resources
    if (b->h_ctr) (void)hipHostFree(b->h_ctr);
    b->h_ctr = nullptr;
    if (b->done) (void)hipEventDestroy(b->done);
    b->done = nullptr;
    return;
  }
  free_query_arrays(b);
  free_frontier(b);
  dfree(ix, &b->lvl_count, (size_t)GT_MAX_LEVELS * gt::kMaxSlots);
  dfree(ix, &b->tile_mask, gt::kMaxTiles);
  dfree(ix, &b->hits, (size_t)b->hit_cap);
  dfree(ix, &b->band_idx, (size_t)b->hit_cap);
  dfree(ix, &b->cand, (size_t)b->cand_cap);
  dfree(ix, &b->out_id, (size_t)b->out_cap);
  dfree(ix, &b->out_sim, (size_t)b->out_cap);
  dfree(ix, &b->tmp_id, (size_t)b->out_cap);
  dfree(ix, &b->tmp_sim, (size_t)b->out_cap);
  dfree(ix, &b->fin_id, (size_t)b->out_cap);
  dfree(ix, &b->fin_sim, (size_t)b->out_cap);
  dfree(ix, &b->dmask[0], (size_t)b->dmask_len);
  dfree(ix, &b->dmask[1], (size_t)b->dmask_len);
  dfree(ix, &b->bitmap, (size_t)b->bitmap_words);
  dfree(ix, &b->ctr, 1);
  if (b->h_ctr) (void)hipHostFree(b->h_ctr);
  b->h_ctr = nullptr;
  if (b->done) (void)hipEventDestroy(b->done);
  b->done = nullptr;
  if (b->events) {
    for (auto& e : b->ev) (void)hipEventDestroy(e);
    for (auto& e : b->evw) (void)hipEventDestroy(e);
    b->events = false;
  }
}

void free_tree(Index* ix) {
  const size_t cap = (size_t)ix->cap, dp = (size_t)ix->dp, tree = (cap - 1) * dp;
  dfree(ix, &ix->leaves, cap * dp);
  dfree(ix, &ix->invn, cap);
  dfree(ix, &ix->ff, cap);
  dfree(ix, &ix->nf, cap);
  dfree(ix, &ix->d_mmin, 2);
  dfree(ix, &ix->master, tree);
  dfree(ix, &ix->pbf16, tree);
  dfree(ix, &ix->pfp8, tree);
  const size_t mtree = (cap - 1) * (size_t)ix->pw;
  dfree(ix, &ix->mmax, mtree);
  dfree(ix, &ix->pmax16, mtree);
  dfree(ix, &ix->d_absmax, 1);
  dfree(ix, &ix->d_lexp, GT_MAX_LEVELS);
  dfree(ix, &ix->d_levelmax, GT_MAX_LEVELS);
  dfree(ix, &ix->d_flags, GT_MAX_LEVELS);
}

gt_status batch_init(Batch* b) {
  Index* ix = b->ix;
  TRY(dalloc(ix, &b->ctr, 1));
  HIPCHK(hipHostMalloc((void**)&b->h_ctr, sizeof(gt::DevCounters), hipHostMallocDefault));
  TRY(dalloc(ix, &b->lvl_count, (size_t)GT_MAX_LEVELS * gt::kMaxSlots));
  TRY(dalloc(ix, &b->tile_mask, gt::kMaxTiles));
  b->hit_cap = int64_t(1) << 20;
  TRY(dalloc(ix, &b->hits, (size_t)b->hit_cap));
  TRY(dalloc(ix, &b->band_idx, (size_t)b->hit_cap));
  HIPCHK(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
  return GT_OK;
}

// Query arrays for nq_pad queries and frontiers for nt tiles.
gt_status batch_reserve(Batch* b, int nq_pad, int nt) {
  Index* ix = b->ix;
  const size_t dp = (size_t)ix->dp;
  if (b->fixed) {
    if (nq_pad > b->nq_alloc || nt > b->nt_alloc || b->fr_cap < 1)
      return fail(GT_ERR_CAPACITY, "the call does not fit the buffers carved for it");
    return GT_OK;
  }
  if (nq_pad > b->nq_alloc) {
    free_query_arrays(b);
    const size_t nqa = (size_t)nq_pad;
    TRY(dalloc(ix, &b->qf, nqa * dp));
    if (ix->signed_mode) TRY(dalloc(ix, &b->qw, nqa * (size_t)ix->pw));
    TRY(dalloc(ix, &b->qbf, nqa * (size_t)ix->pw));
    TRY(dalloc(ix, &b->q8, nqa * dp));
    TRY(dalloc(ix, &b->qexp, nqa));
    TRY(dalloc(ix, &b->invn_q, nqa));
    TRY(dalloc(ix, &b->qq, nqa));
    TRY(dalloc(ix, &b->rho, nqa));
    TRY(dalloc(ix, &b->thr, nqa));
    TRY(dalloc(ix, &b->thr_gemm, nqa));
    TRY(dalloc(ix, &b->sabs, nqa));
    TRY(dalloc(ix, &b->qcount, nqa));
    TRY(dalloc(ix, &b->offs, nqa + 1));
    HIPCHK(hipHostMalloc((void**)&b->h_rho, nqa * sizeof(double), hipHostMallocDefault));
    b->nq_alloc = nq_pad;
  }
  const int64_t fr_cap = int64_t(1) << std::max(0, ix->depth - 1);
  if (nt > b->nt_alloc || fr_cap != b->fr_cap) {
    free_frontier(b);
    for (int k = 0; k < 2; ++k) {
      TRY(dalloc(ix, &b->fr_node[k], (size_t)nt * fr_cap));
      TRY(dalloc(ix, &b->fr_mask[k], (size_t)nt * fr_cap));
    }
    b->nt_alloc = nt;
    b->fr_cap = fr_cap;
  }
  return GT_OK;
}

gt_status grow_hits(Batch* b, int64_t need) {
  Index* ix = b->ix;
  if (b->fixed) {
    b->hits_overflowed = true;
    return fail(GT_ERR_CAPACITY, "the call's " + std::to_string(need) +
                                     " leaf candidates exceed the fixed scratch (room for " +
                                     std::to_string(b->hit_cap) + "); use fewer queries per call");
  }
  dfree(ix, &b->hits, (size_t)b->hit_cap);
  dfree(ix, &b->band_idx, (size_t)b->hit_cap);
  b->hit_cap = 0;
  const int64_t cap = need + need / 4 + 1024;
  if (cap >= (int64_t(1) << 32)) return fail(GT_ERR_OUT_OF_MEMORY, "more than 2^32 candidates");
  TRY(dalloc(ix, &b->hits, (size_t)cap));
  TRY(dalloc(ix, &b->band_idx, (size_t)cap));
  b->hit_cap = cap;
  return GT_OK;
}

gt_status ensure_out(Batch* b, int64_t need) {
  if (need <= b->out_cap && b->out_id) return GT_OK;
  if (b->fixed)
    return fail(GT_ERR_CAPACITY, "the call's " + std::to_string(need) +
                                     " results exceed the fixed scratch (room for " +
                                     std::to_string(b->out_cap) + "); use fewer queries per call");
  Index* ix = b->ix;
  const size_t o = (size_t)b->out_cap;
  dfree(ix, &b->out_id, o);
  dfree(ix, &b->out_sim, o);
  dfree(ix, &b->tmp_id, o);
  dfree(ix, &b->tmp_sim, o);
  dfree(ix, &b->fin_id, o);
  dfree(ix, &b->fin_sim, o);
  b->out_cap = 0;
  const int64_t cap = std::max<int64_t>(need + need / 4, int64_t(1) << 16);
  TRY(dalloc(ix, &b->out_id, (size_t)cap));
  TRY(dalloc(ix, &b->out_sim, (size_t)cap));
  TRY(dalloc(ix, &b->tmp_id, (size_t)cap));
  TRY(dalloc(ix, &b->tmp_sim, (size_t)cap));
  TRY(dalloc(ix, &b->fin_id, (size_t)cap));
  TRY(dalloc(ix, &b->fin_sim, (size_t)cap));
  b->out_cap = cap;
  return GT_OK;
}

// --------------------------------------------------------------- event timing
void ev_mark(Batch* b, int k) {
  if (b->profile) (void)hipEventRecord(b->ev[k], b->stream);
}
void ev_launch_begin(Batch* b) {
  if (b->profile && b->nw < GT_MAX_LEVELS) (void)hipEventRecord(b->evw[2 * b->nw], b->stream);
}
void ev_launch_end(Batch* b, bool dense) {
  if (b->profile && b->nw < GT_MAX_LEVELS) {
    (void)hipEventRecord(b->evw[2 * b->nw + 1], b->stream);
    b->evw_dense[b->nw] = dense;
    ++b->nw;
  }
}
float ev_between(Batch* b, int x, int y) {
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, b->ev[x], b->ev[y]);
  return ms;
}
float ev_walk(Batch* b, bool dense) {
  float t = 0.0f;
  for (int i = 0; i < b->nw; ++i) {
    if (b->evw_dense[i] != dense) continue;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, b->evw[2 * i], b->evw[2 * i + 1]);
    t += ms;
  }
  return t;
}

// ------------------------------------------------------------- launch stages
gt_status enqueue_walk(Index* ix, Batch* b) {
  hipStream_t s = b->stream;
  const int f = b->fmt, nt = b->nt, D = ix->depth, h = b->head, dl = b->dense_last;
  const int grid = ix->grid > 0 ? ix->grid : ix->n_cu;
  // pool row length: d_pad, or 2 d_pad for the shifted max/min rows of a
  // signed index, whose walk queries are [max(q,0) | max(-q,0)]
  const size_t dp = (size_t)(b->maxpool ? ix->pw : ix->dp);
  const void* qtile = f == GT_POOL_F32 ? (const void*)(ix->signed_mode ? b->qw : b->qf)
                      : f == GT_POOL_BF16 ? (const void*)b->qbf : (const void*)b->q8;
  const size_t esz = f == GT_POOL_F32 ? 4 : f == GT_POOL_BF16 ? 2 : 1;
  const unsigned char* pool_base =
      b->maxpool ? (f == GT_POOL_F32 ? (const unsigned char*)ix->mmax
                                     : (const unsigned char*)ix->pmax16)
      : f == GT_POOL_F32  ? (const unsigned char*)ix->master
      : f == GT_POOL_BF16 ? (const unsigned char*)ix->pbf16
                          : (const unsigned char*)ix->pfp8;
  uint32_t* bitmap = b->counted ? b->bitmap : nullptr;
  b->frontier_launches = 0;
  b->dense_launches = 0;
  // Subtraction step (bfloat16 pools, score records from a dense step):
  // sparse levels sub_from .. sub_to read only the right children.
  const int ws = ix->walk_subtract < 0 ? 1 : ix->walk_subtract;
  // (sum pools only: a max pool is not its halves' combination)
  // (and rows whose whole query tile fits in LDS)
  bool sub = f == GT_POOL_BF16 && !b->maxpool && dl >= 0 && ws > 0 && dl <= D - 2 &&
             (int)dp <= gt::kMaxDpBf16;
  int sub_to = !sub ? -1 : (ws == 2 ? D - 3 : D - 2);
  // A workspace with a query limit takes its score records and dense masks
  // for its largest call at once: growing them call by call would free and
  // reallocate (gigabytes, for the records), and every free waits for the
  // whole device.
  const int nt_res = b->max_queries > 0
                         ? std::max(nt, (b->max_queries + gt::kQueriesPerTile16 - 1) /
                                            gt::kQueriesPerTile16)
                         : nt;
  if (sub && sub_to >= dl && b->fixed && (int64_t)nt_res * b->fr_cap > b->rec_len) {
    // no room for score records in the fixed buffers: direct tests (same
    // results, both children read)
    sub = false;
    sub_to = -1;
  }
  if (sub && sub_to >= dl) {
    const int64_t need = (int64_t)nt_res * b->fr_cap;
    if (need > b->rec_len) {
      dfree(ix, &b->fr_rec[0], (size_t)b->rec_len * 64);
      dfree(ix, &b->fr_rec[1], (size_t)b->rec_len * 64);
      b->rec_len = 0;
      TRY(dalloc(ix, &b->fr_rec[0], (size_t)need * 64));
      TRY(dalloc(ix, &b->fr_rec[1], (size_t)need * 64));
      b->rec_len = need;
    }
  }
  const bool use_rec = sub && sub_to >= dl;
  if (dl >= 0) {
    // per-(pool, tile) masks only pass between chained dense steps (an
    // explicit head more than one level above the last dense level)
    const size_t need = h + 1 < dl ? ((size_t)1 << std::max(0, dl - 1)) * (size_t)nt_res : 0;
    if ((int64_t)need > b->dmask_len && b->fixed)
      return fail(GT_ERR_CAPACITY, "chained dense steps need dense masks the fixed buffers lack");
    if ((int64_t)need > b->dmask_len) {
      dfree(ix, &b->dmask[0], (size_t)b->dmask_len);
      dfree(ix, &b->dmask[1], (size_t)b->dmask_len);
      b->dmask_len = 0;
      TRY(dalloc(ix, &b->dmask[0], need));
      TRY(dalloc(ix, &b->dmask[1], need));
      b->dmask_len = (int64_t)need;
    }
    for (int L = h + 1; L <= dl; ++L) {
      gt::DenseLevelArgs a{};
      a.level = L;
      // pools beyond the last one holding a row below the epoch are all zero
      // and can hold no result: they are not tested
      a.rows = std::max<int64_t>(1, std::min<int64_t>(int64_t(1) << L,
                                                     (b->n_epoch + (int64_t(1) << (D - L)) - 1) >> (D - L)));
      a.nt = nt;
      a.dp = (int)dp;
      a.nb = b->nb;
      a.bcap = b->fr_cap >> b->nb;
      a.child_rows = pool_base + (size_t)level_row(L) * dp * esz;
      a.qtile = qtile;
      a.thr = b->thr;
      a.qexp = b->qexp;
      a.lexp = ix->lexp[L];
      a.parent = L == h + 1 ? nullptr : b->dmask[(L - 1) & 1];
      a.tile_mask = b->tile_mask;
      a.out_dense = L < dl ? b->dmask[L & 1] : nullptr;
      a.out_node = b->fr_node[L & 1];
      a.out_mask = b->fr_mask[L & 1];
      a.out_count = b->lvl_count + (size_t)L * gt::kMaxSlots;
      a.stat_pairs = &b->ctr->pairs[L];
      a.bitmap = bitmap;
      a.bit_base = level_row(L);
      a.out_rec = (use_rec && L == dl) ? b->fr_rec[L & 1] : nullptr;
      a.over = &b->ctr->fr_over;
      ev_launch_begin(b);
      HIPCHK(gt::launch_dense_level(f, a, s));
      ev_launch_end(b, true);
      b->dense_launches++;
    }
  }
  const int sparse_from = dl >= 0 ? dl : h;
  for (int l = sparse_from; l <= D - 2; ++l) {
    gt::WalkLevelArgs a{};
    a.level = l;
    a.dense = (l == h);
    a.nt = nt;
    a.dp = (int)dp;
    a.nb = b->nb;
    a.bcap = b->fr_cap >> b->nb;
    a.child_rows = pool_base + (size_t)level_row(l + 1) * dp * esz;
    a.in_node = b->fr_node[l & 1];
    a.in_mask = b->fr_mask[l & 1];
    a.in_count = b->lvl_count + (size_t)l * gt::kMaxSlots;
    a.out_node = b->fr_node[(l + 1) & 1];
    a.out_mask = b->fr_mask[(l + 1) & 1];
    a.out_count = b->lvl_count + (size_t)(l + 1) * gt::kMaxSlots;
    a.tile_mask = b->tile_mask;
    a.qtile = qtile;
    a.thr = b->thr;
    a.qexp = b->qexp;
    a.lexp = ix->lexp[l + 1];
    a.stat_pairs = &b->ctr->pairs[l + 1];
    a.bitmap = bitmap;
    a.bit_base = level_row(l + 1);
    a.over = &b->ctr->fr_over;
    ev_launch_begin(b);
    if (use_rec && l <= sub_to) {
      a.in_rec = b->fr_rec[l & 1];
      a.out_rec = l + 1 <= sub_to ? b->fr_rec[(l + 1) & 1] : nullptr;
      a.sabs = b->sabs;
      a.n_epoch = b->n_epoch;
      a.depth = D;
      HIPCHK(gt::launch_walk_sub(a, grid, s));
    } else {
      HIPCHK(gt::launch_walk_level(f, a, grid, s));
    }
    ev_launch_end(b, false);
    b->frontier_launches++;
  }
  return GT_OK;
}

gt_status enqueue_leaf(Index* ix, Batch* b) {
  const int D = ix->depth;
  const int sparse_from = b->dense_last >= 0 ? b->dense_last : b->head;
  gt::LeafArgs la{};
  la.level = D - 1;
  la.dense = (sparse_from == D - 1) && b->dense_last < 0;
  la.nt = b->nt;
  la.dp = ix->dp;
  la.nb = b->nb;
  la.bcap = b->fr_cap >> b->nb;
  la.tq = b->tq;
  la.in_node = b->fr_node[(D - 1) & 1];
  la.in_mask = b->fr_mask[(D - 1) & 1];
  la.in_count = b->lvl_count + (size_t)(D - 1) * gt::kMaxSlots;
  la.tile_mask = b->tile_mask;
  la.leaves = ix->leaves;
  la.invn_f = ix->invn;
  la.qf = b->qf;
  la.invn_q = b->invn_q;
  la.rho = b->rho;
  la.n_epoch = b->n_epoch;
  la.hits = b->hits;
  la.band_idx = b->band_idx;
  la.hit_cap = (unsigned long long)b->hit_cap;
  la.qcount = b->qcount;
  la.ctr = b->ctr;
  la.bitmap = b->counted ? b->bitmap : nullptr;
  la.bit_base = level_row(D);
  // two workgroups (eight waves) per CU: measured faster than one, three,
  // four or eight per CU on this kernel, whose loads already fill the CU's
  // outstanding-request budget
  HIPCHK(gt::launch_leaf(la, ix->n_cu * 2, b->stream));
  return GT_OK;
}

gt_status enqueue_exhaustive(Index* ix, Batch* b) {
  if (!b->cand) {
    b->cand_cap = int64_t(1) << 20;
    TRY(dalloc(ix, &b->cand, (size_t)b->cand_cap));
  }
  ev_launch_begin(b);
  HIPCHK(gt::launch_exhaustive_gemm(b->qf, b->nq_pad, ix->leaves, b->n_epoch, ix->dp, b->thr_gemm,
                                    ix->nf, b->cand, (unsigned long long)b->cand_cap, b->ctr,
                                    b->nq, b->stream));
  ev_launch_end(b, true);
  return GT_OK;
}

gt_status enqueue_pair_check(Index* ix, Batch* b) {
  HIPCHK(gt::launch_pair_check(b->cand, &b->ctr->ncand, (unsigned long long)b->cand_cap, b->qf,
                               ix->leaves, b->invn_q, ix->invn, b->rho, ix->dp, b->hits,
                               (unsigned long long)b->hit_cap, b->band_idx, b->qcount, b->ctr,
                               ix->n_cu * 4, b->stream));
  return GT_OK;
}

// Placement of the accepted pairs by query and the per-query sort by id.
// lim: largest result count the outputs can take; the kernels check the
// count on the device and do nothing when it is larger.
gt_status enqueue_place(Batch* b, int64_t lim, int64_t* ids, float* sims) {
  hipStream_t s = b->stream;
  const unsigned long long hc = (unsigned long long)b->hit_cap, l = (unsigned long long)lim;
  HIPCHK(gt::launch_scatter(b->hits, b->ctr, hc, l, b->offs, b->out_id, b->out_sim, s));
  HIPCHK(gt::launch_sort_segments(b->offs, b->nq, b->out_id, b->out_sim, b->tmp_id, b->tmp_sim,
                                  ids, sims, b->ctr, hc, l, b->n_epoch, s));
  return GT_OK;
}

// recheck, offsets, placement and sort of the results (before the host has
// seen their count, so that a call needs one wait), and the copy of the
// counters the host needs
gt_status enqueue_tail(Index* ix, Batch* b) {
  hipStream_t s = b->stream;
  HIPCHK(gt::launch_recheck(b->hits, b->band_idx, &b->ctr->nband, (unsigned long long)b->hit_cap,
                            b->qf, ix->leaves, ix->d, ix->dp, ix->ff, b->rho, b->qcount,
                            b->ctr, s));
  ev_mark(b, 4);
  HIPCHK(gt::launch_scan_offsets(b->qcount, b->nq, b->offs, nullptr, b->ctr, s));
  TRY(ensure_out(b, 1));
  b->spec_direct = b->tgt_ids != nullptr;
  // (a fixed batch has no staging of its own for the sorted results: without
  // caller buffers nothing is placed)
  b->spec_lim = b->spec_direct ? std::min(b->out_cap, b->tgt_max) : b->fixed ? 0 : b->out_cap;
  TRY(enqueue_place(b, b->spec_lim, b->spec_direct ? b->tgt_ids : b->fin_id,
                    b->spec_direct ? b->tgt_sims : b->fin_sim));
  HIPCHK(hipMemcpyAsync(b->h_ctr, b->ctr, sizeof(gt::DevCounters), hipMemcpyDeviceToHost, s));
  if (b->done) HIPCHK(hipEventRecord(b->done, s));
  ev_mark(b, 5);
  return GT_OK;
}

// candidate stage again after the candidate buffers grew
void set_targets(Batch* b, int64_t max_results, int64_t* ids, float* sims) {
  b->tgt_ids = max_results > 0 ? ids : nullptr;
  b->tgt_sims = max_results > 0 ? sims : nullptr;
  b->tgt_max = max_results;
}

gt_status redo_candidates(Index* ix, Batch* b) {
  hipStream_t s = b->stream;
  TRY(zero_dev(b->qcount, (size_t)b->nq_pad * 4, s));
  TRY(zero_dev(&b->ctr->nhits, 8, s));
  TRY(zero_dev(&b->ctr->leaf_pairs, 8, s));
  TRY(zero_dev(&b->ctr->rechecked, 8, s));
  TRY(zero_dev(&b->ctr->nband, 8, s));
  if (b->kind == 1) {
    TRY(enqueue_leaf(ix, b));
  } else {
    TRY(zero_dev(&b->ctr->ncand, 8, s));
    TRY(enqueue_exhaustive(ix, b));
    TRY(enqueue_pair_check(ix, b));
  }
  return enqueue_tail(ix, b);
}

gt_status check_query_args(const Index* ix, const float* q, int nq, const double* rho, int tq) {
  if (!ix) return fail(GT_ERR_INVALID_ARG, "index is NULL");
  if (nq < 0) return fail(GT_ERR_INVALID_ARG, "nq < 0");
  if ((int64_t)nq > (int64_t)gt::kMaxTiles * tq)
    return fail(GT_ERR_INVALID_ARG, "nq exceeds " + std::to_string(gt::kMaxTiles * tq) +
                                        " queries per call for this format");
  if (nq > 0 && (!q || !rho)) return fail(GT_ERR_INVALID_ARG, "NULL query argument");
  for (int i = 0; i < nq; ++i)
    if (isnan(rho[i])) return fail(GT_ERR_INVALID_ARG, "rho is NaN");
  return GT_OK;
}

// ------------------------------------------------------ fixed (carved) batches
void* arena_take(Batch* b, size_t bytes) {
  const size_t off = (b->arena_used + 255) & ~size_t(255);
  if (off > b->arena_size || bytes > b->arena_size - off) return nullptr;
  b->arena_used = off + bytes;
  return b->arena + off;
}

constexpr size_t kPerPair = sizeof(gt::Hit) + 4 + 4 * 4;  // hit, band index, 4 staging words
constexpr size_t kPerEntry = 2 * (4 + 8);                   // node and mask, two levels
constexpr size_t kPerRecord = 2 * 64 * 2;                   // 64 bf16 bounds, two levels

// Call shape of a walk in user pool format fmt: the walked format, tiles.
struct CallShape {
  bool maxp;
  int wf, tq, nt, nq_pad, h, dl;
  bool want_rec;
};
CallShape call_shape(const Index* ix, int nq, int fmt) {
  CallShape c{};
  c.maxp = fmt == GT_POOL_MAX_F32 || fmt == GT_POOL_MAX_BF16;
  c.wf = c.maxp ? (fmt == GT_POOL_MAX_F32 ? GT_POOL_F32 : GT_POOL_BF16) : fmt;
  c.tq = tq_of(c.wf);
  c.nt = std::max(1, (nq + c.tq - 1) / c.tq);
  c.nq_pad = std::max(128, (nq + 127) / 128 * 128);
  c.h = head_of(ix);
  c.dl = dense_last_of(ix, c.wf, c.h);
  c.want_rec = c.wf == GT_POOL_BF16 && !c.maxp && c.dl >= 0 && ix->walk_subtract != 0 &&
               c.dl <= ix->depth - 2 && ix->dp <= gt::kMaxDpBf16;
  return c;
}

template <class T>
void take(Batch* b, T*& p, size_t count, bool& ok) {
  p = static_cast<T*>(arena_take(b, std::max<size_t>(count, 1) * sizeof(T)));
  ok = ok && p != nullptr;
}

// The buffers of a walk call other than its frontier, records and candidates:
// counters, query copies, and the dense masks of chained dense steps.
void carve_common(Index* ix, Batch* b, void* base, size_t bytes, int nq, const CallShape& c,
                  bool& ok) {
  b->ix = ix;
  b->fixed = true;
  b->arena = static_cast<unsigned char*>(base);
  b->arena_size = bytes;
  b->arena_used = 0;
  b->max_queries = std::max(nq, 1);
  b->rec_len = 0;
  b->dmask_len = 0;
  b->fr_rec[0] = b->fr_rec[1] = nullptr;
  b->dmask[0] = b->dmask[1] = nullptr;
  const size_t dp = (size_t)ix->dp, pw = (size_t)ix->pw, nqa = (size_t)c.nq_pad;
  take(b, b->ctr, 1, ok);
  take(b, b->lvl_count, (size_t)GT_MAX_LEVELS * gt::kMaxSlots, ok);
  take(b, b->tile_mask, gt::kMaxTiles, ok);
  take(b, b->qf, nqa * dp, ok);
  if (ix->signed_mode) take(b, b->qw, nqa * pw, ok);
  take(b, b->qbf, nqa * pw, ok);
  take(b, b->q8, nqa * dp, ok);
  take(b, b->qexp, nqa, ok);
  take(b, b->invn_q, nqa, ok);
  take(b, b->qq, nqa, ok);
  take(b, b->rho, nqa, ok);
  take(b, b->thr, nqa, ok);
  take(b, b->thr_gemm, nqa, ok);
  take(b, b->sabs, nqa, ok);
  take(b, b->qcount, nqa, ok);
  take(b, b->offs, nqa + 1, ok);
  b->nq_alloc = c.nq_pad;
  b->nt_alloc = c.nt;
  if (c.dl >= 0 && ix->head_level >= 0 && c.h + 1 < c.dl) {
    const size_t need = ((size_t)1 << std::max(0, c.dl - 1)) * (size_t)c.nt;
    take(b, b->dmask[0], need, ok);
    take(b, b->dmask[1], need, ok);
    b->dmask_len = (int64_t)need;
  }
}

void carve_pairs(Batch* b, size_t pairs, bool& ok) {
  take(b, b->hits, pairs, ok);
  take(b, b->band_idx, pairs, ok);
  take(b, b->out_id, pairs, ok);
  take(b, b->out_sim, pairs, ok);
  take(b, b->tmp_id, pairs, ok);
  take(b, b->tmp_sim, pairs, ok);
  b->hit_cap = (int64_t)pairs;
  b->out_cap = (int64_t)pairs;
}

// Frontier of fr_cap entries per tile (two levels), with score records if asked.
void carve_frontier(Batch* b, int nt, int64_t fr_cap, bool rec, bool& ok) {
  for (int k = 0; k < 2; ++k) {
    take(b, b->fr_node[k], (size_t)nt * fr_cap, ok);
    take(b, b->fr_mask[k], (size_t)nt * fr_cap, ok);
  }
  if (rec) {
    take(b, b->fr_rec[0], (size_t)nt * fr_cap * 64, ok);
    take(b, b->fr_rec[1], (size_t)nt * fr_cap * 64, ok);
    b->rec_len = (int64_t)nt * fr_cap;
  }
  b->fr_cap = fr_cap;
}

// Carves every buffer of one walk call of nq queries in pool format fmt out of
// [base, base + bytes): counters, query copies, the frontier at its worst case
// (every pool of the deepest level for every tile, so no level can overflow),
// dense masks if chained dense steps are configured, score records of the
// subtraction step if they fit beside at least 2^20 candidates, and the rest
// split between candidates and result staging.  GT_ERR_CAPACITY if the
// frontier alone does not fit.
gt_status carve_fixed(Index* ix, Batch* b, void* base, size_t bytes, int nq, int fmt) {
  constexpr size_t kMinPairs = size_t(1) << 20;
  const CallShape c = call_shape(ix, nq, fmt);
  const int64_t fr_cap = int64_t(1) << std::max(0, ix->depth - 1);
  bool ok = true;
  carve_common(ix, b, base, bytes, nq, c, ok);
  carve_frontier(b, c.nt, fr_cap, false, ok);
  if (!ok)
    return fail(GT_ERR_CAPACITY,
                "a call of " + std::to_string(nq) + " queries on an index of depth " +
                    std::to_string(ix->depth) + " needs more than the " +
                    std::to_string(bytes >> 20) + " MiB of fixed scratch for its frontier; " +
                    "use fewer queries per call");
  const size_t rec = (size_t)c.nt * (size_t)fr_cap * 64 * sizeof(uint16_t);
  const size_t left0 = bytes - b->arena_used;
  if (c.want_rec && left0 > 2 * rec + 2 * 256 + kMinPairs * kPerPair + 8 * 256) {
    take(b, b->fr_rec[0], rec / 2, ok);
    take(b, b->fr_rec[1], rec / 2, ok);
    b->rec_len = (int64_t)c.nt * fr_cap;
  }
  const size_t left = bytes - b->arena_used;
  const size_t pairs = left > 8 * 256 ? (left - 8 * 256) / kPerPair : 0;
  if (pairs < 1024)
    return fail(GT_ERR_CAPACITY, "no room for candidates in the fixed scratch beside a call of " +
                                     std::to_string(nq) + " queries; use fewer queries per call");
  carve_pairs(b, pairs, ok);
  if (!ok) return fail(GT_ERR_CAPACITY, "fixed scratch carve failed");
  return GT_OK;
}

// Bytes of the common buffers of a call (with their alignment).
size_t common_bytes(Index* ix, int nq, const CallShape& c) {
  Batch dry;
  bool ok = true;
  carve_common(ix, &dry, reinterpret_cast<void*>(uintptr_t(256)), SIZE_MAX / 4, nq, c, ok);
  return dry.arena_used + 256;
}

// Carve of an external workspace's call: the common buffers, `pairs`
// candidates and results, and a frontier of whatever the memory leaves (at
// most the worst case), with score records only if allowed and wanted.
gt_status carve_budget(Index* ix, Batch* b, void* base, size_t bytes, int nq, int fmt,
                       int64_t pairs, bool allow_rec) {
  const CallShape c = call_shape(ix, nq, fmt);
  bool ok = true;
  carve_common(ix, b, base, bytes, nq, c, ok);
  if (pairs < 0) {
    // continuation: the worst-case frontier of the call's tiles, without
    // records, and every remaining byte for candidates and results
    const int64_t worst = int64_t(1) << std::max(0, ix->depth - 1);
    carve_frontier(b, c.nt, worst, false, ok);
    const size_t left = ok ? bytes - b->arena_used : 0;
    const size_t np = left > 8 * 256 ? (left - 8 * 256) / kPerPair : 0;
    if (!ok || np < 1024)
      return fail(GT_ERR_CAPACITY, "the call's memory does not hold one tile's worst case");
    carve_pairs(b, np, ok);
    if (!ok) return fail(GT_ERR_CAPACITY, "continuation carve failed");
    return GT_OK;
  }
  carve_pairs(b, (size_t)std::max<int64_t>(pairs, 1024), ok);
  if (!ok) return fail(GT_ERR_CAPACITY, "the call's memory does not hold its query and candidate buffers");
  const bool rec = allow_rec && c.want_rec;
  const size_t per = kPerEntry + (rec ? kPerRecord : 0);
  const size_t left = bytes - b->arena_used;
  const size_t usable = left > 8 * 256 ? left - 8 * 256 : 0;
  const int64_t worst = int64_t(1) << std::max(0, ix->depth - 1);
  const int64_t fr_cap = std::min<int64_t>(worst, (int64_t)(usable / per / (size_t)c.nt));
  if (fr_cap < 64) return fail(GT_ERR_CAPACITY, "the call's memory leaves no room for its frontier");
  carve_frontier(b, c.nt, fr_cap, rec, ok);
  if (!ok) return fail(GT_ERR_CAPACITY, "frontier carve failed");
  return GT_OK;
}

// Enqueues a whole call up to the counter readback.  kind 1: walk, 2: exhaustive.
gt_status submit(Index* ix, Batch* b, int kind, const float* q, int nq, const double* rho,
                 int fmt, hipStream_t s) {
  if (b->pending) return fail(GT_ERR_INVALID_ARG, "the workspace has a call in flight");
  // max pools run the kernels of their storage format on the max tree
  const int user_fmt = fmt;
  const bool maxp = kind == 1 && (fmt == GT_POOL_MAX_F32 || fmt == GT_POOL_MAX_BF16);
  if (maxp) fmt = fmt == GT_POOL_MAX_F32 ? GT_POOL_F32 : GT_POOL_BF16;
  const int tq = kind == 1 ? tq_of(fmt) : gt::kQueriesPerTile16;
  if (kind == 1) {
    if (fmt != GT_POOL_F32 && fmt != GT_POOL_BF16 && fmt != GT_POOL_FP8E4M3)
      return fail(GT_ERR_INVALID_ARG, "unknown pool format");
    if (!(ix->formats & (uint32_t)user_fmt))
      return fail(GT_ERR_INVALID_ARG, "pool format was not built");
    if ((maxp ? ix->pw : ix->dp) > gt::kMaxWalkWidth)
      return fail(GT_ERR_INVALID_ARG, "pool rows wider than " +
                                          std::to_string(gt::kMaxWalkWidth) + " columns");
  }
  TRY(check_query_args(ix, q, nq, rho, tq));
  if (ix->signed_mode)
    for (int i = 0; i < nq; ++i)
      if (!(rho[i] > 0.0))
        return fail(GT_ERR_INVALID_ARG, "rho must be > 0 on an index of signed vectors");
  const int nt = (nq + tq - 1) / tq;
  const int nq_pad = std::max(128, (nq + 127) / 128 * 128);
  if (b->max_queries > 0 && nq > b->max_queries)
    return fail(GT_ERR_CAPACITY, "batch of " + std::to_string(nq) +
                                     " queries exceeds the workspace's " +
                                     std::to_string(b->max_queries));
  TRY(batch_reserve(b, nq_pad, std::max(nt, 1)));
  b->kind = kind;
  b->stream = s;
  b->fmt = fmt;
  b->maxpool = maxp;
  b->nq = nq;
  b->nq_pad = nq_pad;
  b->nt = nt;
  b->tq = tq;
  // a continuation tile sees the rows its call saw, whatever was inserted since
  b->n_epoch = b->cont ? b->ext_epoch : ix->n;
  b->head = head_of(ix);
  b->dense_last = kind == 1 ? dense_last_of(ix, fmt, b->head) : -1;
  if (kind == 1) b->dense_last = adapt_dense_last(ix, b, fmt, maxp, b->dense_last, b->head);
  // A dense step computes every pool of its level against every query, and
  // a pool's score never exceeds its parent's (non-negative rows, sums
  // rounded up), so a chain of dense steps keeps the same (pool, query) pairs
  // as its last step alone, up to rounding, which only keeps more.  With an
  // automatic head only the last dense level is tested.
  if (b->dense_last >= 0 && ix->head_level < 0) b->head = b->dense_last - 1;
  b->nb = bucket_bits_of(b->dense_last >= 0 ? b->dense_last : b->head, nt);
  b->profile = ix->profile && !b->fixed;
  b->nw = 0;
  if (b->profile && !b->events) {
    for (auto& e : b->ev) HIPCHK(hipEventCreate(&e));
    for (auto& e : b->evw) HIPCHK(hipEventCreate(&e));
    b->events = true;
  }
  ev_mark(b, 0);
  TRY(zero_dev(b->ctr, sizeof(gt::DevCounters), s));
  TRY(zero_dev(b->qcount, (size_t)nq_pad * 4, s));
  TRY(zero_dev(b->tile_mask, (size_t)gt::kMaxTiles * 8, s));
  if (kind == 1) TRY(zero_dev(b->lvl_count, (size_t)GT_MAX_LEVELS * gt::kMaxSlots * 4, s));
  b->counted = ix->count_unique && kind == 1 && !b->fixed;
  if (b->counted) {
    const int64_t words = (int64_t(2) << ix->depth) / 32 + 1;
    if (!b->bitmap) {
      TRY(dalloc(ix, &b->bitmap, (size_t)words));
      b->bitmap_words = words;
    }
    TRY(zero_dev(b->bitmap, (size_t)words * 4, s));
  }
  if (nq > 0) {
    if (b->h_rho) {
      memcpy(b->h_rho, rho, (size_t)nq * 8);
      HIPCHK(hipMemcpyAsync(b->rho, b->h_rho, (size_t)nq * 8, hipMemcpyHostToDevice, s));
    } else {
      HIPCHK(hipMemcpyAsync(b->rho, rho, (size_t)nq * 8, hipMemcpyHostToDevice, s));
    }
    // reduced query copies only for the call's pool format; the absolute
    // terms of the subtraction step only for bfloat16 sum pools
    const bool w16 = kind == 1 && fmt == GT_POOL_BF16, w8 = kind == 1 && fmt == GT_POOL_FP8E4M3;
    const bool w32s = kind == 1 && fmt == GT_POOL_F32 && ix->signed_mode;
    HIPCHK(gt::launch_query_prep(q, nq, ix->d, ix->dp, tq, b->rho, ix->d_mmin, b->qf,
                                 w16 ? b->qbf : nullptr, w8 ? b->q8 : nullptr, b->qexp, b->invn_q,
                                 b->qq, b->thr, b->thr_gemm, b->tile_mask,
                                 w16 && !maxp ? ix->master + level_row(0) * ix->dp : nullptr,
                                 w16 && !maxp ? b->sabs : nullptr, w32s ? b->qw : nullptr, ix->pw,
                                 ix->signed_mode ? ix->sbound : 0.0f, &b->ctr->err, nq_pad, s));
  }
  ev_mark(b, 1);
  if (nq > 0 && b->n_epoch > 0) {
    if (kind == 1) {
      TRY(enqueue_walk(ix, b));
      ev_mark(b, 2);
      TRY(enqueue_leaf(ix, b));
      // entries of every walked level (the automatic dense level and the
      // memory estimates of a server read them)
      HIPCHK(gt::launch_level_entries(b->lvl_count, b->dense_last >= 0 ? b->dense_last : b->head,
                                      ix->depth, b->ctr, s));
    } else {
      TRY(enqueue_exhaustive(ix, b));
      ev_mark(b, 2);
      TRY(enqueue_pair_check(ix, b));
    }
  } else {
    ev_mark(b, 2);
  }
  ev_mark(b, 3);
  TRY(enqueue_tail(ix, b));
  b->pending = true;
  b->last_nq = nq;
  b->last_nt = nt;
  b->last_fmt = kind == 1 ? user_fmt : 0;
  b->last_head = b->head;
  return GT_OK;
}

// Waits for the counters, handles buffer overflow, writes offsets, ids and sims.
// keep_on_overflow: after GT_ERR_RESULT_OVERFLOW the call stays in flight, so
// finish can be called again with larger buffers without recomputing it.
gt_status continue_by_tiles(Index* ix, Batch* b, int64_t max_results, int64_t* offsets,
                            int64_t* ids, float* sims, int64_t* total_out, bool keep_on_overflow);

gt_status finish(Index* ix, Batch* b, int64_t max_results, int64_t* offsets, int64_t* ids,
                 float* sims, int64_t* total_out, bool keep_on_overflow) {
  if (!b->pending) return fail(GT_ERR_INVALID_ARG, "no call in flight on this workspace");
  b->pending = false;
  if (b->cont_again) {
    if (!total_out || !offsets || max_results < 0 || (max_results > 0 && (!ids || !sims)))
      return fail(GT_ERR_INVALID_ARG, "bad output arguments");
    return continue_by_tiles(ix, b, max_results, offsets, ids, sims, total_out, keep_on_overflow);
  }
  if (!total_out) return fail(GT_ERR_INVALID_ARG, "total_out is NULL");
  if (max_results < 0) return fail(GT_ERR_INVALID_ARG, "max_results < 0");
  if (!offsets) return fail(GT_ERR_INVALID_ARG, "offsets is NULL");
  if (max_results > 0 && (!ids || !sims)) return fail(GT_ERR_INVALID_ARG, "NULL output buffer");
  hipStream_t s = b->stream;
  *total_out = 0;
  for (int attempt = 0;; ++attempt) {
    if (b->done)
      HIPCHK(hipEventSynchronize(b->done));
    else
      HIPCHK(hipStreamSynchronize(s));
    const gt::DevCounters& c = *b->h_ctr;
    if (c.err)
      return fail(GT_ERR_INVALID_INPUT, ix->signed_mode
                                            ? "query contains a NaN or infinite value"
                                            : "query contains a NaN, infinite or negative value");
    if (c.slot_over)
      return fail(GT_ERR_CAPACITY, "a query has more than 2^30 results");
    const bool cand_over = b->kind == 2 && (int64_t)c.ncand > b->cand_cap;
    const bool hit_over = (int64_t)c.nhits > b->hit_cap;
    if (b->external && !b->cont && (c.fr_over || hit_over))
      return continue_by_tiles(ix, b, max_results, offsets, ids, sims, total_out, keep_on_overflow);
    if (c.fr_over)
      return fail(GT_ERR_CAPACITY, "a frontier level outgrew the memory given to one query tile");
    if (!cand_over && !hit_over) break;
    if (attempt > 3) return fail(GT_ERR_DEVICE, "candidate buffers did not converge");
    if (cand_over) {
      const int64_t need = (int64_t)c.ncand;
      dfree(ix, &b->cand, (size_t)b->cand_cap);
      b->cand_cap = 0;
      TRY(dalloc(ix, &b->cand, (size_t)(need + need / 4 + 1024)));
      b->cand_cap = need + need / 4 + 1024;
    }
    if (hit_over) TRY(grow_hits(b, (int64_t)c.nhits));
    TRY(redo_candidates(ix, b));
  }
  if (b->kind == 1) {
    // state for the next call's automatic dense level
    b->have_last = true;
    b->last_dl = b->dense_last;
    b->last_walk_fmt = b->fmt;
    b->last_maxpool = b->maxpool;
    b->last_walk_nt = b->nt;
    b->last_n_epoch = b->n_epoch;
    memcpy(b->last_entries, b->h_ctr->entries, sizeof(b->last_entries));
    int64_t mx = 0;
    for (int l = 0; l < GT_MAX_LEVELS; ++l) mx = std::max(mx, (int64_t)b->h_ctr->entries[l]);
    b->last_max_entries = mx;
    b->last_results = (int64_t)b->h_ctr->total;
  }
  const int64_t total = (int64_t)b->h_ctr->total;
  *total_out = total;
  HIPCHK(hipMemcpyAsync(offsets, b->offs, (size_t)(b->nq + 1) * 8, hipMemcpyDeviceToDevice, s));
  if (total > max_results) {
    b->pending = keep_on_overflow;
    return fail(GT_ERR_RESULT_OVERFLOW, "need max_results >= " + std::to_string(total));
  }
  if (total > 0) {
    if (total > b->spec_lim) {
      // the enqueued placement did nothing: buffers were too small
      TRY(ensure_out(b, total));
      TRY(enqueue_place(b, total, ids, sims));
    } else if (!(b->spec_direct && ids == b->tgt_ids && sims == b->tgt_sims)) {
      HIPCHK(hipMemcpyAsync(ids, b->fin_id, (size_t)total * 8, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(sims, b->fin_sim, (size_t)total * 4, hipMemcpyDeviceToDevice, s));
    }
  }
  ev_mark(b, 6);
  if (b->profile) {
    HIPCHK(hipStreamSynchronize(s));
    b->ms[0] = ev_between(b, 0, 1);                          // query prep
    b->ms[1] = b->kind == 1 ? ev_walk(b, false) : 0.0;       // sparse walk levels
    b->ms[2] = ev_between(b, 2, 3);                          // leaf / pair test
    b->ms[3] = ev_between(b, 3, 4);                          // float64 recheck
    b->ms[4] = ev_between(b, 4, 5) + ev_between(b, 5, 6);    // offsets, compaction
    b->ms[5] = b->kind == 2 ? ev_walk(b, true) : 0.0;        // exhaustive GEMM
    b->ms[6] = ev_between(b, 0, 6);
    b->ms[7] = b->kind == 1 ? ev_walk(b, true) : 0.0;        // dense levels
  }
  return GT_OK;
}

// An external workspace's call whose frontier (or candidates) outgrew its
// memory: the same call again, one query tile at a time, each tile with the
// worst-case frontier of one tile (the submit checked that it fits) and every
// other byte for candidates; a tile whose candidates still do not fit runs
// query by query.  A query's result does not depend on the other queries of
// its call, so the results are those of the call; each part's results go
// straight to the caller's buffers after the earlier parts', and its offsets
// are shifted by the results before it.
gt_status continue_by_tiles(Index* ix, Batch* b, int64_t max_results, int64_t* offsets,
                            int64_t* ids, float* sims, int64_t* total_out, bool keep_on_overflow) {
  const int tq = call_shape(ix, 1, b->user_fmt).tq;
  const int nq = (int)b->rho_in.size();
  const hipStream_t s = b->stream;
  const std::vector<double> rho = b->rho_in;
  std::vector<std::pair<int, int>> work;  // query ranges [first, first + count), in order
  for (int a = 0; a < nq; a += tq) work.emplace_back(a, std::min(tq, nq - a));
  std::vector<int64_t> hoff((size_t)tq + 1);
  int64_t total = 0;
  unsigned long long level_sum[GT_MAX_LEVELS] = {};
  bool over = false;
  b->cont = true;
  b->cont_again = false;
  b->continued_tiles = (int)work.size();
  gt_status st = GT_OK;
  for (size_t w = 0; w < work.size() && st == GT_OK; ++w) {
    const int a = work[w].first, n = work[w].second;
    const int64_t room = max_results > total ? max_results - total : 0;
    int64_t* ids_t = room > 0 ? ids + total : nullptr;
    float* sims_t = room > 0 ? sims + total : nullptr;
    int64_t tot_t = 0;
    b->hits_overflowed = false;
    st = carve_budget(ix, b, b->ext_mem, b->ext_bytes, n, b->user_fmt, -1, false);
    if (st == GT_OK) {
      set_targets(b, room, ids_t, sims_t);
      st = submit(ix, b, 1, b->q_in + (size_t)a * ix->d, n, rho.data() + a, b->user_fmt, s);
    }
    if (st == GT_OK) st = finish(ix, b, room, offsets + a, ids_t, sims_t, &tot_t, false);
    if (st == GT_ERR_CAPACITY && b->hits_overflowed && n > 1) {
      // too many candidates for one tile: its queries one by one
      std::vector<std::pair<int, int>> singles;
      for (int k = 0; k < n; ++k) singles.emplace_back(a + k, 1);
      work.insert(work.begin() + (long)w + 1, singles.begin(), singles.end());
      st = GT_OK;
      continue;
    }
    if (st == GT_ERR_RESULT_OVERFLOW) {
      over = true;
      st = GT_OK;
    }
    if (st != GT_OK) break;
    for (int l = 0; l < GT_MAX_LEVELS; ++l) level_sum[l] += b->h_ctr->entries[l];
    // the part's offsets start at 0: shift them past the earlier parts' results
    const hipError_t e1 = hipMemcpyAsync(hoff.data(), offsets + a, (size_t)(n + 1) * 8,
                                         hipMemcpyDeviceToHost, s);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(s) : e1;
    if (e2 != hipSuccess) {
      st = fail(GT_ERR_DEVICE, std::string("continuation offsets: ") + hipGetErrorString(e2));
      break;
    }
    for (int k = 0; k <= n; ++k) hoff[k] += total;
    const hipError_t e3 = hipMemcpyAsync(offsets + a, hoff.data(), (size_t)(n + 1) * 8,
                                         hipMemcpyHostToDevice, s);
    const hipError_t e4 = e3 == hipSuccess ? hipStreamSynchronize(s) : e3;
    if (e4 != hipSuccess) {
      st = fail(GT_ERR_DEVICE, std::string("continuation offsets: ") + hipGetErrorString(e4));
      break;
    }
    total += tot_t;
  }
  b->cont = false;
  b->rho_in = rho;
  b->nq = nq;
  if (st != GT_OK) return st;
  int64_t mx = 0;
  for (int l = 0; l < GT_MAX_LEVELS; ++l) mx = std::max(mx, (int64_t)level_sum[l]);
  b->last_max_entries = mx;
  b->last_results = total;
  *total_out = total;
  if (over) {
    // the next finish, with larger buffers, runs the parts again
    b->pending = keep_on_overflow;
    b->cont_again = keep_on_overflow;
    return fail(GT_ERR_RESULT_OVERFLOW, "need max_results >= " + std::to_string(total));
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
  if (pool_formats & ~(uint32_t)(GT_POOL_F32 | GT_POOL_BF16 | GT_POOL_FP8E4M3 | GT_POOL_MAX_F32 |
                                 GT_POOL_MAX_BF16 | GT_POOL_SIGNED))
    return fail(GT_ERR_INVALID_ARG, "unknown pool format bits");
  const bool sgn = (pool_formats & GT_POOL_SIGNED) != 0;
  if (sgn && (pool_formats & (GT_POOL_F32 | GT_POOL_BF16 | GT_POOL_FP8E4M3)))
    return fail(GT_ERR_INVALID_ARG, "an index of signed vectors keeps max/min pools only");
  if (capacity == 0) {
    capacity = 2;
    while (capacity < n) capacity <<= 1;
  }
  if (capacity < 2 || (capacity & (capacity - 1)) || capacity < n)
    return fail(GT_ERR_INVALID_ARG, "capacity must be a power of two >= max(n, 2)");
  if (capacity > (int64_t(1) << 31)) return fail(GT_ERR_INVALID_ARG, "capacity above 2^31");

  hipStream_t s = (hipStream_t)stream;
  gt_index* ix = new gt_index();
  auto bail = [&](gt_status st) {
    std::string keep = g_err;
    if (ix->def) {
      free_batch(ix->def);
      delete static_cast<gt_batch*>(ix->def);
    }
    free_tree(ix);
    delete ix;
    g_err = keep;
    return st;
  };
#define BTRY(expr)                    \
  do {                                \
    gt_status s_ = (expr);            \
    if (s_ != GT_OK) return bail(s_); \
  } while (0)
#define BHIP(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return bail(fail(GT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)

  BHIP(hipGetDevice(&ix->device));
  // the device scratch of gt_query_batch_noalloc, once per device
  ix->scratch_err = gt::scratch_setup(ix->device);
  if (ix->scratch_err != hipSuccess) (void)hipGetLastError();
  hipDeviceProp_t prop;
  BHIP(hipGetDeviceProperties(&prop, ix->device));
  ix->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  ix->d = d;
  ix->dp = (d + 127) / 128 * 128;
  ix->cap = capacity;
  ix->depth = 0;
  while ((int64_t(1) << ix->depth) < capacity) ++ix->depth;
  ix->dtype = dtype;
  // signed vectors: max/min pools only (a float32 tree always); otherwise the
  // float32 sums always, and a float32 max tree whenever a max format is asked for
  ix->signed_mode = sgn;
  ix->pw = sgn ? 2 * ix->dp : ix->dp;
  ix->formats = sgn ? (pool_formats | GT_POOL_MAX_F32) : (pool_formats | GT_POOL_F32);
  if (ix->formats & GT_POOL_MAX_BF16) ix->formats |= GT_POOL_MAX_F32;

  const size_t cap = (size_t)capacity, dp = (size_t)ix->dp, tree = (cap - 1) * dp;
  const size_t pw = (size_t)ix->pw, mtree = (cap - 1) * pw;
  BTRY(dalloc(ix, &ix->leaves, cap * dp));
  BTRY(dalloc(ix, &ix->invn, cap));
  BTRY(dalloc(ix, &ix->ff, cap));
  BTRY(dalloc(ix, &ix->nf, cap));
  BTRY(dalloc(ix, &ix->d_mmin, 2));
  BTRY(dalloc(ix, &ix->d_absmax, 1));
  if (ix->formats & GT_POOL_F32) BTRY(dalloc(ix, &ix->master, tree));
  if (ix->formats & GT_POOL_BF16) BTRY(dalloc(ix, &ix->pbf16, tree));
  if (ix->formats & GT_POOL_FP8E4M3) BTRY(dalloc(ix, &ix->pfp8, tree));
  if (ix->formats & GT_POOL_MAX_F32) BTRY(dalloc(ix, &ix->mmax, mtree));
  if (ix->formats & GT_POOL_MAX_BF16) BTRY(dalloc(ix, &ix->pmax16, mtree));
  BTRY(dalloc(ix, &ix->d_lexp, GT_MAX_LEVELS));
  BTRY(dalloc(ix, &ix->d_levelmax, GT_MAX_LEVELS));
  BTRY(dalloc(ix, &ix->d_flags, GT_MAX_LEVELS));
  BHIP(hipMemsetAsync(ix->leaves, 0, cap * dp * 4, s));
  BHIP(hipMemsetAsync(ix->invn, 0, cap * 4, s));
  BHIP(hipMemsetAsync(ix->ff, 0, cap * 8, s));
  BHIP(hipMemsetAsync(ix->nf, 0, cap * 4, s));
  if (ix->master) BHIP(hipMemsetAsync(ix->master, 0, tree * 4, s));
  if (ix->mmax) BHIP(hipMemsetAsync(ix->mmax, 0, mtree * 4, s));
  BHIP(hipMemsetAsync(ix->d_absmax, 0, 4, s));
  BHIP(hipMemsetAsync(ix->d_flags, 0, GT_MAX_LEVELS * 4, s));
  BHIP(hipMemsetAsync(ix->d_lexp, 0, GT_MAX_LEVELS * 4, s));
  const double inf = INFINITY;
  BHIP(hipMemcpyAsync(ix->d_mmin, &inf, 8, hipMemcpyHostToDevice, s));
  unsigned int* derr = ix->d_flags + (GT_MAX_LEVELS - 1);
  BHIP(gt::launch_ingest(feats_dev, dtype, n, d, ix->dp, ix->leaves, ix->ff, ix->invn, ix->nf,
                         ix->d_mmin, derr, sgn, sgn ? ix->d_absmax : nullptr, s));
  unsigned int herr = 0, habs = 0;
  BHIP(hipMemcpyAsync(&herr, derr, 4, hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(&habs, ix->d_absmax, 4, hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  if (herr)
    return bail(fail(GT_ERR_INVALID_INPUT, sgn ? "features contain a NaN or infinite value"
                                               : "features contain a NaN, infinite or negative value"));
  ix->n = n;
  if (sgn) {
    // B: the smallest power of two >= the largest |value| (1 if all are zero)
    float amax;
    memcpy(&amax, &habs, 4);
    int ex = 0;
    const double m = amax > 0.0f ? frexp((double)amax, &ex) : 0.5;
    ix->sbound = amax > 0.0f ? (float)ldexp(1.0, m == 0.5 ? ex - 1 : ex) : 1.0f;
  }

  // pools, bottom-up; only pools covering some of the first n leaves are non-zero
  for (int l = ix->depth - 1; l >= 0; --l) {
    const int64_t span = int64_t(1) << (ix->depth - l);
    const int64_t nodes = (n + span - 1) / span;
    if (ix->master) {
      const float* child = (l == ix->depth - 1) ? ix->leaves : ix->master + level_row(l + 1) * dp;
      BHIP(gt::launch_build_level(child, ix->master + level_row(l) * dp, nodes, ix->dp, 0, s,
                                  false));
    }
    if (ix->mmax) {
      float* mpar = ix->mmax + level_row(l) * pw;
      if (sgn && l == ix->depth - 1) {
        BHIP(gt::launch_signed_bottom(ix->leaves, mpar, 0, nodes, ix->dp, ix->d, n, ix->sbound, s));
      } else {
        const float* mchild = (l == ix->depth - 1) ? ix->leaves : ix->mmax + level_row(l + 1) * pw;
        BHIP(gt::launch_build_level(mchild, mpar, nodes, ix->pw, 0, s, true));
      }
    }
  }
  if (ix->pbf16) BHIP(gt::launch_quant_bf16(ix->master, ix->pbf16, (int64_t)tree, s));
  if (ix->pmax16) BHIP(gt::launch_quant_bf16(ix->mmax, ix->pmax16, (int64_t)mtree, s));
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
  gt_batch* def = new gt_batch();
  def->ix = ix;
  ix->def = def;
  BTRY(batch_init(def));
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
  const size_t dp = (size_t)ix->dp, pw = (size_t)ix->pw;
  const int64_t lo = ix->n, hi = ix->n + n_new;
  unsigned int* derr = ix->d_flags + (GT_MAX_LEVELS - 1);
  double* tmp_mmin = ix->d_mmin + 1;
  const double inf = INFINITY;
  const bool sgn = ix->signed_mode;
  HIPCHK(hipMemsetAsync(derr, 0, 4, s));
  HIPCHK(hipMemsetAsync(ix->d_absmax, 0, 4, s));
  HIPCHK(hipMemcpyAsync(tmp_mmin, &inf, 8, hipMemcpyHostToDevice, s));
  HIPCHK(gt::launch_ingest(feats_dev, ix->dtype, n_new, ix->d, ix->dp, ix->leaves + lo * dp,
                           ix->ff + lo, ix->invn + lo, ix->nf + lo, tmp_mmin, derr, sgn,
                           sgn ? ix->d_absmax : nullptr, s));
  unsigned int herr = 0, habs = 0;
  double mnew = inf;
  HIPCHK(hipMemcpyAsync(&herr, derr, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&habs, ix->d_absmax, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&mnew, tmp_mmin, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float amax = 0.0f;
  memcpy(&amax, &habs, 4);
  // a signed index's shifted rows need every |value| <= B
  const bool beyond = sgn && amax > ix->sbound;
  if (herr || beyond) {
    // leave the unused leaf slots zero, as they were
    HIPCHK(hipMemsetAsync(ix->leaves + lo * dp, 0, (size_t)n_new * dp * 4, s));
    HIPCHK(hipMemsetAsync(ix->ff + lo, 0, (size_t)n_new * 8, s));
    HIPCHK(hipMemsetAsync(ix->invn + lo, 0, (size_t)n_new * 4, s));
    HIPCHK(hipMemsetAsync(ix->nf + lo, 0, (size_t)n_new * 4, s));
    HIPCHK(hipStreamSynchronize(s));
    if (herr)
      return fail(GT_ERR_INVALID_INPUT, sgn ? "inserted rows contain a NaN or infinite value"
                                            : "inserted rows contain a NaN, infinite or negative value");
    return fail(GT_ERR_INVALID_INPUT, "an inserted value exceeds the index's shift bound " +
                                          std::to_string(ix->sbound) + " in absolute value");
  }
  // A float8 level that must be rescaled is rewritten whole; calls in flight
  // on other streams must not read it meanwhile, so the device is drained
  // first when float8 pools exist.  Float32 and bfloat16 pools only grow
  // (upward-rounded sums of non-negative rows), which in-flight calls tolerate.
  if (ix->pfp8) HIPCHK(hipDeviceSynchronize());
  // pools on the root-to-leaf paths of the new rows, re-derived bottom-up
  for (int l = ix->depth - 1; l >= 0; --l) {
    const int sh = ix->depth - l;
    const int64_t a = lo >> sh, b = (hi - 1) >> sh;
    float* par = ix->master ? ix->master + level_row(l) * dp : nullptr;
    if (par) {
      const float* child = (l == ix->depth - 1) ? ix->leaves : ix->master + level_row(l + 1) * dp;
      HIPCHK(gt::launch_build_level(child, par, b - a + 1, ix->dp, a, s, false));
    }
    if (ix->mmax) {
      float* mpar = ix->mmax + level_row(l) * pw;
      if (sgn && l == ix->depth - 1) {
        HIPCHK(gt::launch_signed_bottom(ix->leaves, mpar, a, b - a + 1, ix->dp, ix->d, hi,
                                        ix->sbound, s));
      } else {
        const float* mchild = (l == ix->depth - 1) ? ix->leaves : ix->mmax + level_row(l + 1) * pw;
        HIPCHK(gt::launch_build_level(mchild, mpar, b - a + 1, ix->pw, a, s, true));
      }
      if (ix->pmax16)
        HIPCHK(gt::launch_quant_bf16(mpar + a * pw, ix->pmax16 + (level_row(l) + a) * pw,
                                     (b - a + 1) * ix->pw, s));
    }
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
  if (!ix) return fail(GT_ERR_INVALID_ARG, "index is NULL");
  if (!total_out) return fail(GT_ERR_INVALID_ARG, "total_out is NULL");
  if (!offsets_dev) return fail(GT_ERR_INVALID_ARG, "offsets is NULL");
  if (max_results < 0) return fail(GT_ERR_INVALID_ARG, "max_results < 0");
  if (max_results > 0 && (!ids_dev || !sims_dev)) return fail(GT_ERR_INVALID_ARG, "NULL output buffer");
  set_targets(ix->def, max_results, ids_dev, sims_dev);
  TRY(submit(ix, ix->def, 1, q_dev, nq, rho_host, (int)fmt, (hipStream_t)stream));
  return finish(ix, ix->def, max_results, offsets_dev, ids_dev, sims_dev, total_out, false);
}

gt_status gt_exhaustive(gt_index* ix, const float* q_dev, int32_t nq, const double* rho_host,
                        int64_t max_results, int64_t* offsets_dev, int64_t* ids_dev,
                        float* sims_dev, int64_t* total_out, void* stream) {
  g_err.clear();
  if (!ix) return fail(GT_ERR_INVALID_ARG, "index is NULL");
  if (!total_out) return fail(GT_ERR_INVALID_ARG, "total_out is NULL");
  if (!offsets_dev) return fail(GT_ERR_INVALID_ARG, "offsets is NULL");
  if (max_results < 0) return fail(GT_ERR_INVALID_ARG, "max_results < 0");
  if (max_results > 0 && (!ids_dev || !sims_dev)) return fail(GT_ERR_INVALID_ARG, "NULL output buffer");
  set_targets(ix->def, max_results, ids_dev, sims_dev);
  TRY(submit(ix, ix->def, 2, q_dev, nq, rho_host, 0, (hipStream_t)stream));
  return finish(ix, ix->def, max_results, offsets_dev, ids_dev, sims_dev, total_out, false);
}

gt_status gt_query_batch_noalloc(gt_index* ix, const float* q_dev, int32_t nq,
                                 const double* rho_host, gt_pool fmt, int64_t max_results,
                                 int64_t* offsets_dev, int64_t* ids_dev, float* sims_dev,
                                 int64_t* total_out, void* stream) {
  g_err.clear();
  if (!ix) return fail(GT_ERR_INVALID_ARG, "index is NULL");
  if (!total_out) return fail(GT_ERR_INVALID_ARG, "total_out is NULL");
  if (!offsets_dev) return fail(GT_ERR_INVALID_ARG, "offsets is NULL");
  if (max_results < 0) return fail(GT_ERR_INVALID_ARG, "max_results < 0");
  if (max_results > 0 && (!ids_dev || !sims_dev)) return fail(GT_ERR_INVALID_ARG, "NULL output buffer");
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != ix->device) return fail(GT_ERR_INVALID_ARG, "the index's device must be current");
  void* base = gt::scratch_of(ix->device);
  if (!base)
    return fail(GT_ERR_DEVICE, std::string("device scratch was not set up: ") +
                                   hipGetErrorString(ix->scratch_err));
  if (nq < 0) return fail(GT_ERR_INVALID_ARG, "nq < 0");
  // buffers carved from the device's scratch; the host copy of the counters
  // lives on this stack frame (pageable)
  Batch fb;
  gt::DevCounters host_ctr;
  TRY(carve_fixed(ix, &fb, base, gt::kScratchBytes, nq, (int)fmt));
  fb.h_ctr = &host_ctr;
  set_targets(&fb, max_results, ids_dev, sims_dev);
  TRY(submit(ix, &fb, 1, q_dev, nq, rho_host, (int)fmt, (hipStream_t)stream));
  const gt_status st = finish(ix, &fb, max_results, offsets_dev, ids_dev, sims_dev, total_out, false);
  // the copies out of the scratch are done before the next call may reuse it
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return st;
}

gt_status gt_batch_create(gt_index* ix, int32_t max_queries, gt_batch** out) {
  g_err.clear();
  if (!ix || !out) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (max_queries < 1 || max_queries > gt::kMaxTiles * gt::kQueriesPerTileF32)
    return fail(GT_ERR_INVALID_ARG, "max_queries out of range");
  gt_batch* b = new gt_batch();
  b->ix = ix;
  b->max_queries = max_queries;
  gt_status st = batch_init(b);
  const int nq_pad = (max_queries + 127) / 128 * 128;
  const int nt = (max_queries + gt::kQueriesPerTileF32 - 1) / gt::kQueriesPerTileF32;
  if (st == GT_OK) st = batch_reserve(b, nq_pad, nt);
  if (st != GT_OK) {
    std::string keep = g_err;
    free_batch(b);
    delete b;
    g_err = keep;
    return st;
  }
  *out = b;
  return GT_OK;
}

gt_status gt_call_bytes(const gt_index* cix, int32_t nq, gt_pool fmt, int64_t frontier_entries,
                        int64_t pairs, int64_t* bytes_out, int64_t* min_bytes_out) {
  g_err.clear();
  if (!cix || !bytes_out) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  if (nq < 1 || nq > gt::kMaxTiles * gt::kQueriesPerTileF32) return fail(GT_ERR_INVALID_ARG, "nq out of range");
  if (frontier_entries < 0 || pairs < 0) return fail(GT_ERR_INVALID_ARG, "negative capacity");
  Index* ix = const_cast<gt_index*>(cix);
  const CallShape c = call_shape(ix, nq, (int)fmt);
  const CallShape c1 = call_shape(ix, std::min(nq, c.tq), (int)fmt);
  const int64_t worst = int64_t(1) << std::max(0, ix->depth - 1);
  const size_t per = kPerEntry + (c.want_rec ? kPerRecord : 0);
  const size_t slack = 24 * 256;
  const size_t pr = (size_t)std::max<int64_t>(pairs, 1024) * kPerPair;
  // Entries fall only into subtrees that hold rows (rows fill the tree from
  // the left), while every subtree's slot gets the same room: scale by the
  // populated share of the 2^7 subtrees.  At least 64 entries per slot
  // (small calls spread their entries unevenly).
  const int64_t nbk = int64_t(1) << gt::kMaxBucketBits;
  const int64_t span = std::max<int64_t>(1, ix->cap / nbk);
  const int64_t populated = std::max<int64_t>(1, std::min<int64_t>(nbk, (ix->n + span - 1) / span));
  const int64_t per_tile = (frontier_entries + c.nt - 1) / c.nt;
  const int64_t floor_cap = std::min<int64_t>(worst, int64_t(64) << gt::kMaxBucketBits);
  const int64_t fr_cap = std::max<int64_t>(
      floor_cap, std::min<int64_t>(worst, (per_tile * nbk + populated - 1) / populated));
  const size_t want = common_bytes(ix, nq, c) + pr + (size_t)c.nt * (size_t)fr_cap * per + slack;
  const size_t min_first = common_bytes(ix, nq, c) + pr + (size_t)c.nt * 64 * per + slack;
  const size_t min_cont = common_bytes(ix, std::min(nq, c.tq), c1) + pr + (size_t)worst * kPerEntry + slack;
  const size_t mn = std::max(min_first, min_cont);
  *bytes_out = (int64_t)std::max(want, mn);
  if (min_bytes_out) *min_bytes_out = (int64_t)mn;
  return GT_OK;
}

gt_status gt_batch_create_external(gt_index* ix, int32_t max_queries, gt_batch** out) {
  g_err.clear();
  if (!ix || !out) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (max_queries < 1 || max_queries > gt::kMaxTiles * gt::kQueriesPerTileF32)
    return fail(GT_ERR_INVALID_ARG, "max_queries out of range");
  gt_batch* b = new gt_batch();
  b->ix = ix;
  b->external = true;
  b->max_queries = max_queries;
  b->ext_max_queries = max_queries;
  hipError_t e = hipHostMalloc((void**)&b->h_ctr, sizeof(gt::DevCounters), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    free_batch(b);
    delete b;
    return fail(GT_ERR_DEVICE, std::string("workspace set-up: ") + hipGetErrorString(e));
  }
  *out = b;
  return GT_OK;
}

gt_status gt_batch_submit_external(gt_batch* b, const float* q_dev, int32_t nq,
                                   const double* rho_host, gt_pool fmt, void* mem_dev,
                                   int64_t mem_bytes, int64_t pairs, void* stream) {
  g_err.clear();
  if (!b) return fail(GT_ERR_INVALID_ARG, "batch is NULL");
  if (!b->external) return fail(GT_ERR_INVALID_ARG, "not an external workspace");
  if (b->pending) return fail(GT_ERR_INVALID_ARG, "the workspace has a call in flight");
  Index* ix = b->ix;
  if (nq < 1) return fail(GT_ERR_INVALID_ARG, "nq < 1");
  if (nq > b->ext_max_queries)
    return fail(GT_ERR_CAPACITY, "batch of " + std::to_string(nq) + " queries exceeds the workspace's " +
                                     std::to_string(b->ext_max_queries));
  if (!q_dev || !rho_host || !mem_dev) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(mem_dev) % 256) return fail(GT_ERR_INVALID_ARG, "memory not 256-byte aligned");
  if (pairs < 0 || mem_bytes < 0) return fail(GT_ERR_INVALID_ARG, "negative size");
  int64_t need = 0, mn = 0;
  TRY(gt_call_bytes(static_cast<gt_index*>(ix), nq, fmt, 0, pairs, &need, &mn));
  if (mem_bytes < mn)
    return fail(GT_ERR_CAPACITY, "a call of " + std::to_string(nq) + " queries needs at least " +
                                     std::to_string(mn) + " bytes of workspace memory (given " +
                                     std::to_string(mem_bytes) + ")");
  b->q_in = q_dev;
  b->rho_in.assign(rho_host, rho_host + nq);
  b->user_fmt = (int)fmt;
  b->ext_mem = static_cast<unsigned char*>(mem_dev);
  b->ext_bytes = (size_t)mem_bytes;
  b->ext_pairs = std::max<int64_t>(pairs, 1024);
  b->cont_again = false;
  b->continued_tiles = 0;
  b->ext_epoch = ix->n;
  TRY(carve_budget(ix, b, mem_dev, (size_t)mem_bytes, nq, (int)fmt, b->ext_pairs, true));
  set_targets(b, 0, nullptr, nullptr);
  return submit(ix, b, 1, q_dev, nq, b->rho_in.data(), (int)fmt, (hipStream_t)stream);
}

gt_status gt_batch_info(const gt_batch* b, int64_t* max_level_entries, int64_t* results,
                        int32_t* continued_tiles) {
  g_err.clear();
  if (!b) return fail(GT_ERR_INVALID_ARG, "batch is NULL");
  if (max_level_entries) *max_level_entries = b->last_max_entries;
  if (results) *results = b->last_results;
  if (continued_tiles) *continued_tiles = b->continued_tiles;
  return GT_OK;
}

gt_status gt_batch_submit(gt_batch* b, const float* q_dev, int32_t nq, const double* rho_host,
                          gt_pool fmt, void* stream) {
  g_err.clear();
  if (!b) return fail(GT_ERR_INVALID_ARG, "batch is NULL");
  if (b->external) return fail(GT_ERR_INVALID_ARG, "an external workspace takes gt_batch_submit_external");
  if (!b->pending) set_targets(b, 0, nullptr, nullptr);
  return submit(b->ix, b, 1, q_dev, nq, rho_host, (int)fmt, (hipStream_t)stream);
}

gt_status gt_batch_poll(gt_batch* b, int32_t* done_out) {
  g_err.clear();
  if (!b || !done_out) return fail(GT_ERR_INVALID_ARG, "NULL argument");
  if (!b->pending) return fail(GT_ERR_INVALID_ARG, "no call in flight on this workspace");
  const hipError_t e = hipEventQuery(b->done);
  if (e == hipSuccess) {
    *done_out = 1;
  } else if (e == hipErrorNotReady) {
    *done_out = 0;
  } else {
    return fail(GT_ERR_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
  }
  return GT_OK;
}

gt_status gt_batch_finish(gt_batch* b, int64_t max_results, int64_t* offsets_dev, int64_t* ids_dev,
                          float* sims_dev, int64_t* total_out) {
  g_err.clear();
  if (!b) return fail(GT_ERR_INVALID_ARG, "batch is NULL");
  return finish(b->ix, b, max_results, offsets_dev, ids_dev, sims_dev, total_out, true);
}

void gt_batch_destroy(gt_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_batch(b);
  delete b;
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
  out->pool_formats = ix->formats;
  out->m_min = ix->m_min;
  out->epoch = ix->epoch;
  out->bytes_device = ix->bytes;
  for (int l = 0; l < GT_MAX_LEVELS; ++l) out->fp8_exp[l] = ix->lexp[l];
  const Batch* b = ix->def;
  out->last_nq = b->last_nq;
  out->last_tiles = b->last_nt;
  out->last_format = b->last_fmt;
  out->head_level = b->last_nt > 0 && b->last_head >= 0 ? b->last_head : head_of(ix);
  if (b->ctr && b->last_nt > 0) {
    HIPCHK(hipDeviceSynchronize());
    std::vector<uint32_t> cnt((size_t)GT_MAX_LEVELS * gt::kMaxSlots);
    HIPCHK(hipMemcpy(cnt.data(), b->lvl_count, cnt.size() * 4, hipMemcpyDeviceToHost));
    gt::DevCounters c;
    HIPCHK(hipMemcpy(&c, b->ctr, sizeof(c), hipMemcpyDeviceToHost));
    for (int l = 0; l < ix->depth && l < GT_MAX_LEVELS; ++l) {
      int64_t e = 0;
      for (int k = 0; k < gt::kMaxSlots; ++k) e += cnt[(size_t)l * gt::kMaxSlots + k];
      out->entries[l] = e;
      out->pairs[l] = (int64_t)c.pairs[l];
    }
    out->leaf_pairs = (int64_t)c.leaf_pairs;
    out->candidates = (int64_t)c.nhits;
    out->rechecked = (int64_t)c.rechecked;
    out->results = (int64_t)c.total;
    if (b->counted && b->bitmap) {
      std::vector<uint32_t> bm((size_t)b->bitmap_words);
      HIPCHK(hipMemcpy(bm.data(), b->bitmap, bm.size() * 4, hipMemcpyDeviceToHost));
      for (int l = 0; l <= ix->depth && l < GT_MAX_LEVELS; ++l) {
        int64_t k = 0;
        for (int64_t r = level_row(l); r < level_row(l + 1); ++r) k += (bm[r >> 5] >> (r & 31)) & 1u;
        out->unique_rows[l] = k;
      }
    }
  }
  out->ms_prep = b->ms[0];
  out->ms_frontier = b->ms[1];
  out->ms_leaf = b->ms[2];
  out->ms_recheck = b->ms[3];
  out->ms_compact = b->ms[4];
  out->ms_gemm = b->ms[5];
  out->ms_total = b->ms[6];
  out->ms_dense = b->ms[7];
  out->frontier_launches = b->frontier_launches;
  out->dense_launches = b->dense_launches;
  out->pool_width = ix->pw;
  out->shift_bound = ix->signed_mode ? ix->sbound : 0.0f;
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
  if (!(ix->formats & (uint32_t)f) ||
      (level == ix->depth && f != GT_POOL_F32 && f != GT_POOL_MAX_F32))
    return fail(GT_ERR_INVALID_ARG, "format not available for this level");
  const size_t esz = (f == GT_POOL_F32 || f == GT_POOL_MAX_F32) ? 4
                     : (f == GT_POOL_BF16 || f == GT_POOL_MAX_BF16) ? 2 : 1;
  const bool mx = f == GT_POOL_MAX_F32 || f == GT_POOL_MAX_BF16;
  const size_t w = (mx && level < ix->depth) ? (size_t)ix->pw : (size_t)ix->dp;
  const size_t off = (size_t)level_row(level) * w;
  const unsigned char* base =
      level == ix->depth     ? (const unsigned char*)ix->leaves
      : f == GT_POOL_F32     ? (const unsigned char*)(ix->master + off)
      : f == GT_POOL_BF16    ? (const unsigned char*)(ix->pbf16 + off)
      : f == GT_POOL_MAX_F32 ? (const unsigned char*)(ix->mmax + off)
      : f == GT_POOL_MAX_BF16 ? (const unsigned char*)(ix->pmax16 + off)
                              : (const unsigned char*)(ix->pfp8 + off);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(host_out, base + (size_t)first * w * esz, (size_t)count * w * esz,
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
  } else if (!strcmp(key, "dense_last")) {
    if (value < -2 || value > ix->depth - 1) return fail(GT_ERR_INVALID_ARG, "dense_last out of range");
    ix->dense_last = (int)value;
  } else if (!strcmp(key, "dense_start")) {
    if (value < -1 || value > ix->depth - 1) return fail(GT_ERR_INVALID_ARG, "dense_start out of range");
    ix->dense_start = (int)value;
  } else if (!strcmp(key, "walk_subtract")) {
    if (value < -1 || value > 2) return fail(GT_ERR_INVALID_ARG, "walk_subtract out of range");
    ix->walk_subtract = (int)value;
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
  if (ix->def) {
    free_batch(ix->def);
    delete static_cast<gt_batch*>(ix->def);
  }
  free_tree(ix);
  delete ix;
}

}  // extern "C"
