/*
 * gt.h -- exact range search by adaptive group testing (binary splitting with
 * sum pools) on one AMD MI355X (gfx950).
 *
 * Problem (paper Sec. 1): given database vectors f_1..f_N in R^d, a query q and
 * a threshold rho, return every i with sim(q, f_i) >= rho.  Similarity is the
 * cosine; the paper works with non-negative unit vectors, for which it is the
 * dot product (Sec. 2).  Method (Sec. 2, Alg. 1): a pool is the sum of its
 * members; because every term q_k * f_ik is non-negative, a pool whose score is
 * below the threshold holds no neighbour and is discarded whole, and surviving
 * pools are halved down to single vectors, which get an exact test.  The
 * method is exact: its result is the brute-force set.
 *
 * Conventions for every entry point:
 *  - Returns a gt_status; nothing is thrown across this interface.  On any
 *    error the index is left as it was.  gt_last_error() gives a message for
 *    the calling thread.
 *  - Pointers named *_dev are device pointers (HIP device memory on the
 *    current device); *_host are host pointers.  Inputs are borrowed and read
 *    in stream order: the caller keeps them alive until `stream` reaches the
 *    call.  Outputs are caller-owned device buffers.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are asynchronous except where a host value is returned (documented).
 *  - One host thread may use an index at a time.
 *  - Matrices are row-major with row stride d (elements).
 */
#ifndef GT_H
#define GT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gt_index gt_index; /* opaque, owned by the library */
typedef struct gt_batch gt_batch; /* opaque per-call device workspace */

typedef enum {
  GT_OK = 0,
  GT_ERR_INVALID_ARG = 1,      /* bad size, pointer, dtype or format */
  GT_ERR_INVALID_INPUT = 2,    /* a NaN, infinite or negative value (the prune
                                  rule needs non-negative vectors, Sec. 2); for an
                                  index built with GT_POOL_SIGNED, a NaN or
                                  infinite value, or an inserted value beyond
                                  the index's shift bound */
  GT_ERR_OUT_OF_MEMORY = 3,
  GT_ERR_CAPACITY = 4,         /* insert beyond the capacity given at build */
  GT_ERR_RESULT_OVERFLOW = 5,  /* more results than max_results; see queries */
  GT_ERR_DEVICE = 6            /* a HIP runtime error */
} gt_status;

typedef enum { GT_F32 = 0, GT_F16 = 1, GT_BF16 = 2 } gt_dtype; /* feature storage */

/* Pool storage formats.  Pool sums are kept as float32 master values rounded
 * upward; the reduced formats are upward-rounded copies (bfloat16, and float8
 * e4m3 with one power-of-two scale per tree level).  The MAX formats are a
 * second tree whose pools are the element-wise maximum of their members
 * (paper Sec. 2, Our-Max: a query scores a max pool at least as high as any
 * member, so the same prune rule holds), float32 (exact) and a bfloat16 copy
 * rounded upward; asking for GT_POOL_MAX_BF16 also builds GT_POOL_MAX_F32.
 * Bit mask at build time, one value per query call.
 *
 * GT_POOL_SIGNED (build-time flag only): vectors and queries may have values
 * of any sign (paper Sec. 2, negative descriptors: a pool keeps the
 * element-wise maximum and minimum of its members and a query scores it with
 * the maximum where its component is >= 0 and the minimum where it is < 0,
 * which bounds every member's dot product from above).  Sums no longer bound
 * anything, so such an index keeps only the MAX formats (GT_POOL_MAX_F32
 * always, GT_POOL_MAX_BF16 if asked; asking for a sum format is INVALID_ARG).
 * Their rows are 2 x d_pad wide: pool row [max_k + B | B - min_k] over the
 * members (columns k < d; zero past d and for a pool without members), B the
 * smallest power of two >= the largest |value| at build (1 for an all-zero
 * build), the additions rounded up.  A query q is walked as [max(q,0) |
 * max(-q,0)] against the threshold tau + B |q|_1: the same test as the
 * max/min score against tau, with every operand non-negative.  Limits: every
 * rho > 0 (also for gt_exhaustive on such an index); inserted values must lie
 * in [-B, B]. */
typedef enum {
  GT_POOL_F32 = 1,
  GT_POOL_BF16 = 2,
  GT_POOL_FP8E4M3 = 4,
  GT_POOL_MAX_F32 = 8,
  GT_POOL_MAX_BF16 = 16,
  GT_POOL_SIGNED = 32
} gt_pool;

#define GT_MAX_LEVELS 40

typedef struct {
  int64_t n;              /* vectors currently indexed (ids 0..n-1) */
  int64_t capacity;       /* leaves of the tree (power of two) */
  int32_t d, d_pad;       /* dimension and padded row length */
  int32_t depth;          /* log2(capacity): leaves are at this level */
  int32_t head_level;     /* pools of this level are all taken as live; tests start
                           * at its children (the last call's, else the index default) */
  uint32_t pool_formats;
  double m_min;           /* smallest norm over non-zero rows */
  uint64_t epoch;         /* bumped by every successful insert */
  int64_t bytes_device;   /* device memory held by the index */
  /* last gt_query_batch / gt_exhaustive call */
  int32_t last_nq, last_tiles, last_format;
  int64_t entries[GT_MAX_LEVELS]; /* (tile, pool) frontier entries per level */
  int64_t pairs[GT_MAX_LEVELS];   /* (query, pool) tests per level */
  int64_t leaf_pairs;     /* (query, vector) exact tests */
  int64_t candidates;     /* leaf tests that passed or fell in the recheck band */
  int64_t rechecked;      /* candidates re-decided in float64 */
  int64_t results;        /* total neighbours returned */
  /* device time of the last call, per kernel group, from HIP events on the
   * call's stream; zero unless profiling is on (gt_set_option "profile") */
  double ms_prep, ms_frontier, ms_leaf, ms_recheck, ms_compact, ms_gemm, ms_total;
  int32_t frontier_launches;
  int32_t fp8_exp[GT_MAX_LEVELS]; /* float8 pools of level l are code * 2^fp8_exp[l] */
  /* distinct rows of each level read by the last gt_query_batch (level depth =
   * leaves); filled only while option "count_unique" is on */
  int64_t unique_rows[GT_MAX_LEVELS];
  int32_t dense_launches;  /* dense level steps of the last gt_query_batch */
  double ms_dense;         /* their device time (profiling on) */
  int32_t pool_width;      /* row length of the MAX pools: d_pad, or 2 d_pad with
                            * GT_POOL_SIGNED */
  float shift_bound;       /* B of a GT_POOL_SIGNED index, else 0 */
} gt_stats;

/* Build the index (paper Sec. 2: pools of the binary-splitting tree, created
 * offline; explicit pool sums replace the prefix sums of Eq. 1).
 *   feats_dev  [n x d] features of type `dtype`; every value finite and >= 0
 *              (finite, of any sign, with GT_POOL_SIGNED).
 *   capacity   number of leaves; 0 = smallest power of two >= n, else a power
 *              of two >= n.  Room for later inserts.
 *   pool_formats  bit mask of gt_pool (GT_POOL_F32 is always built).
 * Copies the features; the index owns all its device memory until
 * gt_destroy.  Synchronises `stream` (validation result).  Errors:
 * INVALID_ARG (d < 1 or d > 4096, n < 0, n > capacity, capacity not a power of
 * two, dtype; with GT_POOL_SIGNED: a sum format asked for),
 * INVALID_INPUT, OUT_OF_MEMORY, DEVICE. */
gt_status gt_build_tree(const void* feats_dev, int64_t n, int32_t d, gt_dtype dtype,
                        int64_t capacity, uint32_t pool_formats, void* stream,
                        gt_index** out);

/* Append n_new vectors (paper Sec. 4, streaming setting: the database grows
 * between queries).  Ids n..n+n_new-1 are assigned in order; *first_id_out
 * (host, may be NULL) receives n.  Every pool on a root-to-leaf path of a new
 * vector is re-derived from its two children, so the index equals one built
 * from scratch over the same rows.  Queries issued after this call returns see
 * the new vectors.  Synchronises `stream`.  Errors: CAPACITY (n + n_new >
 * capacity), INVALID_INPUT (index unchanged), DEVICE. */
gt_status gt_insert(gt_index* index, const void* feats_dev, int64_t n_new, void* stream,
                    int64_t* first_id_out);

/* Range query by the level-wise binary-splitting walk (paper Sec. 2, Alg. 1,
 * visited one level per round as analysed in Sec. 4).
 *   q_dev      [nq x d] float32 queries, finite and >= 0 (finite, of any
 *              sign, on a GT_POOL_SIGNED index).
 *   rho_host   [nq] float64 thresholds.  rho <= 0 returns every non-zero row
 *              (INVALID_ARG on a GT_POOL_SIGNED index, where it must be > 0).
 *   fmt        pool format for the walk (must have been built).
 *   offsets_dev [nq + 1] int64: query b's results are ids[offsets[b] ..
 *              offsets[b+1]).
 *   ids_dev    [max_results] int64, ascending within each query.
 *   sims_dev   [max_results] float32 cosines: the float32 value, or the
 *              float64 value rounded to float32 where it was re-decided.
 *   total_out  host: number of results.
 * Membership is decided exactly as the float64 definition
 *   cos = dot / (sqrt(qq) * sqrt(ff)),  sums sequential over k,
 * so the id sets equal a float64 brute-force scan; a zero query or row never
 * matches.  Synchronises `stream` once (result count).  On
 * GT_ERR_RESULT_OVERFLOW, *total_out holds the required max_results and
 * offsets_dev is valid; ids/sims are not written.  Other errors:
 * INVALID_ARG (format not built), INVALID_INPUT (a NaN/Inf/negative query
 * value), OUT_OF_MEMORY, DEVICE.  Every d <= 4096 and every pool format is
 * served; rows of more than 1152 padded columns (2304 for float8) stream the
 * queries through on-chip memory in windows and take no subtraction step. */
gt_status gt_query_batch(gt_index* index, const float* q_dev, int32_t nq, const double* rho_host,
                         gt_pool fmt, int64_t max_results, int64_t* offsets_dev, int64_t* ids_dev,
                         float* sims_dev, int64_t* total_out, void* stream);

/* Exhaustive baseline (the paper's Exh, Sec. 4): every (query, vector) dot
 * product by a float32 matrix-core GEMM with a threshold epilogue, followed by
 * the same exact test as gt_query_batch, so results are identical to it.
 * Arguments, synchronisation and errors as gt_query_batch. */
gt_status gt_exhaustive(gt_index* index, const float* q_dev, int32_t nq, const double* rho_host,
                        int64_t max_results, int64_t* offsets_dev, int64_t* ids_dev,
                        float* sims_dev, int64_t* total_out, void* stream);

/* gt_query_batch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, results and errors as gt_query_batch, but every per-call
 * buffer (query copies, frontiers, counters, candidates, result staging) is
 * carved out of one fixed device array of 256 MiB that the library holds per
 * device until the process ends; the call makes no hipMalloc or hipFree.  The
 * frontier is reserved for its worst case (every pool of the deepest level
 * for every query tile: 24 * 2^(depth-1) bytes per tile of 64 queries, 32 for
 * float32 pools), so a call that does not fit, or whose candidates or results
 * outgrow the rest of the array, fails with GT_ERR_CAPACITY and a message
 * naming the limit (use fewer queries per call).  Without room for the
 * subtraction step's score records the bfloat16 walk tests both children
 * directly (same results).  Every call on a device shares the array, which
 * keeps the last call's contents (a call clears what must start at zero):
 * calls that overlap on one device, from several threads or streams, race.
 * The index's device must be current.  Synchronises `stream` before
 * returning.  No profiling or count_unique counters. */
gt_status gt_query_batch_noalloc(gt_index* index, const float* q_dev, int32_t nq,
                                 const double* rho_host, gt_pool fmt, int64_t max_results,
                                 int64_t* offsets_dev, int64_t* ids_dev, float* sims_dev,
                                 int64_t* total_out, void* stream);

/* Device workspace for one query call at a time, so that several calls can
 * be in flight on different streams (continuous batching: a server admits
 * newly arrived requests into a free workspace while others are still on the
 * device, and their kernels overlap).  gt_query_batch uses the index's own
 * workspace; these use a caller-made one.
 *   gt_batch_create  max_queries = the largest call (1 .. 32768); allocates
 *                    the workspace (frontiers sized for the index depth).
 *   gt_batch_submit  enqueues the whole walk of gt_query_batch on `stream`
 *                    and returns without waiting; arguments as there.  The
 *                    call sees the vectors indexed at submit time (ids below
 *                    gt_stats.n then).  Errors: INVALID_ARG (a call already in
 *                    flight on this workspace, format), CAPACITY (nq above
 *                    max_queries), DEVICE.
 *   gt_batch_poll    *done_out = 1 once the device has reached the result
 *                    count of the call in flight (non-blocking).
 *   gt_batch_finish  completes the call as gt_query_batch does (waits,
 *                    writes offsets, ids, sims; same errors) and frees the
 *                    workspace for the next call.  On RESULT_OVERFLOW the
 *                    call stays in flight with its results kept: *total_out
 *                    and offsets are written, and gt_batch_finish may be
 *                    called again with max_results >= *total_out (nothing is
 *                    recomputed).
 * Inserts may run between submit and finish: the call keeps its epoch, and
 * float32 / bfloat16 pools only grow, which keeps its pruning sound; with
 * float8 pools built, gt_insert first waits for the device.  One host thread
 * drives the index and its workspaces. */
gt_status gt_batch_create(gt_index* index, int32_t max_queries, gt_batch** out);
gt_status gt_batch_submit(gt_batch* batch, const float* q_dev, int32_t nq, const double* rho_host,
                          gt_pool fmt, void* stream);
gt_status gt_batch_poll(gt_batch* batch, int32_t* done_out);
gt_status gt_batch_finish(gt_batch* batch, int64_t max_results, int64_t* offsets_dev,
                          int64_t* ids_dev, float* sims_dev, int64_t* total_out);
void gt_batch_destroy(gt_batch* batch);

/* Admission by memory (continuous batching, paper Sec. 4 streaming setting):
 * workspaces whose device memory the caller hands to each call, so that a
 * server can hold one device arena and admit a call only while its memory
 * fits.  Such a call's frontier gets what its memory leaves after its other
 * buffers -- a budget, not the worst case -- and its kernels check every
 * frontier write against it.  When a level outgrows the budget (or the
 * candidates outgrow `pairs`), gt_batch_finish runs the call again one query
 * tile (64 queries; 32 for float32 pools) at a time, each tile with the whole
 * memory, which always holds one tile's worst case (the submit checks it):
 * the results are the same, only later.
 *
 * gt_call_bytes  device bytes for a call of nq queries in format fmt with room
 *                for frontier_entries entries per frontier level (all tiles
 *                together, spread over the subtrees that hold rows; 0 = the
 *                least) and `pairs` leaf candidates and results (at least
 *                1024).  *min_bytes_out (may be NULL): the
 *                least memory any such call accepts.  bf16 sum-pool calls
 *                with a dense step keep 280 bytes per frontier entry
 *                (subtraction-step score records), others 24.
 * gt_batch_create_external  a workspace without device memory of its own
 *                (an event and pinned counters only); calls up to max_queries.
 * gt_batch_submit_external  as gt_batch_submit, with the call's device
 *                memory [mem_dev, mem_dev + mem_bytes) (256-byte aligned,
 *                owned by the caller, not touched by anything else until
 *                gt_batch_finish returns) and its candidate room `pairs`.  The
 *                queries q_dev must stay valid until gt_batch_finish returns
 *                (a continuation reads them again).  Errors: CAPACITY
 *                (mem_bytes below the call's least, nq above max_queries),
 *                INVALID_ARG, DEVICE.
 *   gt_batch_poll / gt_batch_finish / gt_batch_destroy as for any workspace;
 *   after a result overflow of a continued call, the next finish runs its
 *   tiles again.  A tile whose candidates outgrow `pairs` fails with CAPACITY.
 * gt_batch_info  of the workspace's last finished call: the largest number
 *                of frontier entries at any level, the results, and how many
 *                tiles ran one by one (0: the call fitted its memory).  Any
 *                output may be NULL. */
gt_status gt_call_bytes(const gt_index* index, int32_t nq, gt_pool fmt, int64_t frontier_entries,
                        int64_t pairs, int64_t* bytes_out, int64_t* min_bytes_out);
gt_status gt_batch_create_external(gt_index* index, int32_t max_queries, gt_batch** out);
gt_status gt_batch_submit_external(gt_batch* batch, const float* q_dev, int32_t nq,
                                   const double* rho_host, gt_pool fmt, void* mem_dev,
                                   int64_t mem_bytes, int64_t pairs, void* stream);
gt_status gt_batch_info(const gt_batch* batch, int64_t* max_level_entries, int64_t* results,
                        int32_t* continued_tiles);

/* Counters of the index and of its last query call.  Synchronises the device
 * stream of the last call.  Errors: INVALID_ARG. */
gt_status gt_get_stats(const gt_index* index, gt_stats* out);

/* Copies stored pool sums of one tree level to host memory (inspection and
 * tests).  level in [0, depth]; level == depth gives the float32 leaf rows.
 * Rows first .. first+count-1 of the level, each d_pad values:
 *   GT_POOL_F32 -> float32 master sums (upward-rounded, >= the exact sums),
 *   GT_POOL_BF16 -> uint16 bfloat16 codes, GT_POOL_FP8E4M3 -> uint8 e4m3 codes
 *   (value = decoded code * 2^fp8_exp[level], see gt_stats),
 *   GT_POOL_MAX_F32 -> float32 element-wise maxima (exact; level == depth gives
 *   the leaf rows), GT_POOL_MAX_BF16 -> their bfloat16 codes, rounded up; on a
 *   GT_POOL_SIGNED index the MAX rows are the shifted max/min rows described
 *   at gt_pool, pool_width (= 2 d_pad) values each.
 * host_out must hold count * d_pad elements of that type (count * pool_width
 * for MAX rows below the leaves).  Synchronises the
 * device.  Errors: INVALID_ARG (range, format not built), DEVICE. */
gt_status gt_read_pools(const gt_index* index, int32_t level, int64_t first, int64_t count,
                        gt_pool fmt, void* host_out);

/* Runtime knobs (benchmarking and tests; results never depend on them):
 *   "profile"     0/1: time kernel groups with HIP events (gt_stats.ms_*)
 *   "head_level"  level whose pools are all taken as live, 0..depth-1; tests
 *                 start at level head_level + 1 (-1 = automatic: with dense
 *                 steps only the last dense level is tested)
 *   "grid"        workgroups of the persistent walk kernels (0 = one per CU)
 *   "dense_last"  last level tested with dense steps, every pool against every
 *                 query (-2 = automatic, -1 = none; bf16 and fp8 pools only).
 *                 Automatic: the level whose pools hold about 16 populated
 *                 rows; for rows of 512 or more columns each workspace then
 *                 moves it from call to call by the frontier density its last
 *                 call of the same format met (deeper while the entries of a
 *                 level fill more than 4.6e-4 x row length of its populated
 *                 (pool, query tile) pairs)
 *   "dense_start" the automatic dense level's level for a workspace's first
 *                 call, before it has measured a frontier (-1 = the fixed
 *                 rule above); a cost model's prediction (paper Sec. 5, Eq. 3)
 *                 goes here
 *   "walk_subtract" subtraction step of the bf16 walk after a dense step (paper
 *                 Sec. 2, Alg. 1: one dot product per split, the other half
 *                 bounded by the pool's score minus it): 0 off, 1 every sparse
 *                 level, 2 all but the last, -1 automatic (= 1).  Each frontier
 *                 entry then carries 64 bf16 score bounds (128 bytes).
 *   "count_unique" 0/1: count distinct rows read per level (gt_stats.unique_rows);
 *                 adds atomics to the walk, for measurement runs only
 * Errors: INVALID_ARG for an unknown key or a value out of range. */
gt_status gt_set_option(gt_index* index, const char* key, int64_t value);

/* Frees every device allocation of the index.  NULL is ignored. */
void gt_destroy(gt_index* index);

/* Message for the last error on the calling thread ("" if none).  The string
 * stays valid until the next call on this thread. */
const char* gt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GT_H */
