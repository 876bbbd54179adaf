/*
 * CPU oracle for range-based near-neighbour search (test infrastructure only).
 *
 * Computes, by brute force over every database row, the set
 *     { i : cos(q, f_i) >= rho }
 * which is the problem statement of the paper (Sec. 1, the similarity-threshold
 * query; Sec. 2, where sim is the dot product of unit, non-negative vectors and
 * therefore the cosine).  The search method of the paper is exact (its tables
 * report precision = recall = 1), so the oracle is the plain definition, not
 * the method.
 *
 * Canonical value, used everywhere a float decides membership:
 *     dot = sum_k q_k * f_k     sequential in k, float64
 *     qq  = sum_k q_k * q_k     sequential in k, float64
 *     ff  = sum_k f_k * f_k     sequential in k, float64
 *     cos = dot / (sqrt(qq) * sqrt(ff))     IEEE round-to-nearest-even
 *     member iff cos >= rho    (a NaN from a zero vector is never a member)
 * Inputs are at most float32 wide, so every product is exact in float64.
 *
 * Nothing here is shared with the GPU library; only the seeded input generator
 * feeds both.  Build: gcc -O2 -ffp-contract=off -shared -fPIC -pthread.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_F32 = 0, OR_F16 = 1, OR_BF16 = 2 };

/* IEEE binary16 -> double, from the format definition (1/5/10, bias 15). */
static double half_to_double(uint16_t h) {
  int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
  double v;
  if (e == 0) v = ldexp((double)m, -24);
  else if (e == 31) v = m ? NAN : INFINITY;
  else v = ldexp((double)(m + 1024), e - 25);
  return s ? -v : v;
}

/* bfloat16 -> double: the upper 16 bits of a binary32. */
static double bf16_to_double(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

static inline double load_elem(const void* base, int dtype, int64_t idx) {
  switch (dtype) {
    case OR_F16: return half_to_double(((const uint16_t*)base)[idx]);
    case OR_BF16: return bf16_to_double(((const uint16_t*)base)[idx]);
    default: return (double)((const float*)base)[idx];
  }
}

typedef struct { int64_t n, cap; int64_t* ids; double* sims; } vec_t;

static void vec_push(vec_t* v, int64_t id, double s) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->ids = (int64_t*)realloc(v->ids, (size_t)v->cap * sizeof(int64_t));
    v->sims = (double*)realloc(v->sims, (size_t)v->cap * sizeof(double));
  }
  v->ids[v->n] = id;
  v->sims[v->n] = s;
  v->n++;
}

typedef struct {
  int nq, nthreads;
  vec_t* res; /* [nthreads][nq] */
} oracle_result;

typedef struct {
  const void* feats; int dtype; int64_t n; int32_t d;
  const float* q; int32_t nq; const double* rho;
  const double* qq;
  int64_t lo, hi;
  vec_t* out; /* [nq] for this thread */
} job_t;

#define RB 8 /* rows per block: independent sequential chains, one per row */

static void* scan_rows(void* arg) {
  job_t* J = (job_t*)arg;
  const int32_t d = J->d;
  double* rows = (double*)calloc((size_t)RB * (d > 0 ? d : 1), sizeof(double));
  double ff[RB];
  for (int64_t i0 = J->lo; i0 < J->hi; i0 += RB) {
    int nb = (int)((J->hi - i0) < RB ? (J->hi - i0) : RB);
    for (int r = 0; r < nb; ++r) {
      double acc = 0.0;
      for (int32_t k = 0; k < d; ++k) {
        double x = load_elem(J->feats, J->dtype, (i0 + r) * (int64_t)d + k);
        rows[r * d + k] = x;
        acc = acc + x * x;
      }
      ff[r] = acc;
    }
    for (int32_t j = 0; j < J->nq; ++j) {
      const float* qj = J->q + (int64_t)j * d;
      double dot[RB] = {0};
      for (int32_t k = 0; k < d; ++k) {
        double qk = (double)qj[k];
        for (int r = 0; r < RB; ++r) dot[r] = dot[r] + qk * rows[r * d + k];
      }
      double nq_ = sqrt(J->qq[j]);
      for (int r = 0; r < nb; ++r) {
        double c = dot[r] / (nq_ * sqrt(ff[r]));
        if (c >= J->rho[j]) vec_push(&J->out[j], i0 + r, c);
      }
    }
  }
  free(rows);
  return NULL;
}

/* Brute-force scan.  Returns an opaque result; rows are split into contiguous
 * ranges per thread so per-query ids come out ascending after concatenation. */
oracle_result* oracle_range_search(const void* feats, int dtype, int64_t n, int32_t d,
                                   const float* q, int32_t nq, const double* rho,
                                   int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (n < (int64_t)nthreads * RB) nthreads = n > 0 ? (int)((n + RB - 1) / RB) : 1;
  if (nthreads > 256) nthreads = 256;
  oracle_result* R = (oracle_result*)calloc(1, sizeof(oracle_result));
  R->nq = nq;
  R->nthreads = nthreads;
  R->res = (vec_t*)calloc((size_t)nthreads * (nq > 0 ? nq : 1), sizeof(vec_t));
  double* qq = (double*)calloc(nq > 0 ? nq : 1, sizeof(double));
  for (int32_t j = 0; j < nq; ++j) {
    double acc = 0.0;
    for (int32_t k = 0; k < d; ++k) {
      double x = (double)q[(int64_t)j * d + k];
      acc = acc + x * x;
    }
    qq[j] = acc;
  }
  pthread_t* th = (pthread_t*)calloc(nthreads, sizeof(pthread_t));
  job_t* jobs = (job_t*)calloc(nthreads, sizeof(job_t));
  int64_t per = (n + nthreads - 1) / nthreads;
  per = (per + RB - 1) / RB * RB;
  for (int t = 0; t < nthreads; ++t) {
    job_t* J = &jobs[t];
    J->feats = feats; J->dtype = dtype; J->n = n; J->d = d;
    J->q = q; J->nq = nq; J->rho = rho; J->qq = qq;
    J->lo = (int64_t)t * per < n ? (int64_t)t * per : n;
    J->hi = (int64_t)(t + 1) * per < n ? (int64_t)(t + 1) * per : n;
    J->out = &R->res[(size_t)t * nq];
    pthread_create(&th[t], NULL, scan_rows, J);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  free(qq);
  return R;
}

int64_t oracle_result_count(const oracle_result* R, int32_t j) {
  int64_t c = 0;
  for (int t = 0; t < R->nthreads; ++t) c += R->res[(size_t)t * R->nq + j].n;
  return c;
}

void oracle_result_copy(const oracle_result* R, int32_t j, int64_t* ids, double* sims) {
  int64_t o = 0;
  for (int t = 0; t < R->nthreads; ++t) {
    const vec_t* v = &R->res[(size_t)t * R->nq + j];
    memcpy(ids + o, v->ids, (size_t)v->n * sizeof(int64_t));
    memcpy(sims + o, v->sims, (size_t)v->n * sizeof(double));
    o += v->n;
  }
}

void oracle_result_free(oracle_result* R) {
  if (!R) return;
  for (int64_t i = 0; i < (int64_t)R->nthreads * R->nq; ++i) {
    free(R->res[i].ids);
    free(R->res[i].sims);
  }
  free(R->res);
  free(R);
}

/* Canonical float64 cosine of individual (query, row) pairs. */
void oracle_pair_cos(const void* feats, int dtype, int32_t d, const float* q,
                     const int64_t* qidx, const int64_t* rows, int64_t npairs, double* out) {
  for (int64_t p = 0; p < npairs; ++p) {
    const float* qj = q + qidx[p] * (int64_t)d;
    double dot = 0.0, qq = 0.0, ff = 0.0;
    for (int32_t k = 0; k < d; ++k) {
      double a = (double)qj[k], b = load_elem(feats, dtype, rows[p] * (int64_t)d + k);
      dot = dot + a * b;
      qq = qq + a * a;
      ff = ff + b * b;
    }
    out[p] = dot / (sqrt(qq) * sqrt(ff));
  }
}
