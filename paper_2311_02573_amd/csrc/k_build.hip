// Index construction and query preparation kernels.
//
// Tree layout (paper Sec. 2: the pools of binary splitting are fixed offline):
// level l (0 = root) has 2^l pools; pool j of level l covers leaves
// [j * 2^(depth-l), (j+1) * 2^(depth-l)).  Level l is stored at rows
// (2^l - 1) .. (2^(l+1) - 2) of one array, so the two children of a pool are
// adjacent rows.  Leaves (level `depth`) are the float32 feature rows.
#include <float.h>
#include <hip/hip_fp16.h>
#include <math.h>

#include "gt_internal.h"
#include "gt_numerics.h"

namespace gt {

namespace {

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__device__ __forceinline__ float load_feature(const void* src, int dtype, int64_t idx) {
  if (dtype == GT_F16) return __half2float(reinterpret_cast<const __half*>(src)[idx]);
  if (dtype == GT_BF16)
    return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(src)[idx] << 16);
  return reinterpret_cast<const float*>(src)[idx];
}

// One workgroup of 64 threads per 64 rows.  Column tiles of 64 are staged
// through LDS so that loads and stores are coalesced while each thread still
// sums its own row sequentially in float64 (the canonical squared norm).
// Values must be finite and >= 0, or only finite with allow_negative (then
// the largest |value| is folded into *absmax as float bits).
__global__ __launch_bounds__(64) void k_ingest(const void* src, int dtype, int64_t rows, int d,
                                               int dp, float* leaves, double* ff, float* invn,
                                               float* nf, double* mmin, unsigned int* err,
                                               int allow_negative, unsigned int* absmax) {
  __shared__ float tile[64][65];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  double acc = 0.0;
  bool bad = false;
  float amax = 0.0f;
  for (int c0 = 0; c0 < dp; c0 += 64) {
    const int c = c0 + t;
    for (int r = 0; r < 64; ++r) {
      const int64_t row = r0 + r;
      if (row >= rows) break;
      float v = 0.0f;
      if (c < d) {
        v = load_feature(src, dtype, row * d + c);
        if (allow_negative) {
          if (!isfinite(v)) bad = true;
          amax = fmaxf(amax, fabsf(v));
        } else if (!(v >= 0.0f) || isinf(v)) {
          bad = true;
        }
      }
      if (c < dp) leaves[row * dp + c] = v;
      tile[r][t] = v;
    }
    __syncthreads();
    if (r0 + t < rows) {
      const int lim = min(64, d - c0);
      for (int k = 0; k < lim; ++k) {
        const double x = (double)tile[t][k];
        acc = __dadd_rn(acc, __dmul_rn(x, x));
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(err, 1u);
  if (absmax) {
    for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    if (t == 0 && amax > 0.0f) atomicMax(absmax, __float_as_uint(amax));
  }
  const int64_t row = r0 + t;
  if (row < rows) {
    ff[row] = acc;
    const double nrm = __dsqrt_rn(acc);
    invn[row] = acc > 0.0 ? (float)__ddiv_rn(1.0, nrm) : 0.0f;
    nf[row] = acc > 0.0 ? f64_to_f32_down(nrm) : 0.0f;
    if (acc > 0.0 && !bad)
      atomicMin(reinterpret_cast<unsigned long long*>(mmin),
                (unsigned long long)__double_as_longlong(nrm));
  }
}

// parent = children summed with upward rounding, 4 columns per thread.
// Parent pools of `nodes` nodes from their two children: the element-wise sum
// rounded up (sum pooling, paper Sec. 2) or the element-wise maximum, which is
// exact (Our-Max pooling, Sec. 2).
template <bool MAXP>
__global__ void k_build_level(const float* __restrict__ child, float* __restrict__ parent,
                              int64_t first, int64_t nodes, int dp) {
  const int q = dp / 4;
  const int64_t total = nodes * q;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = first + i / q;
    const int k = (int)(i % q) * 4;
    const float4 a = *reinterpret_cast<const float4*>(child + (2 * j) * dp + k);
    const float4 b = *reinterpret_cast<const float4*>(child + (2 * j + 1) * dp + k);
    float4 s;
    if (MAXP) {
      s.x = fmaxf(a.x, b.x);
      s.y = fmaxf(a.y, b.y);
      s.z = fmaxf(a.z, b.z);
      s.w = fmaxf(a.w, b.w);
    } else {
      s.x = add_up(a.x, b.x);
      s.y = add_up(a.y, b.y);
      s.z = add_up(a.z, b.z);
      s.w = add_up(a.w, b.w);
    }
    *reinterpret_cast<float4*>(parent + j * dp + k) = s;
  }
}

// Bottom level of the max/min tree of a signed index (paper Sec. 2, negative
// descriptors).  Pool j of level depth-1 holds leaves 2j and 2j+1; only leaves
// below n are members.  Row j gets [max_k + B | B - min_k] over its members in
// columns k < d, each term rounded up (every term is >= 0 because |f_k| <= B),
// zero in the padding columns and for a pool without members.  The maximum of
// the shifted rows is taken term by term, which is the shifted max and min.
__global__ void k_signed_bottom(const float* __restrict__ leaves, float* __restrict__ parent,
                                int64_t first, int64_t nodes, int dp, int d, int64_t n,
                                float bound) {
  const int pw = 2 * dp, qd = pw / 4;
  const int64_t total = nodes * qd;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = first + i / qd;
    const int k = (int)(i % qd) * 4;          // column of the shifted row
    const bool hi = k >= dp;                  // second half: B - f
    const int c = hi ? k - dp : k;            // feature column
    float o[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int m = 0; m < 2; ++m) {
      const int64_t leaf = 2 * j + m;
      if (leaf >= n) break;
      const float4 v = *reinterpret_cast<const float4*>(leaves + leaf * dp + c);
      const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (c + e < d) {
          const float t = hi ? add_up(bound, -x[e]) : add_up(x[e], bound);
          o[e] = fmaxf(o[e], t);
        }
      }
    }
    *reinterpret_cast<float4*>(parent + j * pw + k) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

// Frontier entries per level of a call: the sum of the level's per-slot
// counters (one workgroup per level, levels first .. levels-1; 16-byte loads).
__global__ __launch_bounds__(1024) void k_level_entries(const uint32_t* __restrict__ counts,
                                                        int first, DevCounters* ctr) {
  __shared__ unsigned long long part[16];
  const int l = first + blockIdx.x, t = threadIdx.x;
  const uint4* c4 = reinterpret_cast<const uint4*>(counts + (size_t)l * kMaxSlots);
  unsigned long long sum = 0;
  for (int k = t; k < kMaxSlots / 4; k += blockDim.x) {
    const uint4 v = c4[k];
    sum += (unsigned long long)v.x + v.y + v.z + v.w;
  }
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((t & 63) == 0) part[t >> 6] = sum;
  __syncthreads();
  if (t == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
    ctr->entries[l] = tot;
  }
}

__global__ void k_level_max(const float* __restrict__ rows, int64_t count, float* out) {
  float m = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, rows[i]);
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int*>(out), __float_as_uint(m));
}

__global__ void k_quant_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst,
                             int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = bf16_up(src[i]);
}

__global__ void k_quant_fp8(const float* __restrict__ src, uint8_t* __restrict__ dst,
                            int64_t count, int lexp, unsigned int* overflow) {
  bool over = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c = e4m3_up(ldexp((double)src[i], -lexp));
    if (c == 0xFFu) {
      over = true;
      c = 0x7Eu;
    }
    dst[i] = (uint8_t)c;
  }
  if (over) atomicOr(overflow, 1u);
}

// One workgroup of 256 threads per (padded) query.
__global__ __launch_bounds__(256) void k_query_prep(
    const float* __restrict__ q, int nq, int d, int dp, int tq, const double* __restrict__ rho,
    const double* __restrict__ mmin, float* qf, uint16_t* qbf, uint8_t* q8, int* qexp,
    float* invn_q, double* qq_out, float* thr, float* thr_gemm, uint64_t* tile_mask,
    const float* __restrict__ root, float* sabs, float* qw, int pw, float sbound,
    unsigned int* err) {
  __shared__ float qs[4096];
  __shared__ float red[4];
  __shared__ double l1red[4], l2red[4];
  const int b = blockIdx.x, t = threadIdx.x;
  const bool real = b < nq;
  float mx = 0.0f;
  bool bad = false;
  const bool sgn = sbound > 0.0f;  // signed index: any finite value
  for (int k = t; k < d; k += blockDim.x) {
    const float v = real ? q[(int64_t)b * d + k] : 0.0f;
    if (sgn ? !isfinite(v) : (!(v >= 0.0f) || isinf(v))) bad = true;
    qs[k] = v;
    mx = fmaxf(mx, v);
  }
  if (bad) atomicOr(err, 1u);
  // |q|_1 + |root pool|_1 (any order: only an upper bound is needed); for a
  // signed index |q|_1 alone, which sets the threshold's shift B |q|_1
  double l1 = 0.0;
  for (int k = t; k < d; k += blockDim.x) l1 += (double)fabsf(qs[k]);
  if (root)
    for (int k = t; k < dp; k += blockDim.x) l1 += (double)root[k];
  // |q|^2 by a fixed-order parallel sum (deterministic, relative error below
  // 2^-40 for d <= 4096; the thresholds' slack covers far more).  The
  // canonical sequential sum, which the float64 recheck needs bit for bit,
  // is formed there for the few candidates that reach it.
  double l2 = 0.0;
  for (int k = t; k < d; k += blockDim.x) l2 = __fma_rn((double)qs[k], (double)qs[k], l2);
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  for (int o = 32; o >= 1; o >>= 1) l1 += __shfl_xor(l1, o, 64);
  for (int o = 32; o >= 1; o >>= 1) l2 += __shfl_xor(l2, o, 64);
  if ((t & 63) == 0) {
    red[t >> 6] = mx;
    l1red[t >> 6] = l1;
    l2red[t >> 6] = l2;
  }
  __syncthreads();
  const double qq = (l2red[0] + l2red[1]) + (l2red[2] + l2red[3]);
  const float qmax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  // float8 query scale 2^e with qmax / 2^e in (224, 448]
  int e = 0;
  if (qmax > 0.0f) {
    int ex;
    const double m = frexp((double)qmax / 448.0, &ex);
    e = (m == 0.5) ? ex - 1 : ex;
  }
  for (int k = t; k < dp; k += blockDim.x) {
    const float v = k < d ? qs[k] : 0.0f;
    qf[(int64_t)b * dp + k] = v;
    if (sgn) {
      // walk query [max(q,0) | max(-q,0)] against rows [max + B | B - min]
      const float vp = fmaxf(v, 0.0f), vn = fmaxf(-v, 0.0f);
      if (qw) {
        qw[(int64_t)b * pw + k] = vp;
        qw[(int64_t)b * pw + dp + k] = vn;
      }
      if (qbf) {
        qbf[(int64_t)b * pw + k] = bf16_up(vp);
        qbf[(int64_t)b * pw + dp + k] = bf16_up(vn);
      }
    } else {
      if (qbf) qbf[(int64_t)b * dp + k] = bf16_up(v);
      if (q8) q8[(int64_t)b * dp + k] = (uint8_t)e4m3_up(ldexp((double)v, -e));
    }
  }
  if (t == 0) {
    const bool live = real && qq > 0.0 && !bad;
    const double nrm = __dsqrt_rn(qq);
    qq_out[b] = qq;
    qexp[b] = e;
    invn_q[b] = qq > 0.0 ? (float)__ddiv_rn(1.0, nrm) : 0.0f;
    float th = INFINITY, tg = INFINITY;
    if (live) {
      const double r = rho[b];
      if (r <= 0.0) {
        th = -INFINITY;
        tg = -INFINITY;
      } else {
        // cos >= rho with the float64 definition implies the real cosine is
        // at least rho * (1 - 2e-11) for d <= 4096; every member norm is at
        // least m_min, so a pool holding a neighbour scores >= tau (reals).
        const double reff = r * (1.0 - 4e-11);
        const double tau = reff * nrm * (*mmin) * (1.0 - 4e-11);
        if (sgn) {
          // A member's q.f is at most the pool's max/min score U, and the
          // walk computes [q+ | q-] . [max + B | B - min] = U + B |q|_1 over
          // pw non-negative products.  The shift is taken slightly low (the
          // float64 |q|_1 of <= 4096 terms is within 2^-40 of the real one).
          // Products of mixed sign in the leaf GEMM carry an error relative
          // to sum |q_k f_k| <= |q| |f|, hence rho - slack there.
          const double sl = pool_slack(pw);
          const double l1s = (l1red[0] + l1red[1]) + (l1red[2] + l1red[3]);
          const double kappa = (double)sbound * l1s * (1.0 - 1e-12);
          th = f64_to_f32_down((tau + kappa) * (1.0 - sl) - 2.0 * pw * 0x1p-126);
          const double cg = reff * (1.0 - 4e-11) - pool_slack(dp);
          tg = cg > 0.0 ? f64_to_f32_down(cg * nrm) : -INFINITY;
        } else {
          const double sl = pool_slack(dp);
          th = f64_to_f32_down(tau * (1.0 - sl) - 2.0 * dp * 0x1p-126);
          tg = f64_to_f32_down(reff * nrm * (1.0 - 4e-11) * (1.0 - sl));
        }
      }
      atomicOr(reinterpret_cast<unsigned long long*>(&tile_mask[b / tq]),
               (unsigned long long)(1ull << (b % tq)));
    }
    thr[b] = th;
    thr_gemm[b] = tg;
    if (sabs && !sgn) {
      // absolute term of the subtraction step's lower bound: 2^-125 (|S|_1 +
      // |q|_1 + dp 2^-126) + 2^-126, a normal float32 rounded up
      const double l1s = (l1red[0] + l1red[1]) + (l1red[2] + l1red[3]);
      const double v = ldexp(1.01 * l1s + (double)dp * 0x1p-126, -125) + 0x1p-126;
      float f = (float)v;
      if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
      sabs[b] = f;
    }
  }
}

inline int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_ingest(const void* src, int dtype, int64_t rows, int d, int dp, float* leaves,
                         double* ff, float* invn, float* nf, double* mmin, unsigned int* err,
                         bool allow_negative, unsigned int* absmax, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ingest, dim3((unsigned)((rows + 63) / 64)), dim3(64), 0, s, src, dtype, rows,
                     d, dp, leaves, ff, invn, nf, mmin, err, allow_negative ? 1 : 0, absmax);
  return hipGetLastError();
}

hipError_t launch_signed_bottom(const float* leaves, float* parent, int64_t first, int64_t nodes,
                                int dp, int d, int64_t n, float bound, hipStream_t s) {
  if (nodes <= 0) return hipSuccess;
  if (dp % 4 || d > dp || first < 0 || n < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_signed_bottom, dim3(grid_for(nodes * (2 * dp / 4), 256)), dim3(256), 0, s,
                     leaves, parent, first, nodes, dp, d, n, bound);
  return hipGetLastError();
}

hipError_t launch_build_level(const float* child, float* parent, int64_t nodes, int dp,
                              int64_t first, hipStream_t s, bool max_pool) {
  if (nodes <= 0) return hipSuccess;
  if (max_pool)
    hipLaunchKernelGGL(k_build_level<true>, dim3(grid_for(nodes * (dp / 4), 256)), dim3(256), 0, s,
                       child, parent, first, nodes, dp);
  else
    hipLaunchKernelGGL(k_build_level<false>, dim3(grid_for(nodes * (dp / 4), 256)), dim3(256), 0, s,
                       child, parent, first, nodes, dp);
  return hipGetLastError();
}

hipError_t launch_level_entries(const uint32_t* lvl_count, int first, int levels,
                                DevCounters* ctr, hipStream_t s) {
  if (first < 0 || levels > GT_MAX_LEVELS) return hipErrorInvalidValue;
  if (first >= levels) return hipSuccess;
  hipLaunchKernelGGL(k_level_entries, dim3(levels - first), dim3(1024), 0, s, lvl_count, first,
                     ctr);
  return hipGetLastError();
}

hipError_t launch_level_max(const float* rows, int64_t nrows, int dp, float* out_max,
                            hipStream_t s) {
  const int64_t count = nrows * dp;
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_max, dim3(grid_for(count, 256 * 8)), dim3(256), 0, s, rows, count,
                     out_max);
  return hipGetLastError();
}

hipError_t launch_quant_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quant_bf16, dim3(grid_for(count, 256 * 4)), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_quant_fp8(const float* src, uint8_t* dst, int64_t count, int lexp,
                            unsigned int* overflow, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quant_fp8, dim3(grid_for(count, 256 * 4)), dim3(256), 0, s, src, dst, count,
                     lexp, overflow);
  return hipGetLastError();
}

hipError_t launch_query_prep(const float* q, int nq, int d, int dp, int tq, const double* rho,
                             const double* mmin, float* qf, uint16_t* qbf, uint8_t* q8, int* qexp,
                             float* invn_q, double* qq, float* thr, float* thr_gemm,
                             uint64_t* tile_mask, const float* root, float* sabs,
                             float* qw, int pw, float sbound,
                             unsigned int* err, int nq_pad, hipStream_t s) {
  if (nq_pad <= 0) return hipSuccess;
  if (sbound > 0.0f && pw != 2 * dp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_query_prep, dim3(nq_pad), dim3(256), 0, s, q, nq, d, dp, tq, rho, mmin, qf,
                     qbf, q8, qexp, invn_q, qq, thr, thr_gemm, tile_mask, root, sabs, qw, pw,
                     sbound, err);
  return hipGetLastError();
}

}  // namespace gt
