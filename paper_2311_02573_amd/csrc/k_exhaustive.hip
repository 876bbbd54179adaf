// Exhaustive baseline (the paper's Exh comparison, Sec. 4): every (query,
// vector) dot product with a float32 matrix-core GEMM [nq x d] . [d x n], and
// a threshold epilogue that keeps pairs which may reach rho.  Kept pairs go
// through the same exact test as the leaves of the walk, so both paths return
// identical results.
#include <math.h>

#include "gt_internal.h"
#include "gt_device.h"
#include "gt_numerics.h"

namespace gt {

namespace {

typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int GT_ = 128;   // output tile edge (queries x vectors)
constexpr int KC = 32;     // dimensions per LDS stage
constexpr int LDSW = KC + 4;

// One workgroup (4 waves) per 128 x 128 output tile; each wave owns 64 x 64 as
// 2 x 2 blocks of 32 x 32.  Workgroups are dispatched round-robin over the 8
// XCDs; consecutive workgroups of one XCD take the query tiles of one vector
// tile in turn, so each vector tile is fetched into that XCD's L2 once.
__global__ __launch_bounds__(256) void k_gemm_threshold(const float* __restrict__ qf, int nq_pad,
                                                        const float* __restrict__ rows, int64_t n,
                                                        int dp, const float* __restrict__ thr,
                                                        const float* __restrict__ nf, uint2* cand,
                                                        unsigned long long cap, DevCounters* ctr,
                                                        int nq) {
  __shared__ __attribute__((aligned(16))) float As[GT_ * LDSW];
  __shared__ __attribute__((aligned(16))) float Bs[GT_ * LDSW];
  const int QT = nq_pad / GT_;
  const int64_t RT = (n + GT_ - 1) / GT_;
  const int64_t total = RT * QT;
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t w = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (w >= total) return;
  const int qt = (int)(w % QT);
  const int64_t rt = w / QT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = (wave >> 1) * 64, wr = (wave & 1) * 64;  // wave's sub-tile origin
  const int c = lane & 31, half = lane >> 5;

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

  // global -> register staging: 128 rows x 32 floats per operand; thread tid
  // moves float4 pieces tid + 256 v (v < 4): row = piece / 8 = tid / 8 + 32 v
  const float* qbase = qf + (size_t)qt * GT_ * dp;
  const int64_t r0 = rt * GT_;
  const int prow = tid >> 3, pcol = (tid & 7) * 4;
  const float* qa = qbase + (size_t)prow * dp + pcol;
  const float* fb[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t rr = r0 + prow + 32 * v < n ? r0 + prow + 32 * v : n - 1;
    fb[v] = rows + (size_t)rr * dp + pcol;
  }
  const size_t q32 = (size_t)32 * dp;
  float4 ra0 = *reinterpret_cast<const float4*>(qa);
  float4 ra1 = *reinterpret_cast<const float4*>(qa + q32);
  float4 ra2 = *reinterpret_cast<const float4*>(qa + 2 * q32);
  float4 ra3 = *reinterpret_cast<const float4*>(qa + 3 * q32);
  float4 rb0 = *reinterpret_cast<const float4*>(fb[0]);
  float4 rb1 = *reinterpret_cast<const float4*>(fb[1]);
  float4 rb2 = *reinterpret_cast<const float4*>(fb[2]);
  float4 rb3 = *reinterpret_cast<const float4*>(fb[3]);
  for (int k0 = 0; k0 < dp; k0 += KC) {
    __syncthreads();
    *reinterpret_cast<float4*>(&As[(prow + 0) * LDSW + pcol]) = ra0;
    *reinterpret_cast<float4*>(&As[(prow + 32) * LDSW + pcol]) = ra1;
    *reinterpret_cast<float4*>(&As[(prow + 64) * LDSW + pcol]) = ra2;
    *reinterpret_cast<float4*>(&As[(prow + 96) * LDSW + pcol]) = ra3;
    *reinterpret_cast<float4*>(&Bs[(prow + 0) * LDSW + pcol]) = rb0;
    *reinterpret_cast<float4*>(&Bs[(prow + 32) * LDSW + pcol]) = rb1;
    *reinterpret_cast<float4*>(&Bs[(prow + 64) * LDSW + pcol]) = rb2;
    *reinterpret_cast<float4*>(&Bs[(prow + 96) * LDSW + pcol]) = rb3;
    __syncthreads();
    if (k0 + KC < dp) {
      const int kn = k0 + KC;
      ra0 = *reinterpret_cast<const float4*>(qa + kn);
      ra1 = *reinterpret_cast<const float4*>(qa + q32 + kn);
      ra2 = *reinterpret_cast<const float4*>(qa + 2 * q32 + kn);
      ra3 = *reinterpret_cast<const float4*>(qa + 3 * q32 + kn);
      rb0 = *reinterpret_cast<const float4*>(fb[0] + kn);
      rb1 = *reinterpret_cast<const float4*>(fb[1] + kn);
      rb2 = *reinterpret_cast<const float4*>(fb[2] + kn);
      rb3 = *reinterpret_cast<const float4*>(fb[3] + kn);
    }
#pragma unroll
    for (int t = 0; t < KC / 8; ++t) {
      float4 fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        fa[a] = *reinterpret_cast<const float4*>(&As[(wq + 32 * a + c) * LDSW + 8 * t + 4 * half]);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        fb[b] = *reinterpret_cast<const float4*>(&Bs[(wr + 32 * b + c) * LDSW + 8 * t + 4 * half]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a].x, fb[b].x, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a].y, fb[b].y, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a].z, fb[b].z, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a].w, fb[b].w, acc[a][b], 0, 0, 0);
        }
    }
  }

  // epilogue: keep (query, vector) if the score may reach rho * |q| * |f|
  float nfv[2];
  int64_t rid[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    rid[b] = r0 + wr + 32 * b + c;
    nfv[b] = rid[b] < n ? nf[rid[b]] : 0.0f;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int qi = qt * GT_ + wq + 32 * a + 8 * (i >> 2) + 4 * half + (i & 3);
      const float th = qi < nq ? thr[qi] : INFINITY;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const bool keep = nfv[b] > 0.0f && acc[a][b][i] >= th * nfv[b] * (1.0f - 0x1p-20f);
        const uint64_t bal = __ballot(keep);
        if (bal) {
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(&ctr->ncand, (unsigned long long)__popcll(bal));
          base = __shfl(base, 0, 64);
          if (keep) {
            const unsigned long long pos = base + __popcll(bal & ((1ull << lane) - 1ull));
            if (pos < cap) cand[pos] = make_uint2((uint32_t)qi, (uint32_t)rid[b]);
          }
        }
      }
    }
}

// Exact test of explicit (query, vector) pairs: the same float32 dot product
// (in-lane pairwise sums, then the lane reduction) and classification as the
// leaf test of the walk, four pairs per wave at a time.
__global__ __launch_bounds__(256) void k_pair_check(const uint2* cand, const unsigned long long* ncand,
                                                    unsigned long long cap, const float* qf,
                                                    const float* leaves, const float* invn_q,
                                                    const float* invn_f, const double* rho, int dp,
                                                    Hit* hits, unsigned long long hit_cap,
                                                    uint32_t* band_idx, unsigned int* qcount,
                                                    DevCounters* ctr) {
  __shared__ Hit hstage[4][kHitStage];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long n = *ncand < cap ? *ncand : cap;
  const unsigned long long nw = blockDim.x >> 6;
  Hit* buf = hstage[w];
  int cnt = 0;
  unsigned long long npairs = 0;
  for (unsigned long long b0 = (blockIdx.x * nw + w) * 4ull; b0 < n; b0 += gridDim.x * nw * 4ull) {
    uint2 pr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pr[k] = cand[b0 + k < n ? b0 + k : b0];
    float acc[8];
    for (int c = 0; c * 1024 < dp; ++c) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float v = lane_partial16(qf + (size_t)pr[k].x * dp, leaves + (size_t)pr[k].y * dp,
                                       c, dp, lane);
        acc[k] = c == 0 ? v : __fadd_rn(acc[k], v);
        acc[k + 4] = 0.0f;
      }
    }
    const float dot = wave_reduce8(acc, lane);
    const int v = lane >> 3;
    const bool mine = (lane & 7) == 0 && v < 4 && b0 + v < n;
    Hit h;
    uint32_t flag = 0;
    if (mine) {
      const uint2 x = pr[v];
      const float invf = invn_f[x.y];
      const float cs = __fmul_rn(__fmul_rn(dot, invn_q[x.x]), invf);
      flag = invf != 0.0f ? classify(cs, rho[x.x]) : 0u;
      h.q = x.x;
      h.id = x.y;
      h.sim = cs;
      h.flag = flag == HIT_ACCEPT ? flag | accept_slot(&qcount[x.x], ctr) : flag;
      ++npairs;
    }
    stage_hits(buf, cnt, flag != 0u, h, false, ctr, hits, hit_cap, band_idx, lane);
  }
  Hit none;
  stage_hits(buf, cnt, false, none, true, ctr, hits, hit_cap, band_idx, lane);
  for (int o = 32; o >= 1; o >>= 1) npairs += __shfl_xor(npairs, o, 64);
  if (lane == 0 && npairs) atomicAdd(&ctr->leaf_pairs, npairs);
}

}  // namespace

hipError_t launch_exhaustive_gemm(const float* qf, int nq_pad, const float* leaves, int64_t n,
                                  int dp, const float* thr_gemm, const float* nf, uint2* cand,
                                  unsigned long long cand_cap, DevCounters* ctr, int nq,
                                  hipStream_t s) {
  if (n <= 0 || nq_pad <= 0) return hipSuccess;
  const int64_t total = ((n + GT_ - 1) / GT_) * (nq_pad / GT_);
  const int64_t grid = 8 * ((total + 7) / 8);
  hipLaunchKernelGGL(k_gemm_threshold, dim3((unsigned)grid), dim3(256), 0, s, qf, nq_pad, leaves, n,
                     dp, thr_gemm, nf, cand, cand_cap, ctr, nq);
  return hipGetLastError();
}

hipError_t launch_pair_check(const uint2* cand, const unsigned long long* ncand,
                             unsigned long long cap, const float* qf, const float* leaves,
                             const float* invn_q, const float* invn_f, const double* rho, int dp,
                             Hit* hits, unsigned long long hit_cap, uint32_t* band_idx,
                             unsigned int* qcount, DevCounters* ctr, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_check, dim3(grid), dim3(256), 0, s, cand, ncand, cap, qf, leaves, invn_q,
                     invn_f, rho, dp, hits, hit_cap, band_idx, qcount, ctr);
  return hipGetLastError();
}

}  // namespace gt
