// The level-wise binary-splitting walk (paper Sec. 2, Alg. 1; one level per
// round as in the pruning analysis of Sec. 4), the exact leaf test, the
// float64 recheck and the result compaction.
//
// Frontier representation.  Queries are grouped in tiles of TQ (64 for bf16 /
// float8 pools, 32 for float32 pools).  The frontier of a tile at level l is a
// list of entries (pool j, mask): pool j of level l survived for the queries
// whose bits are set.  One level step reads both children of every entry (two
// adjacent rows), scores them against all TQ queries of the tile with matrix
// cores, and keeps child c for query b iff the parent's bit b is set and the
// score reaches the query's lowered threshold tau'_b.  Children with a
// non-empty mask are appended to the tile's next frontier.
#include <math.h>

#include "gt_internal.h"
#include "gt_device.h"
#include "gt_numerics.h"

namespace gt {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

template <int FMT>
struct WalkFmt;
template <>
struct WalkFmt<GT_POOL_F32> {
  static constexpr int TQ = kQueriesPerTileF32, ESZ = 4, MAXDP = kMaxDpF32;
};
template <>
struct WalkFmt<GT_POOL_BF16> {
  static constexpr int TQ = kQueriesPerTile16, ESZ = 2, MAXDP = kMaxDpBf16;
};
template <>
struct WalkFmt<GT_POOL_FP8E4M3> {
  static constexpr int TQ = kQueriesPerTile16, ESZ = 1, MAXDP = kMaxDpFp8;
};

// One 16-byte slice of a row (per lane) against the same slice of a query:
// bf16: one 32x32x16 step; float8: two 32x32x16 steps; float32: four 32x32x2
// steps.  Lanes 0-31 and 32-63 carry different slices, and the A (pool) and B
// (query) operands of a lane always hold the same dimensions, so the sum over
// all slices is the full dot product whatever order the hardware uses inside.
template <int FMT>
__device__ __forceinline__ void mma16(const uint4& a, const uint4& b, f32x16& acc);

template <>
__device__ __forceinline__ void mma16<GT_POOL_BF16>(const uint4& a, const uint4& b, f32x16& acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma16<GT_POOL_FP8E4M3>(const uint4& a, const uint4& b,
                                                       f32x16& acc) {
  const long a0 = (long)(((unsigned long)a.y << 32) | a.x);
  const long a1 = (long)(((unsigned long)a.w << 32) | a.z);
  const long b0 = (long)(((unsigned long)b.y << 32) | b.x);
  const long b1 = (long)(((unsigned long)b.w << 32) | b.z);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a0, b0, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a1, b1, acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma16<GT_POOL_F32>(const uint4& a, const uint4& b, f32x16& acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
}

// Exclusive prefix pre[0..n] of the entry counts of bucket slots
// slot0 .. slot0 + n - 1 (n <= 1024), computed by wave 0.  Dense input: every
// pool of the bucket (1 << shift of them) for the tile's queries.
__device__ __forceinline__ void slot_prefix(uint32_t* pre, int n, int slot0, int nt, int dense,
                                            int shift, const uint64_t* tile_mask,
                                            const uint32_t* counts, uint32_t cap) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int per_lane = (n + 63) / 64;
    const int s0 = lane * per_lane;
    uint32_t loc[16];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int sl = s0 + i;
      uint32_t c = 0;
      if (i < per_lane && sl < n) {
        const int gs = slot0 + sl;
        c = dense ? (tile_mask[gs % nt] ? (1u << shift) : 0u) : min(counts[gs], cap);
      }
      loc[i] = sum;
      sum += c;
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    const uint32_t excl = incl - sum;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int sl = s0 + i;
      if (i < per_lane && sl < n) pre[sl] = excl + loc[i];
    }
    if (lane == 63) pre[n] = incl;
  }
  __syncthreads();
}

__device__ __forceinline__ uint4 ld_global16(const unsigned char* p) {
  return *reinterpret_cast<const uint4*>(p);
}
__device__ __forceinline__ uint4 ld_lds16(const unsigned char* p) {
  return *reinterpret_cast<const uint4*>(p);
}

// 16x16 forms: one 16-byte slice per lane, 64 bytes of each of 16 rows per
// wave instruction.  Lane l holds row (l % 16) and slice (l / 16) of a 64-byte
// step; the A and B lanes of the same index hold the same dimensions.
// Accumulator: register i of lane l is row 4 (l / 16) + i, column l % 16.
typedef __attribute__((ext_vector_type(4))) float f32x4;
template <int FMT>
__device__ __forceinline__ void mma16x16(const uint4& a, const uint4& b, f32x4& acc);
template <>
__device__ __forceinline__ void mma16x16<GT_POOL_BF16>(const uint4& a, const uint4& b, f32x4& acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma16x16<GT_POOL_FP8E4M3>(const uint4& a, const uint4& b,
                                                          f32x4& acc) {
  const long a0 = (long)(((unsigned long)a.y << 32) | a.x);
  const long a1 = (long)(((unsigned long)a.w << 32) | a.z);
  const long b0 = (long)(((unsigned long)b.y << 32) | b.x);
  const long b1 = (long)(((unsigned long)b.w << 32) | b.z);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma16x16<GT_POOL_F32>(const uint4& a, const uint4& b, f32x4& acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
}

// gfx950 f8f6f4 forms for float8 (e4m3: format 0 for both operands, no
// block scales): 32 bytes per lane, the lane's two 16-byte slices a0, a1 and
// the matching slices b0, b1 of the other operand, so A and B lanes again
// carry the same dimensions.  Same numerics as the fp8 forms above (measured
// equal), twice the products per instruction.
typedef __attribute__((ext_vector_type(8))) int i32x8;
__device__ __forceinline__ i32x8 pack32(const uint4& x0, const uint4& x1) {
  i32x8 v;
  v[0] = (int)x0.x; v[1] = (int)x0.y; v[2] = (int)x0.z; v[3] = (int)x0.w;
  v[4] = (int)x1.x; v[5] = (int)x1.y; v[6] = (int)x1.z; v[7] = (int)x1.w;
  return v;
}
__device__ __forceinline__ void mma_f8_16x16x128(const uint4& a0, const uint4& a1, const uint4& b0,
                                                 const uint4& b1, f32x4& acc) {
  acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(pack32(a0, a1), pack32(b0, b1), acc, 0, 0,
                                                        0, 0, 0, 0);
}
__device__ __forceinline__ void mma_f8_32x32x64(const uint4& a0, const uint4& a1, const uint4& b0,
                                                const uint4& b1, f32x16& acc) {
  acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(pack32(a0, a1), pack32(b0, b1), acc, 0, 0,
                                                       0, 0, 0, 0);
}

// Index i with pre[i] <= g < pre[i + 1] (pre ascending, n + 1 values).
__device__ __forceinline__ int find_slot(const uint32_t* pre, int n, uint32_t g) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

constexpr int kPipe = 8;  // 64-byte steps of a lane's two rows fetched ahead

// One level step of the sparse walk.  Workgroup -> XCD x = blockIdx % 8 (the
// hardware deals workgroups to XCDs round robin), which owns the buckets
// [x R, x R + R).  Within an XCD the workgroups split the query tiles; when
// there are fewer tiles than workgroups, the c workgroups of a tile each take
// part m of every bucket.  Every workgroup goes through its buckets in
// order, so at any moment the XCD's workgroups read the same subtrees for
// different tiles and the repeated pool rows are found in L2.
template <int FMT, int NSTEPS>
__global__ __launch_bounds__(kWalkThreads, 1) void k_walk_level(WalkLevelArgs a) {
  using F = WalkFmt<FMT>;
  constexpr int TQ = F::TQ;
  constexpr int NQB = TQ / 16;  // 16-query column blocks
  __shared__ __attribute__((aligned(16))) unsigned char qlds[TQ * (F::MAXDP * F::ESZ + 16)];
  static_assert(kMaxBucketsPerXcd <= 64, "one bucket per lane of wave 0");
  __shared__ uint32_t gpre[kMaxBucketsPerXcd + 1];
  __shared__ uint32_t glo[kMaxBucketsPerXcd], ghi[kMaxBucketsPerXcd];
  // Thresholds of the tile.  Read from LDS in the loop: a value loaded from
  // global memory before the loop would make the compiler wait for every
  // load in flight at its first use in each iteration.
  __shared__ float thr_lds[TQ];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const int rowbytes = a.dp * F::ESZ;
  const int rs = rowbytes + 16;           // LDS row stride (bank spread)
  // 64-byte steps per row; a compile-time count (the common padded widths)
  // unrolls the stage loop completely
  const int nsteps = NSTEPS > 0 ? NSTEPS : rowbytes / 64;
  const int c16 = lane & 15, g4 = lane >> 4;

  const int nbk = 1 << a.nb;
  const int xs = nbk < kXcds ? nbk : kXcds;
  const int R = nbk / xs;
  const int x = blockIdx.x % kXcds;
  const int W = gridDim.x / kXcds, j = blockIdx.x / kXcds;
  if (x >= xs) return;
  int t0, tstep, m, c;
  if (a.nt <= W) {
    t0 = j % a.nt;
    tstep = a.nt;
    m = j / a.nt;
    c = (W - 1 - t0) / a.nt + 1;
  } else {
    t0 = j;
    tstep = W;
    m = 0;
    c = 1;
  }
  const int bshift = a.level - a.nb;  // node -> bucket
  unsigned long long pairs = 0;

  for (int t = t0; t < a.nt; t += tstep) {
    const uint64_t tmask = a.tile_mask[t];
    __syncthreads();  // LDS of the previous tile no longer read
    if (wave == 0) {  // groups of this workgroup's share of each bucket (R <= 16)
      uint32_t ng = 0, lo = 0, hi = 0;
      if (lane < R && tmask) {
        const uint32_t n = a.dense ? (1u << bshift)
                                   : min(a.in_count[(size_t)(x * R + lane) * a.nt + t], (uint32_t)a.bcap);
        lo = (uint32_t)(((uint64_t)n * m) / c);
        hi = (uint32_t)(((uint64_t)n * (m + 1)) / c);
        ng = (hi - lo + kGroupEntries - 1) / kGroupEntries;
      }
      uint32_t incl = ng;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane < R) {
        gpre[lane] = incl - ng;
        glo[lane] = lo;
        ghi[lane] = hi;
      }
      if (lane == 63) gpre[R] = incl;
    }
    __syncthreads();
    const uint32_t gtot = gpre[R];
    if (gtot == 0) continue;
    {
      const unsigned char* src =
          reinterpret_cast<const unsigned char*>(a.qtile) + (size_t)t * TQ * rowbytes;
      // 8 loads in flight per thread before their LDS stores (a plain
      // load-store loop would pay one memory latency per 16 bytes)
      const int vec_per_row = rowbytes / 16;
      const int nvec = TQ * vec_per_row;
      for (int v0 = 0; v0 < nvec; v0 += 8 * kWalkThreads) {
        uint4 buf[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int v = v0 + k * kWalkThreads + tid;
          const int vv = v < nvec ? v : nvec - 1;
          const int row = vv / vec_per_row, col = vv - row * vec_per_row;
          buf[k] = *reinterpret_cast<const uint4*>(src + (size_t)row * rowbytes + col * 16);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int v = v0 + k * kWalkThreads + tid;
          if (v < nvec) {
            const int row = v / vec_per_row, col = v - row * vec_per_row;
            *reinterpret_cast<uint4*>(qlds + row * rs + col * 16) = buf[k];
          }
        }
      }
    }
    if (tid < TQ) {
      const int qi = t * TQ + tid;
      float th = a.thr[qi];
      if (FMT == GT_POOL_FP8E4M3) th = ldexpf(th * kFp8ThrFactor, -(a.qexp[qi] + a.lexp));
      thr_lds[tid] = th;
    }
    __syncthreads();

    // entries of group gg held by this lane: rows c16 (entry c16 / 2) and
    // 16 + c16 (entry 8 + c16 / 2) of the group's 32 child rows
    auto fetch = [&](uint32_t gg, uint32_t& p0, uint64_t& pm0, uint32_t& p1, uint64_t& pm1,
                     uint32_t& slot) {
      const int r = find_slot(gpre, R, gg);
      const uint32_t e0 = glo[r] + (gg - gpre[r]) * kGroupEntries + (c16 >> 1);
      const uint32_t e1 = e0 + 8;
      const uint32_t hi = ghi[r];
      const uint32_t bk = (uint32_t)(x * R + r);
      slot = bk * (uint32_t)a.nt + (uint32_t)t;
      // Loads are issued in both input modes and for padding lanes (at the
      // group's first entry, always valid) so that no branch separates them
      // from their use; dense input (every pool of the bucket) ignores them.
      const size_t base = (size_t)slot * a.bcap;
      const uint32_t ef = e0 - (c16 >> 1);
      const uint32_t i0 = e0 < hi ? e0 : ef, i1 = e1 < hi ? e1 : ef;
      const uint32_t ld0 = a.in_node[base + i0], ld1 = a.in_node[base + i1];
      const uint64_t lm0 = a.in_mask[base + i0], lm1 = a.in_mask[base + i1];
      const uint32_t first = bk << bshift;
      p0 = a.dense ? first + i0 : ld0;
      p1 = a.dense ? first + i1 : ld1;
      pm0 = e0 < hi ? (a.dense ? tmask : lm0) : 0ull;
      pm1 = e1 < hi ? (a.dense ? tmask : lm1) : 0ull;
    };
    // Rows this lane loads.  A load instruction gives each 4 consecutive
    // lanes 64 contiguous bytes of one row (lanes 4R .. 4R+3: row R of the
    // block, entry R / 2, child R % 2), so each lane quad touches one cache
    // line; the matrix-core layout (row = lane % 16) would give every quad
    // four rows.  p0 / p1 are the entries of this lane's output rows
    // (c16 / 2 and 8 + c16 / 2); lane 2e holds entry e.
    auto rows_of = [&](uint32_t p0, uint32_t p1, const unsigned char*& r0,
                       const unsigned char*& r1) {
      const int src = 2 * (lane >> 3);
      const uint32_t q0 = (uint32_t)__shfl((int)p0, src, 64);
      const uint32_t q1 = (uint32_t)__shfl((int)p1, src, 64);
      const uint32_t ch = (uint32_t)((lane >> 2) & 1);
      const unsigned char* base = reinterpret_cast<const unsigned char*>(a.child_rows) + 16 * (lane & 3);
      r0 = base + (size_t)(2u * q0 + ch) * rowbytes;
      r1 = base + (size_t)(2u * q1 + ch) * rowbytes;
    };
    // Loaded slice -> matrix-core operand: lane 16 g + i takes row i, 16-byte
    // chunk g of the step, which the load left in lane 4 i + g.
    const int bp_addr = 4 * (4 * c16 + g4);
    auto to_mfma = [&](const uint4& v) {
      uint4 r;
      r.x = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.x);
      r.y = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.y);
      r.z = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.z);
      r.w = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.w);
      return r;
    };
    // The steps of consecutive groups form one pipeline: while a stage is
    // multiplied, the next one (possibly the first stage of the wave's next
    // group) is in flight.  Loads are unconditional (steps past a row re-read
    // its last step) so the number in flight is static and the compiler waits
    // only for the stage it is about to use.
    const int slast = nsteps - 1;
    uint4 bA0[kPipe], bA1[kPipe], bB0[kPipe], bB1[kPipe];
    uint32_t np0 = 0, np1 = 0, nslot = 0;
    uint64_t npm0 = 0ull, npm1 = 0ull;
    if ((uint32_t)wave < gtot) {
      fetch(wave, np0, npm0, np1, npm1, nslot);
      const unsigned char *r0, *r1;
      rows_of(np0, np1, r0, r1);
#pragma unroll
      for (int u = 0; u < kPipe; ++u) {
        const int st = u < slast ? u : slast;
        bA0[u] = ld_global16(r0 + 64 * st);
        bA1[u] = ld_global16(r1 + 64 * st);
      }
    }
    bool pend = false;
    uint32_t pend_child = 0, pend_slot = 0;
    uint64_t pend_mask = 0ull, pend_bal = 0ull;

    for (uint32_t gg = wave; gg < gtot; gg += nwaves) {
      const uint32_t p0 = np0, p1 = np1, slot = nslot;
      const uint64_t pm0 = npm0, pm1 = npm1;
      const uint32_t child0 = 2u * p0 + (uint32_t)(lane & 1);
      const uint32_t child1 = 2u * p1 + (uint32_t)(lane & 1);
      const unsigned char *arow0, *arow1;
      rows_of(p0, p1, arow0, arow1);
      const unsigned char* brow = qlds + c16 * rs + 16 * g4;
      const bool has_next = gg + nwaves < gtot;
      // the next group's entries (this group's again when there is none)
      fetch(has_next ? gg + nwaves : gg, np0, npm0, np1, npm1, nslot);
      // reserve output slots for the previous group; the reply is awaited
      // only after this group's matrix work
      if (a.bitmap && lane < 16) {
        if (pm0) {
          const uint64_t row = (uint64_t)a.bit_base + child0;
          atomicOr(&a.bitmap[row >> 5], 1u << (row & 31));
        }
        if (pm1) {
          const uint64_t row = (uint64_t)a.bit_base + child1;
          atomicOr(&a.bitmap[row >> 5], 1u << (row & 31));
        }
      }
      uint32_t pend_base = 0;
      if (pend && lane == 0) pend_base = atomicAdd(&a.out_count[pend_slot], (uint32_t)__popcll(pend_bal));

      f32x4 acc[2][NQB];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int qb = 0; qb < NQB; ++qb)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[rb][qb][i] = 0.0f;

      auto step = [&](const uint4& l0, const uint4& l1, int s) {
        const uint4 x0 = to_mfma(l0), x1 = to_mfma(l1);
#pragma unroll
        for (int qb = 0; qb < NQB; ++qb) {
          const uint4 bq = ld_lds16(brow + qb * 16 * rs + 64 * s);
          mma16x16<FMT>(x0, bq, acc[0][qb]);
          mma16x16<FMT>(x1, bq, acc[1][qb]);
        }
      };
      // float8: steps s and s + 1 in one 16x16x128 product
      auto step2 = [&](const uint4& l0a, const uint4& l1a, const uint4& l0b, const uint4& l1b,
                       int s) {
        const uint4 x0a = to_mfma(l0a), x1a = to_mfma(l1a);
        const uint4 x0b = to_mfma(l0b), x1b = to_mfma(l1b);
#pragma unroll
        for (int qb = 0; qb < NQB; ++qb) {
          const uint4 bqa = ld_lds16(brow + qb * 16 * rs + 64 * s);
          const uint4 bqb = ld_lds16(brow + qb * 16 * rs + 64 * (s + 1));
          mma_f8_16x16x128(x0a, x0b, bqa, bqb, acc[0][qb]);
          mma_f8_16x16x128(x1a, x1b, bqa, bqb, acc[1][qb]);
        }
      };
#pragma unroll
      for (int s0 = 0; s0 < nsteps; s0 += 2 * kPipe) {
#pragma unroll
        for (int u = 0; u < kPipe; ++u) {
          const int st = s0 + kPipe + u < slast ? s0 + kPipe + u : slast;
          bB0[u] = ld_global16(arow0 + 64 * st);
          bB1[u] = ld_global16(arow1 + 64 * st);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (FMT == GT_POOL_FP8E4M3) {
          // (a float8 row has an even number of 64-byte steps)
#pragma unroll
          for (int u = 0; u < kPipe; u += 2)
            if (s0 + u < nsteps) step2(bA0[u], bA1[u], bA0[u + 1], bA1[u + 1], s0 + u);
        } else {
#pragma unroll
          for (int u = 0; u < kPipe; ++u)
            if (s0 + u < nsteps) step(bA0[u], bA1[u], s0 + u);
        }
        __builtin_amdgcn_sched_barrier(0);
        {
          // next stage of this group, or the first stage of the next group
          const bool same = s0 + 2 * kPipe < nsteps;
          if (!same && pend) {
            // Survivors of the previous group go out here, before the next
            // group's loads are issued: waiting for the slot reservation then
            // only waits for loads that the next stage needs anyway.
            pend_base = __shfl(pend_base, 0, 64);
            if (lane < 32 && pend_mask) {
              const uint32_t pos = pend_base + (uint32_t)__popcll(pend_bal & ((1ull << lane) - 1ull));
              if (pos < a.bcap) {
                const size_t o = (size_t)pend_slot * a.bcap + pos;
                a.out_node[o] = pend_child;
                a.out_mask[o] = pend_mask;
              } else {
                atomicOr(a.over, 1u);
              }
            }
            pend = false;
          }
          const unsigned char *r0 = arow0, *r1 = arow1;
          if (!same) rows_of(np0, np1, r0, r1);
          const int sf = same ? s0 + 2 * kPipe : 0;
#pragma unroll
          for (int u = 0; u < kPipe; ++u) {
            const int st = sf + u < slast ? sf + u : slast;
            bA0[u] = ld_global16(r0 + 64 * st);
            bA1[u] = ld_global16(r1 + 64 * st);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (FMT == GT_POOL_FP8E4M3) {
#pragma unroll
          for (int u = 0; u < kPipe; u += 2)
            if (s0 + kPipe + u < nsteps)
              step2(bB0[u], bB1[u], bB0[u + 1], bB1[u + 1], s0 + kPipe + u);
        } else {
#pragma unroll
          for (int u = 0; u < kPipe; ++u)
            if (s0 + kPipe + u < nsteps) step(bB0[u], bB1[u], s0 + kPipe + u);
        }
        __builtin_amdgcn_sched_barrier(0);
      }

      // Child row r (lane r < 32): block r / 16, register r % 4, lane group
      // (r % 16) / 4; column block qb supplies query bits 16 qb .. 16 qb + 15.
      const int gsel = 16 * ((lane & 15) >> 2);
      uint64_t mine = 0ull;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          uint64_t part = 0ull;
#pragma unroll
          for (int qb = 0; qb < NQB; ++qb) {
            const uint64_t bal = __ballot(acc[rb][qb][i] >= thr_lds[16 * qb + c16]);
            part |= ((bal >> gsel) & 0xffffull) << (16 * qb);
          }
          if ((lane >> 4) == rb && (lane & 3) == i) mine = part;
        }
      const uint64_t pm_own = lane < 16 ? pm0 : pm1;
      mine = lane < 32 ? (mine & pm_own) : 0ull;
      if (lane < 32) pairs += (unsigned long long)__popcll(pm_own);
      pend_bal = __ballot(mine != 0ull);
      pend = pend_bal != 0ull;
      pend_child = lane < 16 ? child0 : child1;
      pend_mask = mine;
      pend_slot = slot;
    }
    if (pend) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&a.out_count[pend_slot], (uint32_t)__popcll(pend_bal));
      base = __shfl(base, 0, 64);
      if (lane < 32 && pend_mask) {
        const uint32_t pos = base + (uint32_t)__popcll(pend_bal & ((1ull << lane) - 1ull));
        if (pos < a.bcap) {
          const size_t o = (size_t)pend_slot * a.bcap + pos;
          a.out_node[o] = pend_child;
          a.out_mask[o] = pend_mask;
        } else {
          atomicOr(a.over, 1u);
        }
      }
    }
  }
  if (a.stat_pairs) {
    for (int o = 32; o >= 1; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
    if (lane == 0 && pairs) atomicAdd(a.stat_pairs, pairs);
  }
}

// Level step for rows wider than the LDS query tile (padded width above
// WalkFmt::MAXDP: the whole tile no longer fits in LDS).  Same buckets, XCD
// split, groups and decisions as k_walk_level, but the tile's query rows pass
// through LDS in windows of kWideWindow bytes: the workgroup's waves work in
// rounds of one group each, and within a round every wave multiplies its
// group's 32 child rows window by window, all waves stepping through the
// windows together (one barrier pair per window).  Each window's 64-byte
// steps are loaded eight at a time.  Scores are the same sums over the same
// dimensions (in another order), so the decisions keep their slack.
constexpr int kWideWindow = 2048;  // bytes of every query row per LDS window

template <int FMT>
__global__ __launch_bounds__(kWalkThreads, 1) void k_walk_wide(WalkLevelArgs a) {
  using F = WalkFmt<FMT>;
  constexpr int TQ = F::TQ;
  constexpr int NQB = TQ / 16;
  constexpr int RS = kWideWindow + 16;  // LDS row stride (bank spread)
  __shared__ __attribute__((aligned(16))) unsigned char qlds[TQ * RS];
  __shared__ uint32_t gpre[kMaxBucketsPerXcd + 1];
  __shared__ uint32_t glo[kMaxBucketsPerXcd], ghi[kMaxBucketsPerXcd];
  __shared__ float thr_lds[TQ];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const int rowbytes = a.dp * F::ESZ;
  const int nwin = (rowbytes + kWideWindow - 1) / kWideWindow;
  const int c16 = lane & 15, g4 = lane >> 4;

  const int nbk = 1 << a.nb;
  const int xs = nbk < kXcds ? nbk : kXcds;
  const int R = nbk / xs;
  const int x = blockIdx.x % kXcds;
  const int W = gridDim.x / kXcds, j = blockIdx.x / kXcds;
  if (x >= xs) return;
  int t0, tstep, m, c;
  if (a.nt <= W) {
    t0 = j % a.nt;
    tstep = a.nt;
    m = j / a.nt;
    c = (W - 1 - t0) / a.nt + 1;
  } else {
    t0 = j;
    tstep = W;
    m = 0;
    c = 1;
  }
  const int bshift = a.level - a.nb;
  unsigned long long pairs = 0;

  for (int t = t0; t < a.nt; t += tstep) {
    const uint64_t tmask = a.tile_mask[t];
    __syncthreads();
    if (wave == 0) {
      uint32_t ng = 0, lo = 0, hi = 0;
      if (lane < R && tmask) {
        const uint32_t n = a.dense ? (1u << bshift)
                                   : min(a.in_count[(size_t)(x * R + lane) * a.nt + t], (uint32_t)a.bcap);
        lo = (uint32_t)(((uint64_t)n * m) / c);
        hi = (uint32_t)(((uint64_t)n * (m + 1)) / c);
        ng = (hi - lo + kGroupEntries - 1) / kGroupEntries;
      }
      uint32_t incl = ng;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane < R) {
        gpre[lane] = incl - ng;
        glo[lane] = lo;
        ghi[lane] = hi;
      }
      if (lane == 63) gpre[R] = incl;
    }
    if (tid < TQ) {
      const int qi = t * TQ + tid;
      float th = a.thr[qi];
      if (FMT == GT_POOL_FP8E4M3) th = ldexpf(th * kFp8ThrFactor, -(a.qexp[qi] + a.lexp));
      thr_lds[tid] = th;
    }
    __syncthreads();
    const uint32_t gtot = gpre[R];
    if (gtot == 0) continue;
    const unsigned char* qsrc = reinterpret_cast<const unsigned char*>(a.qtile) + (size_t)t * TQ * rowbytes;

    for (uint32_t base = 0; base < gtot; base += (uint32_t)nwaves) {
      const uint32_t gg = base + (uint32_t)wave;
      const bool valid = gg < gtot;  // uniform per wave
      // group gg's entries held by this lane (rows c16 and 16 + c16 of the
      // group's 32 child rows), as in k_walk_level; a wave without a group
      // this round takes the last group with empty masks
      const uint32_t ge = valid ? gg : gtot - 1;
      const int r = find_slot(gpre, R, ge);
      const uint32_t e0 = glo[r] + (ge - gpre[r]) * kGroupEntries + (c16 >> 1);
      const uint32_t e1 = e0 + 8;
      const uint32_t ehi = ghi[r];
      const uint32_t bk = (uint32_t)(x * R + r);
      const uint32_t slot = bk * (uint32_t)a.nt + (uint32_t)t;
      const size_t ebase = (size_t)slot * a.bcap;
      const uint32_t ef = e0 - (c16 >> 1);
      const uint32_t i0 = e0 < ehi ? e0 : ef, i1 = e1 < ehi ? e1 : ef;
      const uint32_t first = bk << bshift;
      const uint32_t p0 = a.dense ? first + i0 : a.in_node[ebase + i0];
      const uint32_t p1 = a.dense ? first + i1 : a.in_node[ebase + i1];
      const uint64_t pm0 = (valid && e0 < ehi) ? (a.dense ? tmask : a.in_mask[ebase + i0]) : 0ull;
      const uint64_t pm1 = (valid && e1 < ehi) ? (a.dense ? tmask : a.in_mask[ebase + i1]) : 0ull;
      // rows this lane loads: lanes 4R'..4R'+3 take 64 contiguous bytes of
      // row R' (entry R' / 2, child R' % 2) of each block
      const int src = 2 * (lane >> 3);
      const uint32_t q0 = (uint32_t)__shfl((int)p0, src, 64);
      const uint32_t q1 = (uint32_t)__shfl((int)p1, src, 64);
      const uint32_t ch = (uint32_t)((lane >> 2) & 1);
      const unsigned char* rbase = reinterpret_cast<const unsigned char*>(a.child_rows) + 16 * (lane & 3);
      const unsigned char* arow0 = rbase + (size_t)(2u * q0 + ch) * rowbytes;
      const unsigned char* arow1 = rbase + (size_t)(2u * q1 + ch) * rowbytes;
      const int bp_addr = 4 * (4 * c16 + g4);
      auto to_mfma = [&](const uint4& v) {
        uint4 o;
        o.x = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.x);
        o.y = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.y);
        o.z = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.z);
        o.w = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.w);
        return o;
      };
      f32x4 acc[2][NQB];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int qb = 0; qb < NQB; ++qb)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[rb][qb][i] = 0.0f;

      for (int wi = 0; wi < nwin; ++wi) {
        const int wofs = wi * kWideWindow;
        const int wbytes = rowbytes - wofs < kWideWindow ? rowbytes - wofs : kWideWindow;
        __syncthreads();  // every wave is done with the previous window
        {
          const int vpr = wbytes / 16;  // 16-byte vectors per row in this window
          const int nvec = TQ * vpr;
          for (int v0 = 0; v0 < nvec; v0 += 8 * kWalkThreads) {
            uint4 buf[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int v = v0 + k * kWalkThreads + tid;
              const int vv = v < nvec ? v : nvec - 1;
              const int row = vv / vpr, col = vv - row * vpr;
              buf[k] = *reinterpret_cast<const uint4*>(qsrc + (size_t)row * rowbytes + wofs + col * 16);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int v = v0 + k * kWalkThreads + tid;
              if (v < nvec) {
                const int row = v / vpr, col = v - row * vpr;
                *reinterpret_cast<uint4*>(qlds + row * RS + col * 16) = buf[k];
              }
            }
          }
        }
        __syncthreads();
        if (valid) {
          const int wsteps = wbytes / 64;
          const unsigned char* brow = qlds + c16 * RS + 16 * g4;
          for (int s0 = 0; s0 < wsteps; s0 += 8) {
            uint4 l0[8], l1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int st = s0 + u < wsteps ? s0 + u : wsteps - 1;
              l0[u] = ld_global16(arow0 + wofs + 64 * st);
              l1[u] = ld_global16(arow1 + wofs + 64 * st);
            }
            if constexpr (FMT == GT_POOL_FP8E4M3) {
              // steps s and s + 1 in one 16x16x128 product (an even count per window)
#pragma unroll
              for (int u = 0; u < 8; u += 2) {
                if (s0 + u < wsteps) {
                  const uint4 x0a = to_mfma(l0[u]), x1a = to_mfma(l1[u]);
                  const uint4 x0b = to_mfma(l0[u + 1]), x1b = to_mfma(l1[u + 1]);
#pragma unroll
                  for (int qb = 0; qb < NQB; ++qb) {
                    const uint4 bqa = ld_lds16(brow + qb * 16 * RS + 64 * (s0 + u));
                    const uint4 bqb = ld_lds16(brow + qb * 16 * RS + 64 * (s0 + u + 1));
                    mma_f8_16x16x128(x0a, x0b, bqa, bqb, acc[0][qb]);
                    mma_f8_16x16x128(x1a, x1b, bqa, bqb, acc[1][qb]);
                  }
                }
              }
            } else {
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                if (s0 + u < wsteps) {
                  const uint4 x0 = to_mfma(l0[u]), x1 = to_mfma(l1[u]);
#pragma unroll
                  for (int qb = 0; qb < NQB; ++qb) {
                    const uint4 bq = ld_lds16(brow + qb * 16 * RS + 64 * (s0 + u));
                    mma16x16<FMT>(x0, bq, acc[0][qb]);
                    mma16x16<FMT>(x1, bq, acc[1][qb]);
                  }
                }
              }
            }
          }
        }
      }
      if (!valid) continue;
      if (a.bitmap && lane < 16) {
        const uint32_t child0 = 2u * p0 + (uint32_t)(lane & 1), child1 = 2u * p1 + (uint32_t)(lane & 1);
        if (pm0) {
          const uint64_t row = (uint64_t)a.bit_base + child0;
          atomicOr(&a.bitmap[row >> 5], 1u << (row & 31));
        }
        if (pm1) {
          const uint64_t row = (uint64_t)a.bit_base + child1;
          atomicOr(&a.bitmap[row >> 5], 1u << (row & 31));
        }
      }
      // survival bits as in k_walk_level: lane r < 32 ends with child row r's mask
      const int gsel = 16 * ((lane & 15) >> 2);
      uint64_t mine = 0ull;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          uint64_t part = 0ull;
#pragma unroll
          for (int qb = 0; qb < NQB; ++qb) {
            const uint64_t bal = __ballot(acc[rb][qb][i] >= thr_lds[16 * qb + c16]);
            part |= ((bal >> gsel) & 0xffffull) << (16 * qb);
          }
          if ((lane >> 4) == rb && (lane & 3) == i) mine = part;
        }
      const uint64_t pm_own = lane < 16 ? pm0 : pm1;
      mine = lane < 32 ? (mine & pm_own) : 0ull;
      if (lane < 32) pairs += (unsigned long long)__popcll(pm_own);
      const uint64_t bal = __ballot(mine != 0ull);
      if (bal == 0ull) continue;
      uint32_t obase = 0;
      if (lane == 0) obase = atomicAdd(&a.out_count[slot], (uint32_t)__popcll(bal));
      obase = __shfl(obase, 0, 64);
      if (mine) {
        const uint32_t pos = obase + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (pos < a.bcap) {
          const size_t o = (size_t)slot * a.bcap + pos;
          a.out_node[o] = 2u * (lane < 16 ? p0 : p1) + (uint32_t)(lane & 1);
          a.out_mask[o] = mine;
        } else {
          atomicOr(a.over, 1u);
        }
      }
    }
  }
  if (a.stat_pairs) {
    for (int o = 32; o >= 1; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
    if (lane == 0 && pairs) atomicAdd(a.stat_pairs, pairs);
  }
}

// Level step with subtraction (bfloat16 pools; paper Sec. 2 and Alg. 1 derive
// the score of one half of a pool from the pool's score and the other half's).
// Every entry carries a score record: upper bounds of its pool's real score
// for all 64 queries of the tile, as bfloat16, query q at 4 (q % 16) + q / 16
// (so that a lane's four values of a pool are eight contiguous bytes).  A
// wave takes 32 entries and reads only their right children (one row each):
// the right child's score s is computed with the matrix cores and tested as
// in k_walk_level; the left child's real score is at most
//   U = diff_upper(sp, score_lower(s, a_b))
// (sp the entry's record, a_b the query's absolute term), and the left child
// is kept for query b iff U >= tau'_b.  Where the right child holds rows at
// or beyond the call's epoch (which later inserts may have grown), U is just
// sp: a part of a pool never scores above the pool.  Every kept child gets a
// complete record (score_upper(s) for the right child, U for the left, each
// rounded up to bfloat16), so the values of queries that are not live are
// bounds too.  Halves the pool rows read per level.
constexpr int kSubGroup = 32;  // entries per wave step
constexpr int kSubPipe = 4;   // 64-byte steps of a lane's two rows fetched ahead
constexpr int kSubThreads = kWalkThreads;  // threads per workgroup

template <int NSTEPS, int PIPE>
__global__ __launch_bounds__(kSubThreads, 1) void k_walk_sub(WalkLevelArgs a) {
  constexpr int FMT = GT_POOL_BF16;
  using F = WalkFmt<FMT>;
  constexpr int TQ = F::TQ;
  constexpr int NQB = TQ / 16;
  static_assert(TQ == 64, "records hold 64 queries");
  __shared__ __attribute__((aligned(16))) unsigned char qlds[TQ * (F::MAXDP * F::ESZ + 16)];
  __shared__ uint32_t gpre[kMaxBucketsPerXcd + 1];
  __shared__ uint32_t glo[kMaxBucketsPerXcd], ghi[kMaxBucketsPerXcd];
  __shared__ float thr_lds[TQ], sabs_lds[TQ];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const int rowbytes = a.dp * F::ESZ;
  const int rs = rowbytes + 16;
  const int nsteps = NSTEPS > 0 ? NSTEPS : rowbytes / 64;
  const int c16 = lane & 15, g4 = lane >> 4;
  const int e32 = lane & 31;  // the entry this lane fetches (lanes 32-63 repeat 0-31)

  const int nbk = 1 << a.nb;
  const int xs = nbk < kXcds ? nbk : kXcds;
  const int R = nbk / xs;
  const int x = blockIdx.x % kXcds;
  const int W = gridDim.x / kXcds, j = blockIdx.x / kXcds;
  if (x >= xs) return;
  int t0, tstep, m, c;
  if (a.nt <= W) {
    t0 = j % a.nt;
    tstep = a.nt;
    m = j / a.nt;
    c = (W - 1 - t0) / a.nt + 1;
  } else {
    t0 = j;
    tstep = W;
    m = 0;
    c = 1;
  }
  // right child 2p+1 of a level-l pool p covers leaves [(2p+1) 2^s, (2p+2) 2^s)
  const int lshift = a.depth - a.level - 1;
  // subtraction is used where the right child lies wholly below the epoch:
  // then the parent and both children hold only rows the call sees, none of
  // which an insert changes
  auto sub_ok = [&](uint32_t ep) {
    return ((uint64_t)(2u * ep + 2u) << lshift) <= (uint64_t)a.n_epoch;
  };
  // upper bound of the left child's score from the pool's bound sp and the
  // right child's computed score sr (a right score that overflowed gives no
  // lower bound)
  auto left_ub = [&](float sp, float sr, float sa, bool sub) {
    if (!sub || !(sr < INFINITY)) return sp;
    return diff_upper(sp, score_lower(sr, sa));
  };
  const float aup = score_abs_up(a.dp);
  unsigned long long pairs = 0;

  for (int t = t0; t < a.nt; t += tstep) {
    const uint64_t tmask = a.tile_mask[t];
    __syncthreads();
    if (wave == 0) {
      uint32_t ng = 0, lo = 0, hi = 0;
      if (lane < R && tmask) {
        const uint32_t n = min(a.in_count[(size_t)(x * R + lane) * a.nt + t], (uint32_t)a.bcap);
        lo = (uint32_t)(((uint64_t)n * m) / c);
        hi = (uint32_t)(((uint64_t)n * (m + 1)) / c);
        ng = (hi - lo + kSubGroup - 1) / kSubGroup;
      }
      uint32_t incl = ng;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane < R) {
        gpre[lane] = incl - ng;
        glo[lane] = lo;
        ghi[lane] = hi;
      }
      if (lane == 63) gpre[R] = incl;
    }
    __syncthreads();
    const uint32_t gtot = gpre[R];
    if (gtot == 0) continue;
    {
      const unsigned char* src =
          reinterpret_cast<const unsigned char*>(a.qtile) + (size_t)t * TQ * rowbytes;
      const int vec_per_row = rowbytes / 16;
      const int nvec = TQ * vec_per_row;
      for (int v0 = 0; v0 < nvec; v0 += 8 * kSubThreads) {
        uint4 buf[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int v = v0 + k * kSubThreads + tid;
          const int vv = v < nvec ? v : nvec - 1;
          const int row = vv / vec_per_row, col = vv - row * vec_per_row;
          buf[k] = *reinterpret_cast<const uint4*>(src + (size_t)row * rowbytes + col * 16);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int v = v0 + k * kSubThreads + tid;
          if (v < nvec) {
            const int row = v / vec_per_row, col = v - row * vec_per_row;
            *reinterpret_cast<uint4*>(qlds + row * rs + col * 16) = buf[k];
          }
        }
      }
    }
    if (tid < TQ) {
      thr_lds[tid] = a.thr[t * TQ + tid];
      sabs_lds[tid] = a.sabs[t * TQ + tid];
    }
    __syncthreads();

    // entry e32 of group gg: its pool, mask and position (padding lanes take
    // the group's first entry with an empty mask, so every load is valid)
    auto fetch = [&](uint32_t gg, uint32_t& p, uint64_t& pm, uint32_t& pos, uint32_t& slot) {
      const int r = find_slot(gpre, R, gg);
      const uint32_t ef = glo[r] + (gg - gpre[r]) * kSubGroup;
      const uint32_t e = ef + (uint32_t)e32;
      const uint32_t hi = ghi[r];
      slot = (uint32_t)(x * R + r) * (uint32_t)a.nt + (uint32_t)t;
      const uint32_t ie = e < hi ? e : ef;
      pos = (uint32_t)((size_t)slot * a.bcap + ie);
      p = a.in_node[pos];
      const uint64_t lm = a.in_mask[pos];
      pm = e < hi ? lm : 0ull;
    };
    // The right-child rows this lane loads: lanes 4R' .. 4R'+3 take 64
    // contiguous bytes of entry R' (block 0) and entry 16 + R' (block 1).
    auto rows_of = [&](uint32_t p, const unsigned char*& r0, const unsigned char*& r1) {
      const uint32_t q0 = (uint32_t)__shfl((int)p, lane >> 2, 64);
      const uint32_t q1 = (uint32_t)__shfl((int)p, 16 + (lane >> 2), 64);
      const unsigned char* base = reinterpret_cast<const unsigned char*>(a.child_rows) + 16 * (lane & 3);
      r0 = base + (size_t)(2u * q0 + 1u) * rowbytes;
      r1 = base + (size_t)(2u * q1 + 1u) * rowbytes;
    };
    const int bp_addr = 4 * (4 * c16 + g4);
    auto to_mfma = [&](const uint4& v) {
      uint4 r;
      r.x = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.x);
      r.y = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.y);
      r.z = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.z);
      r.w = (uint32_t)__builtin_amdgcn_ds_bpermute(bp_addr, (int)v.w);
      return r;
    };
    const int slast = nsteps - 1;
    uint4 bA0[PIPE], bA1[PIPE], bB0[PIPE], bB1[PIPE];
    uint32_t np = 0, npos = 0, nslot = 0;
    uint64_t npm = 0ull;
    if ((uint32_t)wave < gtot) {
      fetch(wave, np, npm, npos, nslot);
      const unsigned char *r0, *r1;
      rows_of(np, r0, r1);
#pragma unroll
      for (int u = 0; u < PIPE; ++u) {
        const int st = u < slast ? u : slast;
        bA0[u] = ld_global16(r0 + 64 * st);
        bA1[u] = ld_global16(r1 + 64 * st);
      }
    }

    for (uint32_t gg = wave; gg < gtot; gg += nwaves) {
      const uint32_t p = np, pos = npos, slot = nslot;
      const uint64_t pm = npm;
      const unsigned char *arow0, *arow1;
      rows_of(p, arow0, arow1);
      const unsigned char* brow = qlds + c16 * rs + 16 * g4;
      // the pools' score records, read while the rows are multiplied: for
      // entry 16 rb + 4 (l / 16) + i the bounds of queries c, 16 + c, 32 + c,
      // 48 + c (c = l % 16), eight contiguous bytes
      uint2 prec[2][4];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t eps = (uint32_t)__shfl((int)pos, 16 * rb + 4 * g4 + i, 64);
          prec[rb][i] = *reinterpret_cast<const uint2*>(a.in_rec + (size_t)eps * TQ + 4 * c16);
        }
      const bool has_next = gg + nwaves < gtot;
      fetch(has_next ? gg + nwaves : gg, np, npm, npos, nslot);
      if (a.bitmap && lane < 32 && pm) {
        const uint64_t row = (uint64_t)a.bit_base + 2u * p + 1u;
        atomicOr(&a.bitmap[row >> 5], 1u << (row & 31));
      }

      f32x4 acc[2][NQB];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int qb = 0; qb < NQB; ++qb)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[rb][qb][i] = 0.0f;
      auto step = [&](const uint4& l0, const uint4& l1, int s) {
        const uint4 x0 = to_mfma(l0), x1 = to_mfma(l1);
#pragma unroll
        for (int qb = 0; qb < NQB; ++qb) {
          const uint4 bq = ld_lds16(brow + qb * 16 * rs + 64 * s);
          mma16x16<FMT>(x0, bq, acc[0][qb]);
          mma16x16<FMT>(x1, bq, acc[1][qb]);
        }
      };
#pragma unroll
      for (int s0 = 0; s0 < nsteps; s0 += 2 * PIPE) {
#pragma unroll
        for (int u = 0; u < PIPE; ++u) {
          const int st = s0 + PIPE + u < slast ? s0 + PIPE + u : slast;
          bB0[u] = ld_global16(arow0 + 64 * st);
          bB1[u] = ld_global16(arow1 + 64 * st);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PIPE; ++u)
          if (s0 + u < nsteps) step(bA0[u], bA1[u], s0 + u);
        __builtin_amdgcn_sched_barrier(0);
        {
          const bool same = s0 + 2 * PIPE < nsteps;
          const unsigned char *r0 = arow0, *r1 = arow1;
          if (!same) rows_of(np, r0, r1);
          const int sf = same ? s0 + 2 * PIPE : 0;
#pragma unroll
          for (int u = 0; u < PIPE; ++u) {
            const int st = sf + u < slast ? sf + u : slast;
            bA0[u] = ld_global16(r0 + 64 * st);
            bA1[u] = ld_global16(r1 + 64 * st);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PIPE; ++u)
          if (s0 + PIPE + u < nsteps) step(bB0[u], bB1[u], s0 + PIPE + u);
        __builtin_amdgcn_sched_barrier(0);
      }

      // Element (rb, qb, i) of lane l: entry 16 rb + 4 (l / 16) + i of the
      // group, query 16 qb + l % 16.  Decisions are gathered per entry by
      // ballots (lane j < 32 ends with entry j's masks, as in k_walk_level);
      // then every kept child gets its complete record.
      auto rec_of = [&](int rb, int i, int qb) {
        const uint32_t w = qb < 2 ? prec[rb][i].x : prec[rb][i].y;
        return bf16_to_f32((uint16_t)((qb & 1) ? (w >> 16) : (w & 0xFFFFu)));
      };
      const int gsel = 16 * ((lane & 15) >> 2);
      uint64_t mine_r = 0ull, mine_l = 0ull;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int er = 16 * rb + 4 * g4 + i;
          const uint64_t em = __shfl(pm, er, 64);
          const bool sub = sub_ok((uint32_t)__shfl((int)p, er, 64));
          uint64_t part_r = 0ull, part_l = 0ull;
#pragma unroll
          for (int qb = 0; qb < NQB; ++qb) {
            const int q = 16 * qb + c16;
            const bool live = (em >> q) & 1ull;
            const float sr = acc[rb][qb][i];
            const float th = thr_lds[q];
            const uint64_t br = __ballot(live && sr >= th);
            const uint64_t bl = __ballot(live && left_ub(rec_of(rb, i, qb), sr, sabs_lds[q], sub) >= th);
            part_r |= ((br >> gsel) & 0xffffull) << (16 * qb);
            part_l |= ((bl >> gsel) & 0xffffull) << (16 * qb);
          }
          if ((lane >> 4) == rb && (lane & 3) == i) {
            mine_r = part_r;
            mine_l = part_l;
          }
        }
      // outputs: lane j < 32 the right child of entry j, lane 32 + j its left
      // (the shuffle runs in every lane: a lane that is switched off gives
      // no data to the others)
      const uint64_t left_m = __shfl(mine_l, e32, 64);
      const uint64_t out_m = lane < 32 ? mine_r : left_m;
      if (lane < 32) pairs += 2ull * (unsigned long long)__popcll(pm);
      const uint64_t bal = __ballot(out_m != 0ull);
      if (bal == 0ull) continue;
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&a.out_count[slot], (uint32_t)__popcll(bal));
      base = __shfl(base, 0, 64);
      const uint32_t opos = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
      if (out_m) {
        if (opos < a.bcap) {
          const size_t o = (size_t)slot * a.bcap + opos;
          a.out_node[o] = 2u * p + (lane < 32 ? 1u : 0u);
          a.out_mask[o] = out_m;
        } else {
          atomicOr(a.over, 1u);
        }
      }
      if (!a.out_rec) continue;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int er = 16 * rb + 4 * g4 + i;
          const bool sub = sub_ok((uint32_t)__shfl((int)p, er, 64));
          const bool keep_r = ((bal >> er) & 1ull) != 0ull;
          const bool keep_l = ((bal >> (32 + er)) & 1ull) != 0ull;
          const uint32_t or_ = (uint32_t)__shfl((int)opos, er, 64);
          const uint32_t ol_ = (uint32_t)__shfl((int)opos, 32 + er, 64);
          uint32_t vr[NQB], vl[NQB];
#pragma unroll
          for (int qb = 0; qb < NQB; ++qb) {
            const int q = 16 * qb + c16;
            const float sr = acc[rb][qb][i];
            vr[qb] = bf16_ceil_hi(score_upper(sr, aup));
            vl[qb] = bf16_ceil_hi(left_ub(rec_of(rb, i, qb), sr, sabs_lds[q], sub));
          }
          if (keep_r && or_ < a.bcap)
            *reinterpret_cast<uint2*>(a.out_rec + ((size_t)slot * a.bcap + or_) * TQ + 4 * c16) =
                make_uint2((vr[0] >> 16) | vr[1], (vr[2] >> 16) | vr[3]);
          if (keep_l && ol_ < a.bcap)
            *reinterpret_cast<uint2*>(a.out_rec + ((size_t)slot * a.bcap + ol_) * TQ + 4 * c16) =
                make_uint2((vl[0] >> 16) | vl[1], (vl[2] >> 16) | vl[3]);
        }
    }
  }
  if (a.stat_pairs) {
    for (int o = 32; o >= 1; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
    if (lane == 0 && pairs) atomicAdd(a.stat_pairs, pairs);
  }
}

// Dense level step: every pool of a level against every query, as a matrix
// product with a masked epilogue.  Used where almost every (pool, query tile)
// pair is live (the first tested level): each pool row is read once per
// 256-query column block instead of once per tile.  A workgroup (4 waves, one
// per SIMD) computes 256 pools x 256 queries (4 tiles); wave w owns pools
// 128 (w / 2) .. +127 and tiles 2 (w % 2), 2 (w % 2) + 1: 4 x 4 blocks of
// 32x32 matrix-core tiles whose accumulators fill the wave's accumulation
// registers, so that every 16-byte operand read from LDS feeds four matrix
// products.  K advances 128 bytes per row per stage.  A stage is loaded
// straight from global memory into LDS (no staging registers) one stage
// ahead, into the other of two buffers; within a stage the operands of the
// next K step are read from LDS while the current step's matrix products
// run, and the next stage's first step is read across the stage's barrier.
// Child j of level L survives for query b iff its parent's bit b is set and
// its score reaches tau'_b.  Output: per-(pool, tile) masks for a following
// dense level, or the bucketed sparse frontier for the walk that follows.
//
// LDS layout of a stage: two regions (pool rows, query rows) of 256 rows x
// 128 bytes, each in 32 blocks of 8 rows; row R of a region is row R / 32 of
// block R % 32, and the blocks are 1040 bytes apart.  The 16-byte skew per
// block puts the same chunk of 8 (or 16) consecutive rows on distinct banks,
// so operand reads are conflict-free, and every read of a wave is one base
// register plus an immediate offset.  One direct-to-LDS load instruction
// fills one block (its 64 lanes write 1 KB contiguously).
constexpr int kDM = 256, kDN = 256, kDK = 128;  // pools, queries, K bytes per stage
constexpr int kDBlk = 8 * kDK + 16;             // block pitch
constexpr int kDRegion = 32 * kDBlk;
constexpr int kDStage = 2 * kDRegion;           // 2 x 32.5 KB
constexpr int kDThreads = 256;
constexpr int kDTiles = kDN / 64;  // query tiles per workgroup

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// A thread's 16 direct-to-LDS loads of a stage: instructions j = w + 4 m of
// wave w (j < 32: pool block j, else query block j - 32).  Lane l of an
// instruction writes byte 16 l of its block, i.e. chunk l % 8 of block row
// l / 8, which is region row 32 (l / 8) + block.  Sources are 32-bit offsets
// from the workgroup's first pool row and first query row.  Rows past the
// last pool re-read the last pool; query rows past the last tile re-read the
// last query row (their columns are never tested).
struct DenseLoads {
  const unsigned char* pool;   // first pool row of the workgroup
  const unsigned char* query;  // first query row of the workgroup
  uint32_t off[16];
};
__device__ __forceinline__ void dense_sources(DenseLoads& L, int rowbytes, int64_t row0,
                                              int64_t rows, int q0, int qrows, int wave,
                                              int lane) {
  const int plim = (int)min(rows - row0, (int64_t)kDM), qlim = min(qrows - q0, kDN);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int j = wave + 4 * m;                 // instruction of the stage
    const int R = 32 * (lane >> 3) + (j & 31);  // region row
    const int lim = j < 32 ? plim : qlim;
    const int rr = R < lim ? R : lim - 1;
    L.off[m] = (uint32_t)rr * (uint32_t)rowbytes + 16u * (uint32_t)(lane & 7);
  }
}
// (instruction m of wave w fills block w + 4 m of the pool region for m < 8,
// block w + 4 m - 32 of the query region after; the destination is the
// wave's offset plus a constant.  The empty asm keeps that offset from being
// treated as loop-invariant: otherwise all 32 destinations are precomputed
// and held in scalar registers through the loop.)
__device__ __forceinline__ void dense_issue(const DenseLoads& L, unsigned char* buf, int s,
                                            uint32_t wave_off) {
  asm volatile("" : "+s"(wave_off));
  const unsigned char* ps = L.pool + s * kDK;
  const unsigned char* qs = L.query + s * kDK;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const uint32_t c = m < 8 ? 4 * m * kDBlk : kDRegion + (4 * m - 32) * kDBlk;
    __builtin_amdgcn_global_load_lds((const void*)((m < 8 ? ps : qs) + L.off[m]),
                                     (lds_void_ptr)(buf + wave_off + c), 16, 0, 0);
  }
}

// Thresholds of tile t for the two 32-query halves a lane's accumulator
// columns belong to (query t * 64 + 32 j + r).
template <int FMT>
__device__ __forceinline__ void dense_thresholds(const DenseLevelArgs& a, int t, int r, float (&thr)[2]) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int qi = t * 64 + 32 * j + r;
    float th = a.thr[qi];
    if (FMT == GT_POOL_FP8E4M3) th = ldexpf(th * kFp8ThrFactor, -(a.qexp[qi] + a.lexp));
    thr[j] = th;
  }
}

// Survival mask of one 32-pool block against tile t: c0 and c1 are the
// 32x32 accumulators of the tile's query halves.  Lane l holds query column
// l % 32 of rows 8 (x / 4) + 4 (l / 32) + x % 4 (register x), so the ballot
// of register x over a query half holds, in its low 32 bits, row
// 8 (x / 4) + x % 4 and, in its high 32 bits, the row 4 below; each half is
// selected into that row's lane.  Lane r < 32 ends with row r's
// 64-query mask (other lanes: 0).
__device__ __forceinline__ uint64_t dense_block_mask(const f32x16& c0, const f32x16& c1,
                                                     const float (&thr)[2], int lane) {
  uint32_t mlo = 0u, mhi = 0u;  // queries 0-31 and 32-63
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    const uint64_t b0 = __ballot(c0[x] >= thr[0]);
    const uint64_t b1 = __ballot(c1[x] >= thr[1]);
    const int rr = 8 * (x >> 2) + (x & 3);
    if (lane == rr) {
      mlo = (uint32_t)b0;
      mhi = (uint32_t)b1;
    }
    if (lane == rr + 4) {
      mlo = (uint32_t)(b0 >> 32);
      mhi = (uint32_t)(b1 >> 32);
    }
    // (the empty asm makes each register's ballots be used at once: left to
    // itself the compiler gathers all 32 wave-wide results first, and they
    // overflow the scalar registers)
    asm volatile("" : "+v"(mlo), "+v"(mhi));
  }
  return ((uint64_t)mhi << 32) | mlo;
}

// Score records of the kept pools (subtraction step): upper bounds of each
// pool's real score for all 64 queries of the tile, query q at
// 4 (q % 16) + q / 16 of the pool's 128-byte record.  A block's bounds are
// first written to LDS in record order (32 rows x 128 bytes), then the kept
// rows are copied out with 16-byte accesses.  Lane l holds queries l % 32
// (c0) and 32 + l % 32 (c1) of rows 8 (x / 4) + 4 (l / 32) + x % 4
// (register x): two 16-bit writes per register at fixed offsets from the
// lane's base.
__device__ __forceinline__ void dense_stage_records(unsigned char* blk, float aup,
                                                    const f32x16& c0, const f32x16& c1,
                                                    int lane) {
  const int q = lane & 15, hi16 = (lane >> 4) & 1;
  unsigned char* base = blk + (lane >> 5) * 4 * 128 + 8 * q + 2 * hi16;
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    const int rr = 8 * (x >> 2) + (x & 3);
    const uint32_t v0 = bf16_ceil_hi(score_upper(c0[x], aup));
    const uint32_t v1 = bf16_ceil_hi(score_upper(c1[x], aup));
    *reinterpret_cast<uint16_t*>(base + rr * 128) = (uint16_t)(v0 >> 16);
    *reinterpret_cast<uint16_t*>(base + rr * 128 + 4) = (uint16_t)(v1 >> 16);
  }
}
// Copies the records of the kept rows of a staged block: oe, lane r < 32, is
// the output entry of row r (-1: not kept).  Lane l moves chunk l % 8 of rows
// l / 8 + 8 k.
__device__ __forceinline__ void dense_copy_records(uint16_t* out_rec, const unsigned char* blk,
                                                   int64_t oe, int lane) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int row = (lane >> 3) + 8 * k;
    const int64_t o = __shfl(oe, row, 64);
    const uint4 v = *reinterpret_cast<const uint4*>(blk + row * 128 + 16 * (lane & 7));
    if (o >= 0) *reinterpret_cast<uint4*>(out_rec + (size_t)o * 64 + 8 * (lane & 7)) = v;
  }
}

// Operands of one K step of a wave: bf16, 16 elements (one 32x32x16
// product per block pair); float8, 64 elements (one 32x32x64 product).
// Lanes 0-31 and 32-63 carry different K ranges, the same in A and B.
template <int FMT>
struct DenseOps {
  static constexpr int NC = FMT == GT_POOL_FP8E4M3 ? 2 : 1;  // 16-byte chunks per lane
  uint4 a[4][NC], b[4][NC];
};
// Lane (r, half) reads, for block i of its pool rows (region row
// 128 wr + 32 i + r: block r, block row 4 wr + i) and K step st, chunks
// NC (2 st + half) + h: base + 128 i + 16 (2 NC st + h), with
// base = 1040 r + 512 wr + 16 NC half (queries alike with wq, in the second
// region).
template <int FMT>
__device__ __forceinline__ void dense_read(const unsigned char* buf, int st, uint32_t abase,
                                           uint32_t bbase, DenseOps<FMT>& o) {
  constexpr int NC = DenseOps<FMT>::NC;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int h = 0; h < NC; ++h)
      o.a[i][h] = *reinterpret_cast<const uint4*>(buf + abase + kDK * i + 16 * (2 * NC * st + h));
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int h = 0; h < NC; ++h)
      o.b[j][h] = *reinterpret_cast<const uint4*>(buf + bbase + kDK * j + 16 * (2 * NC * st + h));
}
template <int FMT, int I0, int I1>
__device__ __forceinline__ void dense_mma(const DenseOps<FMT>& o, f32x16 (&acc)[4][4]) {
#pragma unroll
  for (int i = I0; i < I1; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (FMT == GT_POOL_FP8E4M3)
        mma_f8_32x32x64(o.a[i][0], o.a[i][1], o.b[j][0], o.b[j][1], acc[i][j]);
      else
        mma16<FMT>(o.a[i][0], o.b[j][0], acc[i][j]);
    }
}

template <int FMT>
__global__ __launch_bounds__(kDThreads, 1) void k_dense_level(DenseLevelArgs a) {
  using F = WalkFmt<FMT>;
  static_assert(F::TQ == 64, "dense steps use 64-query tiles");
  // K steps per stage: bf16 steps of 32 bytes, float8 steps of 64 bytes
  constexpr int NS = FMT == GT_POOL_FP8E4M3 ? 2 : 4;
  // (two separate arrays: a read of one is then known not to depend on the
  // loads in flight into the other)
  __shared__ __attribute__((aligned(1024))) unsigned char lds0[kDStage];
  __shared__ __attribute__((aligned(1024))) unsigned char lds1[kDStage];
  // output reservations of the workgroup: entries per (tile, bucket) of its
  // 256 pools (at most 8 buckets once a bucket holds 32 pools or more), and
  // the slots' bases
  __shared__ uint32_t wg_cnt[kDTiles][8], wg_base[kDTiles][8];
  const int64_t rows = a.rows;  // pools holding a row below the call's epoch
  const int64_t RB = (rows + kDM - 1) / kDM;
  const int QB = (a.nt + kDTiles - 1) / kDTiles;
  const int64_t total = RB * QB;
  // XCD-aware order: the workgroups of one XCD take consecutive tiles, i.e.
  // all query blocks of a pool block, which then passes through one L2
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t wid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (wid >= total) return;
  const int qb = (int)(wid % QB);
  const int64_t row0 = (wid / QB) * kDM;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wq = wave & 1;
  const int r = lane & 31, half = lane >> 5;
  const int rowbytes = a.dp * F::ESZ;
  const int nst = rowbytes / kDK;

  const uint32_t wave_off = (uint32_t)(wave * kDBlk);
  DenseLoads L;
  L.pool = reinterpret_cast<const unsigned char*>(a.child_rows) + (size_t)row0 * rowbytes;
  L.query = reinterpret_cast<const unsigned char*>(a.qtile) + (size_t)qb * kDN * rowbytes;
  dense_sources(L, rowbytes, row0, rows, qb * kDN, a.nt * 64, wave, lane);
  constexpr int NC = DenseOps<FMT>::NC;
  const uint32_t abase = (uint32_t)(kDBlk * r + 4 * kDK * wr + 16 * NC * half);
  const uint32_t bbase = (uint32_t)(kDRegion + kDBlk * r + 4 * kDK * wq + 16 * NC * half);

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int x = 0; x < 16; ++x) acc[i][j][x] = 0.0f;

  // Stage s sits in buffer s % 2.  Stage s + 1 is loaded while stage s is
  // multiplied.  At the last K step of stage s a barrier, after this wave's
  // reads of stage s and its loads of stage s + 1 are complete, tells that
  // every wave is done with stage s (its buffer then takes stage s + 2) and
  // that stage s + 1 has landed; the first step of stage s + 1 is read while
  // the last step of stage s is multiplied.  The scheduling barriers keep
  // each step's LDS reads ahead of the matrix work that hides them.
  // (operands alternate between two register sets by the parity of the K
  // step, which is static: a stage has an even number of steps.  The loop
  // runs an even number of stages and holds no data-dependent branch around
  // the reads, so that both sets keep their registers: for an odd number of
  // K stages, position 0 is a stage of zeros and position p holds K stage
  // p - 1.  A step issues its first row of products before the next step's
  // reads: with direct-to-LDS loads in flight the compiler waits for all LDS
  // reads before a step's products, and by then they have had the other
  // twelve products' time.)
  DenseOps<FMT> ops[2];
  const int odd = nst & 1, npos = nst + odd;
  L.pool -= odd * kDK;
  L.query -= odd * kDK;
  // One position from buffer cb; with `next`, its last step crosses the
  // barrier into position p + 1 in buffer nb and, if `issue`, loads position
  // p + 2 into cb.
  auto stage = [&](unsigned char* cb, unsigned char* nb, int p, bool next, bool issue) {
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const DenseOps<FMT>& cu = ops[st & 1];
      DenseOps<FMT>& nx = ops[(st + 1) & 1];
      dense_mma<FMT, 0, 1>(cu, acc);
      __builtin_amdgcn_sched_barrier(0);
      if (st + 1 < NS) {
        dense_read<FMT>(cb, st + 1, abase, bbase, nx);
      } else if (next) {
        __builtin_amdgcn_s_waitcnt(0x0070);  // vmcnt(0) lgkmcnt(0)
        __syncthreads();
        if (issue) dense_issue(L, cb, p + 2, wave_off);
        dense_read<FMT>(nb, 0, abase, bbase, nx);
      }
      __builtin_amdgcn_sched_barrier(0);
      dense_mma<FMT, 1, 4>(cu, acc);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  if (tid < kDTiles * 8) (&wg_cnt[0][0])[tid] = 0u;
  if (odd) {
    for (int i = tid; i < kDStage / 16; i += kDThreads)
      *reinterpret_cast<uint4*>(lds0 + 16 * i) = make_uint4(0u, 0u, 0u, 0u);
  } else {
    dense_issue(L, lds0, 0, wave_off);
  }
  __builtin_amdgcn_s_waitcnt(0x0070);
  __syncthreads();
  dense_issue(L, lds1, 1, wave_off);
  dense_read<FMT>(lds0, 0, abase, bbase, ops[0]);
  int p = 0;
  for (; p + 3 < npos; p += 2) {  // positions p + 2 and p + 3 exist
    stage(lds0, lds1, p, true, true);
    stage(lds1, lds0, p + 1, true, true);
  }
  stage(lds0, lds1, p, true, false);
  stage(lds1, lds0, p + 1, false, false);

  // Output: the wave's 8 blocks (tile tt, pool block i).  Child j survives
  // for query b iff its parent's bit b is set and its score reaches tau'_b.
  // All blocks' masks first; the workgroup's frontier reservations are then
  // gathered in LDS and made with one atomic per (bucket, tile) slot (the
  // slot counters share a few cache lines, and one atomic per block and wave
  // queues on them); then the writes: per-(pool, tile) masks for a following
  // dense level, or the bucketed sparse frontier (and, for the subtraction
  // step, the kept pools' score records).
  float thr[2][2];
  uint64_t pm[2][4];  // parent masks (lane r < 32: pool row r of the block)
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t = qb * kDTiles + 2 * wq + tt;
    thr[tt][0] = thr[tt][1] = 0.0f;
    if (t < a.nt) dense_thresholds<FMT>(a, t, r, thr[tt]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = row0 + wr * 128 + i * 32 + r;
      pm[tt][i] = 0ull;
      if (t < a.nt && lane < 32 && row < rows)
        pm[tt][i] = a.parent ? a.parent[(row >> 1) * a.nt + t] : a.tile_mask[t];
    }
  }
  const int bshift = a.level - a.nb;  // node -> bucket of the sparse output
  unsigned long long pairs = 0;
  uint64_t mine[2][4];
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = row0 + wr * 128 + i * 32 + r;
      mine[tt][i] = dense_block_mask(acc[i][2 * tt], acc[i][2 * tt + 1], thr[tt], lane) & pm[tt][i];
      pairs += (unsigned long long)__popcll(pm[tt][i]);
      if (a.bitmap && pm[tt][i])
        atomicOr(&a.bitmap[(a.bit_base + row) >> 5], 1u << ((a.bit_base + row) & 31));
    }
  if (a.out_dense) {
    // non-empty masks per tile, one atomic per tile and workgroup
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = qb * kDTiles + 2 * wq + tt;
        const int64_t row = row0 + wr * 128 + i * 32 + r;
        if (t < a.nt && lane < 32 && row < rows) a.out_dense[row * a.nt + t] = mine[tt][i];
        const uint64_t eb = __ballot(mine[tt][i] != 0ull);
        if (lane == 0 && eb) atomicAdd(&wg_cnt[2 * wq + tt][0], (uint32_t)__popcll(eb));
      }
    __syncthreads();
    if (tid < kDTiles && qb * kDTiles + tid < a.nt && wg_cnt[tid][0])
      atomicAdd(&a.out_count[qb * kDTiles + tid], wg_cnt[tid][0]);
  } else {
    // one reservation per (bucket, tile) slot of the workgroup when a
    // bucket holds 32 pools or more, else one per row
    const bool grouped = bshift >= 5;
    int64_t oe[2][4];    // output entry of this lane's row (-1: none)
    uint32_t off[2][4];  // the block's first entry within the workgroup's slot
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = qb * kDTiles + 2 * wq + tt;
        const int64_t rb0 = row0 + wr * 128 + i * 32;
        const uint64_t eb = __ballot(mine[tt][i] != 0ull);
        oe[tt][i] = -1;
        off[tt][i] = 0u;
        if (grouped) {
          const int bi = (int)((rb0 >> bshift) - (row0 >> bshift));
          if (lane == 0 && eb) off[tt][i] = atomicAdd(&wg_cnt[2 * wq + tt][bi], (uint32_t)__popcll(eb));
        } else if (mine[tt][i]) {
          off[tt][i] = atomicAdd(&a.out_count[(uint32_t)((rb0 + r) >> bshift) * (uint32_t)a.nt + t], 1u);
        }
      }
    if (grouped) {
      __syncthreads();
      if (tid < kDTiles * 8) {
        const int tw = tid >> 3, bi = tid & 7, t = qb * kDTiles + tw;
        const uint32_t c = wg_cnt[tw][bi];
        if (c && t < a.nt)
          wg_base[tw][bi] =
              atomicAdd(&a.out_count[(uint32_t)((row0 >> bshift) + bi) * (uint32_t)a.nt + t], c);
      }
      __syncthreads();
    }
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = qb * kDTiles + 2 * wq + tt;
        const int64_t rb0 = row0 + wr * 128 + i * 32, row = rb0 + r;
        const uint64_t eb = __ballot(mine[tt][i] != 0ull);
        if (!eb) continue;
        const uint32_t slot = (uint32_t)(row >> bshift) * (uint32_t)a.nt + t;
        uint32_t pos = off[tt][i];
        if (grouped) {
          const int bi = (int)((rb0 >> bshift) - (row0 >> bshift));
          pos = wg_base[2 * wq + tt][bi] + (uint32_t)__builtin_amdgcn_readfirstlane(off[tt][i]) +
                (uint32_t)__popcll(eb & ((1ull << lane) - 1ull));
        }
        if (mine[tt][i]) {
          if (pos < a.bcap) {
            const int64_t o = (int64_t)slot * a.bcap + pos;
            oe[tt][i] = o;
            a.out_node[o] = (uint32_t)row;
            a.out_mask[o] = mine[tt][i];
          } else {
            atomicOr(a.over, 1u);
          }
        }
      }
    if (FMT == GT_POOL_BF16 && a.out_rec) {
      // (the stage buffers are free once every wave is past its last reads;
      // each wave stages its 8 blocks in 32 KB of its own)
      __syncthreads();
      unsigned char* region = (wave < 2 ? lds0 : lds1) + (wave & 1) * 32768;
      const float aup = score_abs_up(a.dp);
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dense_stage_records(region + (tt * 4 + i) * 4096, aup, acc[i][2 * tt],
                              acc[i][2 * tt + 1], lane);
      __syncthreads();
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dense_copy_records(a.out_rec, region + (tt * 4 + i) * 4096, oe[tt][i], lane);
    }
  }
  if (a.stat_pairs) {
    for (int o = 32; o >= 1; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
    if (lane == 0 && pairs) atomicAdd(a.stat_pairs, pairs);
  }
}

// Exact leaf test: entries (pool p at level depth-1, mask) -> vectors 2p and
// 2p+1 for every query of the mask.  A wave takes two entries at a time and,
// per round, up to two mask bits of each: 2 entries x 2 queries x 2 vectors =
// eight dot products whose rows are all fetched together and reduced at once.
// The next pair of entries is fetched while the current one is computed.
struct LeafEntry {
  int t;
  uint32_t p;
  uint64_t m;
  float inv0, inv1;  // inverse norms of vectors 2p and 2p+1 (0: beyond the epoch or zero)
};

__device__ __forceinline__ LeafEntry leaf_entry(const LeafArgs& a, const uint32_t* epre, int nsl,
                                                int slot0, uint32_t idx, uint32_t etot) {
  LeafEntry x;
  x.t = 0;
  x.p = 0;
  x.m = 0ull;
  x.inv0 = x.inv1 = 0.0f;
  if (idx >= etot) return x;
  const int sl = find_slot(epre, nsl, idx);
  const int gs = slot0 + sl;
  const uint32_t e = idx - epre[sl];
  x.t = gs % a.nt;
  if (a.dense) {
    x.p = ((uint32_t)(gs / a.nt) << (a.level - a.nb)) + e;
    x.m = a.tile_mask[x.t];
  } else {
    x.p = a.in_node[(size_t)gs * a.bcap + e];
    x.m = a.in_mask[(size_t)gs * a.bcap + e];
  }
  return x;
}

// Inverse norms of an entry's two vectors, fetched one round before its use
// (the entry itself is fetched two rounds before).
__device__ __forceinline__ void leaf_norms(const LeafArgs& a, LeafEntry& x) {
  const int64_t i0 = 2 * (int64_t)x.p;
  x.inv0 = i0 < a.n_epoch ? a.invn_f[i0] : 0.0f;
  x.inv1 = i0 + 1 < a.n_epoch ? a.invn_f[i0 + 1] : 0.0f;
}

// Workgroup -> XCD x = blockIdx % 8, which owns the bucket slots of buckets
// [x R, x R + R) (slots are bucket-major, so they are contiguous); the XCD's
// workgroups sweep its entries in slot order, so the tiles' copies of a leaf
// pair are tested close together in time and share the XCD's L2.
// NV: 16-byte slices per lane and 1024-column chunk that can be non-zero, 4
// in general and 2 for rows of at most 512 columns (whose other two slices
// would only reload the row's last slice).  Each dot product is summed in the
// same order either way: a slice past dp is zero and adds nothing to
// chunk_sum4.
template <int NV>
__global__ __launch_bounds__(256) void k_leaf(LeafArgs a) {
  __shared__ uint32_t epre[kMaxSlotsPerXcd + 1];
  __shared__ Hit hstage[4][kHitStage];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nbk = 1 << a.nb;
  const int xs = nbk < kXcds ? nbk : kXcds;
  const int x = blockIdx.x % kXcds;
  if (x >= xs) return;
  const int nsl = (nbk / xs) * a.nt;
  const int slot0 = x * nsl;
  slot_prefix(epre, nsl, slot0, a.nt, a.dense, a.level - a.nb, a.tile_mask, a.in_count,
              (uint32_t)a.bcap);
  const uint32_t etot = epre[nsl];
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wgs = gridDim.x / kXcds;
  const uint32_t stride = 2u * wgs * nw;
  Hit* buf = hstage[w];
  int cnt = 0;
  unsigned long long npairs = 0;
  const int v = lane >> 3;              // value owned after the reduction
  const int vs = v >> 2, vk = (v >> 1) & 1, vl = v & 1;
  uint32_t idx = 2u * ((blockIdx.x / kXcds) * nw + w);
  LeafEntry nx0 = leaf_entry(a, epre, nsl, slot0, idx, etot);
  LeafEntry nx1 = leaf_entry(a, epre, nsl, slot0, idx + 1, etot);
  leaf_norms(a, nx0);
  leaf_norms(a, nx1);
  LeafEntry nn0 = leaf_entry(a, epre, nsl, slot0, idx + stride, etot);
  LeafEntry nn1 = leaf_entry(a, epre, nsl, slot0, idx + stride + 1, etot);
  for (; idx < etot; idx += stride) {
    LeafEntry en[2] = {nx0, nx1};
    nx0 = nn0;
    nx1 = nn1;
    leaf_norms(a, nx0);
    leaf_norms(a, nx1);
    nn0 = leaf_entry(a, epre, nsl, slot0, idx + 2 * stride, etot);
    nn1 = leaf_entry(a, epre, nsl, slot0, idx + 2 * stride + 1, etot);
    float inv[2][2];
    const float* frow[2][2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int64_t i = 2 * (int64_t)en[s2].p + c;
        inv[s2][c] = en[s2].m ? (c == 0 ? en[s2].inv0 : en[s2].inv1) : 0.0f;
        frow[s2][c] = a.leaves + i * a.dp;
        if (a.bitmap && lane == 0 && inv[s2][c] != 0.0f)
          atomicOr(&a.bitmap[(a.bit_base + i) >> 5], 1u << ((a.bit_base + i) & 31));
      }
      // a zero vector has no cosine and is never a member
      if (inv[s2][0] == 0.0f && inv[s2][1] == 0.0f) en[s2].m = 0ull;
    }
    while (en[0].m | en[1].m) {
      int qs[2][2];
      bool qv[2][2];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          qv[s2][k] = en[s2].m != 0ull;
          qs[s2][k] = qv[s2][k] ? en[s2].t * a.tq + (__ffsll((unsigned long long)en[s2].m) - 1) : 0;
          en[s2].m &= en[s2].m - 1ull;
        }
      // all eight rows' slices are loaded before any arithmetic (rows of
      // unused combinations are valid rows; their sums are dropped below)
      const float4* q4[2][2];
      const float4* f4[2][2];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          q4[s2][k] = reinterpret_cast<const float4*>(a.qf + (size_t)qs[s2][k] * a.dp);
          f4[s2][k] = reinterpret_cast<const float4*>(frow[s2][k]);
        }
      float acc[8];
      for (int c = 0; c * 1024 < a.dp; ++c) {
        float sv[8][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (v >= NV) {
#pragma unroll
            for (int vi = 0; vi < 8; ++vi) sv[vi][v] = 0.0f;
            continue;
          }
          bool ok;
          const int ec = slice_index(c, v, lane, a.dp, ok);
          float4 qx[2][2], fx[2][2];
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              qx[s2][k] = q4[s2][k][ec];
              fx[s2][k] = f4[s2][k][ec];
            }
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
              for (int l = 0; l < 2; ++l)
              {
                // computed for every slice (a redirected slice holds valid
                // data), then selected: no branch per slice
                const float dv = slice_dot4(qx[s2][k], fx[s2][l]);
                sv[4 * s2 + 2 * k + l][v] = ok ? dv : 0.0f;
              }
        }
#pragma unroll
        for (int vi = 0; vi < 8; ++vi) {
          const float part = chunk_sum4(sv[vi][0], sv[vi][1], sv[vi][2], sv[vi][3]);
          acc[vi] = c == 0 ? part : __fadd_rn(acc[vi], part);
        }
      }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int l = 0; l < 2; ++l)
            if (!(qv[s2][k] && inv[s2][l] != 0.0f)) acc[4 * s2 + 2 * k + l] = 0.0f;
      const float dot = wave_reduce8(acc, lane);
      // lane 8v classifies value v = (entry vs, query vk, vector vl)
      int qg = 0;
      bool ok = false;
      float invf = 0.0f;
      uint32_t id = 0;
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int l = 0; l < 2; ++l)
            if (vs == s2 && vk == k && vl == l) {
              qg = qs[s2][k];
              ok = qv[s2][k] && inv[s2][l] != 0.0f;
              invf = inv[s2][l];
              id = 2u * en[s2].p + (uint32_t)l;
            }
      const bool mine = (lane & 7) == 0 && ok;
      Hit h;
      uint32_t flag = 0;
      if (mine) {
        const float cs = __fmul_rn(__fmul_rn(dot, a.invn_q[qg]), invf);
        flag = classify(cs, a.rho[qg]);
        h.q = (uint32_t)qg;
        h.id = id;
        h.sim = cs;
        h.flag = flag == HIT_ACCEPT ? flag | accept_slot(&a.qcount[qg], a.ctr) : flag;
        ++npairs;
      }
      stage_hits(buf, cnt, flag != 0u, h, false, a.ctr, a.hits, a.hit_cap, a.band_idx, lane);
    }
  }
  Hit none;
  stage_hits(buf, cnt, false, none, true, a.ctr, a.hits, a.hit_cap, a.band_idx, lane);
  for (int o = 32; o >= 1; o >>= 1) npairs += __shfl_xor(npairs, o, 64);
  if (lane == 0 && npairs) atomicAdd(&a.ctr->leaf_pairs, npairs);
}

// Candidates within 1e-5 of rho are re-decided with the canonical float64
// cosine, bit-identical to the oracle: the dot product and the query's squared
// norm run sequentially over k, lane by lane (lane l holds elements
// [16 l, 16 l + 16) of each 1024-chunk, so lane order is k order), one wave
// per candidate; the rows' squared norms are the canonical ones of ingest.
__global__ __launch_bounds__(256) void k_recheck(Hit* hits, const uint32_t* band_idx,
                                                 const unsigned long long* nband,
                                                 unsigned long long cap,
                                                 const float* __restrict__ qf,
                                                 const float* __restrict__ leaves, int d, int dp,
                                                 const double* __restrict__ ff,
                                                 const double* __restrict__ rho,
                                                 unsigned int* qcount, DevCounters* ctr) {
  const int lane = threadIdx.x & 63;
  const unsigned long long n = *nband < cap ? *nband : cap;
  const unsigned long long nw = blockDim.x >> 6;
  for (unsigned long long b = blockIdx.x * nw + (threadIdx.x >> 6); b < n; b += gridDim.x * nw) {
    const uint32_t hi = band_idx[b];
    Hit x = hits[hi];
    const float* q = qf + (size_t)x.q * dp;
    const float* f = leaves + (size_t)x.id * dp;
    // dot = sum q_k f_k and qq = sum q_k^2, both sequential over k (two
    // independent chains in step)
    double s = 0.0, sq = 0.0;
    for (int c = 0; c * 1024 < dp; ++c) {
      const int base = c * 1024 + 16 * lane;
      float qv[16], fv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        qv[j] = base + j < d ? q[base + j] : 0.0f;
        fv[j] = base + j < d ? f[base + j] : 0.0f;
      }
      // (values past d are zero: fma(0, 0, s) = s, so no branch splits the
      // two chains)
      for (int L = 0; L < 64; ++L) {
        if (lane == L) {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            s = __fma_rn((double)qv[j], (double)fv[j], s);
            sq = __fma_rn((double)qv[j], (double)qv[j], sq);
          }
        }
        s = __shfl(s, L, 64);
        sq = __shfl(sq, L, 64);
      }
    }
    if (lane == 0) {
      const double cs = __ddiv_rn(s, __dmul_rn(__dsqrt_rn(sq), __dsqrt_rn(ff[x.id])));
      atomicAdd(&ctr->rechecked, 1ull);
      if (cs >= rho[x.q]) {
        x.flag = HIT_ACCEPT | accept_slot(&qcount[x.q], ctr);
        x.sim = (float)cs;
      } else {
        x.flag = HIT_REJECT;
      }
      hits[hi] = x;
    }
  }
}

// Exclusive scan of per-query counts -> offsets (one workgroup of 1024).
__global__ __launch_bounds__(1024) void k_scan_offsets(const unsigned int* qcount, int nq,
                                                       int64_t* offs, int64_t* offs_out,
                                                       DevCounters* ctr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int per = (nq + 1023) / 1024;
  const int lo = t * per, hi = min(nq, lo + per);
  int64_t s = 0;
  for (int i = lo; i < hi; ++i) s += qcount[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    offs[i] = run;
    if (offs_out) offs_out[i] = run;
    run += qcount[i];
  }
  if (t == 1023) {
    offs[nq] = part[1023];
    if (offs_out) offs_out[nq] = part[1023];
    ctr->total = (unsigned long long)part[1023];
  }
}

// Accepted pairs to their query's segment: slot = offset of the query + the
// pair's slot among the query's results.  Enqueued before the host has seen
// the counts; does nothing unless every candidate was kept (hit_cap) and the
// results fit the output (lim).
__device__ __forceinline__ bool results_fit(const DevCounters* ctr, unsigned long long hit_cap,
                                            unsigned long long lim) {
  return ctr->nhits <= hit_cap && ctr->total <= lim && ctr->slot_over == 0u && ctr->err == 0u;
}

__global__ void k_scatter(const Hit* hits, const DevCounters* ctr, unsigned long long hit_cap,
                          unsigned long long lim, const int64_t* offs, uint32_t* out_id,
                          float* out_sim) {
  if (!results_fit(ctr, hit_cap, lim)) return;
  const unsigned long long n = ctr->nhits;
  for (unsigned long long h = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; h < n;
       h += (unsigned long long)gridDim.x * blockDim.x) {
    const Hit x = hits[h];
    if (hit_kind(x.flag) != HIT_ACCEPT) continue;
    const int64_t pos = offs[x.q] + (int64_t)hit_slot(x.flag);
    out_id[pos] = x.id;
    out_sim[pos] = x.sim;
  }
}

// Sort each query's results by id (ids of one query are distinct).  Up to
// 4096 results: a counting sort on the top 8 bits of the id (id >> shift,
// shift chosen by the host so that every id below the call's epoch has a
// top part below 256) groups the ids in LDS, then each id is placed at its
// group's start plus the number of smaller ids in its group.  Larger
// segments: stable 4-bit LSD radix sort by the same workgroup.
constexpr int kSortPerThread = 16;  // 4096 / 256
__global__ __launch_bounds__(256) void k_sort_segments(const int64_t* offs, uint32_t* id,
                                                       float* sim, uint32_t* tmp_id,
                                                       float* tmp_sim, int64_t* ids_out,
                                                       float* sims_out, const DevCounters* ctr,
                                                       unsigned long long hit_cap,
                                                       unsigned long long lim, int shift) {
  __shared__ uint32_t key[4096];
  __shared__ float val[4096];
  __shared__ uint32_t hist[16 * 256];
  __shared__ uint32_t tot[257];
  if (!results_fit(ctr, hit_cap, lim)) return;
  const int q = blockIdx.x, t = threadIdx.x;
  const int64_t lo = offs[q], n = offs[q + 1] - lo;
  if (n <= 0) return;
  if (n <= 4096) {
    const int ni = (int)n;
    tot[t] = 0u;
    if (t == 0) tot[256] = 0u;
    __syncthreads();
    uint32_t k[kSortPerThread], g[kSortPerThread], r[kSortPerThread];
    float v[kSortPerThread];
#pragma unroll
    for (int e = 0; e < kSortPerThread; ++e) {
      const int i = t + 256 * e;
      if (i < ni) {
        k[e] = id[lo + i];
        v[e] = sim[lo + i];
        const uint32_t gg = k[e] >> shift;
        g[e] = gg < 255u ? gg : 255u;
        r[e] = atomicAdd(&tot[g[e]], 1u);
      }
    }
    __syncthreads();
    if (t < 64) {  // exclusive prefix of the 256 group sizes, four per lane
      uint32_t c[4], sum = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c[j] = tot[4 * t + j];
        sum += c[j];
      }
      uint32_t incl = sum;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t x = __shfl_up(incl, o, 64);
        if (t >= o) incl += x;
      }
      uint32_t run = incl - sum;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        hist[4 * t + j] = run;
        run += c[j];
      }
      if (t == 63) hist[256] = incl;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kSortPerThread; ++e) {
      const int i = t + 256 * e;
      if (i < ni) {
        key[hist[g[e]] + r[e]] = k[e];
        val[hist[g[e]] + r[e]] = v[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kSortPerThread; ++e) {
      const int i = t + 256 * e;
      if (i < ni) {
        const uint32_t b0 = hist[g[e]], b1 = hist[g[e] + 1];
        uint32_t pos = b0;
        for (uint32_t j = b0; j < b1; ++j) pos += key[j] < k[e];
        ids_out[lo + pos] = (int64_t)k[e];
        sims_out[lo + pos] = v[e];
      }
    }
    return;
  }
  uint32_t *si = id + lo, *di = tmp_id + lo;
  float *sv = sim + lo, *dv = tmp_sim + lo;
  const int64_t chunk = (n + 255) / 256;
  const int64_t a0 = min(n, t * chunk), a1 = min(n, a0 + chunk);
  for (int pass = 0; pass < 8; ++pass) {
    const int sh = 4 * pass;
    uint32_t h[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) h[b] = 0;
    for (int64_t i = a0; i < a1; ++i) h[(si[i] >> sh) & 15u]++;
#pragma unroll
    for (int b = 0; b < 16; ++b) hist[b * 256 + t] = h[b];
    __syncthreads();
    // exclusive scan over hist in (digit, thread) order: thread t owns 16 slots
    uint32_t s = 0;
    for (int k = 0; k < 16; ++k) s += hist[t * 16 + k];
    tot[t] = s;
    __syncthreads();
    if (t == 0) {
      uint32_t run = 0;
      for (int k = 0; k < 256; ++k) {
        const uint32_t v = tot[k];
        tot[k] = run;
        run += v;
      }
    }
    __syncthreads();
    uint32_t run = tot[t];
    for (int k = 0; k < 16; ++k) {
      const uint32_t v = hist[t * 16 + k];
      hist[t * 16 + k] = run;
      run += v;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 16; ++b) h[b] = hist[b * 256 + t];
    for (int64_t i = a0; i < a1; ++i) {
      const uint32_t k = si[i];
      const uint32_t pos = h[(k >> sh) & 15u]++;
      di[pos] = k;
      dv[pos] = sv[i];
    }
    __syncthreads();
    uint32_t* ti = si; si = di; di = ti;
    float* tv = sv; sv = dv; dv = tv;
  }
  for (int64_t i = t; i < n; i += 256) {
    ids_out[lo + i] = (int64_t)si[i];
    sims_out[lo + i] = sv[i];
  }
}

int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

template <int FMT, int NFAST>
hipError_t launch_walk_fmt(const WalkLevelArgs& a, int grid, hipStream_t s) {
  const int nsteps = a.dp * WalkFmt<FMT>::ESZ / 64;
  if (nsteps == NFAST)
    hipLaunchKernelGGL((k_walk_level<FMT, NFAST>), dim3(grid), dim3(kWalkThreads), 0, s, a);
  else
    hipLaunchKernelGGL((k_walk_level<FMT, 0>), dim3(grid), dim3(kWalkThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_walk_level(int fmt, const WalkLevelArgs& a, int grid, hipStream_t s) {
  // whole workgroups per XCD; bucket and slot limits of the kernels
  grid = kXcds * ((grid + kXcds - 1) / kXcds);
  if (a.nb < 0 || a.nb > kMaxBucketBits || ((int64_t)a.nt << a.nb) > kMaxSlots ||
      a.level < a.nb || a.nt < 1 || a.nt > kMaxTiles || a.dp < 128 || a.dp % 128 != 0 ||
      a.dp > kMaxWalkWidth)
    return hipErrorInvalidValue;
  // rows wider than the LDS query tile: windows of the tile through LDS
  if (a.dp > maxdp_walk(fmt)) {
    switch (fmt) {
      case GT_POOL_BF16:
        hipLaunchKernelGGL(k_walk_wide<GT_POOL_BF16>, dim3(grid), dim3(kWalkThreads), 0, s, a);
        break;
      case GT_POOL_FP8E4M3:
        hipLaunchKernelGGL(k_walk_wide<GT_POOL_FP8E4M3>, dim3(grid), dim3(kWalkThreads), 0, s, a);
        break;
      case GT_POOL_F32:
        hipLaunchKernelGGL(k_walk_wide<GT_POOL_F32>, dim3(grid), dim3(kWalkThreads), 0, s, a);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  // fast paths: padded width 1024
  switch (fmt) {
    case GT_POOL_BF16: return launch_walk_fmt<GT_POOL_BF16, 32>(a, grid, s);
    case GT_POOL_FP8E4M3: return launch_walk_fmt<GT_POOL_FP8E4M3, 16>(a, grid, s);
    case GT_POOL_F32: return launch_walk_fmt<GT_POOL_F32, 64>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_walk_sub(const WalkLevelArgs& a, int grid, hipStream_t s) {
  grid = kXcds * ((grid + kXcds - 1) / kXcds);
  if (a.dp > kMaxDpBf16 || a.dp < 128 || a.dp % 128 != 0 ||
      a.nb < 0 || a.nb > kMaxBucketBits || ((int64_t)a.nt << a.nb) > kMaxSlots ||
      a.level < a.nb || a.nt < 1 || a.nt > kMaxTiles || a.dense || !a.in_rec || !a.sabs ||
      a.level + 1 >= a.depth || a.depth > 32)
    return hipErrorInvalidValue;
  if (a.dp * 2 / 64 == 32)
    hipLaunchKernelGGL((k_walk_sub<32, kSubPipe>), dim3(grid), dim3(kSubThreads), 0, s, a);
  else
    hipLaunchKernelGGL((k_walk_sub<0, kSubPipe>), dim3(grid), dim3(kSubThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_dense_level(int fmt, const DenseLevelArgs& a, hipStream_t s) {
  if (!a.out_dense &&
      (a.nb < 0 || a.nb > kMaxBucketBits || ((int64_t)a.nt << a.nb) > kMaxSlots || a.level < a.nb))
    return hipErrorInvalidValue;
  if (a.rows < 1 || a.rows > (int64_t(1) << a.level)) return hipErrorInvalidValue;
  if ((a.dp * (fmt == GT_POOL_FP8E4M3 ? 1 : 2)) % kDK != 0) return hipErrorInvalidValue;
  const int64_t rows = a.rows;
  const int64_t total = ((rows + kDM - 1) / kDM) * ((a.nt + kDTiles - 1) / kDTiles);
  const int64_t grid = 8 * ((total + 7) / 8);
  switch (fmt) {
    case GT_POOL_BF16:
      hipLaunchKernelGGL(k_dense_level<GT_POOL_BF16>, dim3((unsigned)grid), dim3(kDThreads), 0, s, a);
      break;
    case GT_POOL_FP8E4M3:
      hipLaunchKernelGGL(k_dense_level<GT_POOL_FP8E4M3>, dim3((unsigned)grid), dim3(kDThreads), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_leaf(const LeafArgs& a, int grid, hipStream_t s) {
  grid = kXcds * ((grid + kXcds - 1) / kXcds);
  if (a.nb < 0 || a.nb > kMaxBucketBits || ((int64_t)a.nt << a.nb) > kMaxSlots ||
      a.level < a.nb || a.nt < 1 || a.nt > kMaxTiles)
    return hipErrorInvalidValue;
  // rows of at most 512 columns: two slices per lane, fewer registers
  // (three waves per SIMD instead of two), so three workgroups per CU
  // (the grid stays a multiple of the XCD count: every XCD's workgroups
  // split its entries by blockIdx / 8)
  if (a.dp <= 512)
    hipLaunchKernelGGL(k_leaf<2>, dim3(kXcds * ((grid / 2 * 3 + kXcds - 1) / kXcds)), dim3(256),
                       0, s, a);
  else
    hipLaunchKernelGGL(k_leaf<4>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_recheck(Hit* hits, const uint32_t* band_idx, const unsigned long long* nband,
                          unsigned long long cap, const float* qf, const float* leaves, int d,
                          int dp, const double* ff, const double* rho,
                          unsigned int* qcount, DevCounters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_recheck, dim3(64), dim3(256), 0, s, hits, band_idx, nband, cap, qf, leaves, d,
                     dp, ff, rho, qcount, ctr);
  return hipGetLastError();
}

hipError_t launch_scan_offsets(const unsigned int* qcount, int nq, int64_t* offs_internal,
                               int64_t* offs_out, DevCounters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, qcount, nq, offs_internal, offs_out,
                     ctr);
  return hipGetLastError();
}

hipError_t launch_scatter(const Hit* hits, const DevCounters* ctr, unsigned long long hit_cap,
                          unsigned long long lim, const int64_t* offs, uint32_t* out_id,
                          float* out_sim, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(1024), dim3(256), 0, s, hits, ctr, hit_cap, lim, offs, out_id,
                     out_sim);
  return hipGetLastError();
}

hipError_t launch_sort_segments(const int64_t* offs, int nq, uint32_t* id, float* sim,
                                uint32_t* tmp_id, float* tmp_sim, int64_t* ids_out,
                                float* sims_out, const DevCounters* ctr,
                                unsigned long long hit_cap, unsigned long long lim,
                                int64_t id_bound, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  // top 8 bits of the ids below id_bound
  int bits = 0;
  while (bits < 32 && (int64_t(1) << bits) < id_bound) ++bits;
  const int shift = bits > 8 ? bits - 8 : 0;
  hipLaunchKernelGGL(k_sort_segments, dim3(nq), dim3(256), 0, s, offs, id, sim, tmp_id, tmp_sim,
                     ids_out, sims_out, ctr, hit_cap, lim, shift);
  return hipGetLastError();
}

}  // namespace gt
