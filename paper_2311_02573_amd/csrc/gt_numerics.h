// Device-side numerics shared by the kernels: upward-rounded conversions and
// additions, and the fixed-order float32 dot product of the exact leaf test.
//
// Soundness of pruning rests on three facts (paper Sec. 2, sum pooling):
//  (1) every stored pool value is >= the exact sum of its members' values,
//  (2) every stored query value is >= the query value,
//  (3) all values are >= 0,
// so the real dot product of the stored vectors is >= q . f_i for every member
// i.  The helpers here provide (1) and (2) by rounding toward +infinity.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

// Next float32 above a finite x >= 0.
__device__ __forceinline__ float next_up_nonneg(float x) {
  return __uint_as_float(__float_as_uint(x) + 1u);
}

// a + b rounded toward +infinity, for finite a, b >= 0.  TwoSum (Knuth) gives
// the exact error of the round-to-nearest sum; a positive error means the
// nearest sum lies below the exact one.
__device__ __forceinline__ float add_up(float a, float b) {
  float s = __fadd_rn(a, b);
  float bv = __fsub_rn(s, a);
  float av = __fsub_rn(s, bv);
  float err = __fadd_rn(__fsub_rn(a, av), __fsub_rn(b, bv));
  return err > 0.0f ? next_up_nonneg(s) : s;
}

// Least bfloat16 >= x for finite x >= 0.  Values below the smallest normal
// (2^-126) go to that normal, so no subnormal reaches the matrix cores.
__device__ __forceinline__ uint16_t bf16_up(float x) {
  uint32_t u = __float_as_uint(x);
  if (u != 0u && u < 0x00800000u) u = 0x00800000u;
  uint32_t hi = u >> 16;
  if (u & 0xFFFFu) hi += 1u;
  return (uint16_t)hi;
}

// Least OCP float8 e4m3 value >= x, for x >= 0 given exactly as a double.
// e4m3: exponent bias 7, 3 mantissa bits, subnormals m * 2^-9, largest finite
// 448 (code 0x7E); 0x7F is NaN.  Returns 0xFF when x > 448.
__device__ __forceinline__ uint32_t e4m3_up(double x) {
  if (!(x > 0.0)) return 0u;
  if (x > 448.0) return 0xFFu;
  int e;
  double m = frexp(x, &e);            // x = m * 2^e, m in [0.5, 1)
  int E = e - 1;                      // x = (2m) * 2^E
  if (E < -6) {                       // below the smallest normal 2^-6
    double k = ceil(ldexp(x, 9));     // multiples of 2^-9; k == 8 is 2^-6 = code 8
    return (uint32_t)k;
  }
  int mm = (int)ceil(ldexp(2.0 * m - 1.0, 3));
  if (mm == 8) { mm = 0; E += 1; }
  uint32_t code = (uint32_t)(((E + 7) << 3) | mm);
  return code > 0x7Eu ? 0xFFu : code;
}

// float64 -> float32 rounded toward -infinity (thresholds are lowered, never
// raised).
__device__ __forceinline__ float f64_to_f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = __uint_as_float(f > 0.0f ? __float_as_uint(f) - 1u
                                                 : (f == 0.0f ? 0x80000001u : __float_as_uint(f) + 1u));
  return f;
}

// Relative slack of a float32-accumulated pool score of K non-negative terms:
// every rounding inside the accumulation (any rounding mode, including
// truncation) loses less than one unit in the last place, 2^-23 relative to a
// partial sum that never exceeds the final sum, so the computed score is at
// least (1 - (K + 1) * 2^-23) times the real one.  A factor of two on top.
__host__ __device__ __forceinline__ double pool_slack(int K) {
  return (double)(K + 2) * 0x1p-22;
}

// Float8 pool scores.  The gfx950 float8 matrix cores (the 32x32x16 /
// 16x16x32 fp8 forms and the f8f6f4 forms, measured alike on this chip) sum
// each group of 8 consecutive products with truncation about 13 bits below
// the group's largest product, then add the group to the float32
// accumulator: measured, one product 2^13 times the other seven of its group
// leaves them exact, 2^14 times drops them.  For non-negative products a
// group so loses less than 7 x 2^-13 of its own sum, and a whole score less
// than 7 x 2^-13 < 2^-10 of the real one, on top of the float32 slack of
// pool_slack.  Float8 thresholds, compared in scaled units, are lowered by a
// further factor 1 - 2^-8 (about four times that loss; rounding the float32
// product can raise it by 2^-24 at most).  The bfloat16 forms keep about 22
// bits below a group's largest product (a loss below 7 x 2^-22, inside
// pool_slack) and the float32 forms round as float32.
constexpr float kFp8ThrFactor = 1.0f - 0x1p-8f;

// Score bounds of the subtraction step (paper Sec. 2 and Alg. 1: the score of
// one half of a pool is the pool's score minus the other half's).  A pool of
// level l holds exactly the members of its two children, so for the real
// scores  q.S_left = q.S_pool - q.S_right.  With an upper bound on q.S_pool
// and a lower bound on q.S_right this bounds the left child from above
// without reading it.  A score s is computed by the matrix cores from
// operands rounded up to bfloat16 (values below 2^-126 raised to 2^-126),
// K <= 4096 products accumulated in float32; the real score q.S uses the
// float32 query and rows.
//  * Upper bound: the rounded-up operands give an exact dot product P >= q.S
//    (all terms >= 0).  Products below 2^-126 may be flushed (each loses less
//    than 2^-126) and the accumulation loses less than (K+1) ulps relative
//    (section on pool slack), so P <= (s + K 2^-126) / (1 - (K+1) 2^-23)
//    <= 1.000489 s + K 2^-126 (1 + 2^-10).  score_upper computes
//    s * 1.0006 + K 2^-125 with one rounding to nearest (2^-24 relative,
//    2^-149 absolute at most), which stays above that.
//  * Lower bound: each stored operand is at most (1 + 2^-7) times the real
//    one plus 2^-126, the master sums exceed the real sums by their upward
//    roundings over at most 40 levels (factor 1 + 40 2^-23), and the
//    accumulation rounds up by less than (K+1) ulps; so
//      q.S >= s / ((1 + (K+1) 2^-23) (1 + 2^-7)^2 (1 + 40 2^-23)) - A
//          >= 0.984071 s - A,
//    A = 2^-126 (c |S|_1 + c |q|_1 + K 2^-126), c < 1.01.  The query
//    preparation gives a = 2 A + 2^-126 (with |S|_1 <= |root|_1), and
//    score_lower computes s * 0.9839 - a with one rounding to nearest, which
//    stays below 0.984071 s - A; a negative value is replaced by 0.
//  * The difference of the two is rounded up explicitly (diff_upper).
constexpr float kScoreUp = 1.0006f;
constexpr float kScoreLow = 0.9839f;
__device__ __forceinline__ float score_abs_up(int K) { return (float)K * 0x1p-125f; }
__device__ __forceinline__ float score_upper(float s, float abs_up) {
  return __fmaf_rn(s, kScoreUp, abs_up);
}
__device__ __forceinline__ float score_lower(float s, float a) {
  return fmaxf(__fmaf_rn(s, kScoreLow, -a), 0.0f);
}
// Upper bound of u - l for u >= 0 (or +infinity) and finite l >= 0, at least
// 0: the nearest difference, moved up by one float when it is positive.
__device__ __forceinline__ float diff_upper(float u, float l) {
  const float d = __fsub_rn(u, l);
  return d > 0.0f ? (d < INFINITY ? __uint_as_float(__float_as_uint(d) + 1u) : d) : 0.0f;
}
// Least bfloat16 >= x for x >= 0 or +infinity, subnormals kept (bounds are
// only used in float32 arithmetic, never as matrix-core operands), as the
// high half of a 32-bit word.
__device__ __forceinline__ uint32_t bf16_ceil_hi(float x) {
  return (__float_as_uint(x) + 0xFFFFu) & 0xFFFF0000u;
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// In-lane part of a fixed-order float32 dot product of two rows, wave-wide
// (64 lanes).  In chunk c (1024 elements), lane l owns the 16 elements
//   c*1024 + 256 v + 4 l + j      (v, j = 0..3),
// so each of the lane's four 16-byte loads belongs to one contiguous 1 KB
// piece read by the whole wave.  The 16 products are summed pairwise, each
// pair by one fused multiply-add (written out, so that no compiler
// contraction can change it):
//   slice v:  fma(x0, y0, x1 y1) + fma(x2, y2, x3 y3)
//   chunk:    (slice 0 + slice 1) + (slice 2 + slice 3)
// Callers add the chunks in order and then sum over the lanes with
// wave_reduce8; the result depends only on the two rows.  Slices past dp
// count as zero; their loads are redirected to the last slice of the row so
// that every load stays in bounds and no branch is needed.
// Each product meets at most three roundings within its slice (as with
// separate products), so
// Bound: |error| <= (5 + (chunks - 1) + 6) * 2^-24 * exact sum.
__device__ __forceinline__ int slice_index(int chunk, int v, int lane, int dp, bool& ok) {
  const int e4 = chunk * 256 + 64 * v + lane;  // float4 index within the row
  ok = 4 * e4 < dp;
  return ok ? e4 : (dp >> 2) - 1;
}
__device__ __forceinline__ float slice_dot4(const float4& x, const float4& y) {
  return __fadd_rn(__builtin_fmaf(x.x, y.x, __fmul_rn(x.y, y.y)),
                   __builtin_fmaf(x.z, y.z, __fmul_rn(x.w, y.w)));
}
__device__ __forceinline__ float chunk_sum4(float s0, float s1, float s2, float s3) {
  return __fadd_rn(__fadd_rn(s0, s1), __fadd_rn(s2, s3));
}
__device__ __forceinline__ float lane_partial16(const float* __restrict__ a,
                                                const float* __restrict__ b, int chunk, int dp,
                                                int lane) {
  float sv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    bool ok;
    const int ec = slice_index(chunk, v, lane, dp, ok);
    const float4 x = reinterpret_cast<const float4*>(a)[ec];
    const float4 y = reinterpret_cast<const float4*>(b)[ec];
    const float dv = slice_dot4(x, y);
    sv[v] = ok ? dv : 0.0f;
  }
  return chunk_sum4(sv[0], sv[1], sv[2], sv[3]);
}

// Sums eight per-lane values over the 64 lanes, each by the same tree
// (partners at lane distance 32, 16, 8, 4, 2, 1), using 10 shuffles instead
// of 6 per value.  Lanes 8v .. 8v+7 receive the sum of value v.
__device__ __forceinline__ float wave_reduce8(const float (&a)[8], int lane) {
  const bool h = (lane >> 5) & 1, g = (lane >> 4) & 1, f = (lane >> 3) & 1;
  float b[4], c[2];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float send = h ? a[j] : a[j + 4];
    const float keep = h ? a[j + 4] : a[j];
    b[j] = __fadd_rn(keep, __shfl_xor(send, 32, 64));
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float send = g ? b[j] : b[j + 2];
    const float keep = g ? b[j + 2] : b[j];
    c[j] = __fadd_rn(keep, __shfl_xor(send, 16, 64));
  }
  float dsum = __fadd_rn(f ? c[1] : c[0], __shfl_xor(f ? c[0] : c[1], 8, 64));
  dsum = __fadd_rn(dsum, __shfl_xor(dsum, 4, 64));
  dsum = __fadd_rn(dsum, __shfl_xor(dsum, 2, 64));
  dsum = __fadd_rn(dsum, __shfl_xor(dsum, 1, 64));
  return dsum;
}

// Canonical float64 cosine: sequential sums over k, then
// dot / (sqrt(qq) * sqrt(ff)).  Products of float32 values are exact in
// float64, so fused or separate multiply-add give the same value.
__device__ __forceinline__ double canonical_cos(const float* __restrict__ q,
                                                const float* __restrict__ f, int d, double qq,
                                                double ff) {
  double dot = 0.0;
  for (int k = 0; k < d; ++k) dot = __dadd_rn(dot, __dmul_rn((double)q[k], (double)f[k]));
  return __ddiv_rn(dot, __dmul_rn(__dsqrt_rn(qq), __dsqrt_rn(ff)));
}

}  // namespace gt
