"""CPU oracle for the group-testing range search -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import,
call, link or execute anything in this package.  The GPU library never does:
its product path has no CPU fallback and fails loudly without its HIP build.

Contents (each function cites the passage of the paper it follows):
  brute    canonical float64 brute-force cosine range scan, in C (range_oracle.c)
  exact    the same decision in exact rational arithmetic; the paper's iterative
           binary-splitting algorithm (Sec. 2, Alg. 1) and its level-wise order
           (Sec. 4), run in rationals, for tiny inputs; the same walk over
           Our-Max pools and over max/min pools of vectors of any sign (Sec. 2)
  pools    explicit pool-sum tree in float64 with error bounds (Sec. 2, Eq. 1),
           Our-Max and max/min trees (Sec. 2)
  formats  bfloat16 / float8 e4m3 value tables and the least representable
           value >= x, from the formats' definitions

The oracle shares no code with the HIP path; both read inputs only from
paper_2311_02573_amd.synth, which draws random data and computes nothing of the
method.
"""
