"""Host-side checks that need no GPU: the benchmark's one-GPU contract and the
binding's pool-format names against the C header."""
import os
import re
import subprocess
import sys

from paper_2311_02573_amd import gt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_pool_format_values_match_the_header():
    src = open(os.path.join(ROOT, "include", "gt.h")).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"\b(GT_POOL_[A-Z0-9_]+)\s*=\s*(\d+)", src))
    want = {"f32": "GT_POOL_F32", "bf16": "GT_POOL_BF16", "fp8": "GT_POOL_FP8E4M3",
            "max_f32": "GT_POOL_MAX_F32", "max_bf16": "GT_POOL_MAX_BF16"}
    assert set(gt.POOLS) == set(want)
    for name, sym in want.items():
        assert gt.POOLS[name] == enum[sym], name
    # distinct single bits (a build-time mask)
    vals = sorted(enum.values())
    assert all(v & (v - 1) == 0 for v in vals) and len(set(vals)) == len(vals)
