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
            "max_f32": "GT_POOL_MAX_F32", "max_bf16": "GT_POOL_MAX_BF16",
            "signed": "GT_POOL_SIGNED"}
    assert set(gt.POOLS) == set(want)
    for name, sym in want.items():
        assert gt.POOLS[name] == enum[sym], name
    # distinct single bits (a build-time mask)
    vals = sorted(enum.values())
    assert all(v & (v - 1) == 0 for v in vals) and len(set(vals)) == len(vals)


def test_stats_struct_fields_match_the_header():
    """The binding's gt_stats mirror has the header's fields, in order, with
    the same C types (a mismatch would shift every later field)."""
    import ctypes

    src = open(os.path.join(ROOT, "include", "gt.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} gt_stats;", src, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    ctype = {"int64_t": ctypes.c_int64, "int32_t": ctypes.c_int32, "uint32_t": ctypes.c_uint32,
             "uint64_t": ctypes.c_uint64, "double": ctypes.c_double, "float": ctypes.c_float}
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, rest = decl.split(None, 1)
        for name in rest.split(","):
            name = name.strip()
            m = re.match(r"(\w+)\[(\w+)\]", name)
            if m:
                fields.append((m.group(1), ctype[typ] * gt.GT_MAX_LEVELS))
                assert m.group(2) == "GT_MAX_LEVELS"
            else:
                fields.append((name, ctype[typ]))
    mine = gt.GTStats._fields_
    assert [f[0] for f in mine] == [f[0] for f in fields]
    for (name, t1), (_, t2) in zip(mine, fields):
        assert ctypes.sizeof(t1) == ctypes.sizeof(t2), name
        assert t1._type_ == t2._type_, name   # element type (arrays too)
