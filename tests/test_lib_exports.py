"""The C-ABI library loads and exports every symbol include/gt.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

from paper_2311_02573_amd import gt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = _strip_comments(open(os.path.join(ROOT, "include", "gt.h")).read())
    return sorted(set(re.findall(r"^(?:gt_status|void|const char\*)\s+(gt_[a-z_]+)\s*\(", src, re.M)))


def _strip_comments(src):
    return re.sub(r"/\*.*?\*/", "", src, flags=re.S)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("gt_build_tree", "gt_insert", "gt_query_batch", "gt_exhaustive"):
        assert n in names
    assert sorted(gt.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(gt.LIB_PATH):
        pytest.fail("libgt.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(gt.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_argtypes_load():
    lib = gt.load_library()
    assert lib.gt_last_error() == b""


def test_stats_struct_matches_header_fields():
    src = _strip_comments(open(os.path.join(ROOT, "include", "gt.h")).read())
    body = src[src.index("typedef struct {", src.index("GT_MAX_LEVELS 40")):src.index("} gt_stats;")]
    names = re.findall(r"\b([a-z_0-9]+)(?:\[[A-Z_]+\])?\s*[,;]", body)
    assert [n for n, _ in gt.GTStats._fields_] == names
