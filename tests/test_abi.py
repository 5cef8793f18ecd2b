"""The C-ABI library loads and exports every symbol include/cc.h declares
(no compute calls: this runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(cc[a-z_]*)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libcc():
    from paper_1602_05232_amd import build as hipbuild
    if not os.path.exists(hipbuild.OUT):
        hipbuild.build()
    import ctypes
    return ctypes.CDLL(hipbuild.OUT)


@pytest.mark.parametrize("header", ["cc.h", "cc_pool.h", "cc_bench.h"])
def test_exports_every_declared_symbol(libcc, header):
    names = declared_functions(header)
    assert len(names) >= 4
    missing = [n for n in names if not hasattr(libcc, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_1602_05232_amd import cc
    assert set(declared_functions("cc.h")) == set(cc.SIGNATURES)
    assert set(declared_functions("cc_bench.h")) == set(cc.BENCH_SIGNATURES)
    assert set(declared_functions("cc_pool.h")) == set(cc.POOL_SIGNATURES)


def test_strerror_and_invalid_args_without_device(libcc):
    # pure host paths: argument checks return before touching the device
    from paper_1602_05232_amd import cc
    L = cc.load_library(cc.LIB_PATH)
    assert L.cc_strerror(0) == b"ok"
    assert L.cc_strerror(-3).startswith(b"vertex id out of range")
    assert L.cc_bulk_update(None, None, 5) == cc.CC_EINVAL
    assert L.cc_bulk_query(None, None, 0, None) == cc.CC_EINVAL
    assert L.cc_destroy(None) == cc.CC_EINVAL
    assert L.cc_num_vertices(None) == 0
    assert not L.cc_create(0)
    assert b"outside" in L.cc_last_error()
    import ctypes
    a, c = ctypes.c_int32(), ctypes.c_int32()
    assert L.cc_filter_state(None, ctypes.byref(a), ctypes.byref(c), None) == cc.CC_EINVAL
    assert L.cc_set_option(None, cc.OPT_FILTER, 1) == cc.CC_EINVAL
    assert L.cc_get_option(None, cc.OPT_QUERY_ITEMS, None) == cc.CC_EINVAL


def test_option_constants_match_the_header():
    """The binding's option numbers and names are those of enum cc_option."""
    from paper_1602_05232_amd import cc
    src = open(os.path.join(ROOT, "include", "cc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    enum = dict((k, int(v)) for k, v in re.findall(r"\b(CC_OPT_[A-Z_]+)\s*=\s*(\d+)", src))
    assert len(enum) >= 13
    for name, value in enum.items():
        assert getattr(cc, name[3:]) == value, name  # CC_OPT_X -> cc.OPT_X
    assert set(cc._OPT_NAMES.values()) == set(enum.values())


def test_tuned_options_are_known_and_in_range():
    """Every stored option set names options of the binding with values the
    library accepts (ranges of include/cc.h), so a lookup never fails at
    graph creation."""
    import json
    from paper_1602_05232_amd import cc, tuning
    allowed = {"update_mode": {0, 1, 2}, "block": set(range(64, 1025, 64)), "items": {0, 1, 2, 4, 8},
               "query_items": {0, 1, 2, 4, 8}, "query_halving": {0, 1}, "hook": {0, 1, 2},
               "compress_linked": {0, 1}, "filter": {0, 1, 2}, "find": {0, 1, 2}, "one_launch": {0, 1},
               "split_below": set(range(0, 101))}
    tab = json.load(open(tuning.CACHE))
    assert "plain/rmat/24" in tab
    for key, opts in list(tab.items()) + [("defaults", tuning.DEFAULTS)]:
        for k, v in opts.items():
            assert k in cc._OPT_NAMES, (key, k)
            if k in allowed:
                assert v in allowed[k], (key, k, v)
            elif k == "grid_cap":
                assert 1 <= v <= 1 << 20
            elif k == "compress_every":
                assert v >= 0
        if key.startswith("plain/") and opts.get("hook") == 2:
            assert opts.get("update_mode", 0) == 0, key  # rank linking takes the fused schedule only
