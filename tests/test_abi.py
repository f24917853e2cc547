"""C ABI: the built library loads on the host and exports every symbol that
include/coremaint.h declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "coremaint.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1612_09368_amd as cm
    if not os.path.exists(cm.LIB_PATH):
        from paper_1612_09368_amd import build
        build.build()
    return cm.library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    import paper_1612_09368_amd as cm
    assert set(cm.EXPORTED) <= set(names)


def test_host_only_calls(lib):
    import paper_1612_09368_amd as cm
    cfg = cm.Config()
    lib.cm_config_default(ctypes.byref(cfg))
    assert cfg.strict == 1 and cfg.mode == cm.MODE_PLAIN and cfg.vertex_capacity == 0
    assert lib.cm_strerror(cm.E_MISSING).decode() == "edge does not exist"
    assert lib.cm_strerror(cm.OK).decode() == "ok"
    # null-handle misuse is rejected on the host before any device work
    assert lib.cm_create(None, None) == cm.E_ARG
    assert lib.cm_load_graph(None, 0, 0, None, None, 0) == cm.E_ARG
    assert lib.cm_insert_edges(None, 0, None, None, 0, None) == cm.E_ARG
    assert lib.cm_last_error(None).decode() == ""
    lib.cm_destroy(None)


def test_status_codes_match_header():
    import paper_1612_09368_amd as cm
    text = open(HEADER).read()
    codes = dict(re.findall(r"#define (CM_E_[A-Z_]+) \((-\d+)\)", text))
    assert int(codes["CM_E_MISSING"]) == cm.E_MISSING
    assert int(codes["CM_E_EXISTS"]) == cm.E_EXISTS
    assert int(codes["CM_E_DEAD"]) == cm.E_DEAD
    assert int(codes["CM_E_INTERNAL"]) == cm.E_INTERNAL
    import oracle
    assert oracle.E_MISSING == cm.E_MISSING and oracle.E_DUP == cm.E_DUP
