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
    assert int(codes["CM_E_IO"]) == cm.E_IO
    import oracle
    assert oracle.E_MISSING == cm.E_MISSING and oracle.E_DUP == cm.E_DUP


def _snapshot_bytes(n_ids, n_alive, m, payload, checksum=None, magic=b"CMSNAP01", version=1):
    import struct
    import numpy as np
    words = np.asarray(payload, dtype=np.int32)
    if checksum is None:
        h = 0xCBF29CE484222325
        for w in words.astype(np.uint32).tolist():
            h = ((h ^ w) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
        checksum = h
    return magic + struct.pack("<iiiiqQ", version, n_ids, n_alive, 0, m, checksum) + words.tobytes()


def test_restore_rejects_bad_files_on_the_host(lib, tmp_path):
    """cm_restore checks the file before it creates a handle: a missing,
    truncated, corrupt or inconsistent snapshot is CM_E_IO and no device
    work starts."""
    import paper_1612_09368_amd as cm
    h = ctypes.c_void_p()
    assert lib.cm_restore(None, str(tmp_path / "missing.snap").encode(), ctypes.byref(h)) == cm.E_IO
    # a path-triangle on 3 ids: cores 2,2,2 and SD 2,2,2, edges (0,1), (0,2), (1,2)
    good = [2, 2, 2, 2, 2, 2, 0, 0, 1, 1, 2, 2]
    cases = {
        "magic": _snapshot_bytes(3, 3, 3, good, magic=b"XXSNAP01"),
        "version": _snapshot_bytes(3, 3, 3, good, version=2),
        "checksum": _snapshot_bytes(3, 3, 3, good, checksum=12345),
        "truncated": _snapshot_bytes(3, 3, 3, good)[:-4],
        "long": _snapshot_bytes(3, 3, 3, good) + b"\0\0\0\0",
        "alive count": _snapshot_bytes(3, 2, 3, good),
        "edge at dead id": _snapshot_bytes(3, 2, 3, [2, 2, -1, 2, 2, 0, 0, 0, 1, 1, 2, 2]),
        "core out of range": _snapshot_bytes(3, 3, 3, [2, 2, 7, 2, 2, 2, 0, 0, 1, 1, 2, 2]),
        "edge out of range": _snapshot_bytes(3, 3, 3, [2, 2, 2, 2, 2, 2, 0, 0, 1, 1, 2, 9]),
    }
    for name, data in cases.items():
        p = tmp_path / f"{name.replace(' ', '_')}.snap"
        p.write_bytes(data)
        h = ctypes.c_void_p()
        assert lib.cm_restore(None, str(p).encode(), ctypes.byref(h)) == cm.E_IO, name
        assert not h.value, name
    assert lib.cm_snapshot(None, b"x") == cm.E_ARG
    assert lib.cm_debug_log(None, None, None, 0, None, None, 0) == cm.E_ARG
    assert lib.cm_strerror(cm.E_IO).decode() == "snapshot file error"
