"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/hloc.h declares, and rejects malformed arguments before any
device work."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2006_08861_amd import hloc

pytestmark = pytest.mark.skipif(not os.path.exists(hloc.LIB_PATH),
                                reason="libhloc.so not built (python -m paper_2006_08861_amd.build)")


def _lib():
    return hloc.load_library()


def test_exports_every_declared_symbol():
    declared = hloc.header_symbols()
    assert len(declared) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", hloc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    lib = _lib()
    for s in declared:
        assert getattr(lib, s) is not None


def test_binding_signatures_cover_header():
    assert sorted(hloc._SIGNATURES) == hloc.header_symbols()


def _build(feats, xy, n=None, d=None, mirrors=0):
    lib = _lib()
    h = ctypes.c_void_p()
    f = None if feats is None else feats.ctypes.data_as(ctypes.c_void_p)
    x = None if xy is None else xy.ctypes.data_as(ctypes.c_void_p)
    n = feats.shape[0] if n is None else n
    d = feats.shape[1] if d is None else d
    rc = lib.hloc_build_db(f, n, d, x, mirrors, ctypes.byref(h))
    return rc, h, lib.hloc_last_error().decode()


def test_build_db_rejects_bad_arguments():
    feats = np.zeros((4, 3), np.float32)
    xy = np.zeros((4, 2), np.float64)
    rc, h, msg = _build(None, xy, 4, 3)
    assert rc == hloc.EINVAL and h.value is None and "NULL" in msg
    rc, h, msg = _build(feats, xy, n=0)
    assert rc == hloc.EINVAL and "n must be" in msg
    rc, h, msg = _build(feats, xy, d=0)
    assert rc == hloc.EINVAL and "d must be" in msg
    rc, h, msg = _build(feats, xy, d=hloc_max_dim() + 1)
    assert rc == hloc.EINVAL
    bad = feats.copy()
    bad[2, 1] = np.nan
    rc, h, msg = _build(bad, xy)
    assert rc == hloc.EINVAL and "row 2" in msg
    badxy = xy.copy()
    badxy[1, 0] = np.inf
    rc, h, msg = _build(feats, badxy)
    assert rc == hloc.EINVAL and "position" in msg
    rc, h, msg = _build(feats, xy, mirrors=0x80)
    assert rc == hloc.EUNSUPPORTED


def hloc_max_dim():
    with open(hloc.HEADER) as f:
        for line in f:
            if line.startswith("#define HLOC_MAX_DIM"):
                return int(line.split()[2])
    raise AssertionError("HLOC_MAX_DIM not found")


def test_calls_on_null_database():
    lib = _lib()
    assert lib.hloc_set_regions(None, None, 1, None) == hloc.EINVAL
    assert lib.hloc_set_aggregation(None, 0.5, 1, 0.0, 0) == hloc.EINVAL
    assert lib.hloc_reserve(None, 1, 1, 1, 1) == hloc.EINVAL
    assert lib.hloc_query_batch(None, None, 0, 1, 1, None, 0, 0, None, None, None, None,
                                None) == hloc.EINVAL
    assert lib.hloc_query_batch_async(None, None, 0, 1, 1, None, 0, 0, None, None, None, None,
                                      None, None) == hloc.EINVAL
    assert lib.hloc_query_windows_async(None, None, 0, 1, 1, None, None, 0, 0, 0, None, None,
                                        None, None, None, None) == hloc.EINVAL
    assert lib.hloc_set_region_labels(None, None, 1) == hloc.EINVAL
    assert lib.hloc_query_labels_async(None, None, 0, 1, 1, 1, None, 0, 0, None, None, None,
                                       None, None, None) == hloc.EINVAL
    out = (ctypes.c_int64 * 6)()
    assert lib.hloc_query_info(None, out, 6) == hloc.EINVAL
    a, b = ctypes.c_int32(), ctypes.c_int32()
    assert lib.hloc_last_regions(None, None, ctypes.byref(a), ctypes.byref(b)) == hloc.EINVAL
    lib.hloc_free_db(None)  # ignored
    assert "NULL" in lib.hloc_last_error().decode()


def test_tile_calls_on_null_handles():
    lib = _lib()
    t = hloc.Tiles(32, 4)
    assert lib.hloc_set_tiles(None, ctypes.byref(t)) == hloc.EINVAL
    assert lib.hloc_get_tiles(None, ctypes.byref(t)) == hloc.EINVAL
    ms = ctypes.c_double()
    assert lib.hloc_autotune(None, None, 1, 1, 1, 0, 1, ctypes.byref(t), ctypes.byref(ms)) == hloc.EINVAL


def test_server_calls_on_null_handles():
    lib = _lib()
    cfg = hloc.ServerConfig(16, 8, 0, 64, 2, 4096, 0)
    h = ctypes.c_void_p()
    assert lib.hloc_server_create(None, ctypes.byref(cfg), ctypes.byref(h)) == hloc.EINVAL
    assert h.value is None
    t = ctypes.c_uint64()
    frames = np.zeros((2, 8), np.float32)
    assert lib.hloc_server_submit(None, frames.ctypes.data_as(ctypes.c_void_p), 2, 4,
                                  ctypes.byref(t)) == hloc.EINVAL
    assert lib.hloc_server_wait(None, 1, 0, None, None, None, None, None, None) == hloc.EINVAL
    out = (ctypes.c_int64 * 10)()
    assert lib.hloc_server_stats(None, out, 10) == hloc.EINVAL
    lib.hloc_server_free(None)  # ignored


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(hloc, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(hloc, "_lib", None)
    with pytest.raises(hloc.HlocError, match="not built"):
        hloc.load_library()


def test_header_limits_match_binding_constants():
    with open(hloc.HEADER) as f:
        text = f.read()
    for name, val in (("HLOC_EINVAL", hloc.EINVAL), ("HLOC_EUNSUPPORTED", hloc.EUNSUPPORTED),
                      ("HLOC_EBUSY", hloc.EBUSY), ("HLOC_ETIMEDOUT", hloc.ETIMEDOUT),
                      ("HLOC_FLAG_EMPTY", hloc.FLAG_EMPTY), ("HLOC_MIRROR_BF16", hloc.MIRROR_BF16)):
        assert f"{name} = {val}" in text


def test_phase_and_info_counts_match_header():
    # the binding names one profile phase per HLOC_PHASE_* and reads as many
    # query counters as the header documents
    import re
    with open(hloc.HEADER) as f:
        text = f.read()
    n_phases = int(re.search(r"HLOC_NUM_PHASES = (\d+)", text).group(1))
    assert len(hloc.HlocDB.PHASES) == n_phases
    n_info = int(re.search(r"Writes min\(n, (\d+)\) values", text).group(1))
    assert len(hloc._INFO_KEYS) == n_info



def test_fft_features_rejects_bad_arguments():
    """Sizes are checked before any device call (safe without a GPU)."""
    lib = _lib()
    P = ctypes.c_void_p
    dummy = P(16)  # never dereferenced: every call below fails validation or does nothing
    for nsig, length, d in ((-1, 8, 2), (4, 3, 2), (4, 1, 1), (4, 4096, 8), (4, 12, 2),
                            (4, 8, 0), (4, 8, 6), (4, 2, 3)):
        rc = lib.hloc_fft_features_async(dummy, nsig, length, d, dummy, None)
        assert rc == hloc.EINVAL, (nsig, length, d)
        assert lib.hloc_last_error().decode()
    assert lib.hloc_fft_features_async(None, 4, 8, 5, None, None) == hloc.EINVAL
    assert lib.hloc_fft_features_async(None, 0, 8, 5, None, None) == hloc.OK
