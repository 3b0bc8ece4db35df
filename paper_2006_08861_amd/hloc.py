"""Python binding of libhloc.so (include/hloc.h) — argument marshalling only.

Every step of the localization runs in the library's HIP kernels. PyTorch is
used for device memory and streams: a query given as a CUDA tensor runs on
torch's current stream and returns CUDA tensors; a query given as a NumPy
array goes through the blocking host-pointer entry point and returns NumPy
arrays. If the library has not been built, loading raises HlocError; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

# the in-tree build; HLOC_LIBRARY names another build of the same sources
LIB_PATH = os.environ.get("HLOC_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libhloc.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "hloc.h")

OK, EINVAL, ENOMEM, ESTATE, EDEVICE, EUNSUPPORTED, EBUSY, ETIMEDOUT = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", ESTATE: "ESTATE",
                EDEVICE: "EDEVICE", EUNSUPPORTED: "EUNSUPPORTED", EBUSY: "EBUSY",
                ETIMEDOUT: "ETIMEDOUT"}
FP32, BF16, FP8 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8}
FLAG_LOW_CONFIDENCE, FLAG_EMPTY, FLAG_BAD_REQUEST = 1, 2, 4
MIRROR_BF16, MIRROR_FP8 = 1, 2

_lib = None

_P = ctypes.c_void_p
_I32, _I64, _U32, _F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
_U64 = ctypes.c_uint64


class Tiles(ctypes.Structure):
    """hloc_tiles."""
    _fields_ = [("rows_per_item", _I32), ("blocks_per_cu", _I32)]


class ServerConfig(ctypes.Structure):
    """hloc_server_config."""
    _fields_ = [("k", _I32), ("n_regions", _I32), ("precision", _I32),
                ("max_batch_frames", _I32), ("max_slots", _I32), ("max_queue_frames", _I32),
                ("hbm_budget_bytes", _I64)]
_SIGNATURES = {
    "hloc_build_db": (ctypes.c_int, [_P, _I64, _I32, _P, _U32, ctypes.POINTER(_P)]),
    "hloc_set_regions": (ctypes.c_int, [_P, _P, _I32, _P]),
    "hloc_set_aggregation": (ctypes.c_int, [_P, _F64, _I32, _F64, _I32]),
    "hloc_query_batch": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _I32, _I32, _P, _P, _P, _P,
                                        _P]),
    "hloc_query_batch_async": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _I32, _I32, _P, _P,
                                              _P, _P, _P, _P]),
    "hloc_query_batch_static_async": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _I32, _I32,
                                                     _P, _P, _P, _P, _P, _P]),
    "hloc_query_windows_async": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _P, _I32, _I32,
                                                _I32, _P, _P, _P, _P, _P, _P]),
    "hloc_streams_create": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, ctypes.POINTER(_P)]),
    "hloc_streams_reset": (ctypes.c_int, [_P]),
    "hloc_streams_free": (None, [_P]),
    "hloc_query_streams_async": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _P, _I32, _P, _P,
                                                _P, _P, _P, _P]),
    "hloc_set_region_labels": (ctypes.c_int, [_P, _P, _I32]),
    "hloc_query_labels_async": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _I32, _P, _I32, _I32,
                                               _P, _P, _P, _P, _P, _P]),
    "hloc_reserve": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32]),
    "hloc_query_info": (ctypes.c_int, [_P, _P, _I32]),
    "hloc_last_regions": (ctypes.c_int, [_P, _P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "hloc_ws_create": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "hloc_ws_free": (None, [_P]),
    "hloc_ws_reserve": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32]),
    "hloc_ws_query_async": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _I32, _I32, _P, _P, _P,
                                           _P, _P, _P]),
    "hloc_ws_query_info": (ctypes.c_int, [_P, _P, _I32]),
    "hloc_ws_capture": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _I32, _I32, _P, _P, _P, _P,
                                       _P]),
    "hloc_ws_replay": (ctypes.c_int, [_P, _P]),
    "hloc_profile": (ctypes.c_int, [_P, _I32]),
    "hloc_profile_read": (ctypes.c_int, [_P, _P, _P, _I32]),
    "hloc_set_tiles": (ctypes.c_int, [_P, ctypes.POINTER(Tiles)]),
    "hloc_get_tiles": (ctypes.c_int, [_P, ctypes.POINTER(Tiles)]),
    "hloc_autotune": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, ctypes.POINTER(Tiles),
                                     ctypes.POINTER(_F64)]),
    "hloc_server_create": (ctypes.c_int, [_P, ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]),
    "hloc_server_submit": (ctypes.c_int, [_P, _P, _I32, _I32, ctypes.POINTER(_U64)]),
    "hloc_server_wait": (ctypes.c_int, [_P, _U64, _I32, _P, _P, _P, _P, _P,
                                        ctypes.POINTER(_F64)]),
    "hloc_server_stats": (ctypes.c_int, [_P, _P, _I32]),
    "hloc_server_free": (None, [_P]),
    "hloc_fft_features_async": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _P]),
    "hloc_free_db": (None, [_P]),
    "hloc_last_error": (ctypes.c_char_p, []),
}


class HlocError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


def header_symbols() -> list[str]:
    """Names of the functions include/hloc.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(hloc_\w+)\s*\(", text,
                                 flags=re.M)))


def load_library():
    """Load libhloc.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HlocError(EDEVICE, f"{LIB_PATH} is not built; run `python -m "
                                 "paper_2006_08861_amd.build`")
    import torch  # noqa: F401  (binds libamdhip64 before the library does)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise HlocError(rc, load_library().hloc_last_error().decode())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _is_torch_cuda(x) -> bool:
    try:
        import torch
    except ImportError:
        return False
    return isinstance(x, torch.Tensor) and x.is_cuda


def fft_features(signals, d: int, stream=None):
    """Fourier-magnitude features (hloc_fft_features_async) of nsig x len
    float32 signals: a CUDA tensor runs on `stream` (default: torch's current
    stream) and returns a CUDA tensor; a NumPy array is copied to the current
    device and back and returns a NumPy array."""
    import torch
    host = not _is_torch_cuda(signals)
    x = (torch.from_numpy(np.ascontiguousarray(signals, dtype=np.float32)).cuda() if host
         else signals.contiguous())
    if x.dtype != torch.float32 or x.dim() != 2:
        raise HlocError(EINVAL, "signals must be a 2-D float32 array")
    nsig, length = x.shape
    out = torch.empty((nsig, d), dtype=torch.float32, device=x.device)
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    lib = load_library()
    with torch.cuda.device(x.device):
        _check(lib.hloc_fft_features_async(_P(x.data_ptr()), nsig, length, d, _P(out.data_ptr()),
                                           _P(stream.cuda_stream)))
    if host:
        stream.synchronize()
        return out.cpu().numpy()
    return out


class HlocDB:
    """A feature database on the current HIP device (see include/hloc.h)."""

    def __init__(self, feats, xy, mirrors: int = 0):
        lib = load_library()
        feats = np.ascontiguousarray(feats, dtype=np.float32)
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        if feats.ndim != 2 or xy.shape != (feats.shape[0], 2):
            raise HlocError(EINVAL, "feats must be n x d and xy n x 2")
        h = ctypes.c_void_p()
        _check(lib.hloc_build_db(_np_ptr(feats), feats.shape[0], feats.shape[1], _np_ptr(xy),
                                 mirrors, ctypes.byref(h)))
        self._h = h
        self.n, self.d = feats.shape
        self.n_regions_total = 0

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().hloc_free_db(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_regions(self, region_of, n_regions_total: int, reps=None):
        region_of = np.ascontiguousarray(region_of, dtype=np.int32)
        if region_of.shape != (self.n,):
            raise HlocError(EINVAL, "region_of must have one entry per row")
        if reps is not None:
            reps = np.ascontiguousarray(reps, dtype=np.float32)
            if reps.shape != (n_regions_total, self.d):
                raise HlocError(EINVAL, "reps must be n_regions_total x d")
        _check(load_library().hloc_set_regions(self._h, _np_ptr(region_of), n_regions_total,
                                               _np_ptr(reps)))
        self.n_regions_total = n_regions_total

    def set_aggregation(self, cell: float, top_c: int, radius: float, toler_pct: int):
        _check(load_library().hloc_set_aggregation(self._h, cell, top_c, radius, toler_pct))

    def reserve(self, nq_max: int, nreq_max: int, k_max: int, n_regions_max: int):
        _check(load_library().hloc_reserve(self._h, nq_max, nreq_max, k_max, n_regions_max))

    def query(self, q, k: int, n_regions: int, req_offsets=None, precision="fp32",
              aggregate: bool = True, stream=None) -> dict:
        """Localize a batch. Returns idx, dist (per frame) and, with
        aggregate=True, xy, tile and flags (per request)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if _is_torch_cuda(q):
            return self._query_device(q, k, n_regions, req_offsets, prec, aggregate, stream)
        return self._query_host(q, k, n_regions, req_offsets, prec, aggregate)

    def query_static(self, q, k: int, n_regions: int, req_offsets=None, precision="fp32",
                     aggregate: bool = True, stream=None) -> dict:
        """As query() on CUDA tensors, through hloc_query_batch_static_async:
        the library allocates no device memory for the batch (its scratch is
        the library's static array; the output tensors are allocated here)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if not _is_torch_cuda(q):
            raise HlocError(EINVAL, "query_static takes a CUDA tensor of frames")
        return self._query_device(q, k, n_regions, req_offsets, prec, aggregate, stream,
                                  entry="hloc_query_batch_static_async")

    def _query_host(self, q, k, n_regions, req_offsets, prec, aggregate):
        lib = load_library()
        q = np.ascontiguousarray(q, dtype=np.float32)
        if q.ndim != 2 or q.shape[1] != self.d:
            raise HlocError(EINVAL, f"q must be nq x {self.d}")
        nq = q.shape[0]
        offs = None if req_offsets is None else np.ascontiguousarray(req_offsets, dtype=np.int32)
        nreq = nq if offs is None else len(offs) - 1
        idx = np.empty((nq, k), np.int64)
        dist = np.empty((nq, k), np.float32)
        out = dict(idx=idx, dist=dist)
        xy = tile = flags = None
        if aggregate:
            xy = np.empty((nreq, 2), np.float64)
            tile = np.empty((nreq, 2), np.int32)
            flags = np.empty(nreq, np.int32)
            out.update(xy=xy, tile=tile, flags=flags)
        _check(lib.hloc_query_batch(self._h, _np_ptr(q), nq, k, n_regions, _np_ptr(offs), nreq,
                                    prec, _np_ptr(idx), _np_ptr(dist), _np_ptr(xy),
                                    _np_ptr(tile), _np_ptr(flags)))
        return out

    def _query_device(self, q, k, n_regions, req_offsets, prec, aggregate, stream,
                      entry="hloc_query_batch_async"):
        import torch
        lib = load_library()
        if q.dtype != torch.float32 or q.dim() != 2 or q.shape[1] != self.d:
            raise HlocError(EINVAL, f"q must be an nq x {self.d} float32 tensor")
        q = q.contiguous()
        dev = q.device
        nq = q.shape[0]
        offs = None
        if req_offsets is not None:
            offs = torch.as_tensor(req_offsets, dtype=torch.int32, device=dev).contiguous()
        nreq = nq if offs is None else offs.numel() - 1
        idx = torch.empty((nq, k), dtype=torch.int64, device=dev)
        dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
        out = dict(idx=idx, dist=dist)
        xy = tile = flags = None
        if aggregate:
            xy = torch.empty((nreq, 2), dtype=torch.float64, device=dev)
            tile = torch.empty((nreq, 2), dtype=torch.int32, device=dev)
            flags = torch.empty(nreq, dtype=torch.int32, device=dev)
            out.update(xy=xy, tile=tile, flags=flags)
        s = stream if stream is not None else torch.cuda.current_stream(dev)

        def p(t):
            return None if t is None else ctypes.c_void_p(t.data_ptr())

        _check(getattr(lib, entry)(self._h, p(q), nq, k, n_regions, p(offs), nreq, prec,
                                   p(idx), p(dist), p(xy), p(tile), p(flags),
                                   ctypes.c_void_p(s.cuda_stream)))
        return out

    def set_region_labels(self, labels, n_labels: int):
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        _check(load_library().hloc_set_region_labels(self._h, _np_ptr(lab), n_labels))
        self.n_labels = int(n_labels)

    def query_labels(self, q, k: int, n_regions: int, n_labels: int, req_offsets=None,
                     precision="fp32", stream=None) -> dict:
        """Top k per (frame, subspace label) and one estimate per request
        pooling frames x labels x k candidates (hloc_query_labels_async).
        idx / dist come back as n_labels x nq x k CUDA tensors."""
        import torch
        dev = q.device if _is_torch_cuda(q) else torch.device("cuda", torch.cuda.current_device())
        qd = q.float().contiguous() if _is_torch_cuda(q) else \
            torch.from_numpy(np.ascontiguousarray(q, dtype=np.float32)).to(dev)
        nq = int(qd.shape[0])
        offs = None
        if req_offsets is not None:
            offs = req_offsets.to(torch.int32).contiguous() if _is_torch_cuda(req_offsets) else \
                torch.from_numpy(np.ascontiguousarray(req_offsets, dtype=np.int32)).to(dev)
        nreq = nq if offs is None else int(offs.shape[0]) - 1
        out = {"idx": torch.empty((n_labels, nq, k), dtype=torch.int64, device=dev),
               "dist": torch.empty((n_labels, nq, k), dtype=torch.float32, device=dev),
               "xy": torch.empty((nreq, 2), dtype=torch.float64, device=dev),
               "tile": torch.empty((nreq, 2), dtype=torch.int32, device=dev),
               "flags": torch.empty(nreq, dtype=torch.int32, device=dev)}
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(load_library().hloc_query_labels_async(
            self._h, _P(qd.data_ptr()), nq, k, n_regions, n_labels,
            None if offs is None else _P(offs.data_ptr()), nreq, PRECISIONS[precision],
            *(_P(out[key].data_ptr()) for key in ("idx", "dist", "xy", "tile", "flags")),
            _P(stream.cuda_stream)))
        return out

    def query_windows(self, q, k: int, n_regions: int, req_offsets, req_frames,
                      precision="fp32", stream=None) -> dict:
        """Sliding-window requests (hloc_query_windows_async): every frame of q
        retrieved once, request i pooling frames req_frames[req_offsets[i] :
        req_offsets[i+1]]. q, req_offsets and req_frames may be CUDA tensors
        or NumPy arrays (copied to the device); returns CUDA tensors."""
        import torch
        dev = q.device if _is_torch_cuda(q) else torch.device("cuda", torch.cuda.current_device())

        def on_dev(a, dtype):
            if _is_torch_cuda(a):
                return a.to(dtype).contiguous()
            return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(dev)

        qd = on_dev(q, torch.float32)
        offs = on_dev(req_offsets, torch.int32)
        frames = on_dev(req_frames, torch.int32)
        nq, nreq = int(qd.shape[0]), int(offs.shape[0]) - 1
        out = {"idx": torch.empty((nq, k), dtype=torch.int64, device=dev),
               "dist": torch.empty((nq, k), dtype=torch.float32, device=dev),
               "xy": torch.empty((nreq, 2), dtype=torch.float64, device=dev),
               "tile": torch.empty((nreq, 2), dtype=torch.int32, device=dev),
               "flags": torch.empty(nreq, dtype=torch.int32, device=dev)}
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(load_library().hloc_query_windows_async(
            self._h, _P(qd.data_ptr()), nq, k, n_regions, _P(offs.data_ptr()),
            _P(frames.data_ptr()), int(frames.shape[0]), nreq, PRECISIONS[precision],
            *(_P(out[key].data_ptr()) for key in ("idx", "dist", "xy", "tile", "flags")),
            _P(stream.cuda_stream)))
        return out

    def info(self) -> dict:
        out = (ctypes.c_int64 * len(_INFO_KEYS))()
        _check(load_library().hloc_query_info(self._h, out, len(_INFO_KEYS)))
        return dict(zip(_INFO_KEYS, list(out)))

    def set_tiles(self, rows_per_item: int, blocks_per_cu: int):
        _check(load_library().hloc_set_tiles(self._h, ctypes.byref(Tiles(rows_per_item,
                                                                          blocks_per_cu))))

    def tiles(self) -> dict:
        t = Tiles()
        _check(load_library().hloc_get_tiles(self._h, ctypes.byref(t)))
        return dict(rows_per_item=t.rows_per_item, blocks_per_cu=t.blocks_per_cu)

    def autotune(self, q, k: int, n_regions: int, precision="fp32", reps: int = 5,
                 cache: str | None = None) -> dict:
        """Choose the fine-screen tiles for batches like q (a CUDA tensor):
        from the JSON cache when it holds this device and shape, else by
        timing every candidate in the library (hloc_autotune), then stored."""
        import json
        import torch
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        key = json.dumps([torch.cuda.get_device_name(q.device), self.n, self.d,
                          self.n_regions_total, int(q.shape[0]), k, n_regions, prec])
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            t = table[key]
            self.set_tiles(t["rows_per_item"], t["blocks_per_cu"])
            return dict(t, source="cache")
        best, ms = Tiles(), ctypes.c_double()
        _check(load_library().hloc_autotune(self._h, ctypes.c_void_p(q.data_ptr()), q.shape[0],
                                            k, n_regions, prec, reps, ctypes.byref(best),
                                            ctypes.byref(ms)))
        t = dict(rows_per_item=best.rows_per_item, blocks_per_cu=best.blocks_per_cu,
                 batch_ms=ms.value)
        if cache:
            table[key] = t
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return dict(t, source="tuned")

    PHASES = ("prep", "coarse", "sched", "screen", "select", "aggregate", "screen_wide",
              "coarse_select", "coarse_defer")

    def profile(self, enable: bool = True):
        """Start (clearing) or stop the per-phase event record."""
        _check(load_library().hloc_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{phase: (milliseconds summed, calls)} since the last read; clears."""
        ms = (ctypes.c_double * len(self.PHASES))()
        calls = (ctypes.c_int64 * len(self.PHASES))()
        _check(load_library().hloc_profile_read(self._h, ms, calls, len(self.PHASES)))
        return {p: (ms[i], calls[i]) for i, p in enumerate(self.PHASES)}

    def last_regions(self) -> np.ndarray:
        """Regions searched by each frame of the last query (nq x n_regions)."""
        lib = load_library()
        nq, nr = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.hloc_last_regions(self._h, None, ctypes.byref(nq), ctypes.byref(nr)))
        out = np.empty((nq.value, nr.value), np.int32)
        if out.size:
            _check(lib.hloc_last_regions(self._h, _np_ptr(out), ctypes.byref(nq), ctypes.byref(nr)))
        return out


_INFO_KEYS = ("items", "coarse_fallbacks", "fine_fallbacks", "max_blocks", "survivors",
              "candidates", "narrow_items", "chunked_bands", "band_rows", "rerank_rows",
              "coarse_deferred")


class Workspace:
    """Scratch memory for one batch in flight on a database (hloc_ws). Several
    workspaces let batches overlap on different streams; a workspace can also
    hold one captured batch (a HIP graph) to replay."""

    def __init__(self, db: HlocDB):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.hloc_ws_create(db._h, ctypes.byref(h)))
        self._h = h
        self.db = db
        self._captured = None

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().hloc_ws_free(self._h)
            self._h = ctypes.c_void_p()
            self._captured = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, nq_max: int, nreq_max: int, k_max: int, n_regions_max: int):
        _check(load_library().hloc_ws_reserve(self._h, nq_max, nreq_max, k_max, n_regions_max))

    @staticmethod
    def outputs(nq: int, nreq: int, k: int, device):
        """Device buffers for one batch's results."""
        import torch
        return dict(idx=torch.empty((nq, k), dtype=torch.int64, device=device),
                    dist=torch.empty((nq, k), dtype=torch.float32, device=device),
                    xy=torch.empty((nreq, 2), dtype=torch.float64, device=device),
                    tile=torch.empty((nreq, 2), dtype=torch.int32, device=device),
                    flags=torch.empty(nreq, dtype=torch.int32, device=device))

    @staticmethod
    def _args(q, k, n_regions, offs, out, precision):
        p = ctypes.c_void_p
        nq = q.shape[0]
        nreq = nq if offs is None else offs.numel() - 1
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        return (p(q.data_ptr()), nq, k, n_regions, None if offs is None else p(offs.data_ptr()),
                nreq, prec, p(out["idx"].data_ptr()), p(out["dist"].data_ptr()),
                p(out["xy"].data_ptr()), p(out["tile"].data_ptr()), p(out["flags"].data_ptr()))

    def query_async(self, q, k: int, n_regions: int, offs, out: dict, stream,
                    precision="fp32"):
        """Enqueue one batch (device tensors) on `stream` into `out`."""
        _check(load_library().hloc_ws_query_async(
            self._h, *self._args(q, k, n_regions, offs, out, precision),
            ctypes.c_void_p(stream.cuda_stream)))

    def capture(self, q, k: int, n_regions: int, offs, out: dict, precision="fp32"):
        """Record one batch on these device buffers for replay()."""
        _check(load_library().hloc_ws_capture(self._h,
                                              *self._args(q, k, n_regions, offs, out, precision)))
        self._captured = (q, offs, out)

    def replay(self, stream):
        _check(load_library().hloc_ws_replay(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def info(self) -> dict:
        out = (ctypes.c_int64 * len(_INFO_KEYS))()
        _check(load_library().hloc_ws_query_info(self._h, out, len(_INFO_KEYS)))
        return dict(zip(_INFO_KEYS, list(out)))


_SERVER_STATS = ("slots", "slot_bytes", "batches", "requests", "frames", "max_batch_frames",
                 "queued_frames", "peak_queued_frames", "max_in_flight", "refused")


class Streams:
    """Sliding windows across calls (hloc_streams): per video stream the
    top-k lists of its last window - 1 frames stay on the device, and each
    new frame's estimate pools its window."""

    def __init__(self, db: HlocDB, n_streams: int, window: int, k: int, max_frames: int):
        self.db, self.k, self.window = db, k, window
        h = _P()
        _check(load_library().hloc_streams_create(db._h, n_streams, window, k, max_frames,
                                                  ctypes.byref(h)))
        self._h = h

    def query(self, q, seg_offsets, seg_stream, n_regions: int, precision="fp32",
              stream=None) -> dict:
        """New frames q in segments (frames seg_offsets[g] : seg_offsets[g+1]
        of stream seg_stream[g], in capture order); CUDA tensors or NumPy
        arrays (copied to the device). Returns CUDA tensors: idx, dist per
        frame and xy, tile, flags of each frame's window."""
        import torch
        dev = q.device if _is_torch_cuda(q) else torch.device("cuda", torch.cuda.current_device())

        def on_dev(a, dtype):
            if _is_torch_cuda(a):
                return a.to(dtype).contiguous()
            return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(dev)

        qd = on_dev(q, torch.float32)
        offs = on_dev(seg_offsets, torch.int32)
        sid = on_dev(seg_stream, torch.int32)
        nq, nseg = int(qd.shape[0]), int(sid.shape[0])
        out = {"idx": torch.empty((nq, self.k), dtype=torch.int64, device=dev),
               "dist": torch.empty((nq, self.k), dtype=torch.float32, device=dev),
               "xy": torch.empty((nq, 2), dtype=torch.float64, device=dev),
               "tile": torch.empty((nq, 2), dtype=torch.int32, device=dev),
               "flags": torch.empty(nq, dtype=torch.int32, device=dev)}
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(load_library().hloc_query_streams_async(
            self._h, _P(qd.data_ptr()), nq, n_regions, PRECISIONS[precision],
            _P(offs.data_ptr()), _P(sid.data_ptr()), nseg,
            *(_P(out[key].data_ptr()) for key in ("idx", "dist", "xy", "tile", "flags")),
            _P(stream.cuda_stream)))
        return out

    def reset(self):
        _check(load_library().hloc_streams_reset(self._h))

    def close(self):
        """Frees the state (before the database is closed)."""
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().hloc_streams_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server over a database (hloc_server): requests of 1 ..
    max_batch_frames frames are batched continuously on up to max_slots
    batches in flight, within an HBM budget (0 = none)."""

    def __init__(self, db: HlocDB, k: int, n_regions: int, precision="fp32",
                 max_batch_frames: int = 256, max_slots: int = 4, max_queue_frames: int = 4096,
                 hbm_budget_bytes: int = 0):
        lib = load_library()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.cfg = ServerConfig(k, n_regions, prec, max_batch_frames, max_slots,
                                max_queue_frames, hbm_budget_bytes)
        h = ctypes.c_void_p()
        _check(lib.hloc_server_create(db._h, ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h
        self.db = db

    def submit(self, frames, k: int | None = None) -> int:
        """Queue one request (frames: F x d); returns its ticket."""
        frames = np.ascontiguousarray(frames, dtype=np.float32)
        t = _U64()
        _check(load_library().hloc_server_submit(self._h, _np_ptr(frames), frames.shape[0],
                                                 self.cfg.k if k is None else k, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, nframes: int, k: int | None = None, timeout_ms: int = -1) -> dict:
        """Results of one request: idx / dist (nframes x k), xy, tile, flags,
        latency_ms (submit to completion)."""
        k = self.cfg.k if k is None else k
        idx = np.empty((nframes, k), np.int64)
        dist = np.empty((nframes, k), np.float32)
        xy = np.empty(2, np.float64)
        tile = np.empty(2, np.int32)
        flags = np.empty(1, np.int32)
        lat = _F64()
        _check(load_library().hloc_server_wait(self._h, ticket, timeout_ms, _np_ptr(idx),
                                               _np_ptr(dist), _np_ptr(xy), _np_ptr(tile),
                                               _np_ptr(flags), ctypes.byref(lat)))
        return dict(idx=idx, dist=dist, xy=xy, tile=tile, flags=int(flags[0]),
                    latency_ms=lat.value)

    def stats(self) -> dict:
        out = (ctypes.c_int64 * len(_SERVER_STATS))()
        _check(load_library().hloc_server_stats(self._h, out, len(_SERVER_STATS)))
        return dict(zip(_SERVER_STATS, list(out)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().hloc_server_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
