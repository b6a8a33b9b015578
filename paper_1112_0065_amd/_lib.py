"""ctypes binding of libdedisp.so: argument marshalling only.

Function names match the C ABI in include/dedisp.h.  Device buffers are
passed as torch tensors on the ROCm device (only their data pointers cross
the boundary) and the stream is torch's current stream unless one is given.
Every computation happens in the library's HIP kernels; there is no Python
or CPU fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdedisp.so")

OK, ERR_INVALID_ARG, ERR_TOO_FEW_SAMPLES, ERR_OUT_OF_MEMORY, ERR_CAPACITY, ERR_HIP, \
    ERR_UNSUPPORTED, ERR_BUSY = range(8)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "TOO_FEW_SAMPLES", 3: "OUT_OF_MEMORY",
                4: "CAPACITY", 5: "HIP", 6: "UNSUPPORTED", 7: "BUSY"}
OUT_I32, OUT_U16 = 0, 1

# dedisp_event, 40 bytes
EVENT_DTYPE = np.dtype([("width_idx", "<i4"), ("dm_idx", "<i4"), ("t_start", "<i8"),
                        ("t_end", "<i8"), ("t_peak", "<i8"), ("b_peak", "<i4"),
                        ("snr", "<f4")])
assert EVENT_DTYPE.itemsize == 40
CLUSTER_DTYPE = np.dtype([("first", "<i8"), ("rep", "<i8"), ("t_lo", "<i8"), ("t_hi", "<i8"),
                          ("t_peak", "<i8"), ("n_members", "<i4"), ("dm_lo", "<i4"),
                          ("dm_hi", "<i4"), ("w_lo", "<i4"), ("w_hi", "<i4"), ("dm_idx", "<i4"),
                          ("width_idx", "<i4"), ("snr", "<f4")])
assert CLUSTER_DTYPE.itemsize == 72
TRIGGER_DTYPE = np.dtype([("start", "<i8"), ("end", "<i8"), ("snr", "<f4"), ("cluster", "<i4"),
                          ("n_clusters", "<i4"), ("reserved", "<i4")])
assert TRIGGER_DTYPE.itemsize == 32


class DedispError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _owned(obj) -> bool:
    """Whether this process created the handle of `obj`.  A process forked
    from one that uses the GPU (a multiprocessing pool) inherits the Python
    objects; their destructors must not call into the library there."""
    return getattr(obj, "_pid", None) == os.getpid()


class _Tile(C.Structure):
    _fields_ = [("dms_per_block", C.c_int32), ("groups", C.c_int32), ("stage_chans", C.c_int32)]


class _ChunkResult(C.Structure):
    _fields_ = [("beam", C.c_int32), ("seq", C.c_int64), ("t_abs0", C.c_int64),
                ("n_bx", C.c_int64), ("n_events", C.c_int64), ("events", C.c_void_p),
                ("scores", C.POINTER(C.c_float)), ("arrival_ns", C.c_int64),
                ("done_ns", C.c_int64), ("flags", C.c_int32), ("n_clusters", C.c_int64),
                ("clusters", C.c_void_p), ("n_candidates", C.c_int64)]


class _ServeStats(C.Structure):
    _fields_ = [("chunks_done", C.c_int64), ("p50_ns", C.c_int64), ("p99_ns", C.c_int64),
                ("max_ns", C.c_int64), ("deadline_ns", C.c_int64),
                ("deadline_misses", C.c_int64), ("batches", C.c_int64),
                ("max_batch", C.c_int64), ("mean_batch", C.c_double), ("slots", C.c_int32)]


class _DeviceProps(C.Structure):
    _fields_ = [("device", C.c_int32), ("compute_units", C.c_int32), ("max_clock_khz", C.c_int32),
                ("memory_clock_khz", C.c_int32), ("memory_bus_bits", C.c_int32),
                ("l2_bytes", C.c_int32), ("wall_clock_khz", C.c_int32), ("reserved", C.c_int32),
                ("lds_bytes_per_cu", C.c_int64), ("total_memory_bytes", C.c_int64),
                ("arch", C.c_char * 64), ("name", C.c_char * 128)]


CHUNK_GAP, CHUNK_LATE, CHUNK_FALLBACK, CHUNK_OVERFLOW, CHUNK_CLUSTERED = 1, 2, 4, 8, 16

_lib = None


def lib() -> C.CDLL:
    """Load libdedisp.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1112_0065_amd.build`")
    # One HIP runtime per process: torch (which supplies device memory and
    # streams) must load its libamdhip64 first, so that the library's
    # dependency on the same soname binds to that copy.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float, C.c_size_t
    P = C.POINTER
    sig = {
        "dedisp_plan_create": (i32, [i32, f64, f64, f64, P(f64), i32, P(vp)]),
        "dedisp_plan_destroy": (i32, [vp]),
        "dedisp_plan_info": (i32, [vp, P(i32), P(i32), P(i64)]),
        "dedisp_plan_copy_delays": (i32, [vp, P(i32)]),
        "dedisp_workspace_bytes": (sz, [vp, i64]),
        "dedisp_execute": (i32, [vp, vp, i64, vp, i32, vp, vp]),
        "dedisp_tile_candidates": (i32, [P(_Tile), i32]),
        "dedisp_default_tile": (i32, [vp, P(_Tile)]),
        "dedisp_execute_tile": (i32, [vp, vp, i64, vp, i32, vp, P(_Tile), vp]),
        "dedisp_repack": (i32, [vp, vp, i64, vp, vp]),
        "dedisp_execute_repacked": (i32, [vp, vp, i64, vp, i32, P(_Tile), vp]),
        "boxcar_filter": (i32, [vp, i32, i32, i64, P(i32), i32, i32, i32, vp, vp]),
        "find_peaks_workspace_bytes": (sz, [i32, i64, P(i32), i32]),
        "find_peaks": (i32, [vp, i32, i32, i64, P(i32), i32, f32, vp, i64, P(i64), vp, vp]),
        "find_peaks_noalloc": (i32, [vp, i32, i32, i64, P(i32), i32, f32, vp, i64, P(i64), vp]),
        "find_peaks_read_stats": (i32, [vp, i32, i64, P(i32), i32, P(i64), P(C.c_uint64),
                                        P(C.c_uint64), P(i64), vp]),
        "dedisp_batch_create": (i32, [P(vp), i32, P(i32), i32, f32, i32, C.c_char_p, P(vp)]),
        "dedisp_batch_execute": (i32, [vp, P(vp), P(i64), P(vp), P(vp), P(i64), P(i64), vp]),
        "dedisp_batch_info": (i32, [vp, P(_Tile), P(i32), P(i32)]),
        "dedisp_batch_set_stages": (i32, [vp, f32, i32, i32]),
        "dedisp_serve_set_stages": (i32, [vp, f32, i32, i32]),
        "dedisp_batch_destroy": (i32, [vp]),
        "dedisp_autotune": (i32, [vp, i64, i32, C.c_char_p, P(_Tile), P(i32)]),
        "dedisp_rfi_mask_workspace_bytes": (sz, [i32, i64]),
        "dedisp_cluster_workspace_bytes": (sz, [i64, i32, i32]),
        "dedisp_subband_create": (i32, [vp, i32, i32, P(vp)]),
        "dedisp_subband_info": (i32, [vp, P(i64), P(i32), P(i32), P(_Tile)]),
        "dedisp_subband_workspace_bytes": (sz, [vp, i64]),
        "dedisp_subband_execute": (i32, [vp, vp, i64, vp, i32, vp, vp]),
        "dedisp_subband_destroy": (i32, [vp]),
        "dedisp_write_candidates": (i32, [C.c_char_p, vp, i64, P(f64), i32, P(i32), i32, f64, i64,
                                          i32]),
        "dedisp_trigger_windows": (i32, [vp, i64, P(i32), i32, i32, f32, i32, i64, i64, vp, i64,
                                         P(i64)]),
        "dedisp_cluster_events": (i32, [vp, i64, i32, P(i32), i32, i32, i32, i64, vp, i64, P(i64),
                                        vp, vp, vp]),
        "baseline_remove": (i32, [vp, i32, i32, i64, i32, i32, vp, i32, vp]),
        "dedisp_rfi_mask": (i32, [P(vp), i32, i32, i64, f32, i32, vp, P(i64), vp, vp]),
        "dedisp_rfi_mask_read_stats": (i32, [vp, i32, i64, P(i32), P(i64), vp]),
        "dedisp_rfi_apply": (i32, [P(vp), i32, i32, i64, vp, vp]),
        "dedisp_serve_slot_bytes": (sz, [P(vp), i32, i64, P(i32), i32]),
        "dedisp_serve_create": (i32, [P(vp), i32, i64, P(i32), i32, f32, sz, vp, P(vp)]),
        "dedisp_serve_submit": (i32, [vp, i32, i64, vp, i64]),
        "dedisp_serve_poll": (i32, [vp, P(_ChunkResult), i32, P(i32), i32]),
        "dedisp_serve_stats": (i32, [vp, P(_ServeStats)]),
        "dedisp_serve_destroy": (i32, [vp]),
        "dedisp_serve_set_clustering": (i32, [vp, i32, i32, i64]),
        "dedisp_now_ns": (i64, []),
        "dedisp_percentile_ns": (i64, [P(i64), i64, f64]),
        "dedisp_serve_admission": (i32, [sz, sz, sz]),
        "triage_create": (i32, [C.c_char_p, C.c_uint64, P(vp)]),
        "triage_destroy": (i32, [vp]),
        "triage_num_params": (i32, []),
        "triage_set_params": (i32, [vp, P(f32), i32]),
        "triage_get_params": (i32, [vp, P(f32), P(f32), i32]),
        "triage_tiles": (i32, [vp, i32, i64, P(i32), i32, vp, vp, i32, vp, vp]),
        "triage_forward": (i32, [vp, vp, i32, vp, vp, vp]),
        "triage_score": (i32, [vp, vp, i32, vp, vp]),
        "triage_forward_backward": (i32, [vp, vp, vp, i32, P(f32), vp]),
        "triage_train_step": (i32, [vp, vp, vp, i32, f32, P(f32), vp]),
        "triage_save": (i32, [vp, C.c_char_p]),
        "dedisp_candidates_nms": (i32, [vp, i64, P(i32), i32, i32, i32, P(i64), P(i64)]),
        "dedisp_device_info": (i32, [P(_DeviceProps)]),
        "dedisp_clock_probe": (i32, [i32, P(f64)]),
        "dedisp_last_error": (C.c_char_p, []),
        "dedisp_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def declared_symbols() -> list:
    """Names of every function include/dedisp.h declares."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "dedisp.h")
    text = open(hdr).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) -
                  {"if", "sizeof", "defined"})


def dedisp_candidates_nms(events: np.ndarray, widths, dm_half: int = 32,
                          t_half_per_width: int = 128) -> np.ndarray:
    """Indices (ascending) of the events kept by per-width non-maximum
    suppression; events: host structured array of EVENT_DTYPE."""
    ev = np.ascontiguousarray(events, dtype=EVENT_DTYPE)
    keep = np.empty(max(len(ev), 1), np.int64)
    nk = C.c_int64()
    _check(lib().dedisp_candidates_nms(ev.ctypes.data if len(ev) else None, len(ev),
                                       _i32arr(widths), len(widths), int(dm_half),
                                       int(t_half_per_width),
                                       keep.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(nk)))
    return keep[:nk.value].copy()


def dedisp_device_info() -> dict:
    p = _DeviceProps()
    _check(lib().dedisp_device_info(C.byref(p)))
    out = {k: getattr(p, k) for k, _ in _DeviceProps._fields_ if k != "reserved"}
    out["arch"] = p.arch.decode()
    out["name"] = p.name.decode()
    return out


def dedisp_clock_probe(wall_us: int = 20000) -> float:
    """Shader clock (GHz) under full vector load, median over waves."""
    g = C.c_double()
    _check(lib().dedisp_clock_probe(int(wall_us), C.byref(g)))
    return float(g.value)


def dedisp_last_error() -> str:
    return lib().dedisp_last_error().decode()


def _check(st: int):
    if st != OK:
        raise DedispError(st, dedisp_last_error())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) or None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


def _i32arr(xs: Sequence[int]):
    a = (C.c_int32 * len(xs))(*[int(x) for x in xs])
    return a


# ---------------------------------------------------------------------------
# Plan
# ---------------------------------------------------------------------------

class Plan:
    """Owns a dedisp_plan handle."""

    def __init__(self, handle: int, nchans: int, ndm: int, max_delay: int):
        self.handle = handle
        self._pid = os.getpid()
        self.nchans = nchans
        self.ndm = ndm
        self.max_delay = max_delay

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None and _owned(self):
            _lib.dedisp_plan_destroy(self.handle)
        self.handle = None

    @property
    def _as_parameter_(self):
        return C.c_void_p(self.handle)


def dedisp_plan_create(nchans: int, f_top: float, df: float, tsamp: float, dm_list) -> Plan:
    dms = np.ascontiguousarray(np.asarray(dm_list, dtype=np.float64))
    h = C.c_void_p()
    _check(lib().dedisp_plan_create(int(nchans), float(f_top), float(df), float(tsamp),
                                    dms.ctypes.data_as(C.POINTER(C.c_double)), len(dms),
                                    C.byref(h)))
    nc, nd, md = dedisp_plan_info_raw(h.value)
    return Plan(h.value, nc, nd, md)


def dedisp_plan_info_raw(handle: int):
    nc, nd, md = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().dedisp_plan_info(handle, C.byref(nc), C.byref(nd), C.byref(md)))
    return nc.value, nd.value, md.value


def dedisp_plan_info(plan: Plan):
    return dedisp_plan_info_raw(plan.handle)


def dedisp_plan_copy_delays(plan: Plan) -> np.ndarray:
    out = np.empty((plan.ndm, plan.nchans), dtype=np.int32)
    _check(lib().dedisp_plan_copy_delays(plan.handle, out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def dedisp_workspace_bytes(plan: Plan, nsamps: int) -> int:
    return int(lib().dedisp_workspace_bytes(plan.handle, int(nsamps)))


# ---------------------------------------------------------------------------
# Dedispersion
# ---------------------------------------------------------------------------

def dedisp_execute(plan: Plan, in_2bit, nsamps: int, out, workspace, stream=None):
    """in_2bit: uint8 device tensor; out: int32 or uint16 device tensor
    [ndm][nsamps - max_delay]; workspace: device tensor of
    dedisp_workspace_bytes(plan, nsamps) bytes."""
    _check(lib().dedisp_execute(plan.handle, _ptr(in_2bit), int(nsamps), _ptr(out),
                                _out_type(out), _ptr(workspace), _stream(stream)))


def dedisp_tile_candidates():
    n = lib().dedisp_tile_candidates(None, 0)
    arr = (_Tile * n)()
    lib().dedisp_tile_candidates(arr, n)
    return [(t.dms_per_block, t.groups, t.stage_chans) for t in arr]


def dedisp_default_tile(plan: Plan):
    t = _Tile()
    _check(lib().dedisp_default_tile(plan.handle, C.byref(t)))
    return (t.dms_per_block, t.groups, t.stage_chans)


def dedisp_execute_tile(plan: Plan, in_2bit, nsamps: int, out, workspace, tile, stream=None):
    t = _Tile(*[int(v) for v in tile])
    _check(lib().dedisp_execute_tile(plan.handle, _ptr(in_2bit), int(nsamps), _ptr(out),
                                     _out_type(out), _ptr(workspace), C.byref(t),
                                     _stream(stream)))


def dedisp_repack(plan: Plan, in_2bit, nsamps: int, workspace, stream=None):
    _check(lib().dedisp_repack(plan.handle, _ptr(in_2bit), int(nsamps), _ptr(workspace),
                               _stream(stream)))


def dedisp_execute_repacked(plan: Plan, workspace, nsamps: int, out, tile=None, stream=None):
    t = None if tile is None else C.byref(_Tile(*[int(v) for v in tile]))
    _check(lib().dedisp_execute_repacked(plan.handle, _ptr(workspace), int(nsamps), _ptr(out),
                                         _out_type(out), t, _stream(stream)))


def _out_type(t) -> int:
    import torch
    if t.dtype == torch.int32:
        return OUT_I32
    if t.dtype in (torch.uint16, torch.int16):
        return OUT_U16
    raise TypeError(f"dedispersed series must be int32 or uint16, got {t.dtype}")


# ---------------------------------------------------------------------------
# Boxcar / peaks
# ---------------------------------------------------------------------------

def boxcar_filter(series, ndm: int, nout: int, widths, dm_first: int, dm_count: int, out,
                  stream=None):
    w = _i32arr(widths)
    _check(lib().boxcar_filter(_ptr(series), _out_type(series), int(ndm), int(nout), w,
                               len(widths), int(dm_first), int(dm_count), _ptr(out),
                               _stream(stream)))


def baseline_remove(series, ndm: int, nout: int, radius: int, offset: int, out, stream=None):
    """out[d][t] = series[d][t+R] - floor(window sum / (2R+1)) + offset over
    nout - 2R positions; series and out are device tensors (int16 = uint16
    bits, or int32)."""
    _check(lib().baseline_remove(_ptr(series), _out_type(series), int(ndm), int(nout), int(radius),
                                 int(offset), _ptr(out), _out_type(out), _stream(stream)))


def find_peaks_workspace_bytes(ndm: int, nout: int, widths) -> int:
    return int(lib().find_peaks_workspace_bytes(int(ndm), int(nout), _i32arr(widths),
                                                len(widths)))


def find_peaks(series, ndm: int, nout: int, widths, snr_thresh: float, events, capacity: int,
               workspace, stream=None) -> int:
    """events: device buffer of capacity*40 bytes.  Returns the number of
    events found (raises DedispError(CAPACITY) when it exceeds capacity,
    after writing the first `capacity`)."""
    n = C.c_int64()
    st = lib().find_peaks(_ptr(series), _out_type(series), int(ndm), int(nout),
                          _i32arr(widths), len(widths), float(snr_thresh), _ptr(events),
                          int(capacity), C.byref(n), _ptr(workspace), _stream(stream))
    if st == ERR_CAPACITY:
        raise DedispError(st, dedisp_last_error() + f" (n_events={n.value})")
    _check(st)
    return int(n.value)


def find_peaks_noalloc(series, ndm: int, nout: int, widths, snr_thresh: float, events,
                       capacity: int, stream=None) -> int:
    """find_peaks with the library's static per-GPU scratch as workspace (no
    allocation; at most 32 MiB of workspace)."""
    n = C.c_int64()
    st = lib().find_peaks_noalloc(_ptr(series), _out_type(series), int(ndm), int(nout),
                                  _i32arr(widths), len(widths), float(snr_thresh), _ptr(events),
                                  int(capacity), C.byref(n), _stream(stream))
    if st == ERR_CAPACITY:
        raise DedispError(st, dedisp_last_error() + f" (n_events={n.value})")
    _check(st)
    return int(n.value)


def find_peaks_read_stats(workspace, ndm: int, nout: int, widths, stream=None):
    """(s1, s2, thr) as [nwidths][ndm] arrays (s2 as Python ints, exact)."""
    nw = len(widths)
    s1 = np.empty(nw * ndm, np.int64)
    lo = np.empty(nw * ndm, np.uint64)
    hi = np.empty(nw * ndm, np.uint64)
    thr = np.empty(nw * ndm, np.int64)
    _check(lib().find_peaks_read_stats(
        _ptr(workspace), int(ndm), int(nout), _i32arr(widths), nw,
        s1.ctypes.data_as(C.POINTER(C.c_int64)), lo.ctypes.data_as(C.POINTER(C.c_uint64)),
        hi.ctypes.data_as(C.POINTER(C.c_uint64)), thr.ctypes.data_as(C.POINTER(C.c_int64)),
        _stream(stream)))
    s2 = np.array([int(h) << 64 | int(l) for h, l in zip(hi.tolist(), lo.tolist())],
                  dtype=object)
    return s1.reshape(nw, ndm), s2.reshape(nw, ndm), thr.reshape(nw, ndm)


def events_from_buffer(buf, n: int) -> np.ndarray:
    """Copy n event records from a device/host byte buffer to a structured array."""
    raw = buf[: n * EVENT_DTYPE.itemsize]
    if hasattr(raw, "cpu"):
        raw = raw.cpu().numpy()
    return np.frombuffer(np.asarray(raw, dtype=np.uint8).tobytes(), dtype=EVENT_DTYPE, count=n)


# ---------------------------------------------------------------------------
# Subband (two-stage) dedispersion
# ---------------------------------------------------------------------------

class Subband:
    def __init__(self, handle: int, plan, nsub: int, group: int):
        self.handle = handle
        self._pid = os.getpid()
        self.plan = plan            # keeps the fine-trial plan alive
        self.nsub = nsub
        self.group = group
        md, nc, sp, t = C.c_int64(), C.c_int32(), C.c_int32(), _Tile()
        _check(lib().dedisp_subband_info(handle, C.byref(md), C.byref(nc), C.byref(sp), C.byref(t)))
        self.max_delay, self.ncoarse, self.span = int(md.value), int(nc.value), int(sp.value)
        self.tile = (t.dms_per_block, t.groups, t.stage_chans)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None and _owned(self):
            _lib.dedisp_subband_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dedisp_subband_create(plan, nsub: int, group: int) -> Subband:
    h = C.c_void_p()
    _check(lib().dedisp_subband_create(plan.handle, int(nsub), int(group), C.byref(h)))
    return Subband(h.value, plan, nsub, group)


def dedisp_subband_workspace_bytes(sb: Subband, nsamps: int) -> int:
    return int(lib().dedisp_subband_workspace_bytes(sb.handle, int(nsamps)))


def dedisp_subband_execute(sb: Subband, packed, nsamps: int, out, workspace, stream=None):
    """packed: device uint8; out: device [ndm][nsamps - sb.max_delay] int16 (uint16 bits) or
    int32."""
    _check(lib().dedisp_subband_execute(sb.handle, _ptr(packed), int(nsamps), _ptr(out),
                                        _out_type(out), _ptr(workspace), _stream(stream)))


# ---------------------------------------------------------------------------
# Event clustering across DM and width
# ---------------------------------------------------------------------------

def dedisp_cluster_workspace_bytes(n_events: int, ndm: int, nwidths: int) -> int:
    return int(lib().dedisp_cluster_workspace_bytes(int(n_events), int(ndm), int(nwidths)))


def dedisp_cluster_events(events, n_events: int, ndm: int, widths, dm_radius: int,
                          width_radius: int, time_tol: int, clusters, capacity: int, workspace,
                          labels=None, stream=None) -> int:
    """events: device buffer of n_events find_peaks records; clusters: device
    buffer of capacity*72 bytes; labels: optional device int32 [n_events].
    Returns the number of clusters (raises DedispError(CAPACITY) when it
    exceeds capacity, after writing the first `capacity`)."""
    n = C.c_int64()
    st = lib().dedisp_cluster_events(_ptr(events), int(n_events), int(ndm), _i32arr(widths),
                                     len(widths), int(dm_radius), int(width_radius),
                                     int(time_tol), _ptr(clusters), int(capacity), C.byref(n),
                                     _ptr(labels), _ptr(workspace), _stream(stream))
    if st == ERR_CAPACITY:
        raise DedispError(st, dedisp_last_error() + f" (n_clusters={n.value})")
    _check(st)
    return int(n.value)


def dedisp_write_candidates(path: str, clusters: np.ndarray, dm_list, widths, tsamp: float,
                            t_offset: int = 0, beam: int = 0):
    """Write the cluster records (host structured array, CLUSTER_DTYPE) as a
    text candidate list."""
    c = np.ascontiguousarray(clusters, dtype=CLUSTER_DTYPE)
    dm = np.ascontiguousarray(dm_list, dtype=np.float64)
    _check(lib().dedisp_write_candidates(str(path).encode(), c.ctypes.data if len(c) else None,
                                         len(c), dm.ctypes.data_as(C.POINTER(C.c_double)), len(dm),
                                         _i32arr(widths), len(widths), float(tsamp), int(t_offset),
                                         int(beam)))


def dedisp_trigger_windows(clusters: np.ndarray, delays: np.ndarray, snr_min: float,
                           min_members: int, pad: int, nsamps: int,
                           capacity: Optional[int] = None) -> np.ndarray:
    """Baseband-dump windows of the clusters (host arrays; delays [ndm][nchans])."""
    c = np.ascontiguousarray(clusters, dtype=CLUSTER_DTYPE)
    d = np.ascontiguousarray(delays, dtype=np.int32)
    cap = len(c) if capacity is None else int(capacity)
    out = np.zeros(max(cap, 1), dtype=TRIGGER_DTYPE)
    n = C.c_int64()
    st = lib().dedisp_trigger_windows(c.ctypes.data if len(c) else None, len(c),
                                      d.ctypes.data_as(C.POINTER(C.c_int32)), d.shape[0],
                                      d.shape[1], float(snr_min), int(min_members), int(pad),
                                      int(nsamps), out.ctypes.data, cap, C.byref(n))
    if st == ERR_CAPACITY:
        raise DedispError(st, dedisp_last_error() + f" (n_windows={n.value})")
    _check(st)
    return out[: n.value].copy()


def clusters_from_buffer(buf, n: int) -> np.ndarray:
    """Copy n cluster records from a device/host byte buffer to a structured array."""
    raw = buf[: n * CLUSTER_DTYPE.itemsize]
    if hasattr(raw, "cpu"):
        raw = raw.cpu().numpy()
    return np.frombuffer(np.asarray(raw, dtype=np.uint8).tobytes(), dtype=CLUSTER_DTYPE, count=n)


# ---------------------------------------------------------------------------
# Multibeam coincidence RFI mask
# ---------------------------------------------------------------------------

def dedisp_rfi_mask_workspace_bytes(nbeams: int, nsamps: int) -> int:
    return int(lib().dedisp_rfi_mask_workspace_bytes(int(nbeams), int(nsamps)))


def dedisp_rfi_mask(inputs, nchans: int, nsamps: int, k_sigma: float, min_beams: int, mask,
                    workspace, stream=None) -> int:
    """inputs: device tensors (one per beam); mask: device uint8 [nsamps].
    Returns the number of masked samples (synchronises)."""
    arr = (C.c_void_p * len(inputs))(*[_ptr(t) for t in inputs])
    n = C.c_int64()
    _check(lib().dedisp_rfi_mask(arr, len(inputs), int(nchans), int(nsamps), float(k_sigma),
                                 int(min_beams), _ptr(mask), C.byref(n), _ptr(workspace),
                                 _stream(stream)))
    return int(n.value)


def dedisp_rfi_apply(beams, nchans: int, nsamps: int, mask, stream=None):
    """Replace the flagged samples of every beam (device uint8 tensors, in
    place) by the mean level in every channel."""
    arr = (C.c_void_p * len(beams))(*[_ptr(t) for t in beams])
    _check(lib().dedisp_rfi_apply(arr, len(beams), int(nchans), int(nsamps), _ptr(mask),
                                  _stream(stream)))


def dedisp_rfi_mask_read_stats(workspace, nbeams: int, nsamps: int, stream=None):
    """(zero-DM series int32 [nbeams][nsamps], cut levels int64 [nbeams])."""
    z = np.empty((nbeams, nsamps), np.int32)
    thr = np.empty(nbeams, np.int64)
    _check(lib().dedisp_rfi_mask_read_stats(_ptr(workspace), int(nbeams), int(nsamps),
                                            z.ctypes.data_as(C.POINTER(C.c_int32)),
                                            thr.ctypes.data_as(C.POINTER(C.c_int64)),
                                            _stream(stream)))
    return z, thr


# ---------------------------------------------------------------------------
# Multibeam batch and autotuner
# ---------------------------------------------------------------------------

class Batch:
    """Owns a dedisp_batch handle (and keeps its plans alive)."""

    def __init__(self, handle: int, plans):
        self.handle = handle
        self._pid = os.getpid()
        self.plans = list(plans)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None and _owned(self):
            _lib.dedisp_batch_destroy(self.handle)
        self.handle = None


def dedisp_batch_create(plans, widths, snr_thresh: float, out_u16: bool = True,
                        tune_cache_path: Optional[str] = None) -> Batch:
    arr = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    h = C.c_void_p()
    path = tune_cache_path.encode() if tune_cache_path else None
    _check(lib().dedisp_batch_create(arr, len(plans), _i32arr(widths), len(widths),
                                     float(snr_thresh), OUT_U16 if out_u16 else OUT_I32, path,
                                     C.byref(h)))
    return Batch(h.value, plans)


def dedisp_batch_execute(batch: Batch, inputs, nsamps, outs, events, capacity, stream=None):
    """inputs/outs/events: lists of device tensors (one per beam); returns the
    list of event counts (raises DedispError(CAPACITY) on overflow)."""
    n = len(batch.plans)
    ins = (C.c_void_p * n)(*[_ptr(t) for t in inputs])
    ns = (C.c_int64 * n)(*[int(v) for v in nsamps])
    os_ = (C.c_void_p * n)(*[_ptr(t) for t in outs])
    evs = (C.c_void_p * n)(*[_ptr(t) for t in events])
    caps = (C.c_int64 * n)(*[int(v) for v in capacity])
    cnt = (C.c_int64 * n)()
    st = lib().dedisp_batch_execute(batch.handle, ins, ns, os_, evs, caps, cnt, _stream(stream))
    if st == ERR_CAPACITY:
        raise DedispError(st, dedisp_last_error() + f" (n_events={list(cnt)})")
    _check(st)
    return list(cnt)


def dedisp_batch_set_stages(batch: Batch, rfi_k_sigma: float = 0.0, rfi_min_beams: int = 0,
                            baseline_radius: int = 0):
    """Coincidence mask before and baseline removal after dedispersion
    (rfi_k_sigma 0 / radius 0 switch a stage off)."""
    _check(lib().dedisp_batch_set_stages(batch.handle, float(rfi_k_sigma), int(rfi_min_beams),
                                         int(baseline_radius)))


def dedisp_batch_info(batch: Batch):
    t, g, c = _Tile(), C.c_int32(), C.c_int32()
    _check(lib().dedisp_batch_info(batch.handle, C.byref(t), C.byref(g), C.byref(c)))
    return (t.dms_per_block, t.groups, t.stage_chans), g.value, c.value


def dedisp_autotune(plan: Plan, nsamps: int, out_u16: bool = True,
                    cache_path: Optional[str] = None):
    """Returns (best_tile, n_rejected)."""
    t, rej = _Tile(), C.c_int32()
    path = cache_path.encode() if cache_path else None
    _check(lib().dedisp_autotune(plan.handle, int(nsamps), OUT_U16 if out_u16 else OUT_I32, path,
                                 C.byref(t), C.byref(rej)))
    return (t.dms_per_block, t.groups, t.stage_chans), rej.value


# ---------------------------------------------------------------------------
# Streaming server
# ---------------------------------------------------------------------------

class Server:
    def __init__(self, handle: int, plans, model=None):
        self.handle = handle
        self._pid = os.getpid()
        self.plans = list(plans)
        self.model = model

    def close(self):
        if getattr(self, "handle", None) and _lib is not None and _owned(self):
            st = _lib.dedisp_serve_destroy(self.handle)
            self.handle = None
            _check(st)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dedisp_serve_slot_bytes(plans, chunk_nsamps: int, widths) -> int:
    arr = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    return int(lib().dedisp_serve_slot_bytes(arr, len(plans), int(chunk_nsamps), _i32arr(widths),
                                             len(widths)))


def dedisp_serve_create(plans, chunk_nsamps: int, widths, snr_thresh: float, hbm_budget: int,
                        model=None) -> Server:
    arr = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    h = C.c_void_p()
    mh = None if model is None else model.handle
    _check(lib().dedisp_serve_create(arr, len(plans), int(chunk_nsamps), _i32arr(widths),
                                     len(widths), float(snr_thresh), int(hbm_budget), mh,
                                     C.byref(h)))
    return Server(h.value, plans, model)


def dedisp_serve_submit(server: Server, beam: int, seq: int, chunk: np.ndarray,
                        arrival_ns: int) -> bool:
    """True when admitted, False on BUSY (retry later)."""
    buf = np.ascontiguousarray(chunk, dtype=np.uint8)
    st = lib().dedisp_serve_submit(server.handle, int(beam), int(seq),
                                   buf.ctypes.data_as(C.c_void_p), int(arrival_ns))
    if st == ERR_BUSY:
        return False
    _check(st)
    return True


def dedisp_serve_poll(server: Server, cap: int = 64, timeout_ms: int = 0):
    arr = (_ChunkResult * cap)()
    n = C.c_int32()
    _check(lib().dedisp_serve_poll(server.handle, arr, cap, C.byref(n), int(timeout_ms)))
    out = []
    for r in arr[: n.value]:
        m = min(r.n_events, 1 << 16)
        ev = np.empty(0, dtype=EVENT_DTYPE)
        if m and r.events:
            raw = C.string_at(r.events, m * EVENT_DTYPE.itemsize)
            ev = np.frombuffer(raw, dtype=EVENT_DTYPE).copy()
        scores = None
        if m and r.scores:
            scores = np.ctypeslib.as_array(r.scores, shape=(m,)).copy()
        clusters = None
        if r.flags & CHUNK_CLUSTERED:
            clusters = np.empty(0, dtype=CLUSTER_DTYPE)
            if r.n_clusters and r.clusters:
                raw = C.string_at(r.clusters, r.n_clusters * CLUSTER_DTYPE.itemsize)
                clusters = np.frombuffer(raw, dtype=CLUSTER_DTYPE).copy()
        out.append(dict(beam=r.beam, seq=r.seq, t_abs0=r.t_abs0, n_bx=r.n_bx,
                        n_events=r.n_events, events=ev, scores=scores,
                        arrival_ns=r.arrival_ns, done_ns=r.done_ns, flags=r.flags,
                        clusters=clusters, n_candidates=r.n_candidates))
    return out


def dedisp_serve_set_stages(server, rfi_k_sigma: float = 0.0, rfi_min_beams: int = 0,
                            baseline_radius: int = 0):
    """Coincidence mask per round of chunks before, baseline removal after
    dedispersion (0 switches a stage off).  Before the first submit."""
    _check(lib().dedisp_serve_set_stages(server.handle, float(rfi_k_sigma), int(rfi_min_beams),
                                         int(baseline_radius)))


def dedisp_serve_set_clustering(server: Server, dm_radius: int, width_radius: int, time_tol: int):
    """Cluster every chunk's events before its result is returned."""
    _check(lib().dedisp_serve_set_clustering(server.handle, int(dm_radius), int(width_radius),
                                             int(time_tol)))


def dedisp_serve_stats(server: Server) -> dict:
    st = _ServeStats()
    _check(lib().dedisp_serve_stats(server.handle, C.byref(st)))
    return {k: getattr(st, k) for k, _ in _ServeStats._fields_}


def dedisp_now_ns() -> int:
    return int(lib().dedisp_now_ns())


def dedisp_percentile_ns(values, q: float) -> int:
    a = np.ascontiguousarray(np.sort(np.asarray(values, dtype=np.int64)))
    return int(lib().dedisp_percentile_ns(a.ctypes.data_as(C.POINTER(C.c_int64)), len(a),
                                          float(q)))


def dedisp_serve_admission(budget: int, resident: int, slot_bytes: int) -> int:
    return int(lib().dedisp_serve_admission(int(budget), int(resident), int(slot_bytes)))


# ---------------------------------------------------------------------------
# Triage network
# ---------------------------------------------------------------------------

class Model:
    def __init__(self, handle: int):
        self.handle = handle
        self._pid = os.getpid()

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None and _owned(self):
            _lib.triage_destroy(self.handle)
        self.handle = None


def triage_create(weights_path: Optional[str] = None, seed: int = 0) -> Model:
    h = C.c_void_p()
    _check(lib().triage_create(weights_path.encode() if weights_path else None, int(seed),
                               C.byref(h)))
    return Model(h.value)


def triage_num_params() -> int:
    return int(lib().triage_num_params())


def triage_set_params(m: Model, params: np.ndarray):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().triage_set_params(m.handle, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))


def triage_get_params(m: Model):
    n = triage_num_params()
    p = np.empty(n, np.float32)
    g = np.empty(n, np.float32)
    _check(lib().triage_get_params(m.handle, p.ctypes.data_as(C.POINTER(C.c_float)),
                                   g.ctypes.data_as(C.POINTER(C.c_float)), n))
    return p, g


def triage_tiles(series, ndm: int, nout: int, widths, peaks_ws, events_dev, n_events: int,
                 tiles_out, stream=None):
    _check(lib().triage_tiles(_ptr(series), int(ndm), int(nout), _i32arr(widths), len(widths),
                              _ptr(peaks_ws), _ptr(events_dev), int(n_events), _ptr(tiles_out),
                              _stream(stream)))


def triage_forward(m: Model, tiles, n: int, logits=None, scores=None, stream=None):
    _check(lib().triage_forward(m.handle, _ptr(tiles), int(n), _ptr(logits), _ptr(scores),
                                _stream(stream)))


def triage_score(m: Model, tiles, n: int, scores, stream=None):
    _check(lib().triage_score(m.handle, _ptr(tiles), int(n), _ptr(scores), _stream(stream)))


def triage_forward_backward(m: Model, tiles, labels, n: int, stream=None) -> float:
    loss = C.c_float()
    _check(lib().triage_forward_backward(m.handle, _ptr(tiles), _ptr(labels), int(n),
                                         C.byref(loss), _stream(stream)))
    return float(loss.value)


def triage_train_step(m: Model, tiles, labels, n: int, lr: float = 1e-3, stream=None) -> float:
    loss = C.c_float()
    _check(lib().triage_train_step(m.handle, _ptr(tiles), _ptr(labels), int(n), float(lr),
                                   C.byref(loss), _stream(stream)))
    return float(loss.value)


def triage_save(m: Model, path: str):
    _check(lib().triage_save(m.handle, path.encode()))
