"""MI355X SneakySnake pre-alignment filter: Python binding of libss.so.

Argument marshalling only: every step of the filter runs in the HIP kernels of
``libss.so`` (see ``include/ss.h`` for the C ABI).  The functions below carry
the C names and forward to them through ctypes; device buffers are passed as
raw pointers or as torch tensors (their ``data_ptr()``), streams as raw HIP
stream handles or ``torch.cuda.Stream`` objects.

There is no CPU fallback: if ``libss.so`` has not been built this module raises
on first use.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libss.so")

SS_OK, SS_EINVAL, SS_EBASE, SS_ELEN, SS_ENOMEM, SS_EBUDGET, SS_EDEVICE, SS_EAGAIN, SS_ETIMEOUT = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
SS_MAX_E_SLICED = 32
SS_MAX_E_PLAIN = 31
SS_MAX_E = 16383
SS_MAX_E_PLANNED = 8191
SS_MAX_LEN = 1 << 24
SS_MAX_LEN_FUSED = 2048
SS_MAX_LEN_VERIFY = 65536
SS_MAX_E_VERIFY_BANDED = 16351
SS_MAX_STREAM_BASES = 32 * ((1 << 30) - 64)
SS_NOALLOC_SCRATCH_BYTES = 32 << 20
SS_RESULT_ACCEPT = 0x8000
SS_RESULT_COUNT = 0x7FFF
SS_INPUT_ASCII, SS_INPUT_PACKED, SS_INPUT_PACKED_SLICED = 0x0, 0x1, 0x2
SS_KERNEL_AUTO, SS_KERNEL_FUSED, SS_KERNEL_SLICED, SS_KERNEL_PLAIN, SS_KERNEL_WAVE, SS_KERNEL_PERSISTENT = (
    0x00, 0x10, 0x20, 0x30, 0x40, 0x50)


class BatchDesc(ctypes.Structure):
    """ss_batch_desc of include/ss.h (field for field)."""
    _fields_ = [("reads", ctypes.c_void_p), ("refs", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("lengths", ctypes.c_void_p), ("ref_offsets", ctypes.c_void_p), ("ref_lengths", ctypes.c_void_p),
                ("E_per_pair", ctypes.c_void_p), ("plan", ctypes.c_void_p), ("n_pairs", ctypes.c_int64),
                ("read_bases", ctypes.c_int64), ("ref_bases", ctypes.c_int64), ("length", ctypes.c_int32),
                ("E", ctypes.c_int32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("out", ctypes.c_void_p), ("err", ctypes.c_void_p)]

_lib = None


class SSError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)}")


def lib():
    """The loaded libss.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1910_09020_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "ss_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "ss_filter_batch": ([vp, vp, vp, i64, i32, vp, vp], ctypes.c_int),
        "ss_filter_batch_var": ([vp, vp, vp, vp, i64, vp, vp], ctypes.c_int),
        "ss_create": ([ctypes.POINTER(vp), ctypes.c_int], ctypes.c_int),
        "ss_destroy": ([vp], ctypes.c_int),
        "ss_sliced_bytes": ([i64, i32], i64),
        "ss_stream_words": ([i64], i64),
        "ss_pack_sliced_async": ([vp, vp, vp, vp, vp, i64, i32, vp, vp, vp], ctypes.c_int),
        "ss_filter_sliced_async": ([vp, vp, i64, i32, i32, vp, vp], ctypes.c_int),
        "ss_filter_sliced_range_async": ([vp, vp, i64, i32, i32, i32, vp, i64, vp], ctypes.c_int),
        "ss_filter_ascii_async": ([vp, vp, vp, i64, i32, i32, i32, vp, vp, vp], ctypes.c_int),
        "ss_verify_async": ([vp, vp, i64, vp, vp, vp, i64, i32, vp, vp], ctypes.c_int),
        "ss_verify_banded_async": ([vp, vp, i64, vp, vp, vp, i32, vp, i64, vp, vp], ctypes.c_int),
        "ss_filter_submaze_async": ([vp, vp, i64, i32, i32, i32, vp, vp], ctypes.c_int),
        "ss_select_accepted_async": ([vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "ss_pack_stream_async": ([vp, vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "ss_filter_plain_async": ([vp, vp, i64, vp, vp, vp, i64, i32, vp, vp], ctypes.c_int),
        "ss_filter_wave_async": ([vp, vp, i64, vp, vp, vp, i64, i32, vp, vp], ctypes.c_int),
        "ss_unpack_results_async": ([vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "ss_plan_create": ([vp, vp, vp, i64, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "ss_plan_destroy": ([vp], ctypes.c_int),
        "ss_plan_items_host": ([vp, vp, i64, i32, vp, vp, i64, vp], ctypes.c_int),
        "ss_plan_info": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "ss_filter_planned_async": ([vp, vp, vp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "ss_plan_capture": ([vp, vp, vp, i64, vp, vp, vp, vp], ctypes.c_int),
        "ss_plan_launch": ([vp, vp], ctypes.c_int),
        "ss_plan_create_tuned": ([vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, ctypes.c_char_p, ctypes.POINTER(vp),
                                  vp], ctypes.c_int),
        "ss_server_create": ([vp, ctypes.c_size_t, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "ss_server_create_loop": ([vp, ctypes.c_size_t, i32, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "ss_server_set_loop_idle": ([vp, i64], ctypes.c_int),
        "ss_server_submit": ([vp, vp, vp, vp, vp, i64, vp, vp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "ss_server_stage_alloc": ([vp, ctypes.c_size_t], vp),
        "ss_server_stage_free": ([vp, vp], ctypes.c_int),
        "ss_server_submit_staged": ([vp, vp, ctypes.c_size_t, vp, vp, i64, vp, vp, ctypes.POINTER(ctypes.c_uint64)],
                                    ctypes.c_int),
        "ss_server_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "ss_server_wait": ([vp, ctypes.c_uint64, i64], ctypes.c_int),
        "ss_server_times": ([vp, ctypes.c_uint64, vp, vp, vp], ctypes.c_int),
        "ss_server_cancel": ([vp, ctypes.c_uint64], ctypes.c_int),
        "ss_server_release": ([vp, ctypes.c_uint64], ctypes.c_int),
        "ss_server_set_hold": ([vp, ctypes.c_int], ctypes.c_int),
        "ss_server_stats": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "ss_server_destroy": ([vp], ctypes.c_int),
        "ss_server_footprint": ([i64, i64], i64),
        "ss_server_set_slices": ([vp, i32], ctypes.c_int),
        "ss_pack_words": ([i64], i64),
        "ss_pack": ([vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "ss_filter_batch_ex": ([vp, ctypes.POINTER(BatchDesc), vp], ctypes.c_int),
        "ss_filter_batch_pairs": ([vp, vp, vp, vp, i64, vp, i32, vp, vp], ctypes.c_int),
        "ss_filter_ascii_noalloc": ([vp, vp, vp, i64, i32, i32, vp, vp, vp], ctypes.c_int),
        "ss_server_stages": ([vp, ctypes.c_uint64, vp, vp, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def exported_symbols():
    """Names of the C entry points this binding declares."""
    return ["ss_status_str", "ss_filter_batch", "ss_filter_batch_var", "ss_create", "ss_destroy",
            "ss_sliced_bytes", "ss_stream_words", "ss_pack_sliced_async", "ss_filter_sliced_async",
            "ss_filter_ascii_async", "ss_pack_stream_async", "ss_filter_plain_async", "ss_filter_wave_async",
            "ss_unpack_results_async", "ss_verify_async", "ss_select_accepted_async", "ss_filter_submaze_async",
            "ss_plan_create", "ss_plan_items_host", "ss_plan_destroy", "ss_plan_info", "ss_filter_planned_async",
            "ss_plan_capture",
            "ss_plan_launch", "ss_plan_create_tuned", "ss_server_create", "ss_server_submit", "ss_server_poll",
            "ss_server_wait", "ss_server_times", "ss_server_cancel", "ss_server_release", "ss_server_set_hold",
            "ss_server_stats", "ss_server_destroy", "ss_server_footprint", "ss_server_set_slices", "ss_pack_words",
            "ss_pack", "ss_filter_batch_ex", "ss_filter_batch_pairs", "ss_filter_ascii_noalloc",
            "ss_server_stages", "ss_server_create_loop", "ss_verify_banded_async", "ss_server_set_loop_idle",
            "ss_server_stage_alloc", "ss_server_stage_free", "ss_server_submit_staged",
            "ss_filter_sliced_range_async"]


def status_str(status: int) -> str:
    try:
        return lib().ss_status_str(status).decode()
    except Exception:
        return f"status {status}"


def _ptr(x):
    """Raw address of a device/host buffer: int, None, torch tensor or numpy array."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)!r}")


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    raise TypeError(f"not a stream: {type(s)!r}")


def _check(rc: int, where: str):
    if rc != SS_OK:
        raise SSError(rc, where)


# ---------------------------------------------------------------- one-call host API
def ss_filter_batch(reads, refs, lengths, E: int):
    """Filter host pairs (numpy uint8 reads/refs, int32 lengths); returns (accept uint8[n], edits int32[n])."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    refs = np.ascontiguousarray(refs, dtype=np.uint8)
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    n = len(lengths)
    acc = np.zeros(n, dtype=np.uint8)
    ed = np.zeros(n, dtype=np.int32)
    rc = lib().ss_filter_batch(_ptr(reads), _ptr(refs), _ptr(lengths), n, int(E), _ptr(acc), _ptr(ed))
    _check(rc, "ss_filter_batch")
    return acc, ed


def ss_filter_batch_var(reads, refs, lengths, E_per_pair):
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    refs = np.ascontiguousarray(refs, dtype=np.uint8)
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    Epp = np.ascontiguousarray(E_per_pair, dtype=np.int32)
    n = len(lengths)
    acc = np.zeros(n, dtype=np.uint8)
    ed = np.zeros(n, dtype=np.int32)
    rc = lib().ss_filter_batch_var(_ptr(reads), _ptr(refs), _ptr(lengths), _ptr(Epp), n, _ptr(acc), _ptr(ed))
    _check(rc, "ss_filter_batch_var")
    return acc, ed


def ss_filter_batch_pairs(reads, read_lengths, refs, ref_lengths, E: int = 0, E_per_pair=None):
    """Pairs of unequal length from host numpy arrays; returns (accept uint8[n], edits int32[n])."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    refs = np.ascontiguousarray(refs, dtype=np.uint8)
    rl = np.ascontiguousarray(read_lengths, dtype=np.int32)
    fl = np.ascontiguousarray(ref_lengths, dtype=np.int32)
    Epp = None if E_per_pair is None else np.ascontiguousarray(E_per_pair, dtype=np.int32)
    n = len(rl)
    acc = np.zeros(n, dtype=np.uint8)
    ed = np.zeros(n, dtype=np.int32)
    rc = lib().ss_filter_batch_pairs(_ptr(reads), _ptr(rl), _ptr(refs), _ptr(fl), n, _ptr(Epp), int(E), _ptr(acc),
                                     _ptr(ed))
    _check(rc, "ss_filter_batch_pairs")
    return acc, ed


# ---------------------------------------------------------------- context and device entry points
def ss_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().ss_create(ctypes.byref(h), int(device)), "ss_create")
    return h.value


def ss_destroy(ctx: int) -> None:
    _check(lib().ss_destroy(ctx), "ss_destroy")


def ss_sliced_bytes(n_pairs: int, m: int) -> int:
    return int(lib().ss_sliced_bytes(int(n_pairs), int(m)))


def ss_stream_words(total_bases: int) -> int:
    return int(lib().ss_stream_words(int(total_bases)))


def ss_pack_sliced_async(ctx, reads, refs, offsets, index, n_pairs, m, packed, err, stream=None):
    _check(lib().ss_pack_sliced_async(ctx, _ptr(reads), _ptr(refs), _ptr(offsets), _ptr(index), int(n_pairs),
                                      int(m), _ptr(packed), _ptr(err), _stream(stream)), "ss_pack_sliced_async")


def ss_filter_sliced_range_async(ctx, packed, n_pairs, m, E_lo, E_hi, out, out_stride, stream=None):
    _check(lib().ss_filter_sliced_range_async(ctx, _ptr(packed), int(n_pairs), int(m), int(E_lo), int(E_hi),
                                              _ptr(out), int(out_stride), _stream(stream)),
           "ss_filter_sliced_range_async")


def ss_filter_sliced_async(ctx, packed, n_pairs, m, E, out, stream=None):
    _check(lib().ss_filter_sliced_async(ctx, _ptr(packed), int(n_pairs), int(m), int(E), _ptr(out),
                                        _stream(stream)), "ss_filter_sliced_async")


def ss_filter_ascii_async(ctx, reads, refs, n_pairs, m, E, tile_groups, out, err, stream=None):
    _check(lib().ss_filter_ascii_async(ctx, _ptr(reads), _ptr(refs), int(n_pairs), int(m), int(E),
                                       int(tile_groups), _ptr(out), _ptr(err), _stream(stream)),
           "ss_filter_ascii_async")


def ss_pack_words(bases: int) -> int:
    return int(lib().ss_pack_words(int(bases)))


def ss_pack(ctx, ascii_dev, bases, packed, err, stream=None):
    _check(lib().ss_pack(ctx, _ptr(ascii_dev), int(bases), _ptr(packed), _ptr(err), _stream(stream)), "ss_pack")


def batch_desc(reads, refs, n_pairs, E, flags, out, err=None, offsets=None, lengths=None, ref_offsets=None,
               ref_lengths=None, E_per_pair=None, plan=None, read_bases=0, ref_bases=0, length=-1) -> BatchDesc:
    """An ss_batch_desc from buffers (torch tensors, raw addresses or None)."""
    return BatchDesc(_ptr(reads), _ptr(refs), _ptr(offsets), _ptr(lengths), _ptr(ref_offsets), _ptr(ref_lengths),
                     _ptr(E_per_pair), plan, int(n_pairs), int(read_bases), int(ref_bases), int(length), int(E),
                     int(flags), 0, _ptr(out), _ptr(err))


def ss_filter_batch_ex(ctx, desc: BatchDesc, stream=None):
    _check(lib().ss_filter_batch_ex(ctx, ctypes.byref(desc), _stream(stream)), "ss_filter_batch_ex")


def ss_filter_ascii_noalloc(ctx, reads, refs, n_pairs, m, E, out, err, stream=None):
    _check(lib().ss_filter_ascii_noalloc(ctx, _ptr(reads), _ptr(refs), int(n_pairs), int(m), int(E), _ptr(out),
                                         _ptr(err), _stream(stream)), "ss_filter_ascii_noalloc")


def ss_filter_submaze_async(ctx, packed, n_pairs, m, E, sub_width, out, stream=None):
    _check(lib().ss_filter_submaze_async(ctx, _ptr(packed), int(n_pairs), int(m), int(E), int(sub_width), _ptr(out),
                                         _stream(stream)), "ss_filter_submaze_async")


def ss_verify_banded_async(ctx, packed, total_bases, offsets, lengths, E_per_pair, E, index, n, ed_out, stream=None):
    _check(lib().ss_verify_banded_async(ctx, _ptr(packed), int(total_bases), _ptr(offsets), _ptr(lengths),
                                        _ptr(E_per_pair), int(E), _ptr(index), int(n), _ptr(ed_out), _stream(stream)),
           "ss_verify_banded_async")


def ss_verify_async(ctx, packed, total_bases, offsets, lengths, index, n, max_len, ed_out, stream=None):
    _check(lib().ss_verify_async(ctx, _ptr(packed), int(total_bases), _ptr(offsets), _ptr(lengths), _ptr(index),
                                 int(n), int(max_len), _ptr(ed_out), _stream(stream)), "ss_verify_async")


def ss_select_accepted_async(ctx, results, n, index_out, count_out, stream=None):
    _check(lib().ss_select_accepted_async(ctx, _ptr(results), int(n), _ptr(index_out), _ptr(count_out),
                                          _stream(stream)), "ss_select_accepted_async")


def ss_pack_stream_async(ctx, reads, refs, total_bases, packed, err, stream=None):
    _check(lib().ss_pack_stream_async(ctx, _ptr(reads), _ptr(refs), int(total_bases), _ptr(packed), _ptr(err),
                                      _stream(stream)), "ss_pack_stream_async")


def ss_filter_plain_async(ctx, packed, total_bases, offsets, lengths, E_per_pair, n_pairs, E, out, stream=None):
    _check(lib().ss_filter_plain_async(ctx, _ptr(packed), int(total_bases), _ptr(offsets), _ptr(lengths),
                                       _ptr(E_per_pair), int(n_pairs), int(E), _ptr(out), _stream(stream)),
           "ss_filter_plain_async")


def ss_filter_wave_async(ctx, packed, total_bases, offsets, lengths, E_per_pair, n_pairs, E, out, stream=None):
    _check(lib().ss_filter_wave_async(ctx, _ptr(packed), int(total_bases), _ptr(offsets), _ptr(lengths),
                                      _ptr(E_per_pair), int(n_pairs), int(E), _ptr(out), _stream(stream)),
           "ss_filter_wave_async")


def ss_unpack_results_async(ctx, results, n_pairs, accept_out, edits_out, stream=None):
    _check(lib().ss_unpack_results_async(ctx, _ptr(results), int(n_pairs), _ptr(accept_out), _ptr(edits_out),
                                         _stream(stream)), "ss_unpack_results_async")


# ---------------------------------------------------------------- batched launch
def ss_plan_create(ctx, lengths, E_per_pair, slices_per_lane: int = 8) -> int:
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    Epp = np.ascontiguousarray(E_per_pair, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().ss_plan_create(ctx, _ptr(lengths), _ptr(Epp), len(lengths), int(slices_per_lane), ctypes.byref(h)),
           "ss_plan_create")
    return h.value


def ss_plan_items_host(lengths, E_per_pair, slices_per_lane: int = 8):
    """The work items (rows: first slot, pairs, lanes per pair, slices per lane, largest E; queue order) and
    the permutation a plan for these pairs holds, computed on the host."""
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    Epp = np.ascontiguousarray(E_per_pair, dtype=np.int32)
    n = len(lengths)
    k = ctypes.c_int64(0)
    _check(lib().ss_plan_items_host(_ptr(lengths), _ptr(Epp), n, int(slices_per_lane), ctypes.addressof(k), None, 0,
                                    None), "ss_plan_items_host")
    items = np.zeros((k.value, 5), dtype=np.int64)
    perm = np.zeros(n, dtype=np.int64)
    _check(lib().ss_plan_items_host(_ptr(lengths), _ptr(Epp), n, int(slices_per_lane), ctypes.addressof(k),
                                    _ptr(items), k.value, _ptr(perm)), "ss_plan_items_host")
    return items, perm


def ss_plan_destroy(plan) -> None:
    _check(lib().ss_plan_destroy(plan), "ss_plan_destroy")


def ss_plan_info(plan) -> dict:
    ni = ctypes.c_int64(0)
    nc, gr, rs = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().ss_plan_info(plan, ctypes.addressof(ni), ctypes.addressof(nc), ctypes.addressof(gr),
                              ctypes.addressof(rs)), "ss_plan_info")
    return dict(items=ni.value, classes=nc.value, grid=gr.value, slices_per_lane=rs.value)


def ss_filter_planned_async(ctx, plan, packed, total_bases, offsets, lengths, E_per_pair, out, stream=None):
    _check(lib().ss_filter_planned_async(ctx, plan, _ptr(packed), int(total_bases), _ptr(offsets), _ptr(lengths),
                                         _ptr(E_per_pair), _ptr(out), _stream(stream)), "ss_filter_planned_async")


def ss_plan_capture(ctx, plan, packed, total_bases, offsets, lengths, E_per_pair, out):
    _check(lib().ss_plan_capture(ctx, plan, _ptr(packed), int(total_bases), _ptr(offsets), _ptr(lengths),
                                 _ptr(E_per_pair), _ptr(out)), "ss_plan_capture")


def ss_plan_launch(plan, stream=None):
    _check(lib().ss_plan_launch(plan, _stream(stream)), "ss_plan_launch")


def ss_plan_create_tuned(ctx, lengths, E_per_pair, packed, total_bases, offsets_dev, lengths_dev, E_dev, out_dev,
                         cache_path=None):
    """Returns (plan handle, chosen slices per lane)."""
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    Epp = np.ascontiguousarray(E_per_pair, dtype=np.int32)
    h = ctypes.c_void_p()
    ch = ctypes.c_int32(0)
    cp = cache_path.encode() if cache_path else None
    _check(lib().ss_plan_create_tuned(ctx, _ptr(lengths), _ptr(Epp), len(lengths), _ptr(packed), int(total_bases),
                                      _ptr(offsets_dev), _ptr(lengths_dev), _ptr(E_dev), _ptr(out_dev), cp,
                                      ctypes.byref(h), ctypes.addressof(ch)), "ss_plan_create_tuned")
    return h.value, ch.value


# ---------------------------------------------------------------- serving
def ss_server_create(ctx, hbm_budget_bytes: int, n_slots: int = 8) -> int:
    h = ctypes.c_void_p()
    _check(lib().ss_server_create(ctx, int(hbm_budget_bytes), int(n_slots), ctypes.byref(h)), "ss_server_create")
    return h.value


def ss_server_create_loop(ctx, hbm_budget_bytes: int, n_slots: int = 32, slices_per_lane: int = 1) -> int:
    """A server whose requests are run by one device-resident loop kernel (see ss.h)."""
    h = ctypes.c_void_p()
    _check(lib().ss_server_create_loop(ctx, int(hbm_budget_bytes), int(n_slots), int(slices_per_lane),
                                       ctypes.byref(h)), "ss_server_create_loop")
    return h.value


def ss_server_set_loop_idle(server, idle_us: int) -> None:
    _check(lib().ss_server_set_loop_idle(server, int(idle_us)), "ss_server_set_loop_idle")


def ss_server_submit(server, reads, refs, lengths, E_per_pair, accept_out, edits_out) -> int:
    """Submit host numpy arrays; accept_out (uint8) and edits_out (int32) must stay alive until done."""
    n = len(lengths)
    t = ctypes.c_uint64(0)
    rc = lib().ss_server_submit(server, _ptr(reads), _ptr(refs), _ptr(lengths), _ptr(E_per_pair), n,
                                _ptr(accept_out), _ptr(edits_out), ctypes.byref(t))
    _check(rc, "ss_server_submit")
    return t.value


def ss_server_stage_alloc(server, nbytes: int):
    """A block of the server's pinned staging (its address, or None when the staging is full)."""
    return lib().ss_server_stage_alloc(server, int(nbytes))


def ss_server_stage_free(server, block) -> None:
    _check(lib().ss_server_stage_free(server, block), "ss_server_stage_free")


def stage_view(block, nbytes: int):
    """A writable numpy view of nbytes of a staging block."""
    return np.ctypeslib.as_array((ctypes.c_uint8 * int(nbytes)).from_address(int(block)))


def ss_server_submit_staged(server, block, refs_offset: int, lengths, E_per_pair, accept_out, edits_out) -> int:
    """Submit a request whose bases were written into a staging block (reads from its start, refs from
    refs_offset); on success the block belongs to the server."""
    n = len(lengths)
    t = ctypes.c_uint64(0)
    rc = lib().ss_server_submit_staged(server, block, int(refs_offset), _ptr(lengths), _ptr(E_per_pair), n,
                                       _ptr(accept_out), _ptr(edits_out), ctypes.byref(t))
    _check(rc, "ss_server_submit_staged")
    return t.value


def ss_server_poll(server, ticket) -> bool:
    d = ctypes.c_int(0)
    _check(lib().ss_server_poll(server, ticket, ctypes.byref(d)), "ss_server_poll")
    return bool(d.value)


def ss_server_wait(server, ticket, timeout_us: int = -1) -> int:
    """Returns the status code (does not raise)."""
    return int(lib().ss_server_wait(server, ticket, int(timeout_us)))


def ss_server_times(server, ticket):
    a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().ss_server_times(server, ticket, ctypes.addressof(a), ctypes.addressof(b), ctypes.addressof(c)),
           "ss_server_times")
    return a.value, b.value, c.value


def ss_server_stages(server, ticket):
    """(enqueue, copy in, encode + filter, copy out) of a finished request, nanoseconds."""
    v = [ctypes.c_int64(0) for _ in range(4)]
    _check(lib().ss_server_stages(server, ticket, *[ctypes.addressof(x) for x in v]), "ss_server_stages")
    return tuple(x.value for x in v)


def ss_server_cancel(server, ticket) -> int:
    return int(lib().ss_server_cancel(server, ticket))


def ss_server_release(server, ticket) -> int:
    return int(lib().ss_server_release(server, ticket))


def ss_server_set_hold(server, hold: bool) -> None:
    _check(lib().ss_server_set_hold(server, 1 if hold else 0), "ss_server_set_hold")


def ss_server_stats(server) -> dict:
    v = [ctypes.c_int64(0) for _ in range(5)]
    _check(lib().ss_server_stats(server, *[ctypes.addressof(x) for x in v]), "ss_server_stats")
    return dict(admitted=v[0].value, deferred=v[1].value, completed=v[2].value, peak_bytes=v[3].value,
                peak_in_flight=v[4].value)


def ss_server_set_slices(server, slices_per_lane: int) -> None:
    _check(lib().ss_server_set_slices(server, int(slices_per_lane)), "ss_server_set_slices")


def ss_server_footprint(n_pairs: int, total_bases: int) -> int:
    return int(lib().ss_server_footprint(int(n_pairs), int(total_bases)))


def ss_server_destroy(server) -> None:
    _check(lib().ss_server_destroy(server), "ss_server_destroy")


def decode_results(res: np.ndarray):
    """Split device result words (uint16) into (accept uint8, edits int32)."""
    res = np.asarray(res).astype(np.uint16, copy=False)
    return (res >> 15).astype(np.uint8), (res & SS_RESULT_COUNT).astype(np.int32)
