"""MI355X (gfx950) decoder for FSST-8 / OnPair-16 string columns.

Thin Python binding over the C ABI of ``libfastdecode.so`` (declared in
``include/fastdecode.h``).  PyTorch supplies device memory and streams only;
every step of the decode runs in the library's HIP kernels.  There is no CPU
fallback: importing works without the library, but every call raises
``LibraryNotBuilt`` until ``python -m paper_2609_15034_amd.build`` has run.

Names follow the C ABI:
  * ``fsst_decode`` / ``onpair_decode``  - one column, raw dictionary;
  * ``Dict`` (fd_dict) + ``decode_into`` - one column, prepared dictionary;
  * ``decode``                           - convenience: sizes and allocates the
                                           outputs (two device passes);
  * ``batch_decode``                     - many columns, one submission (or one
                                           cached HIP graph), autotuned tiles;
  * ``Server`` (fd_server)               - served decode: continuous batching
                                           of requests under an HBM budget.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastdecode.so")

FSST8 = 1
ONPAIR16 = 2
ONPAIR12 = 3          # 12-bit packed codes (OnPair-12, and FSST-12 with tokens of at most 8 bytes)
CODECS = {"fsst8": FSST8, "onpair16": ONPAIR16, "onpair12": ONPAIR12}


def codes_in(codec, codes) -> int:
    """The number of codes in a code tensor: its elements, or for 12-bit
    packed streams (uint8, least significant bit first, two codes in three
    bytes) the whole codes its bytes hold."""
    c = CODECS[codec] if isinstance(codec, str) else int(codec)
    return codes.numel() * 8 // 12 if c == ONPAIR12 else codes.numel()
ASYNC = 1
GRAPH = 2

(OK, EINVAL, EBADCODE, EESCAPE, ECAPACITY, EOVERFLOW, EBADDICT, EOFFSETS, EHIP, ENOMEM, ESIDECAR, ETIMEOUT, ECANCELED,
 EBUSY) = range(14)
STATUS_NAMES = ["FD_OK", "FD_EINVAL", "FD_EBADCODE", "FD_EESCAPE", "FD_ECAPACITY", "FD_EOVERFLOW", "FD_EBADDICT",
                "FD_EOFFSETS", "FD_EHIP", "FD_ENOMEM", "FD_ESIDECAR", "FD_ETIMEOUT", "FD_ECANCELED", "FD_EBUSY"]


class LibraryNotBuilt(RuntimeError):
    pass


class DecodeError(RuntimeError):
    def __init__(self, status: int, what: str = "decode"):
        self.status = int(status)
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{what} failed: {name}")


class Tuning(ctypes.Structure):
    """fd_tuning: mode (0 single pass / 1 three phases), tile_codes (codes per tile, 0 = the largest), grid."""
    _fields_ = [("mode", ctypes.c_int32), ("tile_codes", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Column(ctypes.Structure):
    """fd_column: one column of a batch (device pointers, prepared dictionary)."""
    _fields_ = [("dict", ctypes.c_void_p), ("codes", ctypes.c_void_p), ("n_codes", ctypes.c_int64),
                ("code_offsets", ctypes.c_void_p), ("index_bits", ctypes.c_int32), ("n_strings", ctypes.c_int64),
                ("out_offsets", ctypes.c_void_p), ("out_bytes", ctypes.c_void_p), ("out_capacity", ctypes.c_int64)]


class BatchChoice(ctypes.Structure):
    """fd_batch_choice: the batch autotuner's choice."""
    _fields_ = [("mode", ctypes.c_int32), ("tile_scale_pct", ctypes.c_int32), ("grid_pct", ctypes.c_int32),
                ("source", ctypes.c_int32), ("candidates_timed", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    """fd_server_config: HBM budget (bytes), stream slots, requests per batch (0 = default), queue
    deadline in microseconds (0 = none)."""
    _fields_ = [("max_inflight_bytes", ctypes.c_int64), ("n_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("queue_timeout_us", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("queued", ctypes.c_int64), ("inflight_bytes", ctypes.c_int64),
                ("max_inflight_bytes", ctypes.c_int64), ("canceled", ctypes.c_int64), ("timed_out", ctypes.c_int64)]


_lib = None


def lib():
    """Load libfastdecode.so (raises LibraryNotBuilt when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryNotBuilt(f"{LIB_PATH} is missing: run `python -m paper_2609_15034_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, U = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint
    S = ctypes.c_size_t
    L.fd_status_str.restype = ctypes.c_char_p
    L.fd_status_str.argtypes = [ctypes.c_int]
    L.fd_version.restype = ctypes.c_char_p
    L.fd_workspace_size.restype = ctypes.c_int
    L.fd_workspace_size.argtypes = [ctypes.c_int, I64, I64, ctypes.POINTER(S)]
    L.fd_workspace_size_ex.restype = ctypes.c_int
    L.fd_workspace_size_ex.argtypes = [ctypes.c_int, I64, I64, ctypes.POINTER(Tuning), ctypes.POINTER(S)]
    L.fd_decoded_bound.restype = ctypes.c_int
    L.fd_decoded_bound.argtypes = [ctypes.c_int, I64, ctypes.POINTER(I64)]
    dec = [P, I64, P, ctypes.c_int, I64, P, P, I32, P, P, I64, P, S, P, U, P]
    L.fsst_decode.restype = ctypes.c_int
    L.fsst_decode.argtypes = dec
    L.onpair_decode.restype = ctypes.c_int
    L.onpair_decode.argtypes = dec
    L.fd_dict_create.restype = ctypes.c_int
    L.fd_dict_create.argtypes = [ctypes.c_int, P, P, I32, P, ctypes.POINTER(P)]
    L.fd_dict_destroy.restype = ctypes.c_int
    L.fd_dict_destroy.argtypes = [P]
    L.fd_dict_codec.restype = ctypes.c_int
    L.fd_dict_codec.argtypes = [P]
    L.fd_dict_size.restype = I32
    L.fd_dict_size.argtypes = [P]
    L.fd_decode.restype = ctypes.c_int
    L.fd_decode.argtypes = [P, P, I64, P, ctypes.c_int, I64, P, P, I64, P, S, P, U, P]
    L.fd_decode_ex.restype = ctypes.c_int
    L.fd_decode_ex.argtypes = [P, P, I64, P, ctypes.c_int, I64, P, P, I64, P, S, P, U, ctypes.POINTER(Tuning), P]
    L.fd_debug_graph_hash_bits.restype = ctypes.c_int
    L.fd_debug_graph_hash_bits.argtypes = [I32]
    L.fd_debug_graph_count.restype = ctypes.c_int32
    L.fd_debug_graph_count.argtypes = []
    L.fd_batch_autotune.restype = ctypes.c_int
    L.fd_batch_autotune.argtypes = [ctypes.POINTER(Column), I32, P, S, P, ctypes.POINTER(BatchChoice)]
    L.fd_debug_autotune_forget.restype = ctypes.c_int
    L.fd_debug_autotune_forget.argtypes = []
    L.fd_profile_begin.restype = ctypes.c_int
    L.fd_profile_begin.argtypes = [ctypes.c_uint32, ctypes.c_int32]
    L.fd_profile_end.restype = ctypes.c_int
    L.fd_profile_end.argtypes = [P, P, P, P, P]
    L.fd_decode_noalloc.restype = ctypes.c_int
    L.fd_decode_noalloc.argtypes = [P, P, I64, P, ctypes.c_int, I64, P, P, I64, P, U, ctypes.POINTER(Tuning), P]
    L.fd_sidecar_layout.restype = ctypes.c_int
    L.fd_sidecar_layout.argtypes = [ctypes.c_int, I64, I64, ctypes.POINTER(Tuning), ctypes.POINTER(I32),
                                    ctypes.POINTER(I64)]
    L.fd_sidecar_build.restype = ctypes.c_int
    L.fd_sidecar_build.argtypes = [P, P, I64, P, ctypes.c_int, I64, P, I64, P, S, P, U, ctypes.POINTER(Tuning), P]
    L.fd_decode_sidecar.restype = ctypes.c_int
    L.fd_decode_sidecar.argtypes = [P, P, I64, P, ctypes.c_int, I64, P, I64, P, P, I64, P, S, P, U,
                                    ctypes.POINTER(Tuning), P]
    L.fd_take_workspace_size.restype = ctypes.c_int
    L.fd_take_workspace_size.argtypes = [ctypes.c_int, I64, I64, I64, I64, ctypes.POINTER(Tuning), ctypes.POINTER(S)]
    L.fd_decode_take.restype = ctypes.c_int
    L.fd_decode_take.argtypes = [P, P, I64, P, ctypes.c_int, I64, P, I64, I64, P, P, I64, P, S, P, U,
                                 ctypes.POINTER(Tuning), P]
    L.fd_batch_workspace_size.restype = ctypes.c_int
    L.fd_batch_workspace_size.argtypes = [ctypes.POINTER(Column), I32, ctypes.POINTER(Tuning), ctypes.POINTER(S)]
    L.batch_decode.restype = ctypes.c_int
    L.batch_decode.argtypes = [ctypes.POINTER(Column), I32, ctypes.POINTER(Tuning), P, S, P, U, P]
    L.fd_server_create.restype = ctypes.c_int
    L.fd_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
    L.fd_server_submit.restype = ctypes.c_int
    L.fd_server_submit.argtypes = [P, ctypes.POINTER(Column), ctypes.POINTER(ctypes.c_uint64)]
    L.fd_server_wait.restype = ctypes.c_int
    L.fd_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double)]
    L.fd_server_wait_for.restype = ctypes.c_int
    L.fd_server_wait_for.argtypes = [P, ctypes.c_uint64, I64, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double)]
    L.fd_server_cancel.restype = ctypes.c_int
    L.fd_server_cancel.argtypes = [P, ctypes.c_uint64]
    L.fd_server_get_stats.restype = ctypes.c_int
    L.fd_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    L.fd_server_destroy.restype = ctypes.c_int
    L.fd_server_destroy.argtypes = [P]
    _lib = L
    return L


# --------------------------------------------------------------------------- #
# helpers
# --------------------------------------------------------------------------- #
def _torch():
    import torch
    return torch


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream) -> ctypes.c_void_p:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _codec_id(codec) -> int:
    return CODECS[codec] if isinstance(codec, str) else int(codec)


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, Tuning):
        return ctypes.byref(t)
    return ctypes.byref(Tuning(**t))


def status_str(status: int) -> str:
    return lib().fd_status_str(int(status)).decode()


def version() -> str:
    return lib().fd_version().decode()


def workspace_size(codec, n_codes: int, n_strings: int, tuning=None) -> int:
    out = ctypes.c_size_t(0)
    tu = Tuning(**tuning) if isinstance(tuning, dict) else tuning
    st = lib().fd_workspace_size_ex(_codec_id(codec), int(n_codes), int(n_strings),
                                    ctypes.byref(tu) if tu is not None else None, ctypes.byref(out))
    if st:
        raise DecodeError(st, "fd_workspace_size")
    return int(out.value)


def decoded_bound(codec, n_codes: int) -> int:
    out = ctypes.c_int64(0)
    st = lib().fd_decoded_bound(_codec_id(codec), int(n_codes), ctypes.byref(out))
    if st:
        raise DecodeError(st, "fd_decoded_bound")
    return int(out.value)


def alloc_workspace(codec, n_codes: int, n_strings: int, tuning=None, device=None):
    torch = _torch()
    n = workspace_size(codec, n_codes, n_strings, tuning)
    # 256-byte aligned (the caching allocator returns 512-byte aligned blocks)
    return torch.empty(n, dtype=torch.uint8, device=device or "cuda")


def _index_bits(code_off) -> int:
    torch = _torch()
    if code_off.dtype == torch.int32:
        return 32
    if code_off.dtype == torch.int64:
        return 64
    raise TypeError("code_off must be int32 or int64")


# --------------------------------------------------------------------------- #
# one-shot entry points (raw dictionaries)
# --------------------------------------------------------------------------- #
def fsst_decode(codes, code_off, dict_bytes, dict_lens, out_off, out_bytes, workspace, status=None,
                async_=False, stream=None) -> int:
    """fsst_decode over torch device tensors; returns the fd_status."""
    return lib().fsst_decode(_ptr(codes), codes.numel(), _ptr(code_off), _index_bits(code_off), code_off.numel() - 1,
                             _ptr(dict_bytes), _ptr(dict_lens), dict_lens.numel(), _ptr(out_off), _ptr(out_bytes),
                             out_bytes.numel(), _ptr(workspace), workspace.numel(), _ptr(status),
                             ASYNC if async_ else 0, _stream_handle(stream))


def onpair_decode(codes, code_off, dict_bytes, dict_lens, out_off, out_bytes, workspace, status=None,
                  async_=False, stream=None) -> int:
    """onpair_decode over torch device tensors (codes int16/uint16 storage)."""
    return lib().onpair_decode(_ptr(codes), codes.numel(), _ptr(code_off), _index_bits(code_off),
                               code_off.numel() - 1, _ptr(dict_bytes), _ptr(dict_lens), dict_lens.numel(),
                               _ptr(out_off), _ptr(out_bytes), out_bytes.numel(), _ptr(workspace), workspace.numel(),
                               _ptr(status), ASYNC if async_ else 0, _stream_handle(stream))


# --------------------------------------------------------------------------- #
# prepared dictionaries
# --------------------------------------------------------------------------- #
class Dict:
    """fd_dict: an immutable device-resident dictionary."""

    def __init__(self, codec, dict_bytes, dict_lens, stream=None):
        self._h = ctypes.c_void_p(0)
        self.codec = _codec_id(codec)
        st = lib().fd_dict_create(self.codec, _ptr(dict_bytes), _ptr(dict_lens), dict_lens.numel(),
                                  _stream_handle(stream), ctypes.byref(self._h))
        if st:
            raise DecodeError(st, "fd_dict_create")
        self.size = int(lib().fd_dict_size(self._h))

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise ValueError("dictionary destroyed")
        return self._h

    def close(self):
        if self._h:
            lib().fd_dict_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_into(d: Dict, codes, code_off, out_off, out_bytes, workspace, status=None, async_=False,
                tuning=None, stream=None, n_codes=None) -> int:
    """fd_decode_ex with preallocated outputs; returns the fd_status (FD_OK when
    enqueued with async_=True)."""
    return lib().fd_decode_ex(d.handle, _ptr(codes), int(codes_in(d.codec, codes) if n_codes is None else n_codes),
                              _ptr(code_off), _index_bits(code_off), code_off.numel() - 1, _ptr(out_off),
                              _ptr(out_bytes), out_bytes.numel() if out_bytes is not None else 0, _ptr(workspace),
                              workspace.numel(), _ptr(status), ASYNC if async_ else 0, _tuning(tuning),
                              _stream_handle(stream))


def decode_noalloc_into(d: Dict, codes, code_off, out_off, out_bytes, status=None, async_=False, tuning=None,
                        stream=None, n_codes=None) -> int:
    """fd_decode_noalloc (no workspace: the library's static device scratch);
    returns the fd_status (FD_OK when enqueued with async_=True)."""
    return lib().fd_decode_noalloc(d.handle, _ptr(codes),
                                   int(codes_in(d.codec, codes) if n_codes is None else n_codes), _ptr(code_off),
                                   _index_bits(code_off), code_off.numel() - 1, _ptr(out_off), _ptr(out_bytes),
                                   out_bytes.numel() if out_bytes is not None else 0, _ptr(status),
                                   ASYNC if async_ else 0, _tuning(tuning), _stream_handle(stream))


def decode(d: Dict, codes, code_off, tuning=None, stream=None):
    """Decode a column into new tensors (out_offsets, out_bytes).  Runs a
    first pass with zero capacity to obtain the offsets and the exact size."""
    torch = _torch()
    dev = codes.device
    ws = alloc_workspace(d.codec, codes_in(d.codec, codes), code_off.numel() - 1, tuning, device=dev)
    out_off = torch.empty(code_off.numel(), dtype=code_off.dtype, device=dev)
    empty = torch.empty(0, dtype=torch.uint8, device=dev)
    st = decode_into(d, codes, code_off, out_off, empty, ws, tuning=tuning, stream=stream)
    if st not in (OK, ECAPACITY):
        raise DecodeError(st)
    total = int(out_off[-1].item())
    out = torch.empty(total, dtype=torch.uint8, device=dev)
    st = decode_into(d, codes, code_off, out_off, out, ws, tuning=tuning, stream=stream)
    if st != OK:
        raise DecodeError(st)
    return out_off, out


# --------------------------------------------------------------------------- #
# persisted output positions (sidecar)
# --------------------------------------------------------------------------- #
def sidecar_layout(codec, n_codes: int, n_strings: int, tuning=None):
    """fd_sidecar_layout: (tile_codes, n_entries) of a column's sidecar."""
    sb, n = ctypes.c_int32(0), ctypes.c_int64(0)
    tu = Tuning(**tuning) if isinstance(tuning, dict) else tuning
    st = lib().fd_sidecar_layout(_codec_id(codec), int(n_codes), int(n_strings),
                                 ctypes.byref(tu) if tu is not None else None, ctypes.byref(sb), ctypes.byref(n))
    if st:
        raise DecodeError(st, "fd_sidecar_layout")
    return int(sb.value), int(n.value)


def sidecar_build_into(d: Dict, codes, code_off, sidecar, workspace, status=None, async_=False, tuning=None,
                       stream=None, n_codes=None) -> int:
    """fd_sidecar_build into a preallocated int64 device tensor; returns the fd_status."""
    return lib().fd_sidecar_build(d.handle, _ptr(codes), int(codes_in(d.codec, codes) if n_codes is None else n_codes),
                                  _ptr(code_off), _index_bits(code_off), code_off.numel() - 1, _ptr(sidecar),
                                  sidecar.numel(), _ptr(workspace), workspace.numel(), _ptr(status),
                                  ASYNC if async_ else 0, _tuning(tuning), _stream_handle(stream))


def sidecar_build(d: Dict, codes, code_off, tuning=None, stream=None):
    """The sidecar of a column as a new int64 device tensor (raises on error)."""
    torch = _torch()
    n = codes_in(d.codec, codes)
    _, n_entries = sidecar_layout(d.codec, n, code_off.numel() - 1, tuning)
    sc = torch.empty(n_entries, dtype=torch.int64, device=codes.device)
    ws = alloc_workspace(d.codec, n, code_off.numel() - 1, tuning, device=codes.device)
    st = sidecar_build_into(d, codes, code_off, sc, ws, tuning=tuning, stream=stream)
    if st != OK:
        raise DecodeError(st, "fd_sidecar_build")
    return sc


def decode_sidecar_into(d: Dict, codes, code_off, sidecar, out_off, out_bytes, workspace, status=None, async_=False,
                        tuning=None, stream=None, n_codes=None) -> int:
    """fd_decode_sidecar with preallocated outputs; returns the fd_status."""
    return lib().fd_decode_sidecar(d.handle, _ptr(codes),
                                   int(codes_in(d.codec, codes) if n_codes is None else n_codes), _ptr(code_off),
                                   _index_bits(code_off), code_off.numel() - 1, _ptr(sidecar), sidecar.numel(),
                                   _ptr(out_off), _ptr(out_bytes), out_bytes.numel() if out_bytes is not None else 0,
                                   _ptr(workspace), workspace.numel(), _ptr(status), ASYNC if async_ else 0,
                                   _tuning(tuning), _stream_handle(stream))


# --------------------------------------------------------------------------- #
# selective decode (take)
# --------------------------------------------------------------------------- #
def take_workspace_size(codec, n_codes: int, n_strings: int, n_rows: int, max_codes: int, tuning=None) -> int:
    out = ctypes.c_size_t(0)
    tu = Tuning(**tuning) if isinstance(tuning, dict) else tuning
    st = lib().fd_take_workspace_size(_codec_id(codec), int(n_codes), int(n_strings), int(n_rows), int(max_codes),
                                      ctypes.byref(tu) if tu is not None else None, ctypes.byref(out))
    if st:
        raise DecodeError(st, "fd_take_workspace_size")
    return int(out.value)


def decode_take_into(d: Dict, codes, code_off, rows, max_codes: int, out_off, out_bytes, workspace, status=None,
                     async_=False, tuning=None, stream=None, n_codes=None) -> int:
    """fd_decode_take with preallocated outputs (rows: int64 device tensor);
    returns the fd_status."""
    return lib().fd_decode_take(d.handle, _ptr(codes), int(codes_in(d.codec, codes) if n_codes is None else n_codes),
                                _ptr(code_off), _index_bits(code_off), code_off.numel() - 1, _ptr(rows),
                                rows.numel(), int(max_codes), _ptr(out_off), _ptr(out_bytes),
                                out_bytes.numel() if out_bytes is not None else 0, _ptr(workspace),
                                workspace.numel(), _ptr(status), ASYNC if async_ else 0, _tuning(tuning),
                                _stream_handle(stream))


def decode_take(d: Dict, codes, code_off, rows, tuning=None, stream=None, n_codes=None):
    """The strings `rows` of a column as new tensors (out_offsets, out_bytes);
    rows must not repeat (the workspace holds at most the column's codes).
    Runs a first pass with zero capacity for the exact size."""
    torch = _torch()
    dev = codes.device
    n = codes_in(d.codec, codes) if n_codes is None else int(n_codes)
    ws = torch.empty(take_workspace_size(d.codec, n, code_off.numel() - 1, rows.numel(), n, tuning),
                     dtype=torch.uint8, device=dev)
    out_off = torch.empty(rows.numel() + 1, dtype=code_off.dtype, device=dev)
    empty = torch.empty(0, dtype=torch.uint8, device=dev)
    st = decode_take_into(d, codes, code_off, rows, n, out_off, empty, ws, tuning=tuning, stream=stream, n_codes=n)
    if st not in (OK, ECAPACITY):
        raise DecodeError(st, "fd_decode_take")
    out = torch.empty(int(out_off[-1].item()), dtype=torch.uint8, device=dev)
    st = decode_take_into(d, codes, code_off, rows, n, out_off, out, ws, tuning=tuning, stream=stream, n_codes=n)
    if st != OK:
        raise DecodeError(st, "fd_decode_take")
    return out_off, out


# --------------------------------------------------------------------------- #
# batches
# --------------------------------------------------------------------------- #
def make_columns(cols):
    """fd_column array from a list of (Dict, codes, code_off, out_off, out_bytes)
    tuples of device tensors (out_bytes may be None for capacity 0)."""
    arr = (Column * max(len(cols), 1))()
    for i, (d, codes, code_off, out_off, out_bytes) in enumerate(cols):
        arr[i] = Column(d.handle.value, codes.data_ptr(), codes_in(d.codec, codes), code_off.data_ptr(),
                        _index_bits(code_off),
                        code_off.numel() - 1, out_off.data_ptr(), out_bytes.data_ptr() if out_bytes is not None else 0,
                        out_bytes.numel() if out_bytes is not None else 0)
    return arr


def batch_workspace_size(cols, tuning=None) -> int:
    """fd_batch_workspace_size for a list of column tuples (see make_columns)."""
    arr = make_columns(cols)
    out = ctypes.c_size_t(0)
    tu = Tuning(**tuning) if isinstance(tuning, dict) else tuning
    st = lib().fd_batch_workspace_size(arr, len(cols), ctypes.byref(tu) if tu is not None else None,
                                       ctypes.byref(out))
    if st:
        raise DecodeError(st, "fd_batch_workspace_size")
    return int(out.value)


def batch_autotune(cols, workspace, stream=None) -> dict:
    """fd_batch_autotune: the autotuner's choice for a batch of column tuples
    (timed now if its shape is new)."""
    arr = make_columns(cols)
    out = BatchChoice()
    st = lib().fd_batch_autotune(arr, len(cols), _ptr(workspace), workspace.numel(), _stream_handle(stream),
                                 ctypes.byref(out))
    if st:
        raise DecodeError(st, "fd_batch_autotune")
    return {k: int(getattr(out, k)) for k, _ in BatchChoice._fields_}


def debug_autotune_forget() -> None:
    """Testing hook: clear the process's autotuner cache."""
    st = lib().fd_debug_autotune_forget()
    if st:
        raise DecodeError(st, "fd_debug_autotune_forget")


def debug_graph_hash_bits(bits: int) -> None:
    """Testing hook: keep only `bits` bits of the graph cache's hash (0 makes
    every key collide, so only the full key comparison tells batches apart)."""
    st = lib().fd_debug_graph_hash_bits(int(bits))
    if st:
        raise DecodeError(st, "fd_debug_graph_hash_bits")


def debug_graph_count() -> int:
    """Testing hook: the number of cached batch graphs."""
    return int(lib().fd_debug_graph_count())


PROF_KINDS = ("reset", "coarse", "totals", "scan", "decode", "prepare")   # fd_prof_kind order


def profile_begin(kinds=PROF_KINDS, max_launches: int = 4096) -> None:
    """fd_profile_begin: time every launch of the named kinds (HIP events on
    the launch's stream) until profile_end."""
    mask = 0
    for k in kinds:
        mask |= 1 << PROF_KINDS.index(k)
    st = lib().fd_profile_begin(mask, int(max_launches))
    if st:
        raise DecodeError(st, "fd_profile_begin")


def profile_end() -> dict:
    """fd_profile_end: {kind: {"launches", "total_ms", "mean_us", "min_us",
    "max_us"}} for the kinds launched, plus "dropped"."""
    n = len(PROF_KINDS)
    tot, mn, mx = (ctypes.c_double * n)(), (ctypes.c_double * n)(), (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    dropped = ctypes.c_int64(0)
    st = lib().fd_profile_end(ctypes.cast(tot, ctypes.c_void_p), ctypes.cast(cnt, ctypes.c_void_p),
                              ctypes.cast(mn, ctypes.c_void_p), ctypes.cast(mx, ctypes.c_void_p),
                              ctypes.cast(ctypes.pointer(dropped), ctypes.c_void_p))
    if st:
        raise DecodeError(st, "fd_profile_end")
    out = {"dropped": int(dropped.value)}
    for i, k in enumerate(PROF_KINDS):
        if cnt[i]:
            out[k] = {"launches": int(cnt[i]), "total_ms": tot[i], "mean_us": tot[i] * 1e3 / cnt[i],
                      "min_us": mn[i] * 1e3, "max_us": mx[i] * 1e3}
    return out


def batch_decode(cols, workspace, status=None, tuning=None, async_=False, graph=False, stream=None) -> int:
    """batch_decode over a list of column tuples (Dict, codes, code_off, out_off,
    out_bytes); `status` (device int32, len(cols) + 1) receives the per-column
    statuses and the first error.  Returns the fd_status (FD_OK when enqueued
    with async_=True)."""
    arr = make_columns(cols)
    flags = (ASYNC if async_ else 0) | (GRAPH if graph else 0)
    return lib().batch_decode(arr, len(cols), _tuning(tuning), _ptr(workspace), workspace.numel(), _ptr(status),
                              flags, _stream_handle(stream))


# --------------------------------------------------------------------------- #
# served decode
# --------------------------------------------------------------------------- #
class Server:
    """fd_server: continuous batching of decode requests on the current device.

    ``submit`` takes a column tuple (Dict, codes, code_off, out_off, out_bytes)
    whose tensors must stay alive until ``wait`` returns for its ticket."""

    def __init__(self, max_inflight_bytes: int = 0, n_slots: int = 0, max_batch: int = 0, queue_timeout_us: int = 0):
        self._h = ctypes.c_void_p(0)
        cfg = ServerConfig(int(max_inflight_bytes), int(n_slots), int(max_batch), int(queue_timeout_us))
        st = lib().fd_server_create(ctypes.byref(cfg), ctypes.byref(self._h))
        if st:
            raise DecodeError(st, "fd_server_create")

    @staticmethod
    def prepare(col):
        """A request's column record, built ahead of ``submit`` so that the
        submission costs only the library call (its tensors must stay alive as
        for ``submit``)."""
        return make_columns([col])

    def submit(self, col) -> int:
        """Enqueue a column tuple, or a record from ``prepare``; returns the ticket."""
        arr = col if isinstance(col, ctypes.Array) else make_columns([col])
        t = ctypes.c_uint64(0)
        st = lib().fd_server_submit(self._h, arr, ctypes.byref(t))
        if st:
            raise DecodeError(st, "fd_server_submit")
        return int(t.value)

    def wait(self, ticket: int, timeout_us: int | None = None):
        """(fd_status, latency in microseconds) of a request; with a timeout,
        None if it has not completed by then (wait for the ticket again)."""
        s = ctypes.c_int32(-1)
        lat = ctypes.c_double(0.0)
        st = lib().fd_server_wait_for(self._h, ctypes.c_uint64(ticket), -1 if timeout_us is None else int(timeout_us),
                                      ctypes.byref(s), ctypes.byref(lat))
        if st == ETIMEOUT:
            return None
        if st:
            raise DecodeError(st, "fd_server_wait_for")
        return int(s.value), float(lat.value)

    def cancel(self, ticket: int) -> bool:
        """fd_server_cancel: True if the request was still queued (it then
        completes with ECANCELED), False if it already runs or ran."""
        st = lib().fd_server_cancel(self._h, ctypes.c_uint64(ticket))
        if st == EBUSY:
            return False
        if st:
            raise DecodeError(st, "fd_server_cancel")
        return True

    def stats(self) -> dict:
        out = ServerStats()
        st = lib().fd_server_get_stats(self._h, ctypes.byref(out))
        if st:
            raise DecodeError(st, "fd_server_get_stats")
        return {k: int(getattr(out, k)) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().fd_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
