"""CPU ORACLE - test infrastructure only.

Plain sequential decoders (``oracle.c``, built with gcc -O2) plus a tiny
pure-Python transcription (``spec.py``) for brute force on tiny inputs.  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the library never does, and the oracle
imports nothing from the library.

Status numbering (a convention of the decode interface, restated here):
0 OK, 1 EINVAL, 2 EBADCODE, 3 EESCAPE, 4 ECAPACITY, 5 EOVERFLOW, 6 EBADDICT,
7 EOFFSETS, 9 ENOMEM, 10 ESIDECAR.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, EBADCODE, EESCAPE, ECAPACITY, EOVERFLOW, EBADDICT, EOFFSETS = range(8)
ENOMEM, ESIDECAR = 9, 10


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.oracle_fsst8_decode.restype = ctypes.c_int
        L.oracle_fsst8_decode.argtypes = [P, I64, P, I64, P, P, I32, ctypes.c_int, P, P, I64, P, P]
        L.oracle_onpair16_decode.restype = ctypes.c_int
        L.oracle_onpair16_decode.argtypes = [P, I64, P, I64, P, P, I32, ctypes.c_int, P, P, I64, P, P, P]
        L.oracle_onpair16_decode_copy16.restype = ctypes.c_int
        L.oracle_onpair16_decode_copy16.argtypes = [P, P, I64, P, P, I32, P, P, P]
        _lib = L
    return _lib


@dataclass
class Result:
    status: int
    out_off: np.ndarray     # int64, n_strings + 1 (valid when status in (OK, ECAPACITY, EOVERFLOW))
    out_bytes: np.ndarray   # uint8, min(total, capacity) bytes
    total: int
    err_pos: int


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _as_i64(code_off) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(code_off), dtype=np.int64)


def unpack12(packed, n_codes: int) -> np.ndarray:
    """12-bit codes from their packed byte stream (OnPair-12 / FSST-12, code
    widths table of the Background section).  The paper widens such codes to
    16 bits before decoding (Evaluation, pre-decode preparation) and fixes no
    bit order; the reading here: least significant bit first, code k in bits
    [12k, 12k + 12) of the stream, so two codes fill three bytes.  Written
    from that definition, one code at a time."""
    b = np.ascontiguousarray(packed, dtype=np.uint8)
    if len(b) * 8 < n_codes * 12:
        raise ValueError("packed stream shorter than n_codes codes")
    out = np.zeros(n_codes, np.uint16)
    for k in range(n_codes):
        bit = 12 * k
        byte, sh = bit // 8, bit % 8
        v = int(b[byte]) | (int(b[byte + 1]) << 8) if byte + 1 < len(b) else int(b[byte])
        out[k] = (v >> sh) & 0xFFF
    return out


def unpack12_np(packed, n_codes: int) -> np.ndarray:
    """unpack12 for whole columns: the same definition over pairs of codes
    (three bytes b0 b1 b2 hold b0 | (b1 & 0xf) << 8 and b1 >> 4 | b2 << 4)."""
    b = np.ascontiguousarray(packed, dtype=np.uint8)
    if len(b) * 8 < n_codes * 12:
        raise ValueError("packed stream shorter than n_codes codes")
    n_pairs = (n_codes + 1) // 2
    t = np.zeros(n_pairs * 3, np.uint16)
    t[: min(len(b), n_pairs * 3)] = b[: n_pairs * 3]
    t = t.reshape(-1, 3)
    out = np.empty(n_pairs * 2, np.uint16)
    out[0::2] = t[:, 0] | ((t[:, 1] & 0xF) << 8)
    out[1::2] = (t[:, 1] >> 4) | (t[:, 2] << 4)
    return out[:n_codes]


def pack12(codes) -> np.ndarray:
    """The inverse of unpack12 (test and generator helper): codes < 4096."""
    c = np.asarray(codes, dtype=np.int64)
    if len(c) and (c.min() < 0 or c.max() > 0xFFF):
        raise ValueError("12-bit codes out of range")
    out = np.zeros((len(c) * 12 + 7) // 8, np.uint8)
    for k, v in enumerate(c.tolist()):
        bit = 12 * k
        byte, sh = bit // 8, bit % 8
        w = v << sh
        out[byte] |= w & 0xFF
        out[byte + 1] |= (w >> 8) & 0xFF
        if sh and byte + 2 < len(out):
            out[byte + 2] |= (w >> 16) & 0xFF
    return out


def decode(codec: str, codes, code_off, dict_bytes, dict_lens, index_bits: int | None = None,
           out_capacity: int | None = None, n_codes: int | None = None) -> Result:
    """Decode a whole column.  ``out_capacity=None`` sizes the output exactly
    (an upper bound is used for the call and the result trimmed).  For
    "onpair12" ``codes`` is the packed stream and ``n_codes`` its code count
    (default: every whole code in it); the codes are unpacked (unpack12) and
    decoded as OnPair-16 codes."""
    if codec == "onpair12":
        packed = np.ascontiguousarray(codes, dtype=np.uint8)
        n = (len(packed) * 8) // 12 if n_codes is None else int(n_codes)
        return decode("onpair16", unpack12_np(packed, n), code_off, dict_bytes, dict_lens, index_bits, out_capacity)
    codes = np.ascontiguousarray(codes, dtype=np.uint8 if codec == "fsst8" else np.uint16)
    code_off_arr = np.asarray(code_off)
    if index_bits is None:
        index_bits = 32 if code_off_arr.dtype == np.int32 else 64
    co = _as_i64(code_off_arr)
    db = np.ascontiguousarray(dict_bytes, dtype=np.uint8)
    dl = np.ascontiguousarray(dict_lens, dtype=np.uint8)
    n_strings = len(co) - 1
    maxlen = 8 if codec == "fsst8" else 16
    cap = out_capacity if out_capacity is not None else len(codes) * maxlen
    out_off = np.zeros(max(n_strings + 1, 1), np.int64)
    # guard band after the capacity: the oracle must never write past it
    out = np.full(cap + 64, 0xA5, np.uint8)
    total = ctypes.c_int64(0)
    err = ctypes.c_int64(-1)
    L = lib()
    if codec == "fsst8":
        st = L.oracle_fsst8_decode(_p(codes), len(codes), _p(co), n_strings, _p(db), _p(dl), len(dl), index_bits,
                                   _p(out_off), _p(out), cap, ctypes.byref(total), ctypes.byref(err))
    elif codec == "onpair16":
        scratch = np.zeros(max(len(dl), 1), np.int64)
        st = L.oracle_onpair16_decode(_p(codes), len(codes), _p(co), n_strings, _p(db), _p(dl), len(dl),
                                      index_bits, _p(out_off), _p(out), cap, ctypes.byref(total),
                                      ctypes.byref(err), _p(scratch))
    else:
        raise ValueError(codec)
    t = int(total.value)
    if not np.all(out[cap:] == 0xA5):
        raise AssertionError("oracle wrote past out_capacity")
    return Result(int(st), out_off, out[: min(t, cap)], t, int(err.value))


def code_positions(codec: str, codes, code_off, dict_bytes, dict_lens, positions, n_codes: int | None = None,
                   string_offsets=None):
    """The output position of each code position p in ``positions`` (with
    code_off[0] <= p <= code_off[n]): the bytes the codes at positions
    [code_off[0], p) decode to.  It follows the decode definition (background
    section: tokens concatenated in code order; the escape emits nothing and
    the byte after it is one literal byte) string by string: p lies in the
    string whose codes hold it, and its position is that string's output
    offset plus what the string's codes before p emit, walked in order.  The
    strings' output offsets come from decode(), or from ``string_offsets``
    when given (a column's known string offsets, valid data only).
    Returns (status, int64 positions); None when the data has an error."""
    if codec == "onpair12":
        packed = np.ascontiguousarray(codes, dtype=np.uint8)
        n = (len(packed) * 8) // 12 if n_codes is None else int(n_codes)
        codes, codec = unpack12_np(packed, n), "onpair16"
    if string_offsets is None:
        r = decode(codec, codes, code_off, dict_bytes, dict_lens, index_bits=64)
        if r.status != OK:
            return r.status, None
        soff = r.out_off
    else:
        soff = _as_i64(string_offsets)
    co = _as_i64(code_off)
    dl = np.asarray(dict_lens, dtype=np.int64)
    codes = np.asarray(codes)
    a, b = int(co[0]), int(co[-1])
    out = []
    for p in (int(x) for x in positions):
        if not a <= p <= b:
            raise ValueError("position outside the decode range")
        if p == b:
            out.append(int(soff[-1]))
            continue
        i = int(np.searchsorted(co, p, side="right")) - 1    # the string holding code p
        pos, j = int(soff[i]), int(co[i])
        cl = codes[j:p].tolist()
        j0 = j
        while j < p:
            c = cl[j - j0]
            if codec == "fsst8" and c == 255:      # an escape: its literal follows
                if j + 1 < p:
                    pos += 1
                    j += 2
                else:
                    j += 1
            else:
                pos += int(dl[c])
                j += 1
        out.append(pos)
    return OK, np.array(out, np.int64)


def sidecar(codec: str, codes, code_off, dict_bytes, dict_lens, tile_codes: int, n_codes: int | None = None,
            string_offsets=None):
    """The sidecar of a column: the output position stored for every fixed-size
    group of codes, so that a decoder can start every group at once
    (introduction; design section, overview and placement of the output).  A
    group is a tile of ``tile_codes`` code positions of the code buffer: entry
    k is the output position of code position max(a, min(k T, b)) for
    k < n_tiles = max(1, ceil(n_codes / T)) (n_codes: the buffer's codes), and
    the last entry is the decoded total, where [a, b) = [code_off[0],
    code_off[n]).  Returns (status, int64 entries); None on an error in the
    data."""
    T = int(tile_codes)
    if T < 1:
        raise ValueError("tile_codes must be positive")
    nc = int(n_codes) if n_codes is not None else len(codes)
    co = _as_i64(code_off)
    a, b = int(co[0]), int(co[-1])
    n_tiles = max(1, -(-nc // T))
    pos = [max(a, min(k * T, b)) for k in range(n_tiles)] + [b]
    return code_positions(codec, codes, code_off, dict_bytes, dict_lens, pos, n_codes, string_offsets)


def decode_with_sidecar(codec: str, codes, code_off, dict_bytes, dict_lens, stored, tile_codes: int,
                        index_bits: int | None = None, out_capacity: int | None = None,
                        n_codes: int | None = None) -> Result:
    """Decode with stored output positions: the plain decode's result, except
    that stored positions other than the column's own sidecar give ESIDECAR,
    which ranks after the errors in the data and before EOVERFLOW and
    ECAPACITY (on ESIDECAR nothing of the output is defined)."""
    st, own = sidecar(codec, codes, code_off, dict_bytes, dict_lens, tile_codes, n_codes)
    if st == OK:
        given = np.asarray(stored, dtype=np.int64)
        if len(given) != len(own):
            raise ValueError("a sidecar of another tiling")
        if not np.array_equal(given, own):
            n = len(code_off) - 1
            return Result(ESIDECAR, np.zeros(n + 1, np.int64), np.zeros(0, np.uint8), int(own[-1]), -1)
    return decode(codec, codes, code_off, dict_bytes, dict_lens, index_bits, out_capacity, n_codes)


def take(codec: str, codes, code_off, dict_bytes, dict_lens, rows, max_codes: int | None = None,
         index_bits: int | None = None, out_capacity: int | None = None, n_codes: int | None = None) -> Result:
    """Selective decode: string i of the result is string rows[i] of the
    column (dictionary codecs keep strings independently decodable: the
    random access of the introduction and related work).  The selected
    strings' codes, each string's whole, form a column of their own, which is
    decoded.  A row outside the column, or a selected string whose code
    offsets are not ordered inside [0, n_codes], is EOFFSETS; more than
    ``max_codes`` selected codes is ENOMEM; then the decode's statuses."""
    if codec == "onpair12":
        packed = np.ascontiguousarray(codes, dtype=np.uint8)
        n = (len(packed) * 8) // 12 if n_codes is None else int(n_codes)
        codes, codec = unpack12_np(packed, n), "onpair16"
    codes = np.ascontiguousarray(codes, dtype=np.uint8 if codec == "fsst8" else np.uint16)
    code_off_arr = np.asarray(code_off)
    co = _as_i64(code_off_arr)
    n_strings = len(co) - 1
    rows = np.asarray(rows, dtype=np.int64)
    sel_off = np.zeros(len(rows) + 1, np.int64)
    bad = Result(EOFFSETS, sel_off, np.zeros(0, np.uint8), 0, -1)
    if len(rows) and (rows.min() < 0 or rows.max() >= n_strings):
        return bad
    a, b = co[rows], co[rows + 1]
    if len(rows) and ((a < 0).any() or (b < a).any() or (b > len(codes)).any()):
        return bad
    lens = b - a
    sel_off[1:] = np.cumsum(lens)
    total = int(sel_off[-1])
    if max_codes is not None and total > max_codes:
        return Result(ENOMEM, sel_off, np.zeros(0, np.uint8), 0, -1)
    # code j of the selection is code a[i] + (j - sel_off[i]) of the column, i its string
    idx = np.repeat(a - sel_off[:-1], lens) + np.arange(total, dtype=np.int64)
    return decode(codec, codes[idx], sel_off.astype(code_off_arr.dtype), dict_bytes, dict_lens, index_bits,
                  out_capacity)


def decode_onpair16_copy16(codes, code_off, dict_bytes, dict_lens):
    """The copy-16-and-advance formulation (valid input only)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    co = _as_i64(code_off)
    db = np.ascontiguousarray(dict_bytes, dtype=np.uint8)
    dl = np.ascontiguousarray(dict_lens, dtype=np.uint8)
    n_strings = len(co) - 1
    out_off = np.zeros(n_strings + 1, np.int64)
    out = np.zeros(len(codes) * 16 + 16, np.uint8)
    table = np.zeros(max(len(dl), 1) * 16, np.uint8)
    st = lib().oracle_onpair16_decode_copy16(_p(codes), _p(co), n_strings, _p(db), _p(dl), len(dl), _p(table),
                                            _p(out_off), _p(out))
    return int(st), out_off, out[: int(out_off[-1])]


def time_decode(codec: str, codes, code_off, dict_bytes, dict_lens, threads: int = 1, repeats: int = 1,
                max_strings: int | None = None, n_codes: int | None = None, times: list | None = None):
    """Time the oracle on contiguous string-range shards decoded by `threads`
    threads at once (each shard is an independent oracle call; the calls
    release the GIL).  Returns (best_seconds, decoded_bytes, strings_used);
    every repeat's time is appended to `times` when given.  Only the decode
    calls are timed; outputs are preallocated.  12-bit codes are unpacked
    before the timed region (as the paper widens them before decoding)."""
    if codec == "onpair12":
        packed = np.ascontiguousarray(codes, dtype=np.uint8)
        codes = unpack12_np(packed, (len(packed) * 8) // 12 if n_codes is None else int(n_codes))
        codec = "onpair16"
    codes = np.ascontiguousarray(codes, dtype=np.uint8 if codec == "fsst8" else np.uint16)
    co = _as_i64(code_off)
    if max_strings is not None:
        co = co[: max_strings + 1]
    s = len(co) - 1
    db = np.ascontiguousarray(dict_bytes, dtype=np.uint8)
    dl = np.ascontiguousarray(dict_lens, dtype=np.uint8)
    maxlen = 8 if codec == "fsst8" else 16
    bounds = [s * k // threads for k in range(threads + 1)]
    shards = []
    for k in range(threads):
        a, b = bounds[k], bounds[k + 1]
        sub = np.ascontiguousarray(co[a:b + 1])
        n_c = int(sub[-1] - sub[0]) if b > a else 0
        shards.append((sub, np.zeros(b - a + 1, np.int64), np.zeros(max(n_c * maxlen, 1), np.uint8)))
    L = lib()
    results = [None] * threads

    def run(k):
        sub, oo, ob = shards[k]
        total = ctypes.c_int64(0)
        err = ctypes.c_int64(-1)
        if codec == "fsst8":
            st = L.oracle_fsst8_decode(_p(codes), len(codes), _p(sub), len(sub) - 1, _p(db), _p(dl), len(dl), 64,
                                       _p(oo), _p(ob), len(ob), ctypes.byref(total), ctypes.byref(err))
        else:
            scratch = np.zeros(max(len(dl), 1), np.int64)
            st = L.oracle_onpair16_decode(_p(codes), len(codes), _p(sub), len(sub) - 1, _p(db), _p(dl), len(dl),
                                          64, _p(oo), _p(ob), len(ob), ctypes.byref(total), ctypes.byref(err),
                                          _p(scratch))
        results[k] = (st, int(total.value))

    best = None
    for _ in range(repeats):
        ths = [threading.Thread(target=run, args=(k,)) for k in range(threads)]
        t0 = time.perf_counter()
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
        if times is not None:
            times.append(dt)
    if any(r[0] != OK for r in results):
        raise RuntimeError("oracle failed on a shard: %r" % (results,))
    return best, sum(r[1] for r in results), s
