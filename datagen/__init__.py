"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module generates text columns, trains dictionaries and encodes the text
into code streams.  It holds no decoding arithmetic: neither the CPU oracle nor
the GPU decoder is imported here, and both consume what it produces.

Workload recipes (sizes and distributions follow the paper's workload shapes:
log-like and URL/identifier-like string columns, FSST-style 8-bit codes with an
escape and OnPair-style 16-bit codes):

* ``fsst_small``  - 10,000 printable strings (length U[8, 80]); 255-symbol
  table: 93 single printable bytes (2 of the 95 excluded by seed, which makes
  about 2% of bytes escapes) + 162 random printable symbols of length U[2, 8];
  greedy longest match; uint8 codes, int32 offsets.
* ``fsst_logs_ngram`` - templated log lines, length log-normal (median 120 B,
  sigma 0.5, clamped [32, 2048]); table = the top-255 1..8-byte n-grams of a
  separate 1 MiB sample, scored by count x length; greedy longest match
  (bytes no symbol covers become escapes); uint8 codes, int64 offsets.
* ``fsst_logs``   - the same log lines with a table trained by FSST-style
  rounds on the same sample (parse, count symbols and adjacent symbol pairs
  by bytes covered, keep the best 255): fewer escapes and longer codes.
* ``onpair_urls`` - URL-like (70%) / identifier-like (30%) strings, length
  log-normal (median 30 B, sigma 0.5, clamped [4, 512]); OnPair-style
  dictionary trained on a separate 4 MiB sample (tau = 2, tokens <= 16 B, up
  to 65,536 tokens); uint16 codes, int64 offsets.
* ``random_onpair`` - a random full dictionary (65,536 tokens of length
  U[1, 16]) with uniform random codes (an adversarial gather pattern).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libdatagen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator core with gcc (host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Column(ctypes.Structure):
    _fields_ = [("bytes", ctypes.POINTER(ctypes.c_uint8)), ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("n_strings", ctypes.c_int64), ("n_bytes", ctypes.c_int64)]


class _Codes(ctypes.Structure):
    _fields_ = [("codes", ctypes.c_void_p), ("n_codes", ctypes.c_int64),
                ("code_off", ctypes.POINTER(ctypes.c_int64)), ("n_strings", ctypes.c_int64),
                ("code_bytes", ctypes.c_int), ("n_escapes", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.dg_gen_printable.restype = ctypes.POINTER(_Column)
        L.dg_gen_printable.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        L.dg_gen_logs.restype = ctypes.POINTER(_Column)
        L.dg_gen_logs.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        L.dg_gen_urls.restype = ctypes.POINTER(_Column)
        L.dg_gen_urls.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        L.dg_column_free.argtypes = [ctypes.POINTER(_Column)]
        L.dg_fsst_random_table.restype = ctypes.c_int
        L.dg_fsst_random_table.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, P, P]
        L.dg_fsst_ngram_table.restype = ctypes.c_int
        L.dg_fsst_ngram_table.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P]
        L.dg_fsst_train.restype = ctypes.c_int
        L.dg_fsst_train.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P]
        L.dg_onpair_train.restype = ctypes.c_int
        L.dg_onpair_train.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        L.dg_random_dict.restype = ctypes.c_int
        L.dg_random_dict.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, P, P]
        L.dg_encode_fsst.restype = ctypes.POINTER(_Codes)
        L.dg_encode_fsst.argtypes = [P, P, ctypes.c_int, P, P, ctypes.c_int64, ctypes.c_int]
        L.dg_encode_onpair.restype = ctypes.POINTER(_Codes)
        L.dg_encode_onpair.argtypes = [P, P, ctypes.c_int, P, P, ctypes.c_int64, ctypes.c_int]
        L.dg_codes_free.argtypes = [ctypes.POINTER(_Codes)]
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _take_column(cp) -> tuple[np.ndarray, np.ndarray]:
    c = cp.contents
    nb, ns = c.n_bytes, c.n_strings
    b = np.ctypeslib.as_array(c.bytes, shape=(max(nb, 1),))[:nb].copy()
    o = np.ctypeslib.as_array(c.offsets, shape=(ns + 1,)).copy()
    lib().dg_column_free(cp)
    return b, o


def _take_codes(cp) -> tuple[np.ndarray, np.ndarray, int]:
    c = cp.contents
    dt = np.uint8 if c.code_bytes == 1 else np.uint16
    n = c.n_codes
    raw = (ctypes.c_uint8 * (max(n, 1) * c.code_bytes)).from_address(c.codes)
    codes = np.frombuffer(raw, dtype=dt, count=n).copy()
    off = np.ctypeslib.as_array(c.code_off, shape=(c.n_strings + 1,)).copy()
    esc = c.n_escapes
    lib().dg_codes_free(cp)
    return codes, off, esc


# --------------------------------------------------------------------------- #
# text generators
# --------------------------------------------------------------------------- #
def printable_strings(seed: int, n_strings: int, min_len: int = 8, max_len: int = 80):
    return _take_column(lib().dg_gen_printable(seed, n_strings, min_len, max_len))


# Samples for dictionary training come from the same distribution as the column
# (same seed: same vocabulary and base date) but from disjoint random streams.
SAMPLE_STREAM = 1 << 40


def log_lines(seed: int, target_bytes: int, nchunk: int = 256, threads: int | None = None, stream_base: int = 0):
    nchunk = max(1, min(nchunk, max(1, target_bytes // 4096)))
    return _take_column(lib().dg_gen_logs(seed, stream_base, target_bytes, nchunk, threads or default_threads()))


def url_strings(seed: int, target_bytes: int, nchunk: int = 256, threads: int | None = None, stream_base: int = 0):
    nchunk = max(1, min(nchunk, max(1, target_bytes // 4096)))
    return _take_column(lib().dg_gen_urls(seed, stream_base, target_bytes, nchunk, threads or default_threads()))


# --------------------------------------------------------------------------- #
# dictionaries
# --------------------------------------------------------------------------- #
def fsst_random_table(seed: int, n_sym: int = 255, n_excluded: int = 2):
    out_b = np.zeros(255 * 8, np.uint8)
    out_l = np.zeros(255, np.uint8)
    n = lib().dg_fsst_random_table(seed, n_sym, n_excluded, _ptr(out_b), _ptr(out_l))
    lens = out_l[:n].copy()
    return out_b[: int(lens.sum(dtype=np.int64))].copy(), lens


def fsst_ngram_table(sample_bytes: np.ndarray, sample_off: np.ndarray, max_syms: int = 255):
    out_b = np.zeros(max_syms * 8, np.uint8)
    out_l = np.zeros(max_syms, np.uint8)
    sample_off = np.ascontiguousarray(sample_off, dtype=np.int64)
    n = lib().dg_fsst_ngram_table(_ptr(sample_bytes), _ptr(sample_off), len(sample_off) - 1, max_syms,
                                  _ptr(out_b), _ptr(out_l))
    lens = out_l[:n].copy()
    return out_b[: int(lens.sum(dtype=np.int64))].copy(), lens


def fsst_train(sample_bytes: np.ndarray, sample_off: np.ndarray, max_syms: int = 255, rounds: int = 5):
    out_b = np.zeros(max_syms * 8, np.uint8)
    out_l = np.zeros(max_syms, np.uint8)
    sample_off = np.ascontiguousarray(sample_off, dtype=np.int64)
    n = lib().dg_fsst_train(_ptr(sample_bytes), _ptr(sample_off), len(sample_off) - 1, max_syms, rounds,
                            _ptr(out_b), _ptr(out_l))
    lens = out_l[:n].copy()
    return out_b[: int(lens.sum(dtype=np.int64))].copy(), lens


def onpair_train(sample_bytes: np.ndarray, sample_off: np.ndarray, max_tokens: int = 65536, tau: int = 2,
                 max_len: int = 16):
    out_b = np.zeros(max_tokens * 16, np.uint8)
    out_l = np.zeros(max_tokens, np.uint8)
    sample_off = np.ascontiguousarray(sample_off, dtype=np.int64)
    n = lib().dg_onpair_train(_ptr(sample_bytes), _ptr(sample_off), len(sample_off) - 1, max_tokens, tau,
                              max_len, _ptr(out_b), _ptr(out_l))
    if n < 0:
        raise ValueError("onpair_train: max_tokens must be >= 256")
    lens = out_l[:n].copy()
    return out_b[: int(lens.sum(dtype=np.int64))].copy(), lens


def random_dict(seed: int, n_tok: int = 65536, max_len: int = 16):
    out_b = np.zeros(n_tok * max_len, np.uint8)
    out_l = np.zeros(n_tok, np.uint8)
    lib().dg_random_dict(seed, n_tok, max_len, _ptr(out_b), _ptr(out_l))
    return out_b[: int(out_l.sum(dtype=np.int64))].copy(), out_l


# --------------------------------------------------------------------------- #
# encoders (greedy longest match)
# --------------------------------------------------------------------------- #
def encode_fsst(dict_bytes, dict_lens, text, text_off, threads: int | None = None):
    text_off = np.ascontiguousarray(text_off, dtype=np.int64)
    cp = lib().dg_encode_fsst(_ptr(dict_bytes), _ptr(dict_lens), len(dict_lens), _ptr(text), _ptr(text_off),
                              len(text_off) - 1, threads or default_threads())
    return _take_codes(cp)


def encode_onpair(dict_bytes, dict_lens, text, text_off, threads: int | None = None):
    text_off = np.ascontiguousarray(text_off, dtype=np.int64)
    cp = lib().dg_encode_onpair(_ptr(dict_bytes), _ptr(dict_lens), len(dict_lens), _ptr(text), _ptr(text_off),
                                len(text_off) - 1, threads or default_threads())
    if not cp:
        raise ValueError("encode_onpair: dictionary lacks a single-byte token for some byte value")
    return _take_codes(cp)


# --------------------------------------------------------------------------- #
# workload recipes
# --------------------------------------------------------------------------- #
@dataclass
class Column:
    """An encoded string column plus the text it encodes."""
    name: str
    codec: str                 # "fsst8" | "onpair16"
    codes: np.ndarray          # uint8 / uint16
    code_off: np.ndarray       # int32 / int64, n_strings + 1
    dict_bytes: np.ndarray     # packed token bytes
    dict_lens: np.ndarray      # uint8 token lengths
    text: np.ndarray | None    # the plain bytes (None when not kept)
    text_off: np.ndarray | None
    n_escapes: int = 0
    stats: dict = field(default_factory=dict)

    @property
    def n_strings(self) -> int:
        return len(self.code_off) - 1

    @property
    def decoded_bytes(self) -> int:
        return int(self.stats["decoded_bytes"])


def _stats(codec, codes, code_off, dict_lens, n_escapes, decoded):
    n = int(len(codes))
    s = int(len(code_off) - 1)
    st = {"n_codes": n, "n_strings": s, "decoded_bytes": int(decoded), "n_escapes": int(n_escapes),
          "n_dict": int(len(dict_lens))}
    if n:
        st["bytes_per_code"] = decoded / n
        st["escape_share"] = (n_escapes / n) if codec == "fsst8" else 0.0
    if s:
        st["mean_string_len"] = decoded / s
    if codec == "onpair16" and n:
        used_len = dict_lens[codes]
        st["share_le8"] = float((used_len <= 8).mean())
        st["distinct_codes"] = int(len(np.unique(codes)))
    return st


def fsst_small(seed: int = 1, n_strings: int = 10_000, min_len: int = 8, max_len: int = 80,
               index_bits: int = 32) -> Column:
    text, off = printable_strings(seed, n_strings, min_len, max_len)
    db, dl = fsst_random_table(seed)
    codes, coff, esc = encode_fsst(db, dl, text, off)
    idt = np.int32 if index_bits == 32 else np.int64
    return Column("fsst_small", "fsst8", codes, coff.astype(idt), db, dl, text, off, esc,
                  _stats("fsst8", codes, coff, dl, esc, len(text)))


def fsst_logs(seed: int = 2, target_bytes: int = 1 << 30, sample_bytes: int = 1 << 20,
              threads: int | None = None, keep_text: bool = True) -> Column:
    # separate sample (different seed stream) for the table
    st, so = log_lines(seed, sample_bytes, nchunk=4, threads=threads, stream_base=SAMPLE_STREAM)
    db, dl = fsst_train(st, so, 255)
    text, off = log_lines(seed, target_bytes, threads=threads)
    codes, coff, esc = encode_fsst(db, dl, text, off, threads)
    col = Column("fsst_logs", "fsst8", codes, coff, db, dl, text if keep_text else None,
                 off if keep_text else None, esc, _stats("fsst8", codes, coff, dl, esc, len(text)))
    return col


def fsst_logs_ngram(seed: int = 2, target_bytes: int = 1 << 30, sample_bytes: int = 1 << 20,
                    threads: int | None = None, keep_text: bool = True) -> Column:
    """The log lines of fsst_logs (same seed, same text) with the table built
    as the top-255 frequent 1..8-byte n-grams of the separate 1 MiB sample
    (count x length), greedy longest-match encoded."""
    st, so = log_lines(seed, sample_bytes, nchunk=4, threads=threads, stream_base=SAMPLE_STREAM)
    db, dl = fsst_ngram_table(st, so, 255)
    text, off = log_lines(seed, target_bytes, threads=threads)
    codes, coff, esc = encode_fsst(db, dl, text, off, threads)
    return Column("fsst_logs_ngram", "fsst8", codes, coff, db, dl, text if keep_text else None,
                  off if keep_text else None, esc, _stats("fsst8", codes, coff, dl, esc, len(text)))


def onpair_urls(seed: int = 3, target_bytes: int = 1 << 30, sample_bytes: int = 4 << 20,
                threads: int | None = None, keep_text: bool = True, max_tokens: int = 65536) -> Column:
    st, so = url_strings(seed, sample_bytes, nchunk=16, threads=threads, stream_base=SAMPLE_STREAM)
    db, dl = onpair_train(st, so, max_tokens=max_tokens, tau=2, max_len=16)
    text, off = url_strings(seed, target_bytes, threads=threads)
    codes, coff, _ = encode_onpair(db, dl, text, off, threads)
    return Column("onpair_urls", "onpair16", codes, coff, db, dl, text if keep_text else None,
                  off if keep_text else None, 0, _stats("onpair16", codes, coff, dl, 0, len(text)))


def pack_codes12(codes) -> np.ndarray:
    """Pack codes < 4096 into the 12-bit stream the 12-bit decoders read:
    least significant bit first, two codes in three bytes (a storage format,
    vectorised here; the checker has its own one-code-at-a-time unpacker)."""
    c = np.asarray(codes, dtype=np.uint32)
    n = len(c)
    if n % 2:
        c = np.concatenate([c, np.zeros(1, np.uint32)])
    a, b = c[0::2], c[1::2]
    out = np.empty((len(a), 3), np.uint8)
    out[:, 0] = a & 0xFF
    out[:, 1] = ((a >> 8) & 0xF) | ((b & 0xF) << 4)
    out[:, 2] = (b >> 4) & 0xFF
    return out.reshape(-1)[: (n * 12 + 7) // 8].copy()


def _code12_column(name, codes16, coff, db, dl, text, off, keep_text) -> Column:
    st = _stats("onpair16", codes16, coff, dl, 0, len(text))
    return Column(name, "onpair12", pack_codes12(codes16), coff, db, dl, text if keep_text else None,
                  off if keep_text else None, 0, st)


def onpair12_urls(seed: int = 6, target_bytes: int = 1 << 30, sample_bytes: int = 4 << 20,
                  threads: int | None = None, keep_text: bool = True) -> Column:
    """OnPair-12: the URL / identifier strings of onpair_urls with a 4,096-token
    dictionary (tokens of 1-16 bytes) and 12-bit packed codes."""
    st, so = url_strings(seed, sample_bytes, nchunk=16, threads=threads, stream_base=SAMPLE_STREAM)
    db, dl = onpair_train(st, so, max_tokens=4096, tau=2, max_len=16)
    text, off = url_strings(seed, target_bytes, threads=threads)
    codes, coff, _ = encode_onpair(db, dl, text, off, threads)
    return _code12_column("onpair12_urls", codes, coff, db, dl, text, off, keep_text)


def fsst12_logs(seed: int = 7, target_bytes: int = 1 << 30, sample_bytes: int = 1 << 20,
                threads: int | None = None, keep_text: bool = True) -> Column:
    """FSST-12: the log lines of fsst_logs with a 4,096-symbol table of 1-8 byte
    symbols (all 256 single bytes included, so no escapes) and 12-bit packed
    codes.  It decodes through the 12-bit path like OnPair-12."""
    st, so = log_lines(seed, sample_bytes, nchunk=4, threads=threads, stream_base=SAMPLE_STREAM)
    db, dl = onpair_train(st, so, max_tokens=4096, tau=2, max_len=8)
    text, off = log_lines(seed, target_bytes, threads=threads)
    codes, coff, _ = encode_onpair(db, dl, text, off, threads)
    return _code12_column("fsst12_logs", codes, coff, db, dl, text, off, keep_text)


def random_onpair(seed: int = 33, n_codes: int = 1 << 16, n_strings: int = 1000, n_tok: int = 65536) -> Column:
    """Random full dictionary with uniform random codes (no text kept)."""
    db, dl = random_dict(seed, n_tok, 16)
    rng = np.random.default_rng(seed)
    codes = rng.integers(0, n_tok, size=n_codes, dtype=np.int64).astype(np.uint16)
    cuts = np.sort(rng.integers(0, n_codes + 1, size=n_strings - 1, dtype=np.int64))
    coff = np.concatenate([[0], cuts, [n_codes]]).astype(np.int64)
    decoded = int(dl[codes].sum(dtype=np.int64))
    return Column("random_onpair", "onpair16", codes, coff, db, dl, None, None, 0,
                  _stats("onpair16", codes, coff, dl, 0, decoded))


def batch_columns(seed: int = 4, n_cols: int = 256, min_bytes: int = 4 << 10, max_bytes: int = 64 << 20,
                  threads: int | None = None, keep_text: bool = True) -> list[Column]:
    """The batched workload: n_cols columns, decoded sizes log-uniform in
    [min_bytes, max_bytes], codecs half FSST-8 log lines and half OnPair-16
    URLs (shuffled), every column with its own dictionary trained on its own
    sample (1 MiB for FSST-8, 4 MiB for OnPair-16)."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(min_bytes), np.log(max_bytes), n_cols)).astype(np.int64)
    codecs = rng.permutation(np.array([0] * (n_cols // 2) + [1] * (n_cols - n_cols // 2)))
    cols = []
    for j in range(n_cols):
        cseed = seed * 100_003 + j
        if codecs[j] == 0:
            cols.append(fsst_logs(cseed, int(sizes[j]), 1 << 20, threads, keep_text))
        else:
            cols.append(onpair_urls(cseed, int(sizes[j]), 4 << 20, threads, keep_text))
    return cols


@dataclass
class ServePool:
    """Dictionaries and request chunks of the served workload."""
    dicts: list          # (codec, dict_bytes, dict_lens)
    chunks: list[Column]  # each encoded with dicts[chunk_dict[i]]
    chunk_dict: list[int]


def serve_pool(seed: int = 5, n_dicts: int = 32, n_chunks: int = 128, min_bytes: int = 64 << 10,
               max_bytes: int = 32 << 20, threads: int | None = None, keep_text: bool = True) -> ServePool:
    """The served workload: n_dicts dictionaries (half FSST-8 trained on log
    samples, half OnPair-16 trained on URL samples, each from its own seed) and
    a pool of request chunks with decoded sizes log-uniform in [min_bytes,
    max_bytes].  Chunk i uses dictionary k = i mod n_dicts (128 chunks give 4
    per dictionary) and is fresh text of dictionary k's seed on a random
    stream of its own: the generator draws its vocabularies from the seed, so a
    chunk comes from the distribution its dictionary was trained on, as the
    single columns pair their sample and their text."""
    rng = np.random.default_rng(seed)
    dicts = []
    for k in range(n_dicts):
        dseed = seed * 100_003 + 50_000 + k
        if k % 2 == 0:
            st, so = log_lines(dseed, 1 << 20, nchunk=4, threads=threads, stream_base=SAMPLE_STREAM)
            dicts.append(("fsst8",) + tuple(fsst_train(st, so, 255)))
        else:
            st, so = url_strings(dseed, 4 << 20, nchunk=16, threads=threads, stream_base=SAMPLE_STREAM)
            dicts.append(("onpair16",) + tuple(onpair_train(st, so, max_tokens=65536, tau=2, max_len=16)))
    sizes = np.exp(rng.uniform(np.log(min_bytes), np.log(max_bytes), n_chunks)).astype(np.int64)
    chunks, which = [], []
    for i in range(n_chunks):
        k = i % n_dicts
        codec, db, dl = dicts[k]
        dseed = seed * 100_003 + 50_000 + k
        sbase = (1 + i // n_dicts) << 20          # disjoint from the sample's streams and from each other
        if codec == "fsst8":
            text, off = log_lines(dseed, int(sizes[i]), threads=threads, stream_base=sbase)
            codes, coff, esc = encode_fsst(db, dl, text, off, threads)
        else:
            text, off = url_strings(dseed, int(sizes[i]), threads=threads, stream_base=sbase)
            codes, coff, esc = encode_onpair(db, dl, text, off, threads)
        chunks.append(Column("serve_chunk", codec, codes, coff, db, dl, text if keep_text else None,
                             off if keep_text else None, esc, _stats(codec, codes, coff, dl, esc, len(text))))
        which.append(k)
    return ServePool(dicts, chunks, which)


def column_for(name: str, **kw) -> Column:
    return {"fsst_small": fsst_small, "fsst_logs": fsst_logs, "fsst_logs_ngram": fsst_logs_ngram,
            "onpair_urls": onpair_urls,
            "random_onpair": random_onpair, "onpair12_urls": onpair12_urls, "fsst12_logs": fsst12_logs}[name](**kw)
